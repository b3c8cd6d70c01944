// kernels.hip -- gfx950 kernels of the Oregonator stepper (Sec. 2, Eq. (1)):
// forward Euler on u, v with the five-node Laplacian of u, no-flux edges.
//
//   k_step1  one step per launch, streaming: each thread owns 4 adjacent
//            cells of a row and marches down kStep1Rows rows keeping the
//            north/centre/south rows of u in registers, so u, v and phi are
//            each read from HBM once and u', v' written once (20 B per
//            FP32 cell-update, 40 B in FP64).
//   k_stepT  T steps per launch (FP32): a workgroup of 8 waves loads a
//            256-column by EY-row tile of u (into LDS), v and phi (into
//            registers) including a halo mirrored at the domain edges, runs T
//            steps on chip with the valid region shrinking by one cell per
//            step, and writes the (256-2*HX) x (EY-2*T) interior.  Each wave
//            owns whole 256-cell tile rows (64 lanes x 4 cells), so the east /
//            west neighbours cross lanes by DPP row shifts and only the
//            north / south rows go through LDS.
#include "kernels.h"

namespace rdc {
namespace {

template <typename Real>
struct V4 {
    Real e[4];
};

__device__ __forceinline__ V4<float> load4(const float* p) {
    const float4 t = *reinterpret_cast<const float4*>(p);
    return {{t.x, t.y, t.z, t.w}};
}
__device__ __forceinline__ V4<double> load4(const double* p) {
    const double2 a = reinterpret_cast<const double2*>(p)[0];
    const double2 b = reinterpret_cast<const double2*>(p)[1];
    return {{a.x, a.y, b.x, b.y}};
}
__device__ __forceinline__ void store4(float* p, const V4<float>& v) {
    *reinterpret_cast<float4*>(p) = make_float4(v.e[0], v.e[1], v.e[2], v.e[3]);
}
__device__ __forceinline__ void store4(double* p, const V4<double>& v) {
    reinterpret_cast<double2*>(p)[0] = make_double2(v.e[0], v.e[1]);
    reinterpret_cast<double2*>(p)[1] = make_double2(v.e[2], v.e[3]);
}

__device__ __forceinline__ bool finite2(float a, float b) {
    return __builtin_isfinite(a) && __builtin_isfinite(b);
}
__device__ __forceinline__ bool finite2(double a, double b) {
    return __builtin_isfinite(a) && __builtin_isfinite(b);
}

// ---------------------------------------------------------------- one step

constexpr int kStep1Threads = 256;
constexpr int kStep1Rows = 16;

template <typename Real, bool ARR>
__global__ __launch_bounds__(kStep1Threads) void k_step1(StepArgs<Real> a) {
    const int x0 = (blockIdx.x * kStep1Threads + threadIdx.x) * 4;
    if (x0 >= a.nx) return;
    const int nx = a.nx, ny = a.ny;
    const int64_t P = a.pitch;
    const int y0 = blockIdx.y * kStep1Rows;
    const int yend = min(y0 + kStep1Rows, ny);
    const Real* __restrict__ u = a.u;

    V4<Real> un = load4(u + (int64_t)(y0 > 0 ? y0 - 1 : 0) * P + x0);  // north row
    V4<Real> uc = load4(u + (int64_t)y0 * P + x0);                     // centre row
    bool bad = false;
    for (int y = y0; y < yend; ++y) {
        const int ys = (y + 1 < ny) ? y + 1 : y;                       // south, mirrored
        const V4<Real> us = load4(u + (int64_t)ys * P + x0);
        const Real* row = u + (int64_t)y * P;
        const Real west = (x0 > 0) ? row[x0 - 1] : uc.e[0];
        const Real east = (x0 + 4 < nx) ? row[x0 + 4] : uc.e[3];
        const V4<Real> vc = load4(a.v + (int64_t)y * P + x0);
        const V4<Real> pc = load4(a.phi + (int64_t)y * P + x0);
        V4<Real> uo, vo;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const Real W = (c == 0) ? west : uc.e[c - 1];
            Real E = (c == 3) ? east : uc.e[c + 1];
            if (x0 + c + 1 >= nx) E = uc.e[c];
            cell_update(uc.e[c], W, E, un.e[c], us.e[c], vc.e[c], pc.e[c], a.k, uo.e[c], vo.e[c]);
        }
        Real* uout = a.u_out + (int64_t)y * P + x0;
        Real* vout = a.v_out + (int64_t)y * P + x0;
        if (x0 + 3 < nx) {
            store4(uout, uo);
            store4(vout, vo);
#pragma unroll
            for (int c = 0; c < 4; ++c) bad |= !finite2(uo.e[c], vo.e[c]);
        } else {
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                if (x0 + c < nx) {
                    uout[c] = uo.e[c];
                    vout[c] = vo.e[c];
                    bad |= !finite2(uo.e[c], vo.e[c]);
                }
            }
        }
        if (ARR) {
            int32_t* ar = a.arrival + (int64_t)y * a.apitch + x0;
#pragma unroll
            for (int c = 0; c < 4; ++c)
                if (x0 + c < nx && ar[c] == kNever && uo.e[c] >= a.theta) ar[c] = a.step0 + 1;
        }
        un = uc;
        uc = us;
    }
    if (bad) *a.flag = 1;
}

// ---------------------------------------------------------------- T steps

constexpr int kTileCols = 256;  // 64 lanes x 4 cells: one wave per tile row
constexpr int kTileWaves = 8;

// Lane i receives lane i-1's x (lane 0 keeps its own): DPP wave_shr:1.
__device__ __forceinline__ float from_west_lane(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(x), __float_as_int(x),
                                                      0x138, 0xf, 0xf, false));
}
// Lane i receives lane i+1's x (lane 63 keeps its own): DPP wave_shl:1.
__device__ __forceinline__ float from_east_lane(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(x), __float_as_int(x),
                                                      0x130, 0xf, 0xf, false));
}

template <int T, int R, bool ARR>
__global__ __launch_bounds__(kTileWaves * 64) void k_stepT(StepArgs<float> a, int tiles_x,
                                                          int ntiles, int per_xcd) {
    constexpr int HX = (T + 3) & ~3;          // column halo, rounded to whole lanes
    constexpr int BX = kTileCols - 2 * HX;    // output columns per tile
    constexpr int EY = kTileWaves * R;        // loaded rows
    constexpr int BY = EY - 2 * T;            // output rows per tile
    static_assert(BY > 0 && BX > 0, "tile too small for T");
    __shared__ float4 lds[EY][64];

    // Workgroups are dealt to the 8 XCDs round-robin; renumber so that each
    // XCD walks a contiguous run of the row-major tile order and the halo
    // rows two neighbouring tiles share stay in one XCD's L2.
    const int b = blockIdx.x;
    const int tile = (b & 7) * per_xcd + (b >> 3);
    if (tile >= ntiles) return;
    const int tx = tile % tiles_x, ty = tile / tiles_x;
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nx = a.nx, ny = a.ny;
    const int64_t P = a.pitch;
    const int gx = tx * BX - HX + 4 * lane;   // first global column of this lane
    const int gy0 = ty * BY - T;              // global row of tile row 0
    const bool fast_x = gx >= 0 && gx + 3 < nx;
    int xs[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) xs[c] = reflect_index(gx + c, nx);

    float vr[R][4], pr[R][4], un[R][4];
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int r = w + kTileWaves * k;
        const int64_t off = (int64_t)reflect_index(gy0 + r, ny) * P;
        float4 uu, vv, pp;
        if (fast_x) {
            uu = *reinterpret_cast<const float4*>(a.u + off + gx);
            vv = *reinterpret_cast<const float4*>(a.v + off + gx);
            pp = *reinterpret_cast<const float4*>(a.phi + off + gx);
        } else {
            uu = make_float4(a.u[off + xs[0]], a.u[off + xs[1]], a.u[off + xs[2]], a.u[off + xs[3]]);
            vv = make_float4(a.v[off + xs[0]], a.v[off + xs[1]], a.v[off + xs[2]], a.v[off + xs[3]]);
            pp = make_float4(a.phi[off + xs[0]], a.phi[off + xs[1]], a.phi[off + xs[2]],
                             a.phi[off + xs[3]]);
        }
        lds[r][lane] = uu;
        vr[k][0] = vv.x; vr[k][1] = vv.y; vr[k][2] = vv.z; vr[k][3] = vv.w;
        pr[k][0] = pp.x; pr[k][1] = pp.y; pr[k][2] = pp.z; pr[k][3] = pp.w;
    }

    // Output cells: rows [T, EY-T), lanes [HX/4, 64-HX/4), inside the grid.
    const bool out_lane = lane >= HX / 4 && lane < 64 - HX / 4;
    int ar[ARR ? R : 1][4];
    if (ARR) {
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int r = w + kTileWaves * k;
            const int gy = gy0 + r;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const bool in = out_lane && r >= T && r < EY - T && gy < ny && gx + c < nx;
                ar[k][c] = in ? a.arrival[(int64_t)gy * a.apitch + gx + c] : 0;
            }
        }
    }
    __syncthreads();

#pragma unroll
    for (int t = 1; t <= T; ++t) {
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int r = w + kTileWaves * k;
            if (r >= t && r < EY - t) {
                const float4 c = lds[r][lane];
                const float4 n = lds[r - 1][lane];
                const float4 s = lds[r + 1][lane];
                const float west = from_west_lane(c.w);
                const float east = from_east_lane(c.x);
                cell_update(c.x, west, c.y, n.x, s.x, vr[k][0], pr[k][0], a.k, un[k][0], vr[k][0]);
                cell_update(c.y, c.x, c.z, n.y, s.y, vr[k][1], pr[k][1], a.k, un[k][1], vr[k][1]);
                cell_update(c.z, c.y, c.w, n.z, s.z, vr[k][2], pr[k][2], a.k, un[k][2], vr[k][2]);
                cell_update(c.w, c.z, east, n.w, s.w, vr[k][3], pr[k][3], a.k, un[k][3], vr[k][3]);
                if (ARR && r >= T && r < EY - T) {
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        if (ar[k][e] == kNever && un[k][e] >= a.theta) ar[k][e] = a.step0 + t;
                }
            }
        }
        if (t < T) {
            __syncthreads();
#pragma unroll
            for (int k = 0; k < R; ++k) {
                const int r = w + kTileWaves * k;
                if (r >= t && r < EY - t)
                    lds[r][lane] = make_float4(un[k][0], un[k][1], un[k][2], un[k][3]);
            }
            __syncthreads();
        }
    }

    bool bad = false;
    if (out_lane) {
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int r = w + kTileWaves * k;
            const int gy = gy0 + r;
            if (r < T || r >= EY - T || gy >= ny) continue;
            const int64_t off = (int64_t)gy * P + gx;
            if (gx + 3 < nx) {
                *reinterpret_cast<float4*>(a.u_out + off) =
                    make_float4(un[k][0], un[k][1], un[k][2], un[k][3]);
                *reinterpret_cast<float4*>(a.v_out + off) =
                    make_float4(vr[k][0], vr[k][1], vr[k][2], vr[k][3]);
#pragma unroll
                for (int c = 0; c < 4; ++c) bad |= !finite2(un[k][c], vr[k][c]);
            } else {
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    if (gx + c < nx) {
                        a.u_out[off + c] = un[k][c];
                        a.v_out[off + c] = vr[k][c];
                        bad |= !finite2(un[k][c], vr[k][c]);
                    }
                }
            }
            if (ARR) {
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    if (gx + c < nx) a.arrival[(int64_t)gy * a.apitch + gx + c] = ar[k][c];
            }
        }
    }
    if (bad) *a.flag = 1;
}

// ---------------------------------------------------------------- stimulation etc.

template <typename Real>
__global__ __launch_bounds__(256) void k_stimulate(Real* u, int64_t pitch, int nx, int ny, Disks d,
                                                   int32_t* arrival, int64_t apitch, int step) {
    const int i = blockIdx.x;
    if (i >= d.count) return;
    const int64_t cx = d.cx[i], cy = d.cy[i], r = d.r[i];
    const int64_t x_lo = cx - r > 0 ? cx - r : 0;
    const int64_t x_hi = cx + r < nx - 1 ? cx + r : nx - 1;
    const int64_t y_lo = cy - r > 0 ? cy - r : 0;
    const int64_t y_hi = cy + r < ny - 1 ? cy + r : ny - 1;
    if (x_hi < x_lo || y_hi < y_lo) return;
    const int64_t w = x_hi - x_lo + 1, n = w * (y_hi - y_lo + 1);
    for (int64_t j = threadIdx.x; j < n; j += blockDim.x) {
        const int64_t x = x_lo + j % w, y = y_lo + j / w;
        const int64_t dx = x - cx, dy = y - cy;
        if (dx * dx + dy * dy <= r * r) {
            u[y * pitch + x] = Real(1);
            if (arrival) {
                int32_t* p = arrival + y * apitch + x;
                if (*p == kNever) *p = step;
            }
        }
    }
}

template <typename Real>
__global__ __launch_bounds__(256) void k_arrival_init(const Real* u, int64_t pitch, int nx, int ny,
                                                      Real theta, int32_t* arrival,
                                                      int64_t apitch, int step) {
    const int64_t n = (int64_t)nx * ny;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * blockDim.x) {
        const int64_t x = j % nx, y = j / nx;
        arrival[y * apitch + x] = (u[y * pitch + x] >= theta) ? step : kNever;
    }
}

__global__ void k_clear_flag(int* flag) {
    if (threadIdx.x == 0) *flag = 0;
}

__global__ __launch_bounds__(256) void k_copy16(const float4* __restrict__ src,
                                                float4* __restrict__ dst, int64_t n) {
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * blockDim.x)
        dst[j] = src[j];
}

template <typename Real>
hipError_t step1_impl(const StepArgs<Real>& a, hipStream_t s) {
    const dim3 grid((a.nx + kStep1Threads * 4 - 1) / (kStep1Threads * 4),
                    (a.ny + kStep1Rows - 1) / kStep1Rows);
    if (a.arrival)
        hipLaunchKernelGGL((k_step1<Real, true>), grid, dim3(kStep1Threads), 0, s, a);
    else
        hipLaunchKernelGGL((k_step1<Real, false>), grid, dim3(kStep1Threads), 0, s, a);
    return hipGetLastError();
}

template <int T, int R>
hipError_t stepT_impl(const StepArgs<float>& a, hipStream_t s) {
    constexpr int HX = (T + 3) & ~3;
    constexpr int BX = kTileCols - 2 * HX;
    constexpr int BY = kTileWaves * R - 2 * T;
    const int tiles_x = (a.nx + BX - 1) / BX;
    const int tiles_y = (a.ny + BY - 1) / BY;
    const int ntiles = tiles_x * tiles_y;
    const int per_xcd = (ntiles + 7) / 8;
    const dim3 grid(8 * per_xcd), block(kTileWaves * 64);
    if (a.arrival)
        hipLaunchKernelGGL((k_stepT<T, R, true>), grid, block, 0, s, a, tiles_x, ntiles, per_xcd);
    else
        hipLaunchKernelGGL((k_stepT<T, R, false>), grid, block, 0, s, a, tiles_x, ntiles, per_xcd);
    return hipGetLastError();
}

template <int R>
hipError_t stepT_rows(const StepArgs<float>& a, int T, hipStream_t s) {
    switch (T) {
        case 2: return stepT_impl<2, R>(a, s);
        case 3: return stepT_impl<3, R>(a, s);
        case 4: return stepT_impl<4, R>(a, s);
        case 5: return stepT_impl<5, R>(a, s);
        case 6: return stepT_impl<6, R>(a, s);
        case 7: return stepT_impl<7, R>(a, s);
        case 8: return stepT_impl<8, R>(a, s);
        default: return hipErrorInvalidValue;
    }
}

template <typename Real>
hipError_t stimulate_impl(Real* u, int64_t pitch, int nx, int ny, const Disks& d,
                          int32_t* arrival, int64_t apitch, int step, hipStream_t s) {
    if (d.count <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_stimulate<Real>), dim3(d.count), dim3(256), 0, s, u, pitch, nx, ny, d,
                       arrival, apitch, step);
    return hipGetLastError();
}

template <typename Real>
hipError_t arrival_init_impl(const Real* u, int64_t pitch, int nx, int ny, Real theta,
                             int32_t* arrival, int64_t apitch, int step, hipStream_t s) {
    const int64_t n = (int64_t)nx * ny;
    const int64_t blocks = (n + 255) / 256 < 65536 ? (n + 255) / 256 : 65536;
    hipLaunchKernelGGL((k_arrival_init<Real>), dim3((unsigned)blocks), dim3(256), 0, s, u, pitch,
                       nx, ny, theta, arrival, apitch, step);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_step1(const StepArgs<float>& a, hipStream_t s) { return step1_impl(a, s); }
hipError_t launch_step1(const StepArgs<double>& a, hipStream_t s) { return step1_impl(a, s); }

bool tile_rows_supported(int rows) { return rows == 48 || rows == 64 || rows == 80; }
int tile_rows_default() { return 80; }

hipError_t launch_stepT(const StepArgs<float>& a, int T, int rows, hipStream_t s) {
    switch (rows) {
        case 48: return stepT_rows<6>(a, T, s);
        case 64: return stepT_rows<8>(a, T, s);
        case 80: return stepT_rows<10>(a, T, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_stimulate(float* u, int64_t pitch, int nx, int ny, const Disks& d,
                            int32_t* arrival, int64_t apitch, int step, hipStream_t s) {
    return stimulate_impl(u, pitch, nx, ny, d, arrival, apitch, step, s);
}
hipError_t launch_stimulate(double* u, int64_t pitch, int nx, int ny, const Disks& d,
                            int32_t* arrival, int64_t apitch, int step, hipStream_t s) {
    return stimulate_impl(u, pitch, nx, ny, d, arrival, apitch, step, s);
}

hipError_t launch_arrival_init(const float* u, int64_t pitch, int nx, int ny, float theta,
                               int32_t* arrival, int64_t apitch, int step, hipStream_t s) {
    return arrival_init_impl(u, pitch, nx, ny, theta, arrival, apitch, step, s);
}
hipError_t launch_arrival_init(const double* u, int64_t pitch, int nx, int ny, double theta,
                               int32_t* arrival, int64_t apitch, int step, hipStream_t s) {
    return arrival_init_impl(u, pitch, nx, ny, theta, arrival, apitch, step, s);
}

hipError_t launch_clear_flag(int* flag, hipStream_t s) {
    hipLaunchKernelGGL(k_clear_flag, dim3(1), dim3(64), 0, s, flag);
    return hipGetLastError();
}

hipError_t launch_copy16(const void* src, void* dst, int64_t n16, hipStream_t s) {
    if (n16 <= 0) return hipSuccess;
    const int64_t blocks = (n16 + 255) / 256 < 8192 ? (n16 + 255) / 256 : 8192;
    hipLaunchKernelGGL(k_copy16, dim3((unsigned)blocks), dim3(256), 0, s,
                       static_cast<const float4*>(src), static_cast<float4*>(dst), n16);
    return hipGetLastError();
}

}  // namespace rdc
