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

// ---------------------------------------------------------------- lane exchange, buffers

// Lane i receives lane i-1's x: DPP wave_shr:1.  Lane 0 has no source and
// reads 0 (bound_ctrl); callers overwrite or never use that lane's value,
// which lets the compiler fold the move into the consuming add.
__device__ __forceinline__ float from_west_lane(float x) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0x138, 0xf, 0xf, true));
}
// Lane i receives lane i+1's x: DPP wave_shl:1 (lane 63 reads 0).
__device__ __forceinline__ float from_east_lane(float x) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0x130, 0xf, 0xf, true));
}
__device__ __forceinline__ double from_west_lane(double x) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), 0x138, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), 0x138, 0xf, 0xf, true);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double from_east_lane(double x) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), 0x130, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), 0x130, 0xf, 0xf, true);
    return __hiloint2double(hi, lo);
}

// Cache policy of the streaming stores of u' and v' (buffer "aux" bits).
// The default 2 sets the non-temporal hint: the next step reads these planes
// back from HBM long after they leave the caches.  A build-time tunable.
#ifndef RDC_STORE_AUX
#define RDC_STORE_AUX 2
#endif
constexpr int kStoreAux = RDC_STORE_AUX;

// Buffer resource covering one row of `bytes` bytes from `row` (raw, 32-bit
// elements): loads and stores through it take a 32-bit lane offset against a
// scalar base, and any offset past the row reads 0 / drops the write instead
// of touching memory outside it.
template <typename Real>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_rsrc(const Real* row, int bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<Real*>(row), (short)0, bytes, 0x00020000);
}
__device__ __forceinline__ float4 buf_load4(__amdgpu_buffer_rsrc_t r, int byte_off) {
    const auto v = __builtin_amdgcn_raw_buffer_load_b128(r, byte_off, 0, 0);
    return make_float4(__uint_as_float(v[0]), __uint_as_float(v[1]), __uint_as_float(v[2]),
                       __uint_as_float(v[3]));
}
__device__ __forceinline__ float buf_load1(__amdgpu_buffer_rsrc_t r, int byte_off) {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, byte_off, 0, 0));
}
__device__ __forceinline__ void buf_store4(__amdgpu_buffer_rsrc_t r, int byte_off, float a0,
                                           float a1, float a2, float a3) {
    __attribute__((ext_vector_type(4))) unsigned int v;
    v[0] = __float_as_uint(a0);
    v[1] = __float_as_uint(a1);
    v[2] = __float_as_uint(a2);
    v[3] = __float_as_uint(a3);
    __builtin_amdgcn_raw_buffer_store_b128(v, r, byte_off, 0, kStoreAux);
}
__device__ __forceinline__ void buf_store1(__amdgpu_buffer_rsrc_t r, int byte_off, float a) {
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(a), r, byte_off, 0, kStoreAux);
}

// 4 consecutive cells of a row through a row resource (float: one 16-byte
// access; double: two).
__device__ __forceinline__ V4<float> row_load4(__amdgpu_buffer_rsrc_t r, int x, float) {
    const float4 t = buf_load4(r, 4 * x);
    return {{t.x, t.y, t.z, t.w}};
}
__device__ __forceinline__ V4<double> row_load4(__amdgpu_buffer_rsrc_t r, int x, double) {
    const auto a = __builtin_amdgcn_raw_buffer_load_b128(r, 8 * x, 0, 0);
    const auto b = __builtin_amdgcn_raw_buffer_load_b128(r, 8 * x + 16, 0, 0);
    return {{__hiloint2double(a[1], a[0]), __hiloint2double(a[3], a[2]),
             __hiloint2double(b[1], b[0]), __hiloint2double(b[3], b[2])}};
}
__device__ __forceinline__ float row_load1(__amdgpu_buffer_rsrc_t r, int x, float) {
    return buf_load1(r, 4 * x);
}
__device__ __forceinline__ double row_load1(__amdgpu_buffer_rsrc_t r, int x, double) {
    const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, 8 * x, 0, 0);
    return __hiloint2double(v[1], v[0]);
}
__device__ __forceinline__ void row_store4(__amdgpu_buffer_rsrc_t r, int x, const V4<float>& v) {
    buf_store4(r, 4 * x, v.e[0], v.e[1], v.e[2], v.e[3]);
}
__device__ __forceinline__ void row_store4(__amdgpu_buffer_rsrc_t r, int x, const V4<double>& v) {
    __attribute__((ext_vector_type(4))) unsigned int a, b;
    a[0] = __double2loint(v.e[0]); a[1] = __double2hiint(v.e[0]);
    a[2] = __double2loint(v.e[1]); a[3] = __double2hiint(v.e[1]);
    b[0] = __double2loint(v.e[2]); b[1] = __double2hiint(v.e[2]);
    b[2] = __double2loint(v.e[3]); b[3] = __double2hiint(v.e[3]);
    __builtin_amdgcn_raw_buffer_store_b128(a, r, 8 * x, 0, kStoreAux);
    __builtin_amdgcn_raw_buffer_store_b128(b, r, 8 * x + 16, 0, kStoreAux);
}
__device__ __forceinline__ void row_store1(__amdgpu_buffer_rsrc_t r, int x, float v) {
    buf_store1(r, 4 * x, v);
}
__device__ __forceinline__ void row_store1(__amdgpu_buffer_rsrc_t r, int x, double v) {
    __attribute__((ext_vector_type(2))) unsigned int a;
    a[0] = __double2loint(v);
    a[1] = __double2hiint(v);
    __builtin_amdgcn_raw_buffer_store_b64(a, r, 8 * x, 0, kStoreAux);
}

// ---------------------------------------------------------------- one step

#ifndef RDC_STEP1_ROWS
#define RDC_STEP1_ROWS 16
#endif
constexpr int kStep1Threads = 256;
constexpr int kStep1Rows = RDC_STEP1_ROWS;   // rows one block marches down

// Each lane owns 4 adjacent cells of a row; a wave covers 256 columns.  The
// block marches down kStep1Rows rows keeping the north / centre / south rows
// of u in registers; east / west neighbours cross lanes by DPP and only the
// wave's edge lanes read one extra cell.  Lanes past the east edge still run
// (the lane exchange needs the whole wave) but load through bounds-checked
// row resources and store nothing.
// One output row: north / centre / south rows of u (this lane's 4 cells),
// v and phi of the centre row; east / west across lanes, edge lanes load.
template <typename Real, bool ARR>
__device__ __forceinline__ void step1_row(const StepArgs<Real>& a, int y, int x0, int lane,
                                          int rb, const V4<Real>& un, const V4<Real>& uc,
                                          const V4<Real>& us, const V4<Real>& vc,
                                          const V4<Real>& pc, bool& bad) {
    const int nx = a.nx;
    const int64_t off = (int64_t)y * a.pitch;
    Real west = from_west_lane(uc.e[3]);
    Real east = from_east_lane(uc.e[0]);
    if (lane == 0) west = row_load1(row_rsrc(a.u + off, rb), x0 - 1, Real());
    if (lane == 63) east = row_load1(row_rsrc(a.u + off, rb), x0 + 4, Real());
    if (x0 == 0) west = uc.e[0];                                      // west edge: mirror
    V4<Real> uo, vo;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const Real W = (c == 0) ? west : uc.e[c - 1];
        Real E = (c == 3) ? east : uc.e[c + 1];
        if (x0 + c + 1 >= nx) E = uc.e[c];                            // east edge: mirror
        cell_update(uc.e[c], W, E, un.e[c], us.e[c], vc.e[c], scaled_phi(pc.e[c], a.k), a.k,
                    uo.e[c], vo.e[c]);
    }
    if (x0 >= nx) return;
    const auto ro = row_rsrc(a.u_out + off, rb);
    const auto rv = row_rsrc(a.v_out + off, rb);
    if (x0 + 3 < nx) {
        row_store4(ro, x0, uo);
        row_store4(rv, x0, vo);
#pragma unroll
        for (int c = 0; c < 4; ++c) bad |= !finite2(uo.e[c], vo.e[c]);
    } else {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            if (x0 + c < nx) {
                row_store1(ro, x0 + c, uo.e[c]);
                row_store1(rv, x0 + c, vo.e[c]);
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
}

// Each lane owns 4 adjacent cells of a row; a wave covers 256 columns.  The
// block marches down kStep1Rows rows, two per iteration (all loads of the
// pair issued before any arithmetic), keeping the north / centre / south rows
// of u in registers; east / west neighbours cross lanes by DPP and only the
// wave's edge lanes read one extra cell.  Lanes past the east edge still run
// (the lane exchange needs the whole wave) but load through bounds-checked
// row resources and store nothing.
template <typename Real, bool ARR>
__global__ __launch_bounds__(kStep1Threads) void k_step1(StepArgs<Real> a) {
    const int x0 = (blockIdx.x * kStep1Threads + threadIdx.x) * 4;
    const int lane = threadIdx.x & 63;
    const int ny = a.ny;
    const int64_t P = a.pitch;
    const int rb = static_cast<int>(P * sizeof(Real));
    const int y0 = blockIdx.y * kStep1Rows;
    const int yend = min(y0 + kStep1Rows, ny);
    auto load = [&](const Real* plane, int y) __attribute__((always_inline)) {
        return row_load4(row_rsrc(plane + (int64_t)y * P, rb), x0, Real());
    };

    V4<Real> un = load(a.u, y0 > 0 ? y0 - 1 : 0);
    V4<Real> uc = load(a.u, y0);
    bool bad = false;
    for (int y = y0; y < yend; y += 2) {
        const bool two = y + 1 < yend;
        const int y1 = two ? y + 1 : y;
        const V4<Real> us = load(a.u, y + 1 < ny ? y + 1 : y);       // south, mirrored
        const V4<Real> us2 = load(a.u, y1 + 1 < ny ? y1 + 1 : y1);
        const V4<Real> vc = load(a.v, y), pc = load(a.phi, y);
        const V4<Real> vc1 = load(a.v, y1), pc1 = load(a.phi, y1);
        step1_row<Real, ARR>(a, y, x0, lane, rb, un, uc, us, vc, pc, bad);
        if (two) step1_row<Real, ARR>(a, y1, x0, lane, rb, uc, us, us2, vc1, pc1, bad);
        un = us;
        uc = us2;
    }
    if (bad) *a.flag = 1;
}

// ---------------------------------------------------------------- T steps

constexpr int kTileCols = 256;  // 64 lanes x 4 cells: one wave per tile row
constexpr int kTileWaves = 8;

// Two 8-wave workgroups per CU (4 waves per SIMD, a 128-VGPR budget) when
// the tile's LDS allows it; the second launch-bounds argument is the minimum
// number of waves per SIMD.
// (The arrival-tracking variant keeps 4R more registers and is not held to it.)
template <int R, bool ARR>
constexpr int tile_waves_per_simd() { return (R <= 8 && !ARR) ? 4 : 2; }

template <int T, int R, bool ARR>
__global__ __launch_bounds__(kTileWaves * 64, (tile_waves_per_simd<R, ARR>())) void k_stepT(StepArgs<float> a, int tiles_x,
                                                          int ntiles, int per_xcd) {
    constexpr int HX = (T + 3) & ~3;          // column halo, rounded to whole lanes
    constexpr int BX = kTileCols - 2 * HX;    // output columns per tile
    constexpr int EY = kTileWaves * R;        // loaded rows
    constexpr int BY = EY - 2 * T;            // output rows per tile
    static_assert(BY > 0 && BX > 0, "tile too small for T");
    __shared__ float4 lds[EY][64];

    // Workgroups are dealt to the 8 XCDs round-robin; renumber so that each
    // XCD walks a contiguous run of the row-major tile order: concurrent
    // tiles of one XCD share halo cells in its L2, and their loads sweep long
    // contiguous row segments.  (A column-major walk measured slower.)
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
    int xb[4];                                // byte offsets of this lane's 4 columns
#pragma unroll
    for (int c = 0; c < 4; ++c) xb[c] = 4 * reflect_index(gx + c, nx);
    const int row_bytes = static_cast<int>(P * 4);

    float vr[R][4], pr[R][4], un[R][4];
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int r = w + kTileWaves * k;
        const int64_t off = (int64_t)reflect_index(gy0 + r, ny) * P;
        const auto ru = row_rsrc(a.u + off, row_bytes);
        const auto rv = row_rsrc(a.v + off, row_bytes);
        const auto rp = row_rsrc(a.phi + off, row_bytes);
        float4 uu, vv, pp;
        if (fast_x) {
            uu = buf_load4(ru, xb[0]);
            vv = buf_load4(rv, xb[0]);
            pp = buf_load4(rp, xb[0]);
        } else {
            uu = make_float4(buf_load1(ru, xb[0]), buf_load1(ru, xb[1]), buf_load1(ru, xb[2]),
                             buf_load1(ru, xb[3]));
            vv = make_float4(buf_load1(rv, xb[0]), buf_load1(rv, xb[1]), buf_load1(rv, xb[2]),
                             buf_load1(rv, xb[3]));
            pp = make_float4(buf_load1(rp, xb[0]), buf_load1(rp, xb[1]), buf_load1(rp, xb[2]),
                             buf_load1(rp, xb[3]));
        }
        lds[r][lane] = uu;
        vr[k][0] = vv.x; vr[k][1] = vv.y; vr[k][2] = vv.z; vr[k][3] = vv.w;
        pr[k][0] = scaled_phi(pp.x, a.k);
        pr[k][1] = scaled_phi(pp.y, a.k);
        pr[k][2] = scaled_phi(pp.z, a.k);
        pr[k][3] = scaled_phi(pp.w, a.k);
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
        // Valid rows at sub-step t: [t, EY-t).  The condition is uniform
        // across a wave (rows are dealt to waves round-robin).
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
        const int xo = 4 * gx;   // gx >= 0 for output lanes
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int r = w + kTileWaves * k;
            const int gy = gy0 + r;
            if (r < T || r >= EY - T || gy >= ny) continue;
            const int64_t off = (int64_t)gy * P;
            const auto ru = row_rsrc(a.u_out + off, row_bytes);
            const auto rv = row_rsrc(a.v_out + off, row_bytes);
            if (gx + 3 < nx) {
                buf_store4(ru, xo, un[k][0], un[k][1], un[k][2], un[k][3]);
                buf_store4(rv, xo, vr[k][0], vr[k][1], vr[k][2], vr[k][3]);
#pragma unroll
                for (int c = 0; c < 4; ++c) bad |= !finite2(un[k][c], vr[k][c]);
            } else {
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    if (gx + c < nx) {
                        buf_store1(ru, xo + 4 * c, un[k][c]);
                        buf_store1(rv, xo + 4 * c, vr[k][c]);
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

constexpr int kCopyUnroll = 4;

// Streaming copy: each thread moves kCopyUnroll 16-byte words, all loads
// issued before the stores.
__global__ __launch_bounds__(256) void k_copy16(const float4* __restrict__ src,
                                                float4* __restrict__ dst, int64_t n) {
    const int64_t base = (int64_t)blockIdx.x * 256 * kCopyUnroll + threadIdx.x;
    float4 t[kCopyUnroll];
#pragma unroll
    for (int i = 0; i < kCopyUnroll; ++i) {
        const int64_t j = base + i * 256;
        if (j < n) t[i] = src[j];
    }
#pragma unroll
    for (int i = 0; i < kCopyUnroll; ++i) {
        const int64_t j = base + i * 256;
        if (j < n) dst[j] = t[i];
    }
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

bool tile_rows_supported(int rows) {
    return rows == 48 || rows == 56 || rows == 64 || rows == 80;
}
int tile_rows_default() { return 80; }

hipError_t launch_stepT(const StepArgs<float>& a, int T, int rows, hipStream_t s) {
    switch (rows) {
        case 48: return stepT_rows<6>(a, T, s);
        case 56: return stepT_rows<7>(a, T, s);
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
    const int64_t blocks = (n16 + 256 * kCopyUnroll - 1) / (256 * kCopyUnroll);
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_copy16, dim3((unsigned)blocks), dim3(256), 0, s,
                       static_cast<const float4*>(src), static_cast<float4*>(dst), n16);
    return hipGetLastError();
}

}  // namespace rdc
