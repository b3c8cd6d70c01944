// kernels.hip -- gfx950 kernels of the Oregonator stepper (Sec. 2, Eq. (1)):
// forward Euler on u, v with the five-node Laplacian of u, no-flux edges.
//
//   k_step1  one step per launch, streaming: each thread owns 4 adjacent
//            cells of a row and marches down kStep1Rows rows keeping the
//            north/centre/south rows of u in registers, so u, v and phi are
//            each read from HBM once and u', v' written once (20 B per
//            FP32 cell-update, 40 B in FP64).
// The T-step kernels are in tiles_impl.h (LDS tiles, one translation unit
// per tile height) and stream.hip (row pipelines).
#include "kernels.h"
#include "tile.h"

namespace rdc {
namespace {

using namespace dev;


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
template <typename Real, bool OUT>
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
    if (OUT && a.arrival) {
        int32_t* ar = a.arrival + (int64_t)y * a.apitch + x0;
#pragma unroll
        for (int c = 0; c < 4; ++c)
            if (x0 + c < nx && ar[c] == kNever && uo.e[c] >= a.theta) ar[c] = a.step0 + 1;
    }
    if (OUT && a.tl && (a.step0 + 1) % a.tl_rate == 0) {
        Real* tp = a.tl + (int64_t)y * a.tpitch + x0;
#pragma unroll
        for (int c = 0; c < 4; ++c)
            if (x0 + c < nx && uo.e[c] > tp[c]) tp[c] = uo.e[c];
    }
}

// Each lane owns 4 adjacent cells of a row; a wave covers 256 columns.  The
// block marches down kStep1Rows rows, two per iteration (all loads of the
// pair issued before any arithmetic), keeping the north / centre / south rows
// of u in registers; east / west neighbours cross lanes by DPP and only the
// wave's edge lanes read one extra cell.  Lanes past the east edge still run
// (the lane exchange needs the whole wave) but load through bounds-checked
// row resources and store nothing.
template <typename Real, bool OUT>
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
        step1_row<Real, OUT>(a, y, x0, lane, rb, un, uc, us, vc, pc, bad);
        if (two) step1_row<Real, OUT>(a, y1, x0, lane, rb, uc, us, us2, vc1, pc1, bad);
        un = us;
        uc = us2;
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

// tl := u, row by row (pitches may differ).
template <typename Real>
__global__ __launch_bounds__(256) void k_copy_plane(const Real* u, int64_t pitch, int nx, int ny,
                                                    Real* tl, int64_t tpitch) {
    const int64_t n = (int64_t)nx * ny;
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * blockDim.x) {
        const int64_t y = j / nx, x = j % nx;
        tl[y * tpitch + x] = u[y * pitch + x];
    }
}

template <typename Real>
hipError_t step1_impl(const StepArgs<Real>& a, hipStream_t s) {
    const dim3 grid((a.nx + kStep1Threads * 4 - 1) / (kStep1Threads * 4),
                    (a.ny + kStep1Rows - 1) / kStep1Rows);
    if (a.arrival || a.tl)
        hipLaunchKernelGGL((k_step1<Real, true>), grid, dim3(kStep1Threads), 0, s, a);
    else
        hipLaunchKernelGGL((k_step1<Real, false>), grid, dim3(kStep1Threads), 0, s, a);
    return hipGetLastError();
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
hipError_t copy_plane_impl(const Real* u, int64_t pitch, int nx, int ny, Real* tl,
                           int64_t tpitch, hipStream_t s) {
    const int64_t n = (int64_t)nx * ny;
    const int64_t blocks = (n + 255) / 256 < 65536 ? (n + 255) / 256 : 65536;
    hipLaunchKernelGGL((k_copy_plane<Real>), dim3((unsigned)blocks), dim3(256), 0, s, u, pitch,
                       nx, ny, tl, tpitch);
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
int tile_rows_default() { return 56; }
int max_rows() { return 65535 * kStep1Rows; }

// Tile heights are 8 rows per wave times R; each R's kernels live in their
// own translation unit (tiles_r<R>.hip).
template <typename Real>
hipError_t stepT_any(const StepArgs<Real>& a, int T, int rows, hipStream_t s) {
    switch (rows) {
        case 48: return launch_tiles<6>(a, T, s);
        case 56: return launch_tiles<7>(a, T, s);
        case 64: return launch_tiles<8>(a, T, s);
        case 80: return launch_tiles<10>(a, T, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_stepT(const StepArgs<float>& a, int T, int rows, hipStream_t s) {
    return stepT_any(a, T, rows, s);
}
hipError_t launch_stepT(const StepArgs<double>& a, int T, int rows, hipStream_t s) {
    return stepT_any(a, T, rows, s);
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
hipError_t launch_copy_plane(const float* u, int64_t pitch, int nx, int ny, float* tl,
                             int64_t tpitch, hipStream_t s) {
    return copy_plane_impl(u, pitch, nx, ny, tl, tpitch, s);
}
hipError_t launch_copy_plane(const double* u, int64_t pitch, int nx, int ny, double* tl,
                             int64_t tpitch, hipStream_t s) {
    return copy_plane_impl(u, pitch, nx, ny, tl, tpitch, s);
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
