// tile.h -- device building blocks shared by the single-grid and batched
// kernels: vector and buffer-resource row access, DPP lane exchange, and the
// T-step LDS tile of the Oregonator stepper (Sec. 2, Eq. (1)).
#pragma once

#include <hip/hip_runtime.h>

#include "cell.h"
#include "kernels.h"

namespace rdc {
namespace dev {

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
// The FP64 one-step kernel's lane holds 32 contiguous bytes, stored as two
// 16-byte halves, so each store instruction covers every other 16 bytes of
// the wave's span.  With the non-temporal hint the cache writes such half
// lines out before the other half arrives (counters: +12% bytes written,
// 4.8 TB/s); with the default write-back policy they merge (+0.4%,
// 5.0 TB/s).  Those stores use this policy.
constexpr int kStoreAuxSplit = 0;

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
    __builtin_amdgcn_raw_buffer_store_b128(a, r, 8 * x, 0, kStoreAuxSplit);
    __builtin_amdgcn_raw_buffer_store_b128(b, r, 8 * x + 16, 0, kStoreAuxSplit);
}
__device__ __forceinline__ void row_store1(__amdgpu_buffer_rsrc_t r, int x, float v) {
    buf_store1(r, 4 * x, v);
}
__device__ __forceinline__ void row_store1(__amdgpu_buffer_rsrc_t r, int x, double v) {
    __attribute__((ext_vector_type(2))) unsigned int a;
    a[0] = __double2loint(v);
    a[1] = __double2hiint(v);
    __builtin_amdgcn_raw_buffer_store_b64(a, r, 8 * x, 0, kStoreAuxSplit);
}

constexpr int kTileCols = 256;  // 64 lanes x 4 cells: one wave per tile row
constexpr int kTileWaves = 8;

// Two 8-wave workgroups per CU (4 waves per SIMD, a 128-VGPR budget) when
// the tile's LDS allows it; the second launch-bounds argument is the minimum
// number of waves per SIMD.
// (The output variant -- arrival map and/or timelapse -- keeps up to 8R more
// registers and is not held to it.)
template <int R, bool OUT>
constexpr int tile_waves_per_simd() { return (R <= 8 && !OUT) ? 4 : 2; }

// Output tile of k_stepT / the batched kernel: BX columns by BY rows.
template <int T, int R>
struct TileGeom {
    static constexpr int HX = (T + 3) & ~3;
    static constexpr int BX = kTileCols - 2 * HX;
    static constexpr int BY = kTileWaves * R - 2 * T;
};

// T forward-Euler steps on one tile (tx, ty) of the grid described by `a`:
// load the tile with its mirrored halo, run the sub-steps on chip, store the
// interior.  Called by one 512-thread workgroup; `lds` is that workgroup's
// tile of u.
template <int T, int R, bool OUT>
__device__ __forceinline__ void step_tile(const StepArgs<float>& a, int tx, int ty,
                                          float4 (&lds)[kTileWaves * R][64]) {
    constexpr int HX = (T + 3) & ~3;          // column halo, rounded to whole lanes
    constexpr int BX = kTileCols - 2 * HX;    // output columns per tile
    constexpr int EY = kTileWaves * R;        // loaded rows
    constexpr int BY = EY - 2 * T;            // output rows per tile
    static_assert(BY > 0 && BX > 0, "tile too small for T");
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
    // The output variant carries their arrival times and timelapse maxima
    // through the sub-steps in registers.
    const bool out_lane = lane >= HX / 4 && lane < 64 - HX / 4;
    int ar[OUT ? R : 1][4];
    float tm[OUT ? R : 1][4];
    if (OUT) {
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int r = w + kTileWaves * k;
            const int gy = gy0 + r;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const bool in = out_lane && r >= T && r < EY - T && gy < ny && gx + c < nx;
                ar[k][c] = in && a.arrival ? a.arrival[(int64_t)gy * a.apitch + gx + c] : 0;
                tm[k][c] = in && a.tl ? a.tl[(int64_t)gy * a.tpitch + gx + c] : 0.0f;
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
                // West and east enter the update as a sum.  Each lane shift
                // sits right before the update that takes it: the compiler
                // folds a shift into its add only a few instructions away.
                const float west = from_west_lane(c.w);
                cell_update(c.x, c.y, west, n.x, s.x, vr[k][0], pr[k][0], a.k, un[k][0], vr[k][0]);
                cell_update(c.y, c.x, c.z, n.y, s.y, vr[k][1], pr[k][1], a.k, un[k][1], vr[k][1]);
                cell_update(c.z, c.y, c.w, n.z, s.z, vr[k][2], pr[k][2], a.k, un[k][2], vr[k][2]);
                const float east = from_east_lane(c.x);
                cell_update(c.w, c.z, east, n.w, s.w, vr[k][3], pr[k][3], a.k, un[k][3], vr[k][3]);
                if (OUT && r >= T && r < EY - T) {
                    if (a.arrival) {
#pragma unroll
                        for (int e = 0; e < 4; ++e)
                            if (ar[k][e] == kNever && un[k][e] >= a.theta) ar[k][e] = a.step0 + t;
                    }
                    if (a.tl && (a.step0 + t) % a.tl_rate == 0) {
#pragma unroll
                        for (int e = 0; e < 4; ++e)
                            if (un[k][e] > tm[k][e]) tm[k][e] = un[k][e];
                    }
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
            if (OUT && a.arrival) {
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    if (gx + c < nx) a.arrival[(int64_t)gy * a.apitch + gx + c] = ar[k][c];
            }
            if (OUT && a.tl) {
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    if (gx + c < nx) a.tl[(int64_t)gy * a.tpitch + gx + c] = tm[k][c];
            }
        }
    }
    if (bad) *a.flag = 1;
}


// ---------------------------------------------------------------- FP64 T-step tile

// The FP64 variant of step_tile: each lane owns 2 adjacent cells (16 bytes)
// of a row, so a wave covers 128 columns and an LDS row is 1 KB as in FP32;
// the column halo is T rounded up to whole lanes.  Same per-cell update as
// the one-step FP64 kernel, so every launch shape is bit-identical to it.
constexpr int kTileCols64 = 128;

template <int T, int R>
struct TileGeom64 {
    static constexpr int HX = (T + 1) & ~1;
    static constexpr int BX = kTileCols64 - 2 * HX;
    static constexpr int BY = kTileWaves * R - 2 * T;
};

__device__ __forceinline__ double2 buf_load2d(__amdgpu_buffer_rsrc_t r, int byte_off) {
    const auto v = __builtin_amdgcn_raw_buffer_load_b128(r, byte_off, 0, 0);
    return make_double2(__hiloint2double(v[1], v[0]), __hiloint2double(v[3], v[2]));
}
__device__ __forceinline__ double buf_load1d(__amdgpu_buffer_rsrc_t r, int byte_off) {
    const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, byte_off, 0, 0);
    return __hiloint2double(v[1], v[0]);
}
__device__ __forceinline__ void buf_store2d(__amdgpu_buffer_rsrc_t r, int byte_off, double a0,
                                            double a1) {
    __attribute__((ext_vector_type(4))) unsigned int v;
    v[0] = __double2loint(a0);
    v[1] = __double2hiint(a0);
    v[2] = __double2loint(a1);
    v[3] = __double2hiint(a1);
    __builtin_amdgcn_raw_buffer_store_b128(v, r, byte_off, 0, kStoreAux);
}
__device__ __forceinline__ void buf_store1d(__amdgpu_buffer_rsrc_t r, int byte_off, double a) {
    __attribute__((ext_vector_type(2))) unsigned int v;
    v[0] = __double2loint(a);
    v[1] = __double2hiint(a);
    __builtin_amdgcn_raw_buffer_store_b64(v, r, byte_off, 0, kStoreAux);
}

template <int T, int R, bool OUT>
__device__ __forceinline__ void step_tile64(const StepArgs<double>& a, int tx, int ty,
                                            double2 (&lds)[kTileWaves * R][64]) {
    using G = TileGeom64<T, R>;
    constexpr int HX = G::HX, BX = G::BX;
    constexpr int EY = kTileWaves * R;
    static_assert(G::BY > 0 && BX > 0, "tile too small for T");
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nx = a.nx, ny = a.ny;
    const int64_t P = a.pitch;
    const int gx = tx * BX - HX + 2 * lane;   // first global column of this lane
    const int gy0 = ty * G::BY - T;           // global row of tile row 0
    const bool fast_x = gx >= 0 && gx + 1 < nx;
    int xb[2];                                // byte offsets of this lane's 2 columns
#pragma unroll
    for (int c = 0; c < 2; ++c) xb[c] = 8 * reflect_index(gx + c, nx);
    const int row_bytes = static_cast<int>(P * 8);

    double vr[R][2], pr[R][2], un[R][2];
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int r = w + kTileWaves * k;
        const int64_t off = (int64_t)reflect_index(gy0 + r, ny) * P;
        const auto ru = row_rsrc(a.u + off, row_bytes);
        const auto rv = row_rsrc(a.v + off, row_bytes);
        const auto rp = row_rsrc(a.phi + off, row_bytes);
        double2 uu, vv, pp;
        if (fast_x) {
            uu = buf_load2d(ru, xb[0]);
            vv = buf_load2d(rv, xb[0]);
            pp = buf_load2d(rp, xb[0]);
        } else {
            uu = make_double2(buf_load1d(ru, xb[0]), buf_load1d(ru, xb[1]));
            vv = make_double2(buf_load1d(rv, xb[0]), buf_load1d(rv, xb[1]));
            pp = make_double2(buf_load1d(rp, xb[0]), buf_load1d(rp, xb[1]));
        }
        lds[r][lane] = uu;
        vr[k][0] = vv.x;
        vr[k][1] = vv.y;
        pr[k][0] = scaled_phi(pp.x, a.k);
        pr[k][1] = scaled_phi(pp.y, a.k);
    }

    const bool out_lane = lane >= HX / 2 && lane < 64 - HX / 2;
    int ar[OUT ? R : 1][2];
    double tm[OUT ? R : 1][2];
    if (OUT) {
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int r = w + kTileWaves * k;
            const int gy = gy0 + r;
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const bool in = out_lane && r >= T && r < EY - T && gy < ny && gx + c < nx;
                ar[k][c] = in && a.arrival ? a.arrival[(int64_t)gy * a.apitch + gx + c] : 0;
                tm[k][c] = in && a.tl ? a.tl[(int64_t)gy * a.tpitch + gx + c] : 0.0;
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
                const double2 c = lds[r][lane];
                const double2 n = lds[r - 1][lane];
                const double2 s = lds[r + 1][lane];
                const double west = from_west_lane(c.y);
                const double east = from_east_lane(c.x);
                cell_update(c.x, west, c.y, n.x, s.x, vr[k][0], pr[k][0], a.k, un[k][0], vr[k][0]);
                cell_update(c.y, c.x, east, n.y, s.y, vr[k][1], pr[k][1], a.k, un[k][1], vr[k][1]);
                if (OUT && r >= T && r < EY - T) {
                    if (a.arrival) {
#pragma unroll
                        for (int e = 0; e < 2; ++e)
                            if (ar[k][e] == kNever && un[k][e] >= a.theta) ar[k][e] = a.step0 + t;
                    }
                    if (a.tl && (a.step0 + t) % a.tl_rate == 0) {
#pragma unroll
                        for (int e = 0; e < 2; ++e)
                            if (un[k][e] > tm[k][e]) tm[k][e] = un[k][e];
                    }
                }
            }
        }
        if (t < T) {
            __syncthreads();
#pragma unroll
            for (int k = 0; k < R; ++k) {
                const int r = w + kTileWaves * k;
                if (r >= t && r < EY - t) lds[r][lane] = make_double2(un[k][0], un[k][1]);
            }
            __syncthreads();
        }
    }

    bool bad = false;
    if (out_lane) {
        const int xo = 8 * gx;   // gx >= 0 for output lanes
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int r = w + kTileWaves * k;
            const int gy = gy0 + r;
            if (r < T || r >= EY - T || gy >= ny) continue;
            const int64_t off = (int64_t)gy * P;
            const auto ru = row_rsrc(a.u_out + off, row_bytes);
            const auto rv = row_rsrc(a.v_out + off, row_bytes);
            if (gx + 1 < nx) {
                buf_store2d(ru, xo, un[k][0], un[k][1]);
                buf_store2d(rv, xo, vr[k][0], vr[k][1]);
                bad |= !finite2(un[k][0], vr[k][0]) || !finite2(un[k][1], vr[k][1]);
            } else if (gx < nx) {
                buf_store1d(ru, xo, un[k][0]);
                buf_store1d(rv, xo, vr[k][0]);
                bad |= !finite2(un[k][0], vr[k][0]);
            }
            if (OUT && a.arrival) {
#pragma unroll
                for (int c = 0; c < 2; ++c)
                    if (gx + c < nx) a.arrival[(int64_t)gy * a.apitch + gx + c] = ar[k][c];
            }
            if (OUT && a.tl) {
#pragma unroll
                for (int c = 0; c < 2; ++c)
                    if (gx + c < nx) a.tl[(int64_t)gy * a.tpitch + gx + c] = tm[k][c];
            }
        }
    }
    if (bad) *a.flag = 1;
}

}  // namespace dev
}  // namespace rdc
