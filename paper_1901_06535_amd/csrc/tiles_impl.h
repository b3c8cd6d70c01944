// tiles_impl.h -- the T-step LDS tile kernels (k_stepT, FP32; k_stepT64,
// FP64) and their launchers for one tile height: included by one
// tiles_r<R>.hip per height, so the heights compile in parallel.
//
//   k_stepT  T steps per launch (FP32): a workgroup of 8 waves loads a
//            256-column by EY-row tile of u (into LDS), v and phi (into
//            registers) including a halo mirrored at the domain edges, runs T
//            steps on chip with the valid region shrinking by one cell per
//            step, and writes the (256-2*HX) x (EY-2*T) interior.  Each wave
//            owns whole 256-cell tile rows (64 lanes x 4 cells), so the east /
//            west neighbours cross lanes by DPP row shifts and only the
//            north / south rows go through LDS.
#pragma once

#include "kernels.h"
#include "tile.h"

namespace rdc {
namespace {

using namespace dev;

template <int T, int R, bool OUT>
__global__ __launch_bounds__(kTileWaves * 64, (tile_waves_per_simd<R, OUT>()))
void k_stepT(StepArgs<float> a, int tiles_x, int ntiles, int per_xcd) {
    __shared__ float4 lds[kTileWaves * R][64];
    // Workgroups are dealt to the 8 XCDs round-robin; renumber so that each
    // XCD walks a contiguous run of the row-major tile order: concurrent
    // tiles of one XCD share halo cells in its L2, and their loads sweep long
    // contiguous row segments.  (A column-major walk measured slower.)
    const int b = blockIdx.x;
    const int tile = (b & 7) * per_xcd + (b >> 3);
    if (tile >= ntiles) return;
    step_tile<T, R, OUT>(a, tile % tiles_x, tile / tiles_x, lds);
}

template <int T, int R, bool OUT>
__global__ __launch_bounds__(kTileWaves * 64, (tile_waves_per_simd<R, OUT>()))
void k_stepT64(StepArgs<double> a, int tiles_x, int ntiles, int per_xcd) {
    __shared__ double2 lds[kTileWaves * R][64];
    const int b = blockIdx.x;
    const int tile = (b & 7) * per_xcd + (b >> 3);   // XCD-contiguous runs, as k_stepT
    if (tile >= ntiles) return;
    step_tile64<T, R, OUT>(a, tile % tiles_x, tile / tiles_x, lds);
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
    if (a.arrival || a.tl)
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
        case 9: return stepT_impl<9, R>(a, s);
        case 10: return stepT_impl<10, R>(a, s);
        case 11: return stepT_impl<11, R>(a, s);
        case 12: return stepT_impl<12, R>(a, s);
        default: return hipErrorInvalidValue;
    }
}

template <int T, int R>
hipError_t stepT64_impl(const StepArgs<double>& a, hipStream_t s) {
    using G = TileGeom64<T, R>;
    const int tiles_x = (a.nx + G::BX - 1) / G::BX;
    const int tiles_y = (a.ny + G::BY - 1) / G::BY;
    const int ntiles = tiles_x * tiles_y;
    const int per_xcd = (ntiles + 7) / 8;
    const dim3 grid(8 * per_xcd), block(kTileWaves * 64);
    if (a.arrival || a.tl)
        hipLaunchKernelGGL((k_stepT64<T, R, true>), grid, block, 0, s, a, tiles_x, ntiles, per_xcd);
    else
        hipLaunchKernelGGL((k_stepT64<T, R, false>), grid, block, 0, s, a, tiles_x, ntiles,
                           per_xcd);
    return hipGetLastError();
}

template <int R>
hipError_t stepT64_rows(const StepArgs<double>& a, int T, hipStream_t s) {
    switch (T) {
        case 2: return stepT64_impl<2, R>(a, s);
        case 3: return stepT64_impl<3, R>(a, s);
        case 4: return stepT64_impl<4, R>(a, s);
        case 5: return stepT64_impl<5, R>(a, s);
        case 6: return stepT64_impl<6, R>(a, s);
        case 7: return stepT64_impl<7, R>(a, s);
        case 8: return stepT64_impl<8, R>(a, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

template <int R>
hipError_t launch_tiles(const StepArgs<float>& a, int T, hipStream_t s) {
    return stepT_rows<R>(a, T, s);
}
template <int R>
hipError_t launch_tiles(const StepArgs<double>& a, int T, hipStream_t s) {
    return stepT64_rows<R>(a, T, s);
}

}  // namespace rdc
