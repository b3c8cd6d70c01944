// kernels.h -- internal launch interface between the C ABI (api.hip) and the
// HIP kernels (kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cell.h"

namespace rdc {

constexpr int32_t kNever = 0x7fffffff;  // arrival value of a cell that never arrived

template <typename Real>
struct StepArgs {
    const Real* u;      // current u plane
    const Real* v;      // current v plane
    const Real* phi;    // excitability plane
    Real* u_out;        // next u plane
    Real* v_out;        // next v plane
    int32_t* arrival;   // optional first-arrival plane (nullptr = off)
    Real* tl;           // optional timelapse plane: running max of u over frames (nullptr = off)
    int* flag;          // sticky non-finite flag (device int)
    int64_t pitch;      // elements per row of u, v, phi
    int64_t apitch;     // elements per row of arrival
    int64_t tpitch;     // elements per row of tl
    int nx, ny;
    int step0;          // state index before this launch (for arrival times and frames)
    int tl_rate;        // a frame is taken after every step whose index is a multiple
    Real theta;         // arrival threshold
    Consts<Real> k;
};

// One forward-Euler step per launch, streaming (FP32 or FP64).
hipError_t launch_step1(const StepArgs<float>& a, hipStream_t s);
hipError_t launch_step1(const StepArgs<double>& a, hipStream_t s);

// T forward-Euler steps per launch on LDS tiles of `rows` rows (FP32).
// T in 2..kMaxBlock; `rows` one of tile_rows_supported().
// Most steps one tile launch takes: FP32 (kMaxBlock), FP64 (kMaxBlock64).
constexpr int kMaxBlock = 12;
constexpr int kMaxBlock64 = 8;
hipError_t launch_stepT(const StepArgs<float>& a, int T, int rows, hipStream_t s);
// The same for FP64 (tiles of 128 columns, 2 cells per lane).
hipError_t launch_stepT(const StepArgs<double>& a, int T, int rows, hipStream_t s);
bool tile_rows_supported(int rows);
// The tile kernels of one height (8 waves x R rows), FP32 and FP64; defined
// in tiles_impl.h and instantiated in tiles_r<R>.hip for R = 6, 7, 8, 10.
template <int R>
hipError_t launch_tiles(const StepArgs<float>& a, int T, hipStream_t s);
template <int R>
hipError_t launch_tiles(const StepArgs<double>& a, int T, hipStream_t s);
// Most rows a grid may have: the one-step kernel's launch grid covers
// kStep1Rows rows per block row, at most 65535 block rows.
int max_rows();
int tile_rows_default();

// T forward-Euler steps per launch by register-resident row pipelines
// (FP32, one wave per 256-column strip and segment of rows; no LDS tiles).
// T in 2..kMaxStreamCells on any grid, up to kMaxStream on grids whose
// width is a multiple of 4 and at least 256 (edge strips of mirrored 16-byte
// blocks; the cell-by-cell edge strips of other widths do not fit the
// registers at T = 12); results bit-identical to launch_step1 and
// launch_stepT.
constexpr int kMaxStream = 12;
constexpr int kMaxStreamCells = 11;
struct StreamGeom {
    int bx;        // output columns per strip (a multiple of 4)
    int nstrips;   // strips across the grid
    int seg_rows;  // output rows per segment
    int items;     // strips x segments, one wave each
    int per_xcd;   // workgroups per XCD
};
bool stream_supported(int T, int nx);
hipError_t launch_stream(const StepArgs<float>& a, int T, hipStream_t s);
// The same for FP64 (128-column strips, 2 cells per lane), T in 2..kMaxStream64.
constexpr int kMaxStream64 = 8;
bool stream64_supported(int T);
hipError_t launch_stream(const StepArgs<double>& a, int T, hipStream_t s);
// Strips of `bx` output columns and row segments for the row-pipeline
// kernels (4 waves per workgroup, ticks counted in loop bodies of 12):
// segments of near-equal height, as many as keep lowest the rows walked
// per round of `slots` resident waves.
StreamGeom stream_geom(int nx, int ny, int T, int bx, int slots);
// Resident waves of a row-pipeline launch on the current device (two 4-wave
// workgroups per CU).
int stream_slots();

// Catalytic stimulation: u := 1 on up to kMaxDisks disks per launch.
constexpr int kMaxDisks = 64;
struct Disks {
    int cx[kMaxDisks], cy[kMaxDisks], r[kMaxDisks];
    int count;
};
hipError_t launch_stimulate(float* u, int64_t pitch, int nx, int ny, const Disks& d,
                            int32_t* arrival, int64_t apitch, int step, hipStream_t s);
hipError_t launch_stimulate(double* u, int64_t pitch, int nx, int ny, const Disks& d,
                            int32_t* arrival, int64_t apitch, int step, hipStream_t s);

// arrival := (u >= theta) ? step : kNever over the grid.
hipError_t launch_arrival_init(const float* u, int64_t pitch, int nx, int ny, float theta,
                               int32_t* arrival, int64_t apitch, int step, hipStream_t s);
hipError_t launch_arrival_init(const double* u, int64_t pitch, int nx, int ny, double theta,
                               int32_t* arrival, int64_t apitch, int step, hipStream_t s);

// tl := u over the grid (the timelapse's first frame).
hipError_t launch_copy_plane(const float* u, int64_t pitch, int nx, int ny, float* tl,
                             int64_t tpitch, hipStream_t s);
hipError_t launch_copy_plane(const double* u, int64_t pitch, int nx, int ny, double* tl,
                             int64_t tpitch, hipStream_t s);

// *flag := 0 (a kernel, not a memset, so the call is safe under graph capture).
hipError_t launch_clear_flag(int* flag, hipStream_t s);

// Plain device copy of n16 16-byte words (the measured bandwidth ceiling).
hipError_t launch_copy16(const void* src, void* dst, int64_t n16, hipStream_t s);

}  // namespace rdc
