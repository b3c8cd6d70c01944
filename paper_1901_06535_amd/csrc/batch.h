// batch.h -- internal interface between the batched C ABI (batch.hip) and the
// whole-grid LDS kernel (resident.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "cell.h"

namespace rdc {

// One grid of a batch as the device sees it: size, row pitch and offset of
// its region in the pooled planes (elements), scheme constants.
struct SimDev {
    int nx, ny;
    int64_t pitch, offset;
    Consts<float> k;
};

// Whole-grid LDS kernel.  One workgroup of kResThreads threads takes one
// grid and runs every step of a launch on chip.  Thread t works on column
// x = t mod nx of row group g = t / nx, i.e. on rows [g m, g m + m) of that
// column (fewer in the last group when m does not divide ny), holding u, v
// and c1 phi of those cells in registers; u of the whole grid is mirrored in
// LDS (two planes, one read and one written per step) for the neighbours.
constexpr int kResThreads = 1024;
constexpr int kResRows = 16;          // most rows per thread (LDS: 2 x 16 x 1024 floats, 128 KiB)
constexpr int kResMaxSteps = 16384;   // most steps per launch (a longer call takes several)

struct ResItem {
    int sim;      // grid index in the batch
    int m;        // rows per thread
    int groups;   // row groups, ceil(ny / m); groups * nx <= kResThreads
    int pad;
};

struct ResArgs {
    const float* u;     // pooled planes holding the state on entry
    const float* v;
    const float* phi;
    float* u_out;       // pooled planes receiving it (may equal u, v: each grid is read whole first)
    float* v_out;
    const SimDev* sims;
    const ResItem* items;
    int* flags;         // sticky non-finite flag per grid
    int count;          // items (workgroups)
    int steps;          // 1..kResMaxSteps
};

// Layout of an nx x ny grid on the resident kernel: the fewest rows per
// thread that cover it.  False if the grid does not fit (more than
// kResThreads columns or more than kResRows rows per thread).
bool resident_layout(int nx, int ny, int* m, int* groups);

hipError_t launch_resident(const ResArgs& a, hipStream_t s);

// Row pipelines over many grids (stream.hip): one wave per item, output
// columns [strip * stream_strip_cols(T), + stream_strip_cols(T)) and output
// rows [y0, y1) of grid `sim`; 4 waves per workgroup, workgroups dealt to
// the 8 XCDs in contiguous runs of per_xcd.
struct StreamItem {
    int sim, strip, y0, y1;
};

struct BatchStreamArgs {
    const float* u;     // pooled planes holding the state on entry
    const float* v;
    const float* phi;
    float* u_out;       // pooled planes receiving it (not u, v)
    float* v_out;
    const SimDev* sims;
    const StreamItem* items;
    int* flags;         // sticky non-finite flag per grid
    int nitems;         // work items (waves), >= 1
    int per_xcd;        // workgroups per XCD: 8 * per_xcd * 4 >= nitems
};

// Output columns per strip of the row pipelines at T steps per launch
// (0 outside 2..11).
int stream_strip_cols(int T);
hipError_t launch_batch_stream(const BatchStreamArgs& b, int T, hipStream_t s);

// Work items of the row pipelines at T (2..11) steps per launch over grids
// (batch index, size), `slots` waves resident at a time: every grid's
// strips, its rows cut into segments of near-equal height, all segments
// under one bound chosen to keep lowest the longest wave's work times the
// rounds of resident waves; longest items first.
struct GridShape {
    int sim, nx, ny;
};
std::vector<StreamItem> batch_stream_items(const std::vector<GridShape>& grids, int T,
                                           int slots);

}  // namespace rdc
