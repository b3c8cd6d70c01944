// batch.h -- internal interface between the batched C ABI (batch.hip) and the
// whole-grid LDS kernel (resident.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

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

}  // namespace rdc
