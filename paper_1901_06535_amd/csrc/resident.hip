// resident.hip -- small grids of a batch advanced whole in LDS: forward-Euler
// steps of the Oregonator (Sec. 2, Eq. (1)), every step of a launch on chip.
//
// A grid of at most kResThreads x kResRows cells is read once from the
// pooled planes, stepped `steps` times by one workgroup with one barrier per
// step, and written back once; between the two nothing touches HBM.  Each
// thread keeps u, v and c1 phi of its cells (one column, m consecutive rows)
// in registers.  u is mirrored in LDS for the neighbours' reads, slot
// k * kResThreads + t holding cell k of thread t: the west and east
// neighbours of a cell are the same slot of threads t -+ 1, so every
// neighbour read of a thread is one base address plus the immediate offset
// of its row.  North and south neighbours inside a thread's column come from
// its own registers; the cells above its first row and below its last come
// from the threads of the row groups before and after.  No-flux edges (the
// ghost cell equals the edge cell) are reads of the cell itself: a thread in
// column 0 reads its own slot as its west neighbour, and so on.  The update
// is cell_update, so a grid evolves bit-identically to the same grid stepped
// by any other kernel.
#include "batch.h"

namespace rdc {
namespace {

constexpr int kResPlane = kResRows * kResThreads;   // floats per LDS plane of u

// One grid, M rows per thread.  Every thread steps all M of its row slots
// (in the last row group those past the grid's last row from zero, never
// read back into a row of the grid), so the step has no branches.  Each M
// is a function of its own (not inlined into the kernel): every one then
// gets its own register allocation, while the sixteen bodies inlined into
// one kernel are allocated together and spill.
template <int M>
__device__ __attribute__((noinline)) void resident_grid(const ResArgs& r, const ResItem& it,
                                                        const SimDev& sd, float* lds) {
    const int nx = sd.nx, ny = sd.ny, m = M;
    const int t = threadIdx.x;
    const int g = t / nx;
    const int x = t - g * nx;
    const int y0 = g * m;
    const bool active = g < it.groups;
    const int mt = active ? min(m, ny - y0) : 1;     // rows of this column that exist
    Consts<float> K = sd.k;
    // k0 in a VGPR: an FMA reads one scalar operand at most.
    K.k0 = __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(K.k0), 0xe4, 0xf, 0xf, false));

    // LDS slots of the neighbours (edge cells read themselves).
    const int iW = x > 0 ? t - 1 : t;
    const int iE = x < nx - 1 ? t + 1 : t;
    const int iN = y0 > 0 ? (m - 1) * kResThreads + t - nx : t;
    const int iS = y0 + mt < ny ? t + nx : (mt - 1) * kResThreads + t;

    const int64_t P = sd.pitch;
    const int64_t base = sd.offset + (int64_t)y0 * P + x;
    float u[M], v[M], c1p[M];
#pragma unroll
    for (int k = 0; k < M; ++k) {
        u[k] = 0.0f;
        v[k] = 0.0f;
        c1p[k] = 0.0f;
        if (active && k < mt) {
            const int64_t o = base + k * P;
            u[k] = r.u[o];
            v[k] = r.v[o];
            c1p[k] = scaled_phi(r.phi[o], K);
        }
        if (active) lds[k * kResThreads + t] = u[k];
    }
    __syncthreads();

    // the step count as a wave-uniform value read once (the loop is scalar)
    const int steps = __builtin_amdgcn_readfirstlane(r.steps);
    for (int s = 0; s < steps; ++s) {
        const float* rd = lds + (s & 1) * kResPlane;
        float* wr = lds + kResPlane - (s & 1) * kResPlane;
        if (active) {
            float uW[M], uE[M];
#pragma unroll
            for (int k = 0; k < M; ++k) {
                uW[k] = rd[iW + k * kResThreads];
                uE[k] = rd[iE + k * kResThreads];
            }
            const float above = rd[iN];
            const float below = rd[iS];
            float north = above;
#pragma unroll
            for (int k = 0; k < M; ++k) {
                const float c = u[k];
                // the row below: this thread's next cell, or (after its last
                // row) the next group's first cell or the edge cell itself
                float south = below;
                if (k + 1 < M && k + 1 < mt) south = u[k + 1 < M ? k + 1 : k];
                float un, vn;
                cell_update(c, uW[k], uE[k], north, south, v[k], c1p[k], K, un, vn);
                north = c;
                u[k] = un;
                v[k] = vn;
                wr[k * kResThreads + t] = un;
            }
        }
        __syncthreads();
    }

    if (active) {
        bool bad = false;
#pragma unroll
        for (int k = 0; k < M; ++k) {
            if (k < mt) {
                const int64_t o = base + k * P;
                r.u_out[o] = u[k];
                r.v_out[o] = v[k];
                bad |= !(__builtin_isfinite(u[k]) && __builtin_isfinite(v[k]));
            }
        }
        if (bad) r.flags[it.sim] = 1;
    }
}

__global__ __launch_bounds__(kResThreads) void k_batch_resident(ResArgs r) {
    __shared__ float lds[2 * kResPlane];
    if ((int)blockIdx.x >= r.count) return;
    const ResItem it = r.items[blockIdx.x];
    const SimDev sd = r.sims[it.sim];
    switch (it.m) {
        case 1: resident_grid<1>(r, it, sd, lds); break;
        case 2: resident_grid<2>(r, it, sd, lds); break;
        case 3: resident_grid<3>(r, it, sd, lds); break;
        case 4: resident_grid<4>(r, it, sd, lds); break;
        case 5: resident_grid<5>(r, it, sd, lds); break;
        case 6: resident_grid<6>(r, it, sd, lds); break;
        case 7: resident_grid<7>(r, it, sd, lds); break;
        case 8: resident_grid<8>(r, it, sd, lds); break;
        case 9: resident_grid<9>(r, it, sd, lds); break;
        case 10: resident_grid<10>(r, it, sd, lds); break;
        case 11: resident_grid<11>(r, it, sd, lds); break;
        case 12: resident_grid<12>(r, it, sd, lds); break;
        case 13: resident_grid<13>(r, it, sd, lds); break;
        case 14: resident_grid<14>(r, it, sd, lds); break;
        case 15: resident_grid<15>(r, it, sd, lds); break;
        case 16: resident_grid<16>(r, it, sd, lds); break;
        default: break;
    }
}
static_assert(kResRows == 16, "k_batch_resident dispatches m = 1..16");

}  // namespace

bool resident_layout(int nx, int ny, int* m, int* groups) {
    if (nx < 1 || ny < 1 || nx > kResThreads) return false;
    const int per = kResThreads / nx;                 // row groups that fit
    const int rows = (ny + per - 1) / per;
    if (rows > kResRows) return false;
    *m = rows;
    *groups = (ny + rows - 1) / rows;
    return true;
}

hipError_t launch_resident(const ResArgs& a, hipStream_t s) {
    if (a.count < 1 || a.steps < 1 || a.steps > kResMaxSteps) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_batch_resident, dim3(a.count), dim3(kResThreads), 0, s, a);
    return hipGetLastError();
}

}  // namespace rdc
