// stream_batch.hip -- the grids of a batch on the row pipelines of
// stream_pipe.h: the kernel (one wave per grid, strip and segment), its
// launch and the plan of its work items over all grids.  Compiled with the
// default scheduling: its edge strips (most strips of a batch's narrow
// grids) load cell by cell, and ran slower with the ILP strategy.
#include <algorithm>
#include <vector>

#include "stream_pipe.h"

namespace rdc {
namespace {

// Many grids of a batch (the pooled planes of batch.h): one wave per work
// item (grid, strip, segment), every item's rows planned on the host; the
// same pipeline as k_stream, so each grid evolves bit-identically to the
// same grid stepped alone.  Edge strips go cell by cell (batch grids have
// any width).
template <int T>
__global__ __launch_bounds__(kStreamWaves * 64, 2)
void k_batch_stream(BatchStreamArgs b) {
    static_assert(stream_fits<T>(), "T too large for the row slots");
    __shared__ float4 phs[kStreamWaves][kPhiRows][64];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wg = (blockIdx.x & 7) * b.per_xcd + (blockIdx.x >> 3);
    const int item = wg * kStreamWaves + wave;
    if (item >= b.nitems) return;
    const StreamItem it = b.items[item];
    const SimDev sd = b.sims[it.sim];
    StepArgs<float> a;
    a.u = b.u + sd.offset;
    a.v = b.v + sd.offset;
    a.phi = b.phi + sd.offset;
    a.u_out = b.u_out + sd.offset;
    a.v_out = b.v_out + sd.offset;
    a.arrival = nullptr;
    a.tl = nullptr;
    a.flag = b.flags + it.sim;
    a.pitch = sd.pitch;
    a.apitch = 0;
    a.tpitch = 0;
    a.tl_rate = 1;
    a.nx = sd.nx;
    a.ny = sd.ny;
    a.step0 = 0;
    a.theta = 0.0f;
    a.k = sd.k;
    stream_wave<T, false>(a, it.strip, it.y0, it.y1, phs[wave]);
}

}  // namespace

std::vector<StreamItem> batch_stream_items(const std::vector<GridShape>& grids, int T,
                                           int slots) {
    std::vector<StreamItem> list;
    const int bx = stream_strip_cols(T);
    if (grids.empty() || bx <= 0 || slots < 1) return list;
    int max_ny = 1;
    for (const GridShape& g : grids) max_ny = max(max_ny, g.ny);
    // The most rows a segment may have: every grid is cut into ceil(ny / h)
    // segments of near-equal height (so none has more than h rows); h is
    // the one that keeps lowest the work of the longest wave times the
    // rounds of resident waves.
    int best_h = max_ny;
    double best = -1.0;
    for (int h = max_ny; h >= 1; --h) {
        int64_t items = 0;
        for (const GridShape& g : grids)
            items += (int64_t)((g.nx + bx - 1) / bx) * ((g.ny + h - 1) / h);
        if (items > 64LL * slots) break;
        const int64_t rounds = (items + slots - 1) / slots;
        const double cost = (double)rounds * wave_cost(h, T);
        if (best < 0 || cost <= best) {
            best = cost;
            best_h = h;
        }
    }
    for (const GridShape& g : grids) {
        const int nseg = (g.ny + best_h - 1) / best_h;
        const int rows = (g.ny + nseg - 1) / nseg;
        const int nstrips = (g.nx + bx - 1) / bx;
        for (int y0 = 0; y0 < g.ny; y0 += rows)
            for (int st = 0; st < nstrips; ++st)
                list.push_back({g.sim, st, y0, min(y0 + rows, g.ny)});
    }
    // Longest first: with more items than resident waves, the rounds after
    // the first are the short items (neighbouring strips of a segment stay
    // together, so their halo columns meet in one XCD's L2).
    std::stable_sort(list.begin(), list.end(), [](const StreamItem& a, const StreamItem& c) {
        return a.y1 - a.y0 > c.y1 - c.y0;
    });
    return list;
}

int stream_strip_cols(int T) {
    switch (T) {
        case 2: return stream_bx<2>();
        case 3: return stream_bx<3>();
        case 4: return stream_bx<4>();
        case 5: return stream_bx<5>();
        case 6: return stream_bx<6>();
        case 7: return stream_bx<7>();
        case 8: return stream_bx<8>();
        case 9: return stream_bx<9>();
        case 10: return stream_bx<10>();
        case 11: return stream_bx<11>();
        default: return 0;
    }
}

namespace {
template <int T>
hipError_t batch_stream_impl(const BatchStreamArgs& b, hipStream_t s) {
    const int wgs = (b.nitems + kStreamWaves - 1) / kStreamWaves;
    if (b.nitems < 1 || b.per_xcd * 8 < wgs) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_batch_stream<T>), dim3(8 * b.per_xcd), dim3(kStreamWaves * 64), 0, s,
                       b);
    return hipGetLastError();
}
}  // namespace

hipError_t launch_batch_stream(const BatchStreamArgs& b, int T, hipStream_t s) {
    switch (T) {
        case 2: return batch_stream_impl<2>(b, s);
        case 3: return batch_stream_impl<3>(b, s);
        case 4: return batch_stream_impl<4>(b, s);
        case 5: return batch_stream_impl<5>(b, s);
        case 6: return batch_stream_impl<6>(b, s);
        case 7: return batch_stream_impl<7>(b, s);
        case 8: return batch_stream_impl<8>(b, s);
        case 9: return batch_stream_impl<9>(b, s);
        case 10: return batch_stream_impl<10>(b, s);
        case 11: return batch_stream_impl<11>(b, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace rdc
