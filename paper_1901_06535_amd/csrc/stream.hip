// stream.hip -- single grids on the row pipelines of stream_pipe.h: the
// kernel, its launch and the plan of its work items (strips and segments).
// Compiled with the scheduler's iterative ILP strategy (build.py).
#include "stream_pipe.h"

namespace rdc {
namespace {

template <int T, bool MIRROR>
__global__ __launch_bounds__(kStreamWaves * 64, 2)
void k_stream(StepArgs<float> a, StreamGeom g) {
    static_assert(stream_fits<T>(), "T too large for the row slots");
    __shared__ float4 phs[kStreamWaves][kPhiRows][64];   // each wave's c1*phi ring
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    // Workgroups are dealt to the 8 XCDs round-robin: renumber so that each
    // XCD takes a contiguous run of work items (neighbouring strips of the
    // same rows, whose halo columns then meet in that XCD's L2).
    const int b = blockIdx.x;
    const int wg = (b & 7) * g.per_xcd + (b >> 3);
    const int item = wg * kStreamWaves + wave;
    if (item >= g.items) return;
    const int strip = item % g.nstrips;
    const int seg = item / g.nstrips;
    const int y0 = seg * g.seg_rows;
    const int y1 = min(y0 + g.seg_rows, a.ny);   // output rows [y0, y1)
    stream_wave<T, MIRROR>(a, strip, y0, y1, phs[wave]);
}

template <int T>
hipError_t stream_impl(const StepArgs<float>& a, hipStream_t s) {
    const StreamGeom g = stream_geom(a.nx, a.ny, T, stream_bx<T>(), stream_slots());
    const dim3 grid(8 * g.per_xcd), block(kStreamWaves * 64);
    if (a.nx % 4 == 0 && a.nx >= 256) {
        hipLaunchKernelGGL((k_stream<T, true>), grid, block, 0, s, a, g);
    } else {
        if constexpr (T > kMaxStreamCells)
            return hipErrorInvalidValue;     // cell-by-cell edge strips: T <= 11
        else
            hipLaunchKernelGGL((k_stream<T, false>), grid, block, 0, s, a, g);
    }
    return hipGetLastError();
}

}  // namespace

// Items (strip, segment) for the streaming kernel: strips of `bx` output
// columns; segments of near-equal height, as many as keep lowest the work
// of the longest wave times the rounds of resident waves (`slots` waves at
// a time).
StreamGeom stream_geom(int nx, int ny, int T, int bx, int slots) {
    StreamGeom g{};
    g.bx = bx;
    g.nstrips = (nx + bx - 1) / bx;
    int best_rows = ny;
    double best = -1.0;
    for (int nseg = 1; nseg <= ny; ++nseg) {
        const int rows = (ny + nseg - 1) / nseg;
        const int64_t items = (int64_t)g.nstrips * ((ny + rows - 1) / rows);
        const int64_t rounds = (items + slots - 1) / slots;
        const double cost = (double)rounds * wave_cost(rows, T);
        if (best < 0 || cost < best) {
            best = cost;
            best_rows = rows;
        }
        if (items > 64LL * slots) break;
    }
    g.seg_rows = best_rows;
    g.items = g.nstrips * ((ny + best_rows - 1) / best_rows);
    const int wgs = (g.items + kStreamWaves - 1) / kStreamWaves;
    g.per_xcd = (wgs + 7) / 8;
    return g;
}

int stream_slots() {
    // Resident waves when every CU holds two 4-wave workgroups (the launch
    // bounds ask for two waves per SIMD).
    static int cached_dev = -1, cached = 0;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 2048;
    if (dev != cached_dev) {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            cus <= 0)
            cus = 256;
        cached = cus * 4 * 2;
        cached_dev = dev;
    }
    return cached;
}

bool stream_supported(int T, int nx) {
    return T >= 2 && (T <= kMaxStreamCells || (T <= kMaxStream && nx % 4 == 0 && nx >= 256));
}

hipError_t launch_stream(const StepArgs<float>& a, int T, hipStream_t s) {
    switch (T) {
        case 2: return stream_impl<2>(a, s);
        case 3: return stream_impl<3>(a, s);
        case 4: return stream_impl<4>(a, s);
        case 5: return stream_impl<5>(a, s);
        case 6: return stream_impl<6>(a, s);
        case 7: return stream_impl<7>(a, s);
        case 8: return stream_impl<8>(a, s);
        case 9: return stream_impl<9>(a, s);
        case 10: return stream_impl<10>(a, s);
        case 11: return stream_impl<11>(a, s);
        case 12: return stream_impl<12>(a, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace rdc
