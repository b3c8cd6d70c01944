// stream64.hip -- T forward-Euler steps of the Oregonator (Sec. 2, Eq. (1))
// per launch, FP64, by row pipelines held in registers.
//
// The FP64 counterpart of stream.hip (which describes the scheme): one wave
// per strip of 128 columns (64 lanes x 2 adjacent cells, 16 bytes per lane)
// and segment of rows walks down the segment one row per tick, loading one
// new row of u, v and phi two rows ahead and advancing every level t = 1..T
// by one row (a skew of one row per level).  Every intermediate row stays in
// registers (level 1 keeps u^0 rows mod 6, level t >= 2 three rows of
// u^(t-1), v of the rows in flight in 12 slots); phi of the rows in flight
// sits in a per-wave LDS ring.  Halo: T columns each side (left rounded up
// to whole lanes) and T rows above and below a segment, loaded mirrored at
// the domain edges.  Every cell goes through the FP64 cell_update, so the
// result is bit-identical to the other FP64 kernels and to the oracle.
#include "kernels.h"
#include "tile.h"

namespace rdc {
namespace {

using namespace dev;

constexpr int kWaves = 4;         // waves per workgroup (independent pipelines)
constexpr int kUnroll = 12;       // ticks per unrolled loop body
constexpr int kRowSlots = 12;     // v of the rows in the levels: row index mod 12
constexpr int kU0Slots = 6;       // u^0 rows held by level 1: row index mod 6
constexpr int kAhead = 2;         // a row is loaded this many ticks before it enters level 1
constexpr int kStage = 3;         // v, phi of loaded rows waiting to enter: row index mod 3
constexpr int kPhiRows = 16;      // phi rows in LDS per wave: row index mod 16
// A buffer offset past any row (rows are shorter than 2 GiB): the access is
// dropped.
constexpr int kOff = static_cast<int>(0x80000000u);

constexpr int md(int a, int m) { return ((a % m) + m) % m; }

// Column halo on the left of the strip: T rounded up to whole lanes (2
// cells), so loads and stores stay 16-byte aligned.
template <int T>
constexpr int hx64() { return (T + 1) & ~1; }

template <int T>
constexpr bool fits64() {
    return T >= 2 && T <= kMaxStream64 && T <= kRowSlots && T <= kPhiRows &&
           kAhead + 3 <= kU0Slots && kAhead + 1 <= kStage && kUnroll % kRowSlots == 0 &&
           kUnroll % kU0Slots == 0 && kUnroll % kStage == 0 && kUnroll % 3 == 0;
}

struct Lane64 {
    int gx;          // first global column of this lane's 2 cells
    int xb[2];       // byte offsets of its 2 columns, mirrored at the domain edges
    int so[2];       // byte offsets of its 2 output cells, or kOff where not stored
    int so2;         // byte offset of its 16-byte output word, or kOff
    bool rev;        // (kMirror) its 2 cells are a 16-byte block in reverse order
    uint64_t out;    // lanes holding output cells
};

// How a strip reads its columns (as in stream.hip): kInterior, kCells (cell
// by cell past an edge), or kMirror (even widths from 128 on: 16-byte words
// everywhere, mirrored blocks past an edge reversed on first use).
enum StripMode { kInterior = 0, kCells = 1, kMirror = 2 };

template <int T, int MODE>
__device__ __forceinline__ void pipeline64(const StepArgs<double>& a, const Lane64& ln, int y0,
                                           int y1, double2 (&phs)[kPhiRows][64],
                                           bool edge_wave) {
    constexpr bool EDGE = MODE == kCells;
    const int ny = a.ny;
    const int lane = threadIdx.x & 63;
    const int64_t P = a.pitch;
    const int row_bytes = static_cast<int>(P * 8);
    const int i0 = y0 - T + 1;                 // first tick: level 1 on row y0 - T + 1
    const int i_end = y1 + T - 1;              // ticks [i0, i_end)
    const Consts<double> k = a.k;

    // As in the FP32 kernel: every level runs on every tick from its first
    // row on; only level T's output is checked and written, where it ran on
    // a row of the segment.
    constexpr int kRampBodies = (2 * T - 2 + kUnroll - 1) / kUnroll;
    double u0[kU0Slots][2] = {};               // u^0 rows (level 1's window)
    double uw[T + 1][3][2] = {};               // uw[t]: rows of u^(t-1), t >= 2
    double vr[kRowSlots][2] = {};              // v of the rows in the levels
    double vs[kStage][2] = {};                 // v of loaded rows not yet in level 1
    double ps[kStage][2] = {};                 // phi of loaded rows not yet in level 1

    // Load row r of u (and of v, phi); rows past the last one any level
    // needs (i_end) read nothing.
    auto load_row = [&](int r, double (&uu)[2], double (&vv)[2], double (&pp)[2],
                        bool with_vp) __attribute__((always_inline)) {
        const int64_t off = (int64_t)reflect_index(r, ny) * P;
        const int nb = r <= i_end ? row_bytes : 0;
        const auto ru = row_rsrc(a.u + off, nb);
        const auto rv = row_rsrc(a.v + off, nb);
        const auto rp = row_rsrc(a.phi + off, nb);
        if (!EDGE) {
            const double2 t = buf_load2d(ru, ln.xb[0]);
            uu[0] = t.x;
            uu[1] = t.y;
            if (with_vp) {
                const double2 w = buf_load2d(rv, ln.xb[0]);
                vv[0] = w.x;
                vv[1] = w.y;
                const double2 p = buf_load2d(rp, ln.xb[0]);
                pp[0] = p.x;
                pp[1] = p.y;
            }
        } else {
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                uu[c] = buf_load1d(ru, ln.xb[c]);
                if (with_vp) {
                    vv[c] = buf_load1d(rv, ln.xb[c]);
                    pp[c] = buf_load1d(rp, ln.xb[c]);
                }
            }
        }
    };

    // kMirror: put a mirrored block's 2 cells in order when the row is
    // first used (edge strips only).
    auto unmirror = [&](double (&x)[2]) __attribute__((always_inline)) {
        if (MODE == kMirror && edge_wave) {
            const double x0 = x[0], x1 = x[1];
            x[0] = ln.rev ? x1 : x0;
            x[1] = ln.rev ? x0 : x1;
        }
    };

    load_row(i0 - 1, u0[md(-1, kU0Slots)], vs[md(-1, kStage)], ps[md(-1, kStage)], false);
#pragma unroll
    for (int j = 0; j <= kAhead; ++j)
        load_row(i0 + j, u0[md(j, kU0Slots)], vs[md(j, kStage)], ps[md(j, kStage)], true);
    unmirror(u0[md(-1, kU0Slots)]);
    unmirror(u0[md(0, kU0Slots)]);

    uint64_t bad = 0;
    // One tick, as in the FP32 kernel: s fixes the slots; in the ramp bodies
    // (ramp >= 0, the body's first tick counted from i0) the levels with no
    // row yet are left out, and their results are kept in place there.
    auto tick = [&](const int i, const int s, const int ramp) __attribute__((always_inline)) {
        // Row i enters level 1: v to its row slot, phi to the LDS ring.
        unmirror(vs[md(s, kStage)]);
        unmirror(ps[md(s, kStage)]);
        unmirror(u0[md(s + 1, kU0Slots)]);       // row i + 1: level 1's south from now on
        double pc1[2];
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            vr[md(s, kRowSlots)][c] = vs[md(s, kStage)][c];
            pc1[c] = scaled_phi(ps[md(s, kStage)][c], k);
        }
        phs[i & (kPhiRows - 1)][lane] = make_double2(pc1[0], pc1[1]);
        load_row(i + 1 + kAhead, u0[md(s + 1 + kAhead, kU0Slots)],
                 vs[md(s + 1 + kAhead, kStage)], ps[md(s + 1 + kAhead, kStage)], true);

        double un[2];
        const bool live_T = i >= i0 + 2 * T - 2 && i < i_end;
#pragma unroll
        for (int t = 1; t <= T; ++t) {
            if (ramp >= 0 && ramp + s < 2 * t - 2) continue;   // no row of level t yet
            const int rs = md(s - t + 1, kRowSlots);           // slot of row rho = i - t + 1
            const double* n;
            const double* c;
            const double* so;
            if (t == 1) {
                n = u0[md(s - 1, kU0Slots)];
                c = u0[md(s, kU0Slots)];
                so = u0[md(s + 1, kU0Slots)];
            } else {
                n = uw[t][md(s - t, 3)];
                c = uw[t][md(s - t + 1, 3)];
                so = uw[t][md(s - t + 2, 3)];
            }
            double pc[2];
            if (t == 1) {
                pc[0] = pc1[0];
                pc[1] = pc1[1];
            } else {
                const double2 q = phs[(i - t + 1) & (kPhiRows - 1)][lane];
                pc[0] = q.x;
                pc[1] = q.y;
            }
            const double west = from_west_lane(c[1]);
            const double east = from_east_lane(c[0]);
            // west and east enter the update as a sum (either order)
            cell_update(c[0], west, c[1], n[0], so[0], vr[rs][0], pc[0], k, un[0],
                        vr[rs][0]);
            cell_update(c[1], c[0], east, n[1], so[1], vr[rs][1], pc[1], k, un[1],
                        vr[rs][1]);
            if (ramp >= 0) {
#pragma unroll
                for (int e = 0; e < 2; ++e) asm volatile("" : "+v"(un[e]), "+v"(vr[rs][e]));
            }
            if (t < T) {
#pragma unroll
                for (int e = 0; e < 2; ++e) uw[t < T ? t + 1 : T][md(s - t + 1, 3)][e] = un[e];
            } else if (live_T) {
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                    const bool ok = __builtin_isfinite(un[e]) && __builtin_isfinite(vr[rs][e]);
                    bad |= __builtin_amdgcn_ballot_w64(!ok);
                }
            }
        }
        // Row i - T + 1 of u^T and v^T, written where level T ran on it.
        if (ramp >= 0 && ramp + s < 2 * T - 2) return;
        const int rs = md(s - T + 1, kRowSlots);
        const int64_t off = (int64_t)min(max(i - T + 1, 0), ny - 1) * P;
        const int nb = live_T ? row_bytes : 0;
        const auto ro = row_rsrc(a.u_out + off, nb);
        const auto rv = row_rsrc(a.v_out + off, nb);
        if (!EDGE) {
            buf_store2d(ro, ln.so2, un[0], un[1]);
            buf_store2d(rv, ln.so2, vr[rs][0], vr[rs][1]);
        } else {
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                buf_store1d(ro, ln.so[e], un[e]);
                buf_store1d(rv, ln.so[e], vr[rs][e]);
            }
        }
    };
    auto ramp_body = [&](const int r0) __attribute__((always_inline)) {
#pragma unroll
        for (int s = 0; s < kUnroll; ++s) {
            tick(i0 + r0 + s, s, r0);
            __builtin_amdgcn_sched_barrier(0);
        }
    };
    static_assert(kRampBodies >= 1 && kRampBodies <= 2, "ramp of at most two loop bodies");
    ramp_body(0);
    if constexpr (kRampBodies > 1) ramp_body(kUnroll);
    int ib = i0 + kRampBodies * kUnroll;
    for (; ib + kUnroll <= i_end; ib += kUnroll) {
#pragma unroll
        for (int s = 0; s < kUnroll; ++s) tick(ib + s, s, -1);
    }
    if (ib < i_end) {
#pragma unroll
        for (int s = 0; s < kUnroll; ++s) {
            if (s > 0 && ib + s >= i_end) break;
            tick(ib + s, s, -1);
        }
    }
    if (bad & ln.out) {
        if ((threadIdx.x & 63) == __builtin_ctzll(ln.out)) *a.flag = 1;
    }
}

template <int T, bool MIRROR>
__global__ __launch_bounds__(kWaves * 64, 2)
void k_stream64(StepArgs<double> a, StreamGeom g) {
    static_assert(fits64<T>(), "T too large for the row slots");
    __shared__ double2 phs[kWaves][kPhiRows][64];   // each wave's phi ring
    constexpr int HX = hx64<T>();
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    // Contiguous runs of items per XCD (see k_stream).
    const int b = blockIdx.x;
    const int wg = (b & 7) * g.per_xcd + (b >> 3);
    const int item = wg * kWaves + wave;
    if (item >= g.items) return;
    const int strip = item % g.nstrips;
    const int seg = item / g.nstrips;
    const int nx = a.nx;
    const int x_out0 = strip * g.bx;           // first output column
    const int x_load0 = x_out0 - HX;           // first loaded column
    Lane64 ln;
    ln.gx = x_load0 + 2 * lane;
#pragma unroll
    for (int c = 0; c < 2; ++c) ln.xb[c] = 8 * reflect_index(ln.gx + c, nx);
    ln.rev = false;
    if (MIRROR) {
        // Even width >= 128: a lane's 2 columns are both inside or both past
        // one edge, and their mirror images form one block, reversed.
        if (ln.gx < 0) {
            ln.xb[0] = 8 * (-2 - ln.gx);
            ln.rev = true;
        } else if (ln.gx >= nx) {
            ln.xb[0] = 8 * (2 * nx - 2 - ln.gx);
            ln.rev = true;
        }
    }
    const bool out_lane = lane >= HX / 2 && lane < (HX + g.bx) / 2 && ln.gx < nx;
    ln.so2 = out_lane ? 8 * ln.gx : kOff;
#pragma unroll
    for (int c = 0; c < 2; ++c) ln.so[c] = out_lane && ln.gx + c < nx ? 8 * (ln.gx + c) : kOff;
    ln.out = __builtin_amdgcn_ballot_w64(out_lane);
    const int y0 = seg * g.seg_rows;
    const int y1 = min(y0 + g.seg_rows, a.ny);   // output rows [y0, y1)
    const bool inside = x_load0 >= 0 && x_load0 + 128 <= nx;
    if (MIRROR)
        pipeline64<T, kMirror>(a, ln, y0, y1, phs[wave], !inside);
    else if (inside)
        pipeline64<T, kInterior>(a, ln, y0, y1, phs[wave], false);
    else
        pipeline64<T, kCells>(a, ln, y0, y1, phs[wave], true);
}

template <int T>
hipError_t impl64(const StepArgs<double>& a, hipStream_t s) {
    constexpr int HX = hx64<T>();
    // Output columns: the loaded 128 less the left halo HX and a right halo
    // of at least T, kept a multiple of 2.
    constexpr int bx = (128 - HX - T) & ~1;
    const StreamGeom g = stream_geom(a.nx, a.ny, T, bx, stream_slots());
    const dim3 grid(8 * g.per_xcd), block(kWaves * 64);
    if (a.nx % 2 == 0 && a.nx >= 128)
        hipLaunchKernelGGL((k_stream64<T, true>), grid, block, 0, s, a, g);
    else
        hipLaunchKernelGGL((k_stream64<T, false>), grid, block, 0, s, a, g);
    return hipGetLastError();
}

}  // namespace

bool stream64_supported(int T) { return T >= 2 && T <= kMaxStream64; }

hipError_t launch_stream(const StepArgs<double>& a, int T, hipStream_t s) {
    switch (T) {
        case 2: return impl64<2>(a, s);
        case 3: return impl64<3>(a, s);
        case 4: return impl64<4>(a, s);
        case 5: return impl64<5>(a, s);
        case 6: return impl64<6>(a, s);
        case 7: return impl64<7>(a, s);
        case 8: return impl64<8>(a, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace rdc
