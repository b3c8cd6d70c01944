// stream_pipe.h -- the row pipeline: T forward-Euler steps of the Oregonator
// (Sec. 2, Eq. (1)) per launch, FP32, held in registers.  Included by
// stream.hip (single grids) and stream_batch.hip (the grids of a batch).
//
// Each wave owns a strip of 256 columns (64 lanes x 4 adjacent cells) and a
// segment of rows, and walks down the segment one row per tick.  In every
// tick it first loads one new row of u, v and phi (a few rows ahead of use),
// then advances each time level t = 1..T by one row: level t turns rows
// rho-1, rho, rho+1 of u at step t-1 into row rho of u and v at step t,
// where rho = tick - t + 1 (a skew of one row per level, so level t reads
// the row level t-1 finished earlier in the same tick).  The last level's
// row is written out.  Every intermediate state stays in registers:
//   - each level t keeps the three rows of u^(t-1) its five-node sum needs
//     (row index mod 3; level 1 keeps u^0 rows mod 6 to leave room for the
//     loads in flight),
//   - v of the rows in flight sits in 12 row slots (row index mod 12); each
//     level updates it in place as the row passes it.
// c1*phi of the rows in flight is kept in a per-wave LDS ring of 16 rows.
// The tick loop is unrolled by 12, so every slot index is a compile-time
// constant and no value is ever moved between registers.  A wave's first
// 2T - 2 ticks (where level t has no row of its range before tick 2t - 2)
// are loop bodies of their own that leave those levels out, and its last,
// partial body a copy that stops after the last tick.  There are no LDS
// tiles and no barriers: waves run independently.  East / west neighbours
// cross lanes by DPP; the strip's outer columns are a halo of width >= T
// that goes stale by one column per level and is recomputed by the
// neighbouring strip, and a segment is extended by T rows above and below.
// Halo rows and columns beyond the domain are loaded mirrored (the even
// extension evolves exactly like the interior), so no level needs edge code.
// Every cell goes through cell_update, so the result is bit-identical to the
// one-step kernel and to the LDS tile kernel at any launch shape.
//
// Every tick issues the same memory instructions whatever the row or lane
// (rows past the segment and lanes outside the output use buffer offsets
// past the row's end, which the hardware drops), so the compiler can count
// outstanding loads exactly and wait only for the row a level is about to
// use.  Waves whose strip reaches past a domain edge load mirrored 16-byte
// blocks and put their cells in order on first use, where the width is a
// multiple of 4 (and at least 256); otherwise they take a second copy of the
// loop that loads and stores cell by cell.  The same pipeline also runs the
// grids of a batch (k_batch_stream: one wave per grid, strip and segment).
#pragma once

#include "batch.h"
#include "kernels.h"
#include "tile.h"

namespace rdc {
namespace {

using namespace dev;

constexpr int kStreamWaves = 4;   // waves per workgroup (independent pipelines)
constexpr int kUnroll = 12;       // ticks per unrolled loop body
constexpr int kRowSlots = 12;     // v of the rows in the levels: row index mod 12
constexpr int kU0Slots = 6;       // u^0 rows held by level 1: row index mod 6
constexpr int kAhead = 2;         // a row is loaded this many ticks before it enters level 1
constexpr int kStage = 3;         // v, phi of loaded rows waiting to enter: row index mod 3
constexpr int kPhiRows = 16;      // c1*phi rows in LDS per wave: row index mod 16
// A buffer offset past any row (rows are shorter than 2 GiB): the access is
// dropped.
constexpr int kOff = static_cast<int>(0x80000000u);

constexpr int md(int a, int m) { return ((a % m) + m) % m; }

// Column halo on the left of the strip: T rounded up to whole lanes, so the
// strip's loads and stores stay 16-byte aligned.
template <int T>
constexpr int stream_hx() { return (T + 3) & ~3; }

// Row slots: a row's v sits in its slot from the tick it enters level 1 to
// the tick level T is done with it (T rows at a time); u^0 rows i-1 ..
// i+1+kAhead fit the level-1 window; c1*phi rows in LDS likewise.
template <int T>
constexpr bool stream_fits() {
    return T >= 2 && T <= kRowSlots && T <= kPhiRows && kAhead + 3 <= kU0Slots &&
           kAhead + 1 <= kStage && kUnroll % kRowSlots == 0 && kUnroll % kU0Slots == 0 &&
           kUnroll % kStage == 0 && kUnroll % 3 == 0;
}

struct Lane {
    int gx;          // first global column of this lane's 4 cells
    int xb[4];       // byte offsets of its 4 columns, mirrored at the domain edges
    int so[4];       // byte offsets of its 4 output cells, or kOff where not stored
    int so4;         // byte offset of its 16-byte output word, or kOff
    bool rev;        // (kMirror) its 4 cells are a 16-byte block in reverse order
    uint64_t out;    // lanes holding output cells
};

// How a strip reads its columns:
//   kInterior  the strip lies inside the grid: one 16-byte word per lane;
//   kCells     it reaches past an edge: cell by cell, each column mirrored;
//   kMirror    any strip of a grid whose width is a multiple of 4 (and at
//              least 256): one 16-byte word per lane, which past an edge is
//              the mirrored block of 4 columns, taken in reverse order once a
//              row enters the levels (by the waves of edge strips only).
// kMirror keeps one copy of the loop in the kernel for every strip.
enum StripMode { kInterior = 0, kCells = 1, kMirror = 2 };

template <int T, int MODE>
__device__ __forceinline__ void stream_pipeline(const StepArgs<float>& a, const Lane& ln,
                                                int y0, int y1, float4 (&phs)[kPhiRows][64],
                                                bool edge_wave) {
    constexpr bool EDGE = MODE == kCells;
    const int ny = a.ny;
    const int lane = threadIdx.x & 63;
    const int64_t P = a.pitch;
    const int row_bytes = static_cast<int>(P * 4);
    const int i0 = y0 - T + 1;                 // first tick: level 1 on row y0 - T + 1
    const int i_end = y1 + T - 1;              // ticks [i0, i_end)
    // k0 kept in a VGPR: an FMA reads one scalar operand at most.
    Consts<float> k = a.k;
    k.k0 = __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(k.k0), 0xe4, 0xf, 0xf, false));

    // Every level runs on every tick from its first row on, also after its
    // last (levels t and t+1 stop together apart from one row, so such a row
    // of u^t is never read by level t+1, and a row's v is not touched by any
    // level after it left the range of rows that level owns); only level
    // T's output is checked and written, and only where it ran on a row of
    // the segment.  Slots start at zero.
    constexpr int kRampBodies = (2 * T - 2 + kUnroll - 1) / kUnroll;
    float u0[kU0Slots][4] = {};                // u^0 rows (level 1's window)
    float uw[T + 1][3][4] = {};                // uw[t]: rows of u^(t-1), t >= 2
    float vr[kRowSlots][4] = {};               // v of the rows in the levels
    float vs[kStage][4] = {};                  // v of loaded rows not yet in level 1
    float ps[kStage][4] = {};                  // phi of loaded rows not yet in level 1

    // Load row r of u (and of v, phi); rows past the last one any level
    // needs (i_end) read nothing.
    auto load_row = [&](int r, float (&uu)[4], float (&vv)[4], float (&pp)[4],
                        bool with_vp) __attribute__((always_inline)) {
        const int64_t off = (int64_t)reflect_index(r, ny) * P;
        const int nb = r <= i_end ? row_bytes : 0;
        const auto ru = row_rsrc(a.u + off, nb);
        const auto rv = row_rsrc(a.v + off, nb);
        const auto rp = row_rsrc(a.phi + off, nb);
        if (!EDGE) {
            const float4 t = buf_load4(ru, ln.xb[0]);
            uu[0] = t.x; uu[1] = t.y; uu[2] = t.z; uu[3] = t.w;
            if (with_vp) {
                const float4 w = buf_load4(rv, ln.xb[0]);
                vv[0] = w.x; vv[1] = w.y; vv[2] = w.z; vv[3] = w.w;
                const float4 p = buf_load4(rp, ln.xb[0]);
                pp[0] = p.x; pp[1] = p.y; pp[2] = p.z; pp[3] = p.w;
            }
        } else {
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                uu[c] = buf_load1(ru, ln.xb[c]);
                if (with_vp) {
                    vv[c] = buf_load1(rv, ln.xb[c]);
                    pp[c] = buf_load1(rp, ln.xb[c]);
                }
            }
        }
    };

    // kMirror: a mirrored block as loaded holds this lane's 4 cells in
    // reverse order; it is put right when the row is first used (the load
    // then has to be complete anyway), by the waves of edge strips only.
    auto unmirror = [&](float (&x)[4]) __attribute__((always_inline)) {
        if (MODE == kMirror && edge_wave) {
            const float x0 = x[0], x1 = x[1], x2 = x[2], x3 = x[3];
            x[0] = ln.rev ? x3 : x0;
            x[1] = ln.rev ? x2 : x1;
            x[2] = ln.rev ? x1 : x2;
            x[3] = ln.rev ? x0 : x3;
        }
    };

    // Rows the first ticks need: u^0 rows i0-1 .. i0+kAhead, v and phi rows
    // i0 .. i0+kAhead (relative row j: u^0 slot j mod 6, staging j mod 3).
    load_row(i0 - 1, u0[md(-1, kU0Slots)], vs[md(-1, kStage)], ps[md(-1, kStage)], false);
#pragma unroll
    for (int j = 0; j <= kAhead; ++j)
        load_row(i0 + j, u0[md(j, kU0Slots)], vs[md(j, kStage)], ps[md(j, kStage)], true);
    unmirror(u0[md(-1, kU0Slots)]);          // the first tick's north and centre rows
    unmirror(u0[md(0, kU0Slots)]);

    uint64_t bad = 0;
    // One tick: row i enters level 1.  s is the tick's place in the unrolled
    // body and fixes every slot.  ramp >= 0 in the first bodies a wave walks
    // (the body's first tick counted from i0): there level t has no row of
    // its range before tick i0 + 2t - 2 and is left out, which the compiler
    // settles, since ramp and s are constants once the bodies are unrolled.
    // ramp = -1 in the loop after them, where every level runs.
    auto tick = [&](const int i, const int s, const int ramp) __attribute__((always_inline)) {
        // Row i enters level 1: its v moves to its row slot (which held
        // row i - 12, done with since level T took it), its phi is
        // scaled once and kept in the wave's LDS ring for the levels.
        unmirror(vs[md(s, kStage)]);
        unmirror(ps[md(s, kStage)]);
        unmirror(u0[md(s + 1, kU0Slots)]);       // row i + 1: level 1's south from now on
        float cp[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            vr[md(s, kRowSlots)][c] = vs[md(s, kStage)][c];
            cp[c] = scaled_phi(ps[md(s, kStage)][c], k);
        }
        phs[i & (kPhiRows - 1)][lane] = make_float4(cp[0], cp[1], cp[2], cp[3]);
        // The row first needed kAhead ticks from now.  Its slots held row
        // i + 1 + kAhead - 6 (u^0) and - 3 (staging), both done with.
        load_row(i + 1 + kAhead, u0[md(s + 1 + kAhead, kU0Slots)],
                 vs[md(s + 1 + kAhead, kStage)], ps[md(s + 1 + kAhead, kStage)], true);

        float un[4];
        // level T runs on a row of the segment (uniform)
        const bool live_T = i >= i0 + 2 * T - 2 && i < i_end;
#pragma unroll
        for (int t = 1; t <= T; ++t) {
            if (ramp >= 0 && ramp + s < 2 * t - 2) continue;   // no row of level t yet
            const int rs = md(s - t + 1, kRowSlots);           // slot of row rho = i - t + 1
            const float* n;
            const float* c;
            const float* so;
            if (t == 1) {
                n = u0[md(s - 1, kU0Slots)];
                c = u0[md(s, kU0Slots)];
                so = u0[md(s + 1, kU0Slots)];
            } else {
                n = uw[t][md(s - t, 3)];
                c = uw[t][md(s - t + 1, 3)];
                so = uw[t][md(s - t + 2, 3)];
            }
            float pc[4];
            if (t == 1) {
#pragma unroll
                for (int e = 0; e < 4; ++e) pc[e] = cp[e];
            } else {
                const float4 q = phs[(i - t + 1) & (kPhiRows - 1)][lane];
                pc[0] = q.x; pc[1] = q.y; pc[2] = q.z; pc[3] = q.w;
            }
            // West and east enter the update as a sum.  Each lane shift sits
            // right before the update that takes it: the compiler folds a
            // shift into its add only a few instructions away.
            const float west = from_west_lane(c[3]);
            cell_update(c[0], c[1], west, n[0], so[0], vr[rs][0], pc[0], k, un[0],
                        vr[rs][0]);
            cell_update(c[1], c[0], c[2], n[1], so[1], vr[rs][1], pc[1], k, un[1],
                        vr[rs][1]);
            cell_update(c[2], c[1], c[3], n[2], so[2], vr[rs][2], pc[2], k, un[2],
                        vr[rs][2]);
            const float east = from_east_lane(c[0]);
            cell_update(c[3], c[2], east, n[3], so[3], vr[rs][3], pc[3], k, un[3],
                        vr[rs][3]);
            if (ramp >= 0) {
                // In the ramp bodies (straight-line code) the compiler would
                // otherwise sink a level's work to the tick where its results
                // are first read, holding the rows it reads live meanwhile.
#pragma unroll
                for (int e = 0; e < 4; ++e) asm volatile("" : "+v"(un[e]), "+v"(vr[rs][e]));
            }
            if (t < T) {
                // row rho of u^t: level t+1's newest row
#pragma unroll
                for (int e = 0; e < 4; ++e) uw[t < T ? t + 1 : T][md(s - t + 1, 3)][e] = un[e];
            } else if (live_T) {
#pragma unroll
                for (int e = 0; e < 4; ++e) {
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
            buf_store4(ro, ln.so4, un[0], un[1], un[2], un[3]);
            buf_store4(rv, ln.so4, vr[rs][0], vr[rs][1], vr[rs][2], vr[rs][3]);
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                buf_store1(ro, ln.so[e], un[e]);
                buf_store1(rv, ln.so[e], vr[rs][e]);
            }
        }
    };
    // A wave walks at least 2T - 1 ticks, so it always walks the ramp
    // bodies (as before, ticks past i_end load and store nothing).  Each is
    // written out: unrolling a loop over them would exceed the compiler's
    // limit for forced unrolling and leave `ramp` a run-time value.
    auto ramp_body = [&](const int r0) __attribute__((always_inline)) {
#pragma unroll
        for (int s = 0; s < kUnroll; ++s) {
            tick(i0 + r0 + s, s, r0);
            // keep the scheduler from hoisting later ticks' loads into this
            // one: in straight-line code it would hold many rows at once
            __builtin_amdgcn_sched_barrier(0);
        }
    };
    static_assert(kRampBodies >= 1 && kRampBodies <= 2, "ramp of at most two loop bodies");
    ramp_body(0);
    if constexpr (kRampBodies > 1) ramp_body(kUnroll);
    // Whole bodies, then the ticks left (fewer than kUnroll) by a copy that
    // stops after the last: a segment's ticks need not fill whole bodies.
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

// Output columns per strip: the loaded 256 less the left halo and a right
// halo of at least T, kept a multiple of 4.
template <int T>
constexpr int stream_bx() { return (256 - stream_hx<T>() - T) & ~3; }

// One wave's work item: output columns [strip * bx, strip * bx + bx) and
// output rows [y0, y1) of the grid `a` describes.
template <int T, bool MIRROR>
__device__ __forceinline__ void stream_wave(const StepArgs<float>& a, int strip, int y0, int y1,
                                            float4 (&phs)[kPhiRows][64]) {
    constexpr int HX = stream_hx<T>();
    constexpr int bx = stream_bx<T>();
    const int lane = threadIdx.x & 63;
    const int nx = a.nx;
    const int x_out0 = strip * bx;             // first output column
    const int x_load0 = x_out0 - HX;           // first loaded column
    Lane ln;
    ln.gx = x_load0 + 4 * lane;
#pragma unroll
    for (int c = 0; c < 4; ++c) ln.xb[c] = 4 * reflect_index(ln.gx + c, nx);
    ln.rev = false;
    if (MIRROR) {
        // Width a multiple of 4 and >= 256: a lane's 4 columns are all
        // inside or all past one edge, and their mirror images are the 4
        // columns of one block, in reverse order.
        if (ln.gx < 0) {
            ln.xb[0] = 4 * (-4 - ln.gx);
            ln.rev = true;
        } else if (ln.gx >= nx) {
            ln.xb[0] = 4 * (2 * nx - 4 - ln.gx);
            ln.rev = true;
        }
    }
    const bool out_lane = lane >= HX / 4 && lane < (HX + bx) / 4 && ln.gx < nx;
    ln.so4 = out_lane ? 4 * ln.gx : kOff;
#pragma unroll
    for (int c = 0; c < 4; ++c) ln.so[c] = out_lane && ln.gx + c < nx ? 4 * (ln.gx + c) : kOff;
    ln.out = __builtin_amdgcn_ballot_w64(out_lane);

    const bool inside = x_load0 >= 0 && x_load0 + 256 <= nx;
    if (MIRROR) {
        stream_pipeline<T, kMirror>(a, ln, y0, y1, phs, !inside);
    } else {
        // Interior strips load and store 16-byte words; a strip that reaches
        // past the left or right edge goes cell by cell.
        if (inside)
            stream_pipeline<T, kInterior>(a, ln, y0, y1, phs, false);
        else
            stream_pipeline<T, kCells>(a, ln, y0, y1, phs, true);
    }
}

// Work of one wave on a segment of `rows` output rows, in level-rows: T
// levels on each of its rows + 2T - 2 ticks (at least the ramp bodies) less
// the T(T-1) the ramp leaves out, about half a level per tick for its loads
// and stores, and two ticks for the first rows' load latency.
inline double wave_cost(int rows, int T) {
    const int64_t ticks = max(rows + 2 * T - 2, (2 * T - 2 + kUnroll - 1) / kUnroll * kUnroll);
    return (T + 0.5) * ticks - (double)T * (T - 1) + 2.0 * T;
}

}  // namespace
}  // namespace rdc
