// batch.hip -- many independent Oregonator grids (Sec. 2, Eq. (1)) advanced
// together: the C ABI rdc_batch_* / rdc_graph_* of include/rdc.h and its
// kernels.
//
// Every grid lives in its own region of five pooled planes.  Small grids
// (at most a set number of cells, and a shape the whole-grid LDS kernel of
// resident.hip takes) run every step of a call on chip, one workgroup each,
// on a second stream forked from and joined back into the caller's.  The
// others are stepped T steps per launch: a launch covers a flat list of work
// items (grid, tile column, tile row) built once per (T, tile rows); each
// 512-thread workgroup takes one item, reads that grid's descriptor (size,
// pitch, plane offset, scheme constants) and runs the same tile routine as
// the single-grid kernel.  Both paths use the one cell update, so a grid in
// a batch evolves bit-identically to the same grid stepped alone.  A whole
// run can be recorded into a HIP graph and replayed as one submission.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <map>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "../../include/rdc.h"
#include "batch.h"
#include "kernels.h"
#include "tile.h"

namespace rdc {
namespace {

using namespace dev;

struct Item {
    int sim, tx, ty, pad;
};

struct BatchArgs {
    const float* u;
    const float* v;
    const float* phi;
    float* u_out;
    float* v_out;
    const SimDev* sims;
    const Item* items;
    int* flags;
    int nitems, per_xcd;
};

template <int T, int R>
__global__ __launch_bounds__(kTileWaves * 64, (tile_waves_per_simd<R, false>()))
void k_batch_stepT(BatchArgs b) {
    __shared__ float4 lds[kTileWaves * R][64];
    // Consecutive items are neighbouring tiles of one grid; deal them to the
    // XCDs in contiguous runs (see k_stepT).
    const int item = (blockIdx.x & 7) * b.per_xcd + (blockIdx.x >> 3);
    if (item >= b.nitems) return;
    const Item it = b.items[item];
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
    step_tile<T, R, false>(a, it.tx, it.ty, lds);
}

struct BatchDisks {
    int sim[kMaxDisks], cx[kMaxDisks], cy[kMaxDisks], r[kMaxDisks];
    int count;
};

__global__ __launch_bounds__(256) void k_batch_stimulate(float* u, const SimDev* sims,
                                                         BatchDisks d) {
    const int i = blockIdx.x;
    if (i >= d.count) return;
    const SimDev sd = sims[d.sim[i]];
    const int64_t cx = d.cx[i], cy = d.cy[i], r = d.r[i];
    const int64_t x_lo = cx - r > 0 ? cx - r : 0;
    const int64_t x_hi = cx + r < sd.nx - 1 ? cx + r : sd.nx - 1;
    const int64_t y_lo = cy - r > 0 ? cy - r : 0;
    const int64_t y_hi = cy + r < sd.ny - 1 ? cy + r : sd.ny - 1;
    if (x_hi < x_lo || y_hi < y_lo) return;
    const int64_t w = x_hi - x_lo + 1, n = w * (y_hi - y_lo + 1);
    float* base = u + sd.offset;
    for (int64_t j = threadIdx.x; j < n; j += blockDim.x) {
        const int64_t x = x_lo + j % w, y = y_lo + j / w;
        const int64_t dx = x - cx, dy = y - cy;
        if (dx * dx + dy * dy <= r * r) base[y * sd.pitch + x] = 1.0f;
    }
}

__global__ void k_clear_flags(int* flags, int n) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        flags[i] = 0;
}

template <int T, int R>
hipError_t batch_launch(const BatchArgs& b, hipStream_t s) {
    const dim3 grid(8 * b.per_xcd), block(kTileWaves * 64);
    hipLaunchKernelGGL((k_batch_stepT<T, R>), grid, block, 0, s, b);
    return hipGetLastError();
}

template <int R>
hipError_t batch_launch_T(const BatchArgs& b, int T, hipStream_t s) {
    switch (T) {
        case 1: return batch_launch<1, R>(b, s);
        case 2: return batch_launch<2, R>(b, s);
        case 3: return batch_launch<3, R>(b, s);
        case 4: return batch_launch<4, R>(b, s);
        case 5: return batch_launch<5, R>(b, s);
        case 6: return batch_launch<6, R>(b, s);
        case 7: return batch_launch<7, R>(b, s);
        case 8: return batch_launch<8, R>(b, s);
        case 9: return batch_launch<9, R>(b, s);
        case 10: return batch_launch<10, R>(b, s);
        case 11: return batch_launch<11, R>(b, s);
        case 12: return batch_launch<12, R>(b, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t batch_launch_any(const BatchArgs& b, int T, int rows, hipStream_t s) {
    switch (rows) {
        case 48: return batch_launch_T<6>(b, T, s);
        case 56: return batch_launch_T<7>(b, T, s);
        case 64: return batch_launch_T<8>(b, T, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace
}  // namespace rdc

struct rdc_batch {
    int count = 0;
    std::vector<rdc_sim_desc> sims;
    float* pool[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};  // u0 u1 v0 v1 phi
    int64_t pool_elems = 0;
    hipStream_t stream = nullptr;
    int device = 0;
    int cur = 0;
    int T = 8, rows = 56;
    int64_t step = 0;
    rdc::SimDev* d_sims = nullptr;
    int* d_flags = nullptr;
    // tile work items of the grids not taken by the resident kernel
    std::map<std::pair<int, int>, std::pair<rdc::Item*, int>> items;  // (T, rows) -> list
    // their row-pipeline work items (rows == RDC_TILE_STREAM)
    std::map<int, std::pair<rdc::StreamItem*, int>> sitems;          // T -> list
    // whole-grid LDS path: cell limit, which grids it takes, their items
    int32_t res_max_cells = RDC_BATCH_RESIDENT_DEFAULT;
    std::vector<char> resident;
    rdc::ResItem* d_res = nullptr;
    int nres = 0;
    hipStream_t side = nullptr;            // the resident launches' stream
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    int64_t plan = 0;                      // bumped when the tables above are replaced
    std::string err;
};

// One recording of the launch sequence per ping-pong parity: entry p starts
// from the planes with index p, so a replay is right whichever planes hold
// the state when it is launched (eager steps between replays may flip it).
struct rdc_graph {
    rdc_batch* b = nullptr;
    hipGraph_t graph[2] = {nullptr, nullptr};
    hipGraphExec_t exec[2] = {nullptr, nullptr};
    int64_t n = 0;
    int64_t plan = 0;                      // the batch's plan the recording refers to
};

namespace {

std::string g_batch_error;

rdc_status bfail(rdc_batch* b, rdc_status s, const std::string& m) {
    if (b)
        b->err = m;
    else
        g_batch_error = m;
    return s;
}

rdc_status bhip(rdc_batch* b, hipError_t e, const char* what) {
    return bfail(b, RDC_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

const char* check_sim_params(const rdc_params& p) {
    if (!(p.eps > 0.0)) return "eps must be > 0";
    if (!std::isfinite(p.f)) return "f must be finite";
    if (!(p.q > 0.0) || !std::isfinite(p.q)) return "q must be finite and > 0";
    if (!(p.D_u >= 0.0) || !std::isfinite(p.D_u)) return "D_u must be finite and >= 0";
    if (!(p.dt > 0.0) || !std::isfinite(p.dt)) return "dt must be finite and > 0";
    if (!(p.dx > 0.0) || !std::isfinite(p.dx)) return "dx must be finite and > 0";
    if (p.dt * p.D_u / (p.dx * p.dx) > 0.25)
        return "dt*D_u/dx^2 exceeds 1/4, the explicit five-node diffusion bound";
    return nullptr;
}

rdc::Consts<float> sim_consts(const rdc_params& p) {
    // Same constants as the single-grid path.
    return rdc::make_consts<float>(p.eps, p.f, p.q, p.D_u, p.dt, p.dx);
}

struct Dev {
    int prev = -1;
    explicit Dev(int d) {
        if (hipGetDevice(&prev) == hipSuccess && prev != d) (void)hipSetDevice(d);
    }
    ~Dev() {
        int now = -1;
        if (prev >= 0 && hipGetDevice(&now) == hipSuccess && now != prev) (void)hipSetDevice(prev);
    }
};

// Work items of every grid for (T, rows), built once and kept on the device.
rdc_status items_for(rdc_batch* b, int T, int rows, const rdc::Item** out, int* n) {
    const auto key = std::make_pair(T, rows);
    auto it = b->items.find(key);
    if (it == b->items.end()) {
        const int HX = (T + 3) & ~3;
        const int BX = rdc::dev::kTileCols - 2 * HX;
        const int BY = rows - 2 * T;
        std::vector<rdc::Item> list;
        for (int s = 0; s < b->count; ++s) {
            if (b->resident[s]) continue;
            const int tx_n = (b->sims[s].nx + BX - 1) / BX;
            const int ty_n = (b->sims[s].ny + BY - 1) / BY;
            for (int ty = 0; ty < ty_n; ++ty)
                for (int tx = 0; tx < tx_n; ++tx) list.push_back({s, tx, ty, 0});
        }
        rdc::Item* d = nullptr;
        hipError_t e = hipSuccess;
        if (!list.empty()) e = hipMalloc(&d, sizeof(rdc::Item) * list.size());
        if (e == hipSuccess && !list.empty())
            e = hipMemcpy(d, list.data(), sizeof(rdc::Item) * list.size(), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            if (d) (void)hipFree(d);
            return bhip(b, e, "work-item table");
        }
        it = b->items.emplace(key, std::make_pair(d, static_cast<int>(list.size()))).first;
    }
    *out = it->second.first;
    *n = it->second.second;
    return RDC_OK;
}

rdc::BatchArgs batch_args(const rdc_batch* b, const rdc::Item* items, int n) {
    rdc::BatchArgs a;
    a.u = b->pool[b->cur];
    a.v = b->pool[2 + b->cur];
    a.phi = b->pool[4];
    a.u_out = b->pool[b->cur ^ 1];
    a.v_out = b->pool[2 + (b->cur ^ 1)];
    a.sims = b->d_sims;
    a.items = items;
    a.flags = b->d_flags;
    a.nitems = n;
    a.per_xcd = (n + 7) / 8;
    return a;
}

// Row-pipeline work items of every tiled grid for T steps per launch
// (2..11), built once and kept on the device.
rdc_status stream_items_for(rdc_batch* b, int T, const rdc::StreamItem** out, int* n) {
    auto it = b->sitems.find(T);
    if (it == b->sitems.end()) {
        std::vector<rdc::GridShape> grids;
        for (int s = 0; s < b->count; ++s)
            if (!b->resident[s]) grids.push_back({s, b->sims[s].nx, b->sims[s].ny});
        const std::vector<rdc::StreamItem> list =
            rdc::batch_stream_items(grids, T, rdc::stream_slots());
        rdc::StreamItem* d = nullptr;
        hipError_t e = hipSuccess;
        if (!list.empty()) e = hipMalloc(&d, sizeof(rdc::StreamItem) * list.size());
        if (e == hipSuccess && !list.empty())
            e = hipMemcpy(d, list.data(), sizeof(rdc::StreamItem) * list.size(),
                          hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            if (d) (void)hipFree(d);
            return bhip(b, e, "row-pipeline work-item table");
        }
        it = b->sitems.emplace(T, std::make_pair(d, static_cast<int>(list.size()))).first;
    }
    *out = it->second.first;
    *n = it->second.second;
    return RDC_OK;
}

// Whether a launch of k steps runs on the row pipelines (else on tiles).
bool stream_launch(const rdc_batch* b, int k) {
    return b->rows == RDC_TILE_STREAM && k >= 2 && k <= rdc::kMaxStreamCells;
}

// Tile height of the tiled launches (the row pipelines' batches take 56-row
// tiles for launches the pipelines do not run: one step).
int tile_rows_of(const rdc_batch* b) { return b->rows == RDC_TILE_STREAM ? 56 : b->rows; }

// Builds the work-item table a launch of k steps needs.
rdc_status tables_for(rdc_batch* b, int k) {
    int cnt = 0;
    if (stream_launch(b, k)) {
        const rdc::StreamItem* items = nullptr;
        return stream_items_for(b, k, &items, &cnt);
    }
    const rdc::Item* items = nullptr;
    return items_for(b, k, tile_rows_of(b), &items, &cnt);
}

// One launch of k steps over the tiled grids, from planes b->cur.
rdc_status launch_tiled(rdc_batch* b, int k, hipStream_t s, hipError_t* e) {
    int cnt = 0;
    if (stream_launch(b, k)) {
        const rdc::StreamItem* items = nullptr;
        const rdc_status st = stream_items_for(b, k, &items, &cnt);
        if (st != RDC_OK) return st;
        rdc::BatchStreamArgs a;
        a.u = b->pool[b->cur];
        a.v = b->pool[2 + b->cur];
        a.phi = b->pool[4];
        a.u_out = b->pool[b->cur ^ 1];
        a.v_out = b->pool[2 + (b->cur ^ 1)];
        a.sims = b->d_sims;
        a.items = items;
        a.flags = b->d_flags;
        a.nitems = cnt;
        a.per_xcd = ((cnt + 3) / 4 + 7) / 8;
        *e = rdc::launch_batch_stream(a, k, s);
        return RDC_OK;
    }
    const rdc::Item* items = nullptr;
    const rdc_status st = items_for(b, k, tile_rows_of(b), &items, &cnt);
    if (st != RDC_OK) return st;
    *e = rdc::batch_launch_any(batch_args(b, items, cnt), k, tile_rows_of(b), s);
    return RDC_OK;
}


// Steps per launch for advancing n steps: ceil(n/T) launches of near-equal
// length (a short remainder launch would pay a whole tile load and store for
// a step or two); with `even`, one launch more when that count is odd, so the
// ping-pong index ends where it started (impossible only for T = 1 and odd n).
std::vector<int> plan_launches(int64_t n, int T, bool even) {
    std::vector<int> ks;
    int64_t m = (n + T - 1) / T;
    if (even && m % 2 == 1 && n >= m + 1) ++m;
    while (n > 0) {
        const int k = static_cast<int>((n + m - 1) / m);
        ks.push_back(k);
        n -= k;
        --m;
    }
    return ks;
}

// Advances every grid n steps: the tiled grids by the launches `ks` (steps
// per launch) on stream s, the resident grids meanwhile by whole-grid
// launches on the side stream, forked from s before and joined into s after
// (event record / wait, which a stream capture records as graph edges).  The
// resident grids read the planes the state is in and write the ones the
// tiled grids end in (the same planes when the launch count is even: each
// grid is read whole before any of it is written).
rdc_status run_launches(rdc_batch* b, const std::vector<int>& ks, int64_t n, hipStream_t s) {
    const bool tiled = b->nres < b->count;
    const int start = b->cur;
    const int end = tiled ? start ^ static_cast<int>(ks.size() & 1) : start;
    const bool res = b->nres > 0 && n > 0;
    hipError_t e = hipSuccess;
    const char* what = nullptr;
    bool forked = false;
    if (res) {
        e = hipEventRecord(b->ev_fork, s);
        if (e == hipSuccess) e = hipStreamWaitEvent(b->side, b->ev_fork, 0);
        forked = e == hipSuccess;
        for (int64_t done = 0; e == hipSuccess && done < n;) {
            const int k = static_cast<int>(std::min<int64_t>(n - done, rdc::kResMaxSteps));
            const int from = done == 0 ? start : end;
            rdc::ResArgs a;
            a.u = b->pool[from];
            a.v = b->pool[2 + from];
            a.phi = b->pool[4];
            a.u_out = b->pool[end];
            a.v_out = b->pool[2 + end];
            a.sims = b->d_sims;
            a.items = b->d_res;
            a.flags = b->d_flags;
            a.count = b->nres;
            a.steps = k;
            e = rdc::launch_resident(a, b->side);
            done += k;
        }
        if (forked) {
            const hipError_t ej = hipEventRecord(b->ev_join, b->side);
            if (e == hipSuccess) e = ej;
        }
        if (e != hipSuccess) what = "whole-grid launch";
    }
    rdc_status st = RDC_OK;
    if (tiled && e == hipSuccess) {
        for (const int k : ks) {
            st = launch_tiled(b, k, s, &e);
            if (st != RDC_OK) break;
            if (e != hipSuccess) {
                what = "batched step launch";
                break;
            }
            b->cur ^= 1;
        }
    }
    // The side stream is joined back whatever failed, so it never stays
    // forked (a capture would not end otherwise).
    if (forked) {
        const hipError_t ej = hipStreamWaitEvent(s, b->ev_join, 0);
        if (e == hipSuccess && st == RDC_OK && ej != hipSuccess) {
            e = ej;
            what = "whole-grid join";
        }
    }
    if (e != hipSuccess) return bhip(b, e, what ? what : "whole-grid fork");
    return st;
}

// Which grids the whole-grid kernel takes (nx * ny <= max_cells and a shape
// it holds), and its work-item table; the tile item tables are rebuilt.
rdc_status set_resident(rdc_batch* b, int32_t max_cells) {
    std::vector<rdc::ResItem> list;
    std::vector<char> flag(b->count, 0);
    for (int i = 0; i < b->count; ++i) {
        const rdc_sim_desc& d = b->sims[i];
        int m = 0, groups = 0;
        if ((int64_t)d.nx * d.ny <= max_cells && rdc::resident_layout(d.nx, d.ny, &m, &groups)) {
            list.push_back({i, m, groups, 0});
            flag[i] = 1;
        }
    }
    // Longest first: workgroups start in index order as CUs free up (one
    // grid per CU at a time), and a grid's time is about its rows per thread
    // times its waves, so this order keeps the CUs' finishing times even.
    auto cost = [&](const rdc::ResItem& r) {
        const int64_t waves = ((int64_t)r.groups * b->sims[r.sim].nx + 63) / 64;
        return waves * r.m;
    };
    std::stable_sort(list.begin(), list.end(), [&](const rdc::ResItem& a, const rdc::ResItem& c) {
        return cost(a) > cost(c);
    });
    rdc::ResItem* d = nullptr;
    hipError_t e = hipSuccess;
    if (!list.empty()) e = hipMalloc(&d, sizeof(rdc::ResItem) * list.size());
    if (e == hipSuccess && !list.empty())
        e = hipMemcpy(d, list.data(), sizeof(rdc::ResItem) * list.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        if (d) (void)hipFree(d);
        return bhip(b, e, "whole-grid item table");
    }
    // launches already queued may still read the old tables
    e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) {
        if (d) (void)hipFree(d);
        return bhip(b, e, "device error before re-planning");
    }
    if (b->d_res) (void)hipFree(b->d_res);
    for (auto& kv : b->items) (void)hipFree(kv.second.first);
    b->items.clear();
    for (auto& kv : b->sitems) (void)hipFree(kv.second.first);
    b->sitems.clear();
    b->d_res = d;
    b->nres = static_cast<int>(list.size());
    ++b->plan;
    b->resident.swap(flag);
    b->res_max_cells = max_cells;
    return RDC_OK;
}

rdc_status copy_sim_plane(rdc_batch* b, int sim, float* pool, const void* src, int64_t spitch,
                          rdc_where where, bool to_pool) {
    const rdc_sim_desc& d = b->sims[sim];
    float* region = pool + d.offset;
    hipMemcpyKind kind;
    if (to_pool)
        kind = where == RDC_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    else
        kind = where == RDC_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
    hipError_t e;
    if (to_pool)
        e = hipMemcpy2DAsync(region, d.pitch * 4, src, spitch * 4, d.nx * 4, d.ny, kind, b->stream);
    else
        e = hipMemcpy2DAsync(const_cast<void*>(src), spitch * 4, region, d.pitch * 4, d.nx * 4,
                             d.ny, kind, b->stream);
    if (e == hipSuccess && where == RDC_HOST) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return bhip(b, e, "plane copy");
    return RDC_OK;
}

// Device objects of a batch (also of one whose creation failed part way).
void release(rdc_batch* b) {
    if (b->side) (void)hipStreamSynchronize(b->side);
    for (auto& kv : b->items) (void)hipFree(kv.second.first);
    b->items.clear();
    for (auto& kv : b->sitems) (void)hipFree(kv.second.first);
    b->sitems.clear();
    if (b->d_res) (void)hipFree(b->d_res);
    if (b->d_sims) (void)hipFree(b->d_sims);
    if (b->d_flags) (void)hipFree(b->d_flags);
    if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
    if (b->ev_join) (void)hipEventDestroy(b->ev_join);
    if (b->side) (void)hipStreamDestroy(b->side);
    b->d_res = nullptr;
    b->d_sims = nullptr;
    b->d_flags = nullptr;
    b->ev_fork = b->ev_join = nullptr;
    b->side = nullptr;
}

}  // namespace

extern "C" {

const char* rdc_batch_last_error(const rdc_batch* b) {
    return b ? b->err.c_str() : g_batch_error.c_str();
}

rdc_status rdc_batch_create(int32_t count, const rdc_sim_desc* sims, const rdc_buffers* pool,
                            int64_t pool_elems, void* hip_stream, rdc_batch** out) {
    g_batch_error.clear();
    if (!out) return bfail(nullptr, RDC_E_INVAL, "out is NULL");
    *out = nullptr;
    if (count < 1 || !sims || !pool) return bfail(nullptr, RDC_E_INVAL, "need count >= 1, sims, pool");
    const void* planes[5] = {pool->u[0], pool->u[1], pool->v[0], pool->v[1], pool->phi};
    for (const void* p : planes)
        if (!p || (reinterpret_cast<uintptr_t>(p) & 255u))
            return bfail(nullptr, RDC_E_INVAL, "pool planes must be non-NULL and 256-byte aligned");
    std::vector<std::pair<int64_t, int64_t>> spans;
    for (int i = 0; i < count; ++i) {
        const rdc_sim_desc& d = sims[i];
        if (d.nx < 1 || d.ny < 1) return bfail(nullptr, RDC_E_INVAL, "grid sizes must be >= 1");
        if (d.pitch < d.nx || d.pitch % 64 || d.offset < 0 || d.offset % 64)
            return bfail(nullptr, RDC_E_INVAL, "pitch/offset must be multiples of 64, pitch >= nx");
        if (d.pitch * 4 > INT32_MAX) return bfail(nullptr, RDC_E_INVAL, "row too long");
        if (d.offset + d.pitch * d.ny > pool_elems)
            return bfail(nullptr, RDC_E_INVAL, "a simulation extends past the pool");
        if (const char* why = check_sim_params(d.params)) return bfail(nullptr, RDC_E_INVAL, why);
        spans.push_back({d.offset, d.offset + d.pitch * d.ny});
    }
    std::sort(spans.begin(), spans.end());
    for (size_t i = 1; i < spans.size(); ++i)
        if (spans[i].first < spans[i - 1].second)
            return bfail(nullptr, RDC_E_INVAL, "simulation regions overlap");
    rdc_batch* b = new (std::nothrow) rdc_batch;
    if (!b) return bfail(nullptr, RDC_E_NOMEM, "host allocation failed");
    b->count = count;
    b->sims.assign(sims, sims + count);
    for (int i = 0; i < 5; ++i) b->pool[i] = static_cast<float*>(const_cast<void*>(planes[i]));
    b->pool_elems = pool_elems;
    b->stream = static_cast<hipStream_t>(hip_stream);
    std::vector<rdc::SimDev> host(count);
    for (int i = 0; i < count; ++i)
        host[i] = {sims[i].nx, sims[i].ny, sims[i].pitch, sims[i].offset, sim_consts(sims[i].params)};
    hipError_t e = hipGetDevice(&b->device);
    if (e == hipSuccess) e = hipMalloc(&b->d_sims, sizeof(rdc::SimDev) * count);
    if (e == hipSuccess) e = hipMalloc(&b->d_flags, sizeof(int) * count);
    if (e == hipSuccess)
        e = hipMemcpy(b->d_sims, host.data(), sizeof(rdc::SimDev) * count, hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(rdc::k_clear_flags, dim3((count + 255) / 256), dim3(256), 0, b->stream,
                           b->d_flags, count);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_join, hipEventDisableTiming);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    rdc_status st = RDC_OK;
    if (e == hipSuccess) st = set_resident(b, RDC_BATCH_RESIDENT_DEFAULT);
    if (e != hipSuccess || st != RDC_OK) {
        const std::string m = e != hipSuccess ? std::string("device setup: ") + hipGetErrorString(e)
                                              : b->err;
        release(b);
        delete b;
        if (st != RDC_OK) return bfail(nullptr, st, m);
        return bfail(nullptr, e == hipErrorOutOfMemory ? RDC_E_NOMEM : RDC_E_DEVICE, m);
    }
    *out = b;
    return RDC_OK;
}

rdc_status rdc_batch_destroy(rdc_batch* b) {
    if (!b) return RDC_OK;
    Dev g(b->device);
    (void)hipStreamSynchronize(b->stream);
    release(b);
    delete b;
    return RDC_OK;
}

rdc_status rdc_batch_set_resident(rdc_batch* b, int32_t max_cells) {
    if (!b) return RDC_E_INVAL;
    if (max_cells < 0) return bfail(b, RDC_E_INVAL, "max_cells < 0");
    Dev g(b->device);
    return set_resident(b, max_cells);
}

int32_t rdc_batch_resident_count(const rdc_batch* b) { return b ? b->nres : -1; }

rdc_status rdc_batch_set_block(rdc_batch* b, int32_t T, int32_t rows) {
    if (!b) return RDC_E_INVAL;
    if (T < 1 || T > rdc::kMaxBlock) return bfail(b, RDC_E_INVAL, "T must be in 1..12");
    if (rows != 48 && rows != 56 && rows != 64 && rows != RDC_TILE_STREAM)
        return bfail(b, RDC_E_INVAL, "rows must be 48, 56, 64 or RDC_TILE_STREAM");
    if (rows == RDC_TILE_STREAM && T > rdc::kMaxStreamCells)
        return bfail(b, RDC_E_INVAL, "the row pipelines take at most 11 steps per launch");
    b->T = T;
    b->rows = rows;
    return RDC_OK;
}

rdc_status rdc_batch_set_phi(rdc_batch* b, int32_t sim, const void* phi, int64_t pitch,
                             rdc_where where) {
    if (!b) return RDC_E_INVAL;
    if (sim < 0 || sim >= b->count || !phi || pitch < b->sims[sim].nx)
        return bfail(b, RDC_E_INVAL, "bad simulation index, NULL or pitch < nx");
    Dev g(b->device);
    return copy_sim_plane(b, sim, b->pool[4], phi, pitch, where, true);
}

rdc_status rdc_batch_write(rdc_batch* b, int32_t sim, const void* u, const void* v,
                           int64_t pitch, rdc_where where) {
    if (!b) return RDC_E_INVAL;
    if (sim < 0 || sim >= b->count || !u || !v || pitch < b->sims[sim].nx)
        return bfail(b, RDC_E_INVAL, "bad simulation index, NULL or pitch < nx");
    Dev g(b->device);
    rdc_status s = copy_sim_plane(b, sim, b->pool[b->cur], u, pitch, where, true);
    if (s == RDC_OK) s = copy_sim_plane(b, sim, b->pool[2 + b->cur], v, pitch, where, true);
    if (s != RDC_OK) return s;
    hipLaunchKernelGGL(rdc::k_clear_flags, dim3(1), dim3(64), 0, b->stream, b->d_flags + sim, 1);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return bhip(b, e, "flag reset");
    return RDC_OK;
}

rdc_status rdc_batch_stimulate(rdc_batch* b, const int32_t* sim, const int32_t* cx,
                               const int32_t* cy, const int32_t* r, int32_t k) {
    if (!b) return RDC_E_INVAL;
    if (k < 0) return bfail(b, RDC_E_INVAL, "k < 0");
    if (k == 0) return RDC_OK;
    if (!sim || !cx || !cy || !r) return bfail(b, RDC_E_INVAL, "disk arrays are NULL");
    for (int32_t i = 0; i < k; ++i) {
        if (sim[i] < 0 || sim[i] >= b->count) return bfail(b, RDC_E_INVAL, "bad simulation index");
        if (r[i] < 0) return bfail(b, RDC_E_INVAL, "disk radius < 0");
        const rdc_sim_desc& d = b->sims[sim[i]];
        const int64_t px = std::min<int64_t>(std::max<int64_t>(cx[i], 0), d.nx - 1);
        const int64_t py = std::min<int64_t>(std::max<int64_t>(cy[i], 0), d.ny - 1);
        const int64_t dx = px - cx[i], dy = py - cy[i];
        if (dx * dx + dy * dy > (int64_t)r[i] * r[i])
            return bfail(b, RDC_E_INVAL, "a stimulus disk covers no cell of its grid");
    }
    Dev g(b->device);
    for (int32_t i0 = 0; i0 < k; i0 += rdc::kMaxDisks) {
        rdc::BatchDisks d;
        d.count = std::min<int32_t>(k - i0, rdc::kMaxDisks);
        for (int j = 0; j < d.count; ++j) {
            d.sim[j] = sim[i0 + j];
            d.cx[j] = cx[i0 + j];
            d.cy[j] = cy[i0 + j];
            d.r[j] = r[i0 + j];
        }
        hipLaunchKernelGGL(rdc::k_batch_stimulate, dim3(d.count), dim3(256), 0, b->stream,
                           b->pool[b->cur], b->d_sims, d);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return bhip(b, e, "stimulate launch");
    }
    return RDC_OK;
}

rdc_status rdc_batch_step(rdc_batch* b, int64_t n) {
    if (!b) return RDC_E_INVAL;
    if (n < 0) return bfail(b, RDC_E_INVAL, "n < 0");
    Dev g(b->device);
    rdc_status s = run_launches(b, plan_launches(n, b->T, false), n, b->stream);
    if (s == RDC_OK) b->step += n;
    return s;
}

rdc_status rdc_batch_read(rdc_batch* b, int32_t sim, void* u, void* v, int64_t pitch,
                          rdc_where where) {
    if (!b) return RDC_E_INVAL;
    if (sim < 0 || sim >= b->count || ((u || v) && pitch < b->sims[sim].nx))
        return bfail(b, RDC_E_INVAL, "bad simulation index or pitch < nx");
    Dev g(b->device);
    hipError_t e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return bhip(b, e, "device error before read");
    int flag = 0;
    e = hipMemcpy(&flag, b->d_flags + sim, sizeof(int), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return bhip(b, e, "flag read");
    if (u) {
        rdc_status s = copy_sim_plane(b, sim, b->pool[b->cur], u, pitch, where, false);
        if (s != RDC_OK) return s;
    }
    if (v) {
        rdc_status s = copy_sim_plane(b, sim, b->pool[2 + b->cur], v, pitch, where, false);
        if (s != RDC_OK) return s;
    }
    if (where == RDC_DEVICE) {
        e = hipStreamSynchronize(b->stream);
        if (e != hipSuccess) return bhip(b, e, "read copy");
    }
    if (flag) return bfail(b, RDC_E_NONFINITE, "a non-finite u or v was produced");
    return RDC_OK;
}

rdc_status rdc_batch_current(rdc_batch* b, void** u_pool, void** v_pool) {
    if (!b) return RDC_E_INVAL;
    if (!u_pool || !v_pool) return bfail(b, RDC_E_INVAL, "NULL output");
    *u_pool = b->pool[b->cur];
    *v_pool = b->pool[2 + b->cur];
    return RDC_OK;
}

rdc_status rdc_batch_capture(rdc_batch* b, int64_t n, rdc_graph** out) {
    if (!b) return RDC_E_INVAL;
    if (!out || n < 2) return bfail(b, RDC_E_INVAL, "need an output and n >= 2");
    *out = nullptr;
    const std::vector<int> ks = plan_launches(n, b->T, true);
    if (ks.size() % 2) return bfail(b, RDC_E_INVAL, "with T = 1, n must be even");
    Dev g(b->device);
    // Work-item tables are made before capture: nothing allocates inside it.
    for (const int k : ks) {
        rdc_status s = tables_for(b, k);
        if (s != RDC_OK) return s;
    }
    hipStream_t cs = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e != hipSuccess) return bhip(b, e, "capture stream");
    rdc_graph* gr = new (std::nothrow) rdc_graph;
    if (!gr) {
        (void)hipStreamDestroy(cs);
        return bfail(b, RDC_E_NOMEM, "host allocation failed");
    }
    const int cur0 = b->cur;
    rdc_status s = RDC_OK;
    for (int p = 0; p < 2 && e == hipSuccess && s == RDC_OK; ++p) {
        b->cur = p;
        e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) s = run_launches(b, ks, n, cs);
        const hipError_t e2 = hipStreamEndCapture(cs, &gr->graph[p]);
        if (e == hipSuccess) e = e2;
        if (e == hipSuccess && s == RDC_OK)
            e = hipGraphInstantiate(&gr->exec[p], gr->graph[p], nullptr, nullptr, 0);
    }
    b->cur = cur0;  // capture queues nothing: the state is where it was
    (void)hipStreamDestroy(cs);
    if (e != hipSuccess || s != RDC_OK) {
        for (int p = 0; p < 2; ++p) {
            if (gr->exec[p]) (void)hipGraphExecDestroy(gr->exec[p]);
            if (gr->graph[p]) (void)hipGraphDestroy(gr->graph[p]);
        }
        delete gr;
        return s != RDC_OK ? s : bhip(b, e, "graph capture");
    }
    gr->b = b;
    gr->n = n;
    gr->plan = b->plan;
    *out = gr;
    return RDC_OK;
}

rdc_status rdc_graph_launch(rdc_graph* g) {
    if (!g || !g->b) return RDC_E_INVAL;
    if (g->plan != g->b->plan)
        return bfail(g->b, RDC_E_STATE, "the batch was re-planned (rdc_batch_set_resident) "
                                        "after this graph was captured");
    Dev d(g->b->device);
    hipError_t e = hipGraphLaunch(g->exec[g->b->cur], g->b->stream);
    if (e != hipSuccess) return bhip(g->b, e, "graph launch");
    // an even number of launches: the state ends in the planes it started in
    g->b->step += g->n;
    return RDC_OK;
}

rdc_status rdc_graph_destroy(rdc_graph* g) {
    if (!g) return RDC_OK;
    if (g->b) {
        Dev d(g->b->device);
        (void)hipStreamSynchronize(g->b->stream);
    }
    for (int p = 0; p < 2; ++p) {
        if (g->exec[p]) (void)hipGraphExecDestroy(g->exec[p]);
        if (g->graph[p]) (void)hipGraphDestroy(g->graph[p]);
    }
    delete g;
    return RDC_OK;
}

}  // extern "C"
