// api.hip -- the C ABI of librdc (declared in include/rdc.h): argument
// checking, ping-pong bookkeeping and launch planning around the kernels.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "../../include/rdc.h"
#include "kernels.h"

struct rdc_ctx {
    int nx = 0, ny = 0;
    rdc_dtype dtype = RDC_FP32;
    void* u[2] = {nullptr, nullptr};
    void* v[2] = {nullptr, nullptr};
    void* phi = nullptr;
    int64_t pitch = 0;
    hipStream_t stream = nullptr;
    int device = 0;
    int cur = 0;                    // index of the planes holding the current state
    rdc_params p{};
    int T = 0;                      // steps per launch (0 = auto)
    int tile_rows = 0;              // tile height (0 = auto)
    int64_t step = 0;               // steps taken since creation
    int* d_flag = nullptr;          // sticky non-finite flag
    int32_t* arrival = nullptr;
    int64_t apitch = 0;
    double theta = 0.5;
    void* tl = nullptr;             // timelapse plane (running max of u over frames)
    int64_t tpitch = 0;
    int32_t tl_rate = 1;
    std::string err;
};

namespace {

std::string g_create_error;

size_t elem_size(rdc_dtype d) { return d == RDC_FP64 ? sizeof(double) : sizeof(float); }

rdc_status fail(rdc_ctx* c, rdc_status s, const std::string& msg) {
    if (c)
        c->err = msg;
    else
        g_create_error = msg;
    return s;
}

rdc_status hip_fail(rdc_ctx* c, hipError_t e, const char* what) {
    return fail(c, RDC_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

bool aligned256(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 255u) == 0; }

rdc_params table1() {
    // Table 1 of the paper.
    rdc_params p;
    p.eps = 0.0243;
    p.f = 1.4;
    p.q = 0.002;
    p.D_u = 0.45;
    p.dt = 0.001;
    p.dx = 0.25;
    return p;
}

const char* check_params(const rdc_params& p) {
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

template <typename Real>
rdc::Consts<Real> consts(const rdc_params& p) {
    return rdc::make_consts<Real>(p.eps, p.f, p.q, p.D_u, p.dt, p.dx);
}

template <typename Real>
rdc::StepArgs<Real> step_args(const rdc_ctx* c) {
    rdc::StepArgs<Real> a;
    a.u = static_cast<const Real*>(c->u[c->cur]);
    a.v = static_cast<const Real*>(c->v[c->cur]);
    a.phi = static_cast<const Real*>(c->phi);
    a.u_out = static_cast<Real*>(c->u[c->cur ^ 1]);
    a.v_out = static_cast<Real*>(c->v[c->cur ^ 1]);
    a.arrival = c->arrival;
    a.tl = static_cast<Real*>(c->tl);
    a.flag = c->d_flag;
    a.pitch = c->pitch;
    a.apitch = c->apitch;
    a.tpitch = c->tpitch;
    a.tl_rate = c->tl_rate;
    a.nx = c->nx;
    a.ny = c->ny;
    a.step0 = static_cast<int>(c->step);
    a.theta = static_cast<Real>(c->theta);
    a.k = consts<Real>(c->p);
    return a;
}

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) == hipSuccess && prev != dev) hipSetDevice(dev);
    }
    ~DeviceGuard() {
        int now = -1;
        if (prev >= 0 && hipGetDevice(&now) == hipSuccess && now != prev) hipSetDevice(prev);
    }
};

// Copy a (ny x nx) plane between host/device and a device plane.
rdc_status copy_plane(rdc_ctx* c, void* dst, int64_t dpitch, const void* src, int64_t spitch,
                      hipMemcpyKind kind, bool sync) {
    const size_t es = elem_size(c->dtype);
    hipError_t e = hipMemcpy2DAsync(dst, dpitch * es, src, spitch * es, c->nx * es, c->ny, kind,
                                    c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "hipMemcpy2DAsync");
    if (sync) {
        e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) return hip_fail(c, e, "hipStreamSynchronize");
    }
    return RDC_OK;
}

// Wait for the context's stream; report a device error, else the sticky
// non-finite flag (the checks rdc_read and rdc_current make).
rdc_status sync_and_check(rdc_ctx* c, const char* what) {
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, what);
    int flag = 0;
    e = hipMemcpy(&flag, c->d_flag, sizeof(int), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(c, e, "flag read");
    if (flag) return fail(c, RDC_E_NONFINITE, "a non-finite u or v was produced");
    return RDC_OK;
}

int auto_block(const rdc_ctx* c) {
    // Several steps per launch once the grid is large enough to fill the
    // chip with tiles; one step per launch for small grids.
    const int64_t cells = static_cast<int64_t>(c->nx) * c->ny;
    return cells >= (int64_t)1024 * 1024 ? 8 : 1;
}

}  // namespace

extern "C" {

const char* rdc_status_string(rdc_status s) {
    switch (s) {
        case RDC_OK: return "RDC_OK";
        case RDC_E_INVAL: return "RDC_E_INVAL";
        case RDC_E_NOMEM: return "RDC_E_NOMEM";
        case RDC_E_DEVICE: return "RDC_E_DEVICE";
        case RDC_E_NONFINITE: return "RDC_E_NONFINITE";
        case RDC_E_STATE: return "RDC_E_STATE";
    }
    return "RDC_E_UNKNOWN";
}

const char* rdc_last_error(const rdc_ctx* c) {
    return c ? c->err.c_str() : g_create_error.c_str();
}

rdc_status rdc_create(int32_t nx, int32_t ny, rdc_dtype dtype, const rdc_buffers* b,
                      void* hip_stream, rdc_ctx** out) {
    g_create_error.clear();
    if (!out) return fail(nullptr, RDC_E_INVAL, "out is NULL");
    *out = nullptr;
    if (nx < 1 || ny < 1) return fail(nullptr, RDC_E_INVAL, "nx and ny must be >= 1");
    if (dtype != RDC_FP32 && dtype != RDC_FP64) return fail(nullptr, RDC_E_INVAL, "bad dtype");
    if (!b) return fail(nullptr, RDC_E_INVAL, "buffers is NULL");
    if (b->pitch < nx || b->pitch % 64 != 0)
        return fail(nullptr, RDC_E_INVAL, "pitch must be >= nx and a multiple of 64");
    if (b->pitch > INT32_MAX / (dtype == RDC_FP64 ? 8 : 4))
        return fail(nullptr, RDC_E_INVAL, "row too long: pitch times element size must be < 2 GiB");
    if (ny > rdc::max_rows())
        return fail(nullptr, RDC_E_INVAL, "ny above the launch grid's row limit");
    const void* planes[5] = {b->u[0], b->u[1], b->v[0], b->v[1], b->phi};
    for (const void* p : planes) {
        if (!p) return fail(nullptr, RDC_E_INVAL, "a buffer is NULL");
        if (!aligned256(p)) return fail(nullptr, RDC_E_INVAL, "buffers must be 256-byte aligned");
    }
    for (int i = 0; i < 5; ++i)
        for (int j = i + 1; j < 5; ++j)
            if (planes[i] == planes[j]) return fail(nullptr, RDC_E_INVAL, "buffers must be distinct");
    rdc_ctx* c = new (std::nothrow) rdc_ctx;
    if (!c) return fail(nullptr, RDC_E_NOMEM, "host allocation failed");
    c->nx = nx;
    c->ny = ny;
    c->dtype = dtype;
    c->u[0] = b->u[0];
    c->u[1] = b->u[1];
    c->v[0] = b->v[0];
    c->v[1] = b->v[1];
    c->phi = b->phi;
    c->pitch = b->pitch;
    c->stream = static_cast<hipStream_t>(hip_stream);
    c->p = table1();
    hipError_t e = hipGetDevice(&c->device);
    if (e == hipSuccess) e = hipMalloc(&c->d_flag, sizeof(int) * 64);
    if (e == hipSuccess) e = rdc::launch_clear_flag(c->d_flag, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        std::string msg = std::string("device setup: ") + hipGetErrorString(e);
        if (c->d_flag) hipFree(c->d_flag);
        delete c;
        return fail(nullptr, e == hipErrorOutOfMemory ? RDC_E_NOMEM : RDC_E_DEVICE, msg);
    }
    *out = c;
    return RDC_OK;
}

rdc_status rdc_destroy(rdc_ctx* c) {
    if (!c) return RDC_OK;
    DeviceGuard g(c->device);
    hipStreamSynchronize(c->stream);
    if (c->d_flag) hipFree(c->d_flag);
    delete c;
    return RDC_OK;
}

rdc_status rdc_set_params(rdc_ctx* c, const rdc_params* p) {
    if (!c) return RDC_E_INVAL;
    if (!p) return fail(c, RDC_E_INVAL, "params is NULL");
    if (const char* why = check_params(*p)) return fail(c, RDC_E_INVAL, why);
    c->p = *p;
    return RDC_OK;
}

rdc_status rdc_set_phi(rdc_ctx* c, const void* phi, int64_t pitch, rdc_where where) {
    if (!c) return RDC_E_INVAL;
    if (!phi || pitch < c->nx) return fail(c, RDC_E_INVAL, "phi is NULL or pitch < nx");
    DeviceGuard g(c->device);
    return copy_plane(c, c->phi, c->pitch, phi, pitch,
                      where == RDC_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice,
                      where == RDC_HOST);
}

rdc_status rdc_write(rdc_ctx* c, const void* u, const void* v, int64_t pitch, rdc_where where) {
    if (!c) return RDC_E_INVAL;
    if (!u || !v || pitch < c->nx) return fail(c, RDC_E_INVAL, "u or v is NULL or pitch < nx");
    DeviceGuard g(c->device);
    const hipMemcpyKind kind = where == RDC_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    rdc_status s = copy_plane(c, c->u[c->cur], c->pitch, u, pitch, kind, false);
    if (s == RDC_OK) s = copy_plane(c, c->v[c->cur], c->pitch, v, pitch, kind, where == RDC_HOST);
    if (s != RDC_OK) return s;
    // A fresh state clears the sticky flag (stream-ordered, so it lands
    // after any launch already queued).
    hipError_t e = rdc::launch_clear_flag(c->d_flag, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "flag reset launch");
    return RDC_OK;
}

rdc_status rdc_stimulate(rdc_ctx* c, const int32_t* cx, const int32_t* cy, const int32_t* r,
                         int32_t k) {
    if (!c) return RDC_E_INVAL;
    if (k < 0) return fail(c, RDC_E_INVAL, "k < 0");
    if (k == 0) return RDC_OK;
    if (!cx || !cy || !r) return fail(c, RDC_E_INVAL, "disk arrays are NULL");
    for (int32_t i = 0; i < k; ++i) {
        if (r[i] < 0) return fail(c, RDC_E_INVAL, "disk radius < 0");
        const int64_t nxm = c->nx - 1, nym = c->ny - 1;
        const int64_t px = cx[i] < 0 ? 0 : (cx[i] > nxm ? nxm : cx[i]);
        const int64_t py = cy[i] < 0 ? 0 : (cy[i] > nym ? nym : cy[i]);
        const int64_t dx = px - cx[i], dy = py - cy[i];
        if (dx * dx + dy * dy > (int64_t)r[i] * r[i])
            return fail(c, RDC_E_INVAL, "a stimulus disk covers no cell of the grid");
    }
    DeviceGuard g(c->device);
    for (int32_t i0 = 0; i0 < k; i0 += rdc::kMaxDisks) {
        rdc::Disks d;
        d.count = (k - i0) < rdc::kMaxDisks ? (k - i0) : rdc::kMaxDisks;
        for (int j = 0; j < d.count; ++j) {
            d.cx[j] = cx[i0 + j];
            d.cy[j] = cy[i0 + j];
            d.r[j] = r[i0 + j];
        }
        hipError_t e;
        if (c->dtype == RDC_FP64)
            e = rdc::launch_stimulate(static_cast<double*>(c->u[c->cur]), c->pitch, c->nx, c->ny,
                                      d, c->arrival, c->apitch, (int)c->step, c->stream);
        else
            e = rdc::launch_stimulate(static_cast<float*>(c->u[c->cur]), c->pitch, c->nx, c->ny,
                                      d, c->arrival, c->apitch, (int)c->step, c->stream);
        if (e != hipSuccess) return hip_fail(c, e, "stimulate launch");
    }
    return RDC_OK;
}

rdc_status rdc_step(rdc_ctx* c, int64_t n) {
    if (!c) return RDC_E_INVAL;
    if (n < 0) return fail(c, RDC_E_INVAL, "n < 0");
    if (c->step + n > INT32_MAX - 8)
        return fail(c, RDC_E_STATE, "step counter would overflow the int32 arrival range");
    DeviceGuard g(c->device);
    const int T = c->T > 0 ? c->T : auto_block(c);
    const int rows = c->tile_rows > 0 ? c->tile_rows : rdc::tile_rows_default();
    // LDS tile height for the launches the row pipelines do not take.
    const int tile_rows = rows == RDC_TILE_STREAM ? rdc::tile_rows_default() : rows;
    const bool f64 = c->dtype == RDC_FP64;
    // ceil(n / T) launches of near-equal length (n = 9, T = 8 runs 5 + 4,
    // not 8 + 1): the launch count is the least possible, and no short
    // remainder launch pays a whole tile load and store for one or two steps.
    int64_t launches = (n + T - 1) / T;
    while (n > 0) {
        const int k = static_cast<int>((n + launches - 1) / launches);
        --launches;
        hipError_t e;
        if (k == 1)
            e = f64 ? rdc::launch_step1(step_args<double>(c), c->stream)
                    : rdc::launch_step1(step_args<float>(c), c->stream);
        else if (rows == RDC_TILE_STREAM && !c->arrival && !c->tl &&
                 (f64 ? rdc::stream64_supported(k) : rdc::stream_supported(k, c->nx)))
            e = f64 ? rdc::launch_stream(step_args<double>(c), k, c->stream)
                    : rdc::launch_stream(step_args<float>(c), k, c->stream);
        else
            e = f64 ? rdc::launch_stepT(step_args<double>(c), k, tile_rows, c->stream)
                    : rdc::launch_stepT(step_args<float>(c), k, tile_rows, c->stream);
        if (e != hipSuccess) return hip_fail(c, e, "step launch");
        c->cur ^= 1;
        c->step += k;
        n -= k;
    }
    return RDC_OK;
}

rdc_status rdc_read(rdc_ctx* c, void* u, void* v, int64_t pitch, rdc_where where) {
    if (!c) return RDC_E_INVAL;
    if ((u || v) && pitch < c->nx) return fail(c, RDC_E_INVAL, "pitch < nx");
    DeviceGuard g(c->device);
    const rdc_status st = sync_and_check(c, "device error before read");
    if (st != RDC_OK && st != RDC_E_NONFINITE) return st;
    const hipMemcpyKind kind = where == RDC_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
    if (u) {
        rdc_status s = copy_plane(c, u, pitch, c->u[c->cur], c->pitch, kind, true);
        if (s != RDC_OK) return s;
    }
    if (v) {
        rdc_status s = copy_plane(c, v, pitch, c->v[c->cur], c->pitch, kind, true);
        if (s != RDC_OK) return s;
    }
    return st;
}

rdc_status rdc_set_block(rdc_ctx* c, int32_t T) {
    if (!c) return RDC_E_INVAL;
    const int tmax = c->dtype == RDC_FP64 ? rdc::kMaxBlock64 : rdc::kMaxBlock;
    if (T < 0 || T > tmax)
        return fail(c, RDC_E_INVAL, c->dtype == RDC_FP64 ? "T must be in 0..8 for FP64"
                                                         : "T must be in 0..12");
    c->T = T;
    return RDC_OK;
}

int32_t rdc_tile_rows_supported(int32_t rows) {
    return (rows == RDC_TILE_STREAM || rdc::tile_rows_supported(rows)) ? 1 : 0;
}

rdc_status rdc_set_tile_rows(rdc_ctx* c, int32_t rows) {
    if (!c) return RDC_E_INVAL;
    if (rows != 0 && !rdc_tile_rows_supported(rows))
        return fail(c, RDC_E_INVAL, "unsupported tile height");
    c->tile_rows = rows;
    return RDC_OK;
}


rdc_status rdc_current(rdc_ctx* c, void** u_dev, void** v_dev) {
    if (!c) return RDC_E_INVAL;
    if (!u_dev || !v_dev) return fail(c, RDC_E_INVAL, "NULL output");
    *u_dev = c->u[c->cur];
    *v_dev = c->v[c->cur];
    DeviceGuard g(c->device);
    return sync_and_check(c, "device error before current");
}

rdc_status rdc_set_arrival(rdc_ctx* c, int32_t* arrival, int64_t pitch, double theta) {
    if (!c) return RDC_E_INVAL;
    if (!arrival) {
        c->arrival = nullptr;
        c->apitch = 0;
        return RDC_OK;
    }
    if (pitch < c->nx || pitch % 64 != 0)
        return fail(c, RDC_E_INVAL, "arrival pitch must be >= nx and a multiple of 64");
    if (!aligned256(arrival)) return fail(c, RDC_E_INVAL, "arrival must be 256-byte aligned");
    if (!std::isfinite(theta)) return fail(c, RDC_E_INVAL, "theta must be finite");
    DeviceGuard g(c->device);
    c->arrival = arrival;
    c->apitch = pitch;
    c->theta = theta;
    hipError_t e;
    if (c->dtype == RDC_FP64)
        e = rdc::launch_arrival_init(static_cast<const double*>(c->u[c->cur]), c->pitch, c->nx,
                                     c->ny, theta, arrival, pitch, (int)c->step, c->stream);
    else
        e = rdc::launch_arrival_init(static_cast<const float*>(c->u[c->cur]), c->pitch, c->nx,
                                     c->ny, (float)theta, arrival, pitch, (int)c->step, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "arrival init launch");
    return RDC_OK;
}

rdc_status rdc_set_timelapse(rdc_ctx* c, void* tl, int64_t pitch, int32_t rate) {
    if (!c) return RDC_E_INVAL;
    if (!tl) {
        c->tl = nullptr;
        c->tpitch = 0;
        c->tl_rate = 1;
        return RDC_OK;
    }
    if (rate < 1) return fail(c, RDC_E_INVAL, "timelapse rate must be >= 1");
    if (pitch < c->nx || pitch % 64 != 0)
        return fail(c, RDC_E_INVAL, "timelapse pitch must be >= nx and a multiple of 64");
    if (!aligned256(tl)) return fail(c, RDC_E_INVAL, "timelapse plane must be 256-byte aligned");
    DeviceGuard g(c->device);
    hipError_t e;
    if (c->dtype == RDC_FP64)
        e = rdc::launch_copy_plane(static_cast<const double*>(c->u[c->cur]), c->pitch, c->nx,
                                   c->ny, static_cast<double*>(tl), pitch, c->stream);
    else
        e = rdc::launch_copy_plane(static_cast<const float*>(c->u[c->cur]), c->pitch, c->nx,
                                   c->ny, static_cast<float*>(tl), pitch, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "timelapse init launch");
    c->tl = tl;
    c->tpitch = pitch;
    c->tl_rate = rate;
    return RDC_OK;
}

rdc_status rdc_get_step(const rdc_ctx* c, int64_t* step) {
    if (!c || !step) return RDC_E_INVAL;
    *step = c->step;
    return RDC_OK;
}

rdc_status rdc_set_step(rdc_ctx* c, int64_t step) {
    if (!c) return RDC_E_INVAL;
    if (step < 0 || step > INT32_MAX - 8)
        return fail(c, RDC_E_INVAL, "step must be in 0 .. INT32_MAX - 8 (the arrival range)");
    c->step = step;
    return RDC_OK;
}

rdc_status rdc_copy(void* dst, const void* src, int64_t nbytes, void* hip_stream) {
    if (!dst || !src || nbytes < 0 || nbytes % 16 != 0)
        return fail(nullptr, RDC_E_INVAL, "copy needs non-NULL pointers and nbytes % 16 == 0");
    if ((reinterpret_cast<uintptr_t>(dst) | reinterpret_cast<uintptr_t>(src)) & 15u)
        return fail(nullptr, RDC_E_INVAL, "copy pointers must be 16-byte aligned");
    hipError_t e = rdc::launch_copy16(src, dst, nbytes / 16, static_cast<hipStream_t>(hip_stream));
    if (e != hipSuccess) return hip_fail(nullptr, e, "copy launch");
    return RDC_OK;
}

}  // extern "C"
