// nn_api.hip -- C ABI (include/rdc.h, rdc_nn_*) of the learned coarse
// stepper's kernels: argument checks and launches on the caller's stream.
#include <cstdint>
#include <cstdio>
#include <mutex>

#include "../../include/rdc.h"
#include "nn.h"

// Workspace of rdc_nn_conv3x3_wgrad_noalloc, for callers that cannot
// allocate: one copy per GPU, held until the process ends.
constexpr int64_t kStaticScratchFloats = int64_t(8) << 20;   // 32 MiB
static __device__ __align__(256) float scratch[kStaticScratchFloats];

namespace {

// The last error of this thread, in a fixed buffer (no heap use on any path).
thread_local char g_nn_error[256];

rdc_status nfail(const char* m) {
    std::snprintf(g_nn_error, sizeof g_nn_error, "%s", m);
    return RDC_E_INVAL;
}

rdc_status nhip(hipError_t e) {
    if (e == hipSuccess) return RDC_OK;
    std::snprintf(g_nn_error, sizeof g_nn_error, "launch: %s", hipGetErrorString(e));
    return RDC_E_DEVICE;
}

// Device address of `scratch` on the current device.  In host code the
// array's name stands for no device address, so every use goes through the
// address hipGetSymbolAddress gives, taken once per device (each GPU holds
// its own copy at its own address).
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float* g_scratch_dev[kMaxDevices] = {};

rdc_status static_scratch(float** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return nhip(e);
    if (dev < 0 || dev >= kMaxDevices) return nfail("device index beyond the static scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            std::snprintf(g_nn_error, sizeof g_nn_error, "static scratch address: %s",
                          hipGetErrorString(e));
            return RDC_E_DEVICE;
        }
        g_scratch_dev[dev] = static_cast<float*>(p);
    }
    *out = g_scratch_dev[dev];
    return RDC_OK;
}

bool al16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }
bool al8(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 7u) == 0; }
hipStream_t S(void* s) { return static_cast<hipStream_t>(s); }

}  // namespace

extern "C" {

const char* rdc_nn_last_error(void) { return g_nn_error; }

rdc_status rdc_nn_conv3x3(const void* x, int32_t ldx, const void* w, const float* bias, void* y,
                          int32_t ldy, int32_t n, int32_t h, int32_t wd, int32_t cin,
                          int32_t cout, int32_t cout_store, int32_t relu, void* stream) {
    if (!x || !w || !y) return nfail("NULL tensor");
    if (n < 1 || n > 65535 || h < 1 || h > 262140 || wd < 32 || wd % 32)
        return nfail("need 1 <= n <= 65535, 1 <= h <= 262140 and w a multiple of 32");
    if (cin < 16 || cin % 16 || !(cout == 32 || cout == 64 || cout == 96 || cout == 128 ||
                                   cout == 192 || cout == 256))
        return nfail("need cin % 16 == 0, cout in {32, 64, 96, 128, 192, 256}");
    if (cout_store < 1 || cout_store > cout) return nfail("cout_store must be in 1..cout");
    if (ldx < cin || ldx % 8 || ldy < ((cout_store + 3) & ~3) || ldy % 4)
        return nfail("strides: ldx >= cin, ldx % 8 == 0, ldy >= cout_store rounded to 4, ldy % 4 == 0");
    if (!al16(x) || !al16(w) || !al8(y)) return nfail("x, w need 16-byte and y 8-byte alignment");
    rdc::nn::ConvArgs a;
    a.x = static_cast<const __bf16*>(x);
    a.w = static_cast<const __bf16*>(w);
    a.bias = bias;
    a.y = static_cast<__bf16*>(y);
    a.ldx = ldx;
    a.ldy = ldy;
    a.N = n;
    a.H = h;
    a.W = wd;
    a.cin = cin;
    a.cout = cout;
    a.cout_store = cout_store;
    return nhip(rdc::nn::conv3x3(a, relu != 0, bias != nullptr, S(stream)));
}

rdc_status rdc_nn_conv3x3_up(const void* x, int32_t ldx, const void* xu, int32_t ldu,
                             int32_t up_c, const void* w, const float* bias, void* y,
                             int32_t ldy, int32_t n, int32_t h, int32_t wd, int32_t cin,
                             int32_t cout, int32_t cout_store, void* stream) {
    if (!x || !xu || !w || !bias || !y) return nfail("NULL tensor or bias");
    if (n < 1 || n > 65535 || h < 2 || h > 262140 || h % 2 || wd < 64 || wd % 64)
        return nfail("need 1 <= n <= 65535, even 2 <= h <= 262140 and w a multiple of 64");
    if (cin < 32 || cin % 16 || up_c < 32 || up_c % 32 || up_c > cin ||
        !(cout == 32 || cout == 64 || cout == 128))
        return nfail("need cin % 16 == 0, up_c a multiple of 32 in 32..cin, cout in {32, 64, 128}");
    if (cout_store < 1 || cout_store > cout) return nfail("cout_store must be in 1..cout");
    if (ldx < cin || ldx % 8 || ldu < up_c || ldu % 8 || ldy < ((cout_store + 3) & ~3) ||
        ldy % 4)
        return nfail("strides: ldx >= cin, ldu >= up_c, both % 8 == 0; ldy >= cout_store rounded to 4, % 4 == 0");
    if (!al16(x) || !al16(xu) || !al16(w) || !al8(y))
        return nfail("x, xu, w need 16-byte and y 8-byte alignment");
    rdc::nn::ConvArgs a;
    a.x = static_cast<const __bf16*>(x);
    a.w = static_cast<const __bf16*>(w);
    a.bias = bias;
    a.y = static_cast<__bf16*>(y);
    a.ldx = ldx;
    a.ldy = ldy;
    a.N = n;
    a.H = h;
    a.W = wd;
    a.cin = cin;
    a.cout = cout;
    a.cout_store = cout_store;
    a.xu = static_cast<const __bf16*>(xu);
    a.ldu = ldu;
    a.up_c = up_c;
    return nhip(rdc::nn::conv3x3_up(a, S(stream)));
}

rdc_status rdc_nn_conv3x3_planes(const float* u, const float* v, const float* phi,
                                 int64_t pitch, int64_t plane_stride, float su, float sv,
                                 float sp, const void* w, const float* bias, void* y, int32_t ldy,
                                 int32_t n, int32_t h, int32_t wd, int32_t cin, int32_t cout,
                                 int32_t cout_store, void* stream) {
    if (!u || !v || !phi || !w || !bias || !y) return nfail("NULL plane, tensor or bias");
    if (n < 1 || n > 65535 || h < 1 || h > 262140 || wd < 32 || wd % 32)
        return nfail("need 1 <= n <= 65535, 1 <= h <= 262140 and w a multiple of 32");
    if (pitch < wd || plane_stride < pitch * h) return nfail("need pitch >= w, plane_stride >= pitch*h");
    if (!(cin == 16 || cin == 32) || !(cout == 32 || cout == 64 || cout == 128))
        return nfail("need cin in {16, 32}, cout in {32, 64, 128}");
    if (cout_store < 1 || cout_store > cout) return nfail("cout_store must be in 1..cout");
    if (ldy < ((cout_store + 3) & ~3) || ldy % 4)
        return nfail("ldy >= cout_store rounded to 4, ldy % 4 == 0");
    if (!al16(w) || !al8(y)) return nfail("w needs 16-byte and y 8-byte alignment");
    rdc::nn::ConvArgs a;
    a.x = nullptr;
    a.w = static_cast<const __bf16*>(w);
    a.bias = bias;
    a.y = static_cast<__bf16*>(y);
    a.ldx = cin;
    a.ldy = ldy;
    a.N = n;
    a.H = h;
    a.W = wd;
    a.cin = cin;
    a.cout = cout;
    a.cout_store = cout_store;
    a.pu = u;
    a.pv = v;
    a.pphi = phi;
    a.ppitch = pitch;
    a.pplane = plane_stride;
    a.su = su;
    a.sv = sv;
    a.sp = sp;
    return nhip(rdc::nn::conv3x3_planes(a, S(stream)));
}

rdc_status rdc_nn_conv3x3_apply(const void* x, int32_t ldx, const void* w, const float* bias,
                                const float* u, const float* v, const float* phi, int64_t pitch,
                                int64_t plane_stride, float* uo, float* vo, int32_t n, int32_t h,
                                int32_t wd, int32_t cin, float su, float sv, float f, float cmax,
                                void* stream) {
    if (!x || !w || !bias || !u || !v || !phi || !uo || !vo)
        return nfail("NULL tensor, bias or plane");
    if (n < 1 || n > 65535 || h < 1 || h > 262140 || wd < 32 || wd % 32)
        return nfail("need 1 <= n <= 65535, 1 <= h <= 262140 and w a multiple of 32");
    if (cin < 16 || cin % 16 || ldx < cin || ldx % 8) return nfail("need cin % 16 == 0, ldx >= cin, ldx % 8 == 0");
    if (pitch < wd || plane_stride < pitch * h) return nfail("need pitch >= w, plane_stride >= pitch*h");
    if (!(f > 0.0f) || !(su != 0.0f) || !(sv != 0.0f)) return nfail("need f > 0 and nonzero su, sv");
    if (!al16(x) || !al16(w)) return nfail("x, w need 16-byte alignment");
    rdc::nn::ConvArgs a;
    a.x = static_cast<const __bf16*>(x);
    a.w = static_cast<const __bf16*>(w);
    a.bias = bias;
    a.y = nullptr;
    a.ldx = ldx;
    a.ldy = 32;
    a.N = n;
    a.H = h;
    a.W = wd;
    a.cin = cin;
    a.cout = 32;
    a.cout_store = 32;
    a.pu = u;
    a.pv = v;
    a.pphi = phi;
    a.ppitch = pitch;
    a.pplane = plane_stride;
    a.su = su;
    a.sv = sv;
    a.uo = uo;
    a.vo = vo;
    a.f = f;
    a.cmax = cmax;
    return nhip(rdc::nn::conv3x3_apply(a, S(stream)));
}

rdc_status rdc_nn_dgrad_weights(const float* w, void* wd, int32_t cout, int32_t cin,
                                void* stream) {
    if (!w || !wd || cout < 1 || cin < 1) return nfail("bad dgrad weight arguments");
    return nhip(rdc::nn::flip_weights(w, static_cast<__bf16*>(wd), cout, cin, S(stream)));
}

int64_t rdc_nn_wgrad_scratch_floats(int32_t n, int32_t h, int32_t w, int32_t cin, int32_t cout) {
    if (n < 1 || h < 1 || w < 32 || cin < 1 || cout < 1) return 0;
    return rdc::nn::wgrad_chunks(n, h, w) * (9 * (int64_t)cout * cin + cout);
}

}  // extern "C"

namespace {

// Checks of the weight-gradient calls; the partials go to `work`.
rdc_status wgrad_args(const void* x, int32_t ldx, const void* dy, int32_t lddy, const float* grad,
                      int32_t n, int32_t h, int32_t w, int32_t cin, int32_t cout) {
    if (!x || !dy || !grad) return nfail("NULL tensor");
    if (n < 1 || h < 1 || w < 32 || w % 32) return nfail("need w a multiple of 32");
    if (cin < 32 || cin % 32 || cout < 32 || cout % 32) return nfail("need cin, cout % 32 == 0");
    if (ldx < cin || ldx % 8 || lddy < cout || lddy % 8) return nfail("bad strides");
    if (!al16(x) || !al16(dy)) return nfail("x, dy need 16-byte alignment");
    return RDC_OK;
}

rdc_status wgrad_launch(const void* x, int32_t ldx, const void* dy, int32_t lddy, float* work,
                        float* grad, float* gbias, int32_t n, int32_t h, int32_t w, int32_t cin,
                        int32_t cout, void* stream) {
    rdc::nn::WgradArgs a;
    a.x = static_cast<const __bf16*>(x);
    a.dy = static_cast<const __bf16*>(dy);
    a.part = work;
    a.bpart = gbias ? work + rdc::nn::wgrad_chunks(n, h, w) * 9 * (int64_t)cout * cin : nullptr;
    a.ldx = ldx;
    a.lddy = lddy;
    a.N = n;
    a.H = h;
    a.W = w;
    a.cin = cin;
    a.cout = cout;
    return nhip(rdc::nn::conv3x3_wgrad(a, grad, gbias, S(stream)));
}

}  // namespace

extern "C" {

rdc_status rdc_nn_conv3x3_wgrad(const void* x, int32_t ldx, const void* dy, int32_t lddy,
                                float* scratch_arg, float* grad, float* gbias, int32_t n, int32_t h,
                                int32_t w, int32_t cin, int32_t cout, void* stream) {
    if (!scratch_arg) return nfail("NULL tensor");
    if (rdc_status st = wgrad_args(x, ldx, dy, lddy, grad, n, h, w, cin, cout)) return st;
    return wgrad_launch(x, ldx, dy, lddy, scratch_arg, grad, gbias, n, h, w, cin, cout, stream);
}

int64_t rdc_nn_wgrad_static_floats(void) { return kStaticScratchFloats; }

rdc_status rdc_nn_conv3x3_wgrad_noalloc(const void* x, int32_t ldx, const void* dy, int32_t lddy,
                                        float* grad, float* gbias, int32_t n, int32_t h,
                                        int32_t w, int32_t cin, int32_t cout, void* stream) {
    if (rdc_status st = wgrad_args(x, ldx, dy, lddy, grad, n, h, w, cin, cout)) return st;
    if (rdc_nn_wgrad_scratch_floats(n, h, w, cin, cout) > kStaticScratchFloats)
        return nfail("shape needs more workspace than the static scratch holds "
                     "(rdc_nn_wgrad_scratch_floats > rdc_nn_wgrad_static_floats)");
    float* work = nullptr;
    if (rdc_status st = static_scratch(&work)) return st;
    // Every partial the summing launches read is written first by the
    // partial launch of the same call, so the scratch needs no clearing.
    return wgrad_launch(x, ldx, dy, lddy, work, grad, gbias, n, h, w, cin, cout, stream);
}

rdc_status rdc_nn_to_bf16(const float* src, void* dst, int64_t n, void* stream) {
    if (!src || !dst || n < 0) return nfail("bad conversion arguments");
    return nhip(rdc::nn::to_bf16(src, static_cast<__bf16*>(dst), n, S(stream)));
}

rdc_status rdc_nn_relu_bwd(void* g, int32_t ldg, const void* y, int32_t ldy, int64_t pixels,
                           int32_t c, void* stream) {
    if (!g || !y || pixels < 1 || c < 1 || ldg < c || ldy < c) return nfail("bad relu-bwd arguments");
    return nhip(rdc::nn::relu_bwd(static_cast<__bf16*>(g), ldg, static_cast<const __bf16*>(y),
                                  ldy, pixels, c, S(stream)));
}

rdc_status rdc_nn_pool2(const void* in, int32_t ldi, void* out, int32_t ldo, int32_t n,
                        int32_t ho, int32_t wo, int32_t c, void* stream) {
    if (!in || !out || n < 1 || ho < 1 || wo < 1 || c < 1 || ldi < c || ldo < c)
        return nfail("bad pool arguments");
    return nhip(rdc::nn::pool2(static_cast<const __bf16*>(in), ldi, static_cast<__bf16*>(out), ldo,
                               n, ho, wo, c, S(stream)));
}

rdc_status rdc_nn_pool2_bwd(const void* gout, int32_t ldo, void* gin, int32_t ldi, int32_t n,
                            int32_t ho, int32_t wo, int32_t c, int32_t accumulate, void* stream) {
    if (!gout || !gin || n < 1 || ho < 1 || wo < 1 || c < 1 || ldi < c || ldo < c)
        return nfail("bad pool-bwd arguments");
    return nhip(rdc::nn::pool2_bwd(static_cast<const __bf16*>(gout), ldo, static_cast<__bf16*>(gin),
                                   ldi, n, ho, wo, c, accumulate != 0, S(stream)));
}

rdc_status rdc_nn_up2(const void* in, int32_t ldi, void* out, int32_t ldo, int32_t n, int32_t ho,
                      int32_t wo, int32_t c, void* stream) {
    if (!in || !out || n < 1 || ho < 2 || wo < 2 || ho % 2 || wo % 2 || c < 1 || ldi < c || ldo < c)
        return nfail("bad upsample arguments");
    return nhip(rdc::nn::up2(static_cast<const __bf16*>(in), ldi, static_cast<__bf16*>(out), ldo, n,
                             ho, wo, c, S(stream)));
}

rdc_status rdc_nn_up2_bwd(const void* gout, int32_t ldo, void* gin, int32_t ldi, int32_t n,
                          int32_t hi, int32_t wi, int32_t c, void* stream) {
    if (!gout || !gin || n < 1 || hi < 1 || wi < 1 || c < 1 || ldi < c || ldo < c)
        return nfail("bad upsample-bwd arguments");
    return nhip(rdc::nn::up2_bwd(static_cast<const __bf16*>(gout), ldo, static_cast<__bf16*>(gin),
                                 ldi, n, hi, wi, c, S(stream)));
}

rdc_status rdc_nn_prep(const float* u, const float* v, const float* phi, int64_t pitch,
                       int64_t plane_stride, void* x, int32_t c, int32_t n, int32_t h,
                       int32_t w, float su, float sv, float sp, void* stream) {
    if (!u || !v || !phi || !x || c < 3 || n < 1 || h < 1 || w < 1 || pitch < w)
        return nfail("bad prep arguments");
    return nhip(rdc::nn::prep(u, v, phi, pitch, plane_stride, static_cast<__bf16*>(x), c, n, h, w,
                              su, sv, sp, S(stream)));
}

rdc_status rdc_nn_apply(const float* u, const float* v, const float* phi, const void* head,
                        int32_t ldh, int64_t pitch, int64_t plane_stride, float* uo, float* vo,
                        int32_t n, int32_t h, int32_t w, float su, float sv, float f, float cmax,
                        void* stream) {
    if (!u || !v || !phi || !head || !uo || !vo || ldh < 2 || n < 1 || h < 1 || w < 1 ||
        pitch < w || su == 0.0f || sv == 0.0f || !(f > 0.0f))
        return nfail("bad apply arguments");
    return nhip(rdc::nn::apply(u, v, phi, static_cast<const __bf16*>(head), ldh, pitch,
                               plane_stride, uo, vo, n, h, w, su, sv, f, cmax, S(stream)));
}

int32_t rdc_nn_loss_blocks(int64_t pixels) { return pixels < 1 ? 0 : rdc::nn::loss_blocks(pixels); }

rdc_status rdc_nn_loss(const float* u, const float* v, const float* ut, const float* vt,
                       int64_t pitch, int64_t plane_stride, const void* head, int32_t ldh,
                       void* g, int32_t ldg, int32_t n, int32_t h, int32_t w, float su, float sv,
                       float theta, float front_w, float* partial, void* stream) {
    if (!u || !v || !ut || !vt || !head || !g || !partial || ldh < 2 || ldg < 2 || n < 1 ||
        h < 1 || w < 1 || pitch < w)
        return nfail("bad loss arguments");
    return nhip(rdc::nn::loss(u, v, ut, vt, pitch, plane_stride, static_cast<const __bf16*>(head),
                              ldh, static_cast<__bf16*>(g), ldg, n, h, w, su, sv, theta, front_w,
                              partial, S(stream)));
}

rdc_status rdc_nn_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr_t,
                       float b1, float b2, float eps, float clip, void* stream) {
    if (!p || !g || !m || !v || n < 0) return nfail("bad adam arguments");
    return nhip(rdc::nn::adam(p, g, m, v, n, lr_t, b1, b2, eps, clip, S(stream)));
}

rdc_status rdc_nn_front_check(const float* a, const float* b, int64_t pitch, int32_t nx,
                              int32_t ny, float theta, uint32_t* count, void* stream) {
    if (!a || !b || !count || nx < 1 || ny < 1 || pitch < nx) return nfail("bad front-check arguments");
    return nhip(rdc::nn::front_check(a, b, pitch, nx, ny, theta, count, S(stream)));
}

rdc_status rdc_nn_state_check(const float* u, const float* v, const float* phi, int64_t pitch,
                              int32_t nx, int32_t ny, float ulo, float uhi, float f, float cmax,
                              uint32_t* count, void* stream) {
    if (!u || !v || !phi || !count || nx < 1 || ny < 1 || pitch < nx || !(ulo <= uhi))
        return nfail("bad state-check arguments");
    return nhip(rdc::nn::state_check(u, v, phi, pitch, nx, ny, ulo, uhi, f, cmax, count,
                                     S(stream)));
}

}  // extern "C"
