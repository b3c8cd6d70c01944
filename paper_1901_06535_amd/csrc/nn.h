// nn.h -- internal launch interface of the learned coarse stepper's kernels
// (nn.hip); the C ABI over it is in nn_api.hip.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rdc {
namespace nn {

// 3x3 same convolution, NHWC bf16.  x: N*H*W pixels with stride ldx (reads
// channels [0, cin)); w: bf16 [9][cout][cin]; bias: fp32 [cout] (optional);
// y: stride ldy, writes channels [0, cout_store) (rounded up to 4).
// cin % 16 == 0, cout in {32, 64, 96, 128, 192, 256}, W % 32 == 0.
struct ConvArgs {
    const __bf16* x;
    const __bf16* w;
    const float* bias;
    __bf16* y;
    int ldx, ldy;
    int N, H, W;
    int cin, cout, cout_store;
    // Input stages fused into the loads (off by default):
    //  * upsampled prefix: channels [0, up_c) come from `xu` (pixel stride
    //    ldu, image (H/2) x (W/2)) by nearest 2x upsampling, the rest from x;
    //  * stepper planes: the input is built from fp32 planes u, v, phi (row
    //    pitch `ppitch`, image n at n * pplane): channels bf16(su u),
    //    bf16(sv v), bf16(sp phi), zeros up to cin; x is not read.
    const __bf16* xu = nullptr;
    int ldu = 0, up_c = 0;
    const float* pu = nullptr;
    const float* pv = nullptr;
    const float* pphi = nullptr;
    int64_t ppitch = 0, pplane = 0;
    float su = 0.0f, sv = 0.0f, sp = 0.0f;
    // Prediction epilogue (conv3x3_apply): instead of storing the output,
    // (uo, vo) = the apply kernel's projection of (u, v) + (out0 / su,
    // out1 / sv) from the bf16-rounded first two output channels, on the
    // planes pu, pv, pphi (layout ppitch, pplane).
    float* uo = nullptr;
    float* vo = nullptr;
    float f = 0.0f, cmax = 0.0f;
};
hipError_t conv3x3(const ConvArgs& a, bool relu, bool bias, hipStream_t s);
// The fused-input forms (bias and ReLU always applied; cout in {32, 64, 128}).
hipError_t conv3x3_up(const ConvArgs& a, hipStream_t s);
hipError_t conv3x3_planes(const ConvArgs& a, hipStream_t s);
// cout = 32, bias, no ReLU, prediction epilogue (see ConvArgs).
hipError_t conv3x3_apply(const ConvArgs& a, hipStream_t s);

// Weight gradient of the same convolution: grad[9][cout][cin] (fp32) from
// x (stride ldx) and dy (stride lddy); `part` is scratch of
// wgrad_chunks(N, H, W) * 9 * cout * cin floats, `bpart` (optional) of
// wgrad_chunks(N, H, W) * cout floats for the bias gradient gbias[cout] =
// sum over pixels of dy.  cin, cout % 32 == 0.
struct WgradArgs {
    const __bf16* x;
    const __bf16* dy;
    float* part;
    float* bpart;
    int ldx, lddy;
    int N, H, W;
    int cin, cout;
};
int64_t wgrad_chunks(int N, int H, int W);
hipError_t conv3x3_wgrad(const WgradArgs& a, float* grad, float* gbias, hipStream_t s);

hipError_t flip_weights(const float* w, __bf16* wd, int cout, int cin, hipStream_t s);
hipError_t to_bf16(const float* src, __bf16* dst, int64_t n, hipStream_t s);
hipError_t relu_bwd(__bf16* g, int ldg, const __bf16* y, int ldy, int64_t pixels, int c,
                    hipStream_t s);
hipError_t pool2(const __bf16* in, int ldi, __bf16* out, int ldo, int N, int Ho, int Wo, int c,
                 hipStream_t s);
hipError_t pool2_bwd(const __bf16* gout, int ldo, __bf16* gin, int ldi, int N, int Ho, int Wo,
                     int c, bool accumulate, hipStream_t s);
hipError_t up2(const __bf16* in, int ldi, __bf16* out, int ldo, int N, int Ho, int Wo, int c,
               hipStream_t s);
hipError_t up2_bwd(const __bf16* gout, int ldo, __bf16* gin, int ldi, int N, int Hi, int Wi,
                   int c, hipStream_t s);
hipError_t prep(const float* u, const float* v, const float* phi, int64_t pitch,
                int64_t plane_stride, __bf16* x, int c, int N, int H, int W, float su, float sv,
                float sp, hipStream_t s);
hipError_t apply(const float* u, const float* v, const float* phi, const __bf16* head, int ldh,
                 int64_t pitch, int64_t plane_stride, float* uo, float* vo, int N, int H, int W,
                 float su, float sv, float f, float cmax, hipStream_t s);
int loss_blocks(int64_t pixels);
hipError_t loss(const float* u, const float* v, const float* ut, const float* vt, int64_t pitch,
                int64_t plane_stride, const __bf16* head, int ldh, __bf16* g, int ldg, int N,
                int H, int W, float su, float sv, float theta, float front_w, float* partial,
                hipStream_t s);
hipError_t adam(float* p, const float* g, float* m, float* v, int64_t n, float lr_t, float b1,
                float b2, float eps, float clip, hipStream_t s);
hipError_t front_check(const float* a, const float* b, int64_t pitch, int nx, int ny,
                       float theta, unsigned int* count, hipStream_t s);
hipError_t state_check(const float* u, const float* v, const float* phi, int64_t pitch, int nx,
                       int ny, float ulo, float uhi, float f, float cmax, unsigned int* count,
                       hipStream_t s);

}  // namespace nn
}  // namespace rdc
