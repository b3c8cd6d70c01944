// nn.hip -- kernels of the learned coarse stepper: a 3x3-convolution U-Net
// that maps (u, v, phi) to (u, v) K steps ahead, trained and run on the GPU.
//
// Activations are NHWC bfloat16 with an explicit pixel stride (so a layer can
// read or write a channel slice of a concatenation buffer).  The 3x3 "same"
// convolution is an implicit GEMM on the CDNA3/4 matrix cores
// (v_mfma_f32_32x32x16_bf16: bf16 operands, fp32 accumulation):
//   forward  Y[p, co] = b[co] + sum_{tap, ci} W[tap, co, ci] X[p + off(tap), ci]
//            one wave computes a 32-pixel row segment for all output channels
//            (up to 8 accumulator blocks of 32 channels); A = weights
//            (32 channels x 16 inputs), B = activations (16 inputs x 32 pixels);
//   dgrad    the same kernel on the output gradient with the weights flipped
//            in space and transposed in channels (a small weight kernel);
//   wgrad    dW[tap, co, ci] = sum_p dY[p, co] X[p + off(tap), ci]: pixels
//            are the reduction axis, so 16-pixel slabs are transposed through
//            LDS into the MFMA operand layout; each workgroup reduces a chunk
//            of pixels and a second kernel sums the chunk partials in a fixed
//            order (deterministic).
// Element-wise kernels: input preparation from the stepper planes, residual
// output, 2x2 average pooling and nearest upsampling (and their adjoints),
// ReLU adjoint, bias gradient, the front-weighted squared-error loss and its
// gradient, Adam with fp32 master weights, and the front check used to decide
// fallback to the plain stepper.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <initializer_list>

#include "nn.h"

namespace rdc {
namespace nn {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ float bf2f(__bf16 x) { return static_cast<float>(x); }
__device__ __forceinline__ __bf16 f2bf(float x) { return static_cast<__bf16>(x); }

__device__ __forceinline__ bf16x8 load8(const __bf16* p) {
    return *reinterpret_cast<const bf16x8*>(p);
}
__device__ __forceinline__ bf16x8 zero8() {
    bf16x8 z;
#pragma unroll
    for (int j = 0; j < 8; ++j) z[j] = f2bf(0.0f);
    return z;
}

// ------------------------------------------------------------------ convolution

// 3x3 "same" convolution as an implicit GEMM on v_mfma_f32_32x32x16_bf16
// (D[co, pixel] += W[co, ci] X[ci, pixel] over 9 taps x cin), with memory
// and matrix work in separate waves.  A 768-thread workgroup owns a strip of
// 32*P output columns and sweeps a run of 8-row output tiles down it; the
// work is a sequence of stages (tile, output-channel pass, 32-input-channel
// chunk):
//   * producer waves 8..11 stage the next stage into one of two LDS buffer
//     pairs: the input tile with its one-pixel halo (10 rows x (32P + 2)
//     columns x 32 channels, zeros outside the image and past cin) and the
//     pass's weights (9 taps x 32*NBP output x 32 input channels);
//   * consumer waves 0..7 (one output row each, two per SIMD) multiply the
//     current stage from LDS only: per tap and 16-channel K step, A = 8 input
//     channels of 32 output channels (one 16-byte read), reused over the P
//     pixel blocks, B = 8 channels of the shifted input pixel (one 16-byte
//     read), reused over the NBP channel blocks; after a pass's last chunk
//     they add the bias, apply the ReLU and store NBP x 32 channels as bf16.
// One barrier per stage hands the staged buffers over.  Producers and
// consumers keep separate memory counters, so the consumers never wait on
// global memory and the next stage's loads overlap the current multiplies.
// LDS rows are 64 bytes (32 channels); the four 16-byte slots of row r are
// permuted by XOR with (r >> 2) & 3, so any 16 consecutive rows read at one
// slot cover all 64 banks (gfx950 serves a 16-byte-per-lane LDS access 16
// lanes at a time; hardware counters read zero bank conflicts with it).
// Variants (template arguments): the producers may build the input while
// loading it (SRC: an upsampled channel prefix read from the coarser level,
// or the network input from the stepper's fp32 planes), the consumers may
// apply the prediction instead of storing (EPI), and one pass of weights may
// stay resident in LDS instead of being restaged with every stage (WCH).
// Each variant computes the same bits as the unfused route.
constexpr int kConvRows = 8;                      // output rows per tile = consumer waves
constexpr int kConvProducers = 4;                 // producer waves
constexpr int kConvThreads = (kConvRows + kConvProducers) * 64;
constexpr int kConvKc = 32;                       // input channels per stage
constexpr int kConvPix = 32;                      // LDS elements per staged row

#ifndef RDC_CONV_SWZ_SHIFT
#define RDC_CONV_SWZ_SHIFT 2    // row bits that permute a row's four 16-byte LDS slots
#endif
#ifndef RDC_CONV_WG_PER_CU
#define RDC_CONV_WG_PER_CU 1    // workgroups launched per CU (each sweeps a run of tiles)
#endif

// Pixel blocks per consumer wave and output-channel blocks per pass; cout =
// 32 NB = 32 NBP * passes.  The LDS budget (two stages of input and weights)
// stays under 160 KB.
template <int NB>
constexpr int conv_pixel_blocks() { return 2; }
template <int NB>
constexpr int conv_pass_blocks() { return NB % 2 == 0 ? 2 : 1; }

__device__ __forceinline__ int conv_slot(int row, int slot) { return slot ^ ((row >> RDC_CONV_SWZ_SHIFT) & 3); }

// Where the producers take the input from (ConvArgs): the x tensor, an
// upsampled prefix of channels from xu and the rest from x, or the stepper
// planes.
enum ConvSrc { kSrcX = 0, kSrcUp = 1, kSrcPlanes = 2 };
// What the consumers do with an output tile: store it, or (one 32-channel
// block) apply the prediction to the stepper planes from its channels 0, 1.
enum ConvEpi { kEpiStore = 0, kEpiApply = 1 };

// WCH > 0: the weights of all WCH input-channel chunks (one pass) stay
// resident in LDS, loaded once by the first WCH stages, instead of being
// restaged with every stage.
template <int NBP, int PASSES, int P, bool RELU, bool BIAS, int SRC, int EPI = kEpiStore,
          int WCH = 0>
__global__ __launch_bounds__(kConvThreads) void k_conv3x3(ConvArgs a, int row_tiles, int runs,
                                                          int run_len) {
    constexpr int CT = 32 * P + 2;                       // staged columns
    constexpr int RT = kConvRows + 2;                    // staged rows
    constexpr int kXin = RT * CT * kConvPix;             // input elements per buffer
    constexpr int kWrows = 9 * NBP * 32;                 // weight rows (tap, co) per stage
    constexpr int kWts = kWrows * kConvPix;              // weight elements per buffer
    constexpr int kPiecesX = RT * CT * 4;                // 16-byte pieces per stage
    constexpr int kPiecesW = kWrows * 4;
    constexpr int kPT = kConvProducers * 64;
    constexpr int kPerX = (kPiecesX + kPT - 1) / kPT;
    constexpr int kPerW = (kPiecesW + kPT - 1) / kPT;
    __shared__ __attribute__((aligned(16))) __bf16 xin[2 * kXin];
    static_assert(WCH == 0 || PASSES == 1, "resident weights cover one pass");
    __shared__ __attribute__((aligned(16))) __bf16 wts[(WCH > 0 ? WCH : 2) * kWts];

    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const bool producer = wv >= kConvRows;
    const int lane = threadIdx.x & 63;
    const int x0 = (blockIdx.x / runs) * 32 * P;         // this strip's first column
    const int total_tiles = a.N * row_tiles;
    const int t_begin = (blockIdx.x % runs) * run_len;
    const int t_end = min(t_begin + run_len, total_tiles);
    const int chunks = (a.cin + kConvKc - 1) / kConvKc;
    const int per_tile = PASSES * chunks;                // stages per tile
    const int stages = (t_end - t_begin) * per_tile;

    // Producer: stage s into buffers (s & 1): the input tile's loads, then
    // its LDS stores, and the weights' (only when they change); out-of-range
    // pieces load a clamped address and store 0.
    auto produce = [&](int s) __attribute__((always_inline)) {
        const int t = t_begin + s / per_tile;
        const int pass = (s % per_tile) / chunks;
        const int c0 = (s % chunks) * kConvKc;
        const int n = t / row_tiles;
        const int y0 = (t % row_tiles) * kConvRows;
        const __bf16* X = SRC == kSrcPlanes ? nullptr : a.x + (int64_t)n * a.H * a.W * a.ldx;
        const int tid = threadIdx.x - kConvRows * 64;
        __bf16* bx = xin + (s & 1) * kXin;
        __bf16* bw = wts + (WCH > 0 ? s % chunks : (s & 1)) * kWts;
        // The weights depend only on (pass, chunk): with one stage per tile
        // they are the same for every stage, and both buffers are filled by
        // the first two stages.
        const bool need_w = WCH > 0 ? s < chunks : (per_tile > 1 || s < 2);
        bf16x8 vx[kPerX], vw[kPerW];
        auto load_w = [&]() __attribute__((always_inline)) {
#pragma unroll
            for (int k = 0; k < kPerW; ++k) {
                const int i = tid + k * kPT;
                const int q = i & 3;
                const int row = min(i >> 2, kWrows - 1);      // (tap, co within the pass)
                const int tap = row / (NBP * 32), co = pass * NBP * 32 + row % (NBP * 32);
                const int ch = c0 + 8 * q;
                const bool ok = i < kPiecesW && ch < a.cin;
                const bf16x8 ld =
                    load8(a.w + ((int64_t)tap * a.cout + co) * a.cin + (ch < a.cin ? ch : 0));
                vw[k] = ok ? ld : zero8();
            }
        };
        // Upsampled prefix: this stage's 32 channels all come from xu (up_c
        // is a multiple of 32), pixel (y, x) from xu's pixel (y/2, x/2).
        const bool from_up = SRC == kSrcUp && c0 < a.up_c;
        // Stepper planes (one 32-channel chunk): only each pixel's first
        // 16-byte slot (channels 0..7) carries data, so the producers take one
        // pixel per thread, load u, v, phi as coalesced 4-byte words and
        // write that slot; the other three slots hold zeros, written once per
        // buffer (stages 0 and 1).
        constexpr int kPixT = RT * CT;
        constexpr int kPerP = SRC == kSrcPlanes ? (kPixT + kPT - 1) / kPT : 1;
        float fu[kPerP], fv[kPerP], fp[kPerP];
        if constexpr (SRC == kSrcPlanes) {
#pragma unroll
            for (int k = 0; k < kPerP; ++k) {
                const int pc = min(tid + k * kPT, kPixT - 1);
                const int r = pc / CT, c = pc - (pc / CT) * CT;
                const int yc = min(max(y0 - 1 + r, 0), a.H - 1);
                const int xc = min(max(x0 - 1 + c, 0), a.W - 1);
                const int64_t o = n * a.pplane + (int64_t)yc * a.ppitch + xc;
                fu[k] = a.pu[o];
                fv[k] = a.pv[o];
                fp[k] = a.pphi[o];
            }
        } else {
#pragma unroll
            for (int k = 0; k < kPerX; ++k) {
                const int i = tid + k * kPT;
                const int q = i & 3;
                const int pc = min(i >> 2, RT * CT - 1);
                const int r = pc / CT, c = pc - (pc / CT) * CT;
                const int yy = y0 - 1 + r, xx = x0 - 1 + c;
                const int ch = c0 + 8 * q;
                const bool ok = i < kPiecesX && yy >= 0 && yy < a.H && xx >= 0 && xx < a.W &&
                                ch < a.cin;
                const int yc = min(max(yy, 0), a.H - 1), xc = min(max(xx, 0), a.W - 1);
                bf16x8 ld;
                if (from_up) {
                    const int hw = a.W >> 1;
                    ld = load8(a.xu +
                               (((int64_t)n * (a.H >> 1) + (yc >> 1)) * hw + (xc >> 1)) * a.ldu + ch);
                } else {
                    ld = load8(X + ((int64_t)yc * a.W + xc) * a.ldx + (ch < a.cin ? ch : 0));
                }
                vx[k] = ok ? ld : zero8();
            }
        }
        // One latency phase when the registers allow it (one channel block
        // per pass); two otherwise.
        if constexpr (NBP == 1) {
            if (need_w) load_w();
        }
        if constexpr (SRC == kSrcPlanes) {
#pragma unroll
            for (int k = 0; k < kPerP; ++k) {
                const int p = tid + k * kPT;
                if (p < kPixT) {
                    const int r = p / CT, c = p - (p / CT) * CT;
                    const int yy = y0 - 1 + r, xx = x0 - 1 + c;
                    bf16x8 val = zero8();
                    if (yy >= 0 && yy < a.H && xx >= 0 && xx < a.W) {
                        val[0] = f2bf(a.su * fu[k]);
                        val[1] = f2bf(a.sv * fv[k]);
                        val[2] = f2bf(a.sp * fp[k]);
                    }
                    *reinterpret_cast<bf16x8*>(&bx[p * kConvPix + 8 * conv_slot(p, 0)]) = val;
                    if (s < 2) {
#pragma unroll
                        for (int q = 1; q < 4; ++q)
                            *reinterpret_cast<bf16x8*>(&bx[p * kConvPix + 8 * conv_slot(p, q)]) =
                                zero8();
                    }
                }
            }
        } else {
#pragma unroll
            for (int k = 0; k < kPerX; ++k) {
                const int i = tid + k * kPT;
                if (i < kPiecesX)
                    *reinterpret_cast<bf16x8*>(
                        &bx[(i >> 2) * kConvPix + 8 * conv_slot(i >> 2, i & 3)]) = vx[k];
            }
        }
        if constexpr (NBP != 1) {
            if (need_w) load_w();
        }
        if (need_w) {
#pragma unroll
            for (int k = 0; k < kPerW; ++k) {
                const int i = tid + k * kPT;
                if (i < kPiecesW)
                    *reinterpret_cast<bf16x8*>(
                        &bw[(i >> 2) * kConvPix + 8 * conv_slot(i >> 2, i & 3)]) = vw[k];
            }
        }
    };

    // Producers and consumers run separate loops with the same number of
    // workgroup barriers (the role is uniform per wave), so the consumers'
    // accumulators are not live in the producers' code.
    if (producer) {
        if (stages > 0) produce(0);
        __syncthreads();
        for (int s = 0; s < stages; ++s) {
            if (s + 1 < stages) produce(s + 1);
            __syncthreads();
        }
        return;
    }

    const int kq = (lane >> 5) << 3;                 // this lane's 8-wide slice of a 16-K step
    const int pl = lane & 31;                        // this lane's pixel / output row in a block
    f32x16 acc[P][NBP];
#pragma unroll
    for (int p = 0; p < P; ++p)
#pragma unroll
        for (int b = 0; b < NBP; ++b)
#pragma unroll
            for (int i = 0; i < 16; ++i) acc[p][b][i] = 0.0f;

    __syncthreads();
    for (int s = 0; s < stages; ++s) {
        {
            const __bf16* bx = xin + (s & 1) * kXin;
            const __bf16* bw = wts + (WCH > 0 ? s % chunks : (s & 1)) * kWts;
            // Taps unrolled in groups small enough to keep the operands of
            // the taps in flight within the register budget of 3 waves/SIMD.
            constexpr int kTapUnroll = NBP == 1 ? 3 : 1;
#pragma unroll kTapUnroll
            for (int tap = 0; tap < 9; ++tap) {
                const int ty = tap / 3, tx = tap % 3;   // input = output + (ty - 1, tx - 1)
#pragma unroll
                for (int ks = 0; ks < 2; ++ks) {
                    const int slot = 2 * ks + (kq >> 3);
                    bf16x8 aw[NBP];
#pragma unroll
                    for (int b = 0; b < NBP; ++b) {
                        const int row = tap * NBP * 32 + b * 32 + pl;
                        aw[b] = *reinterpret_cast<const bf16x8*>(
                            &bw[row * kConvPix + 8 * conv_slot(row, slot)]);
                    }
                    // Pixel blocks past the image's right edge multiply the
                    // zeros staged there and are not stored.
#pragma unroll
                    for (int p = 0; p < P; ++p) {
                        const int pix = (wv + ty) * CT + p * 32 + pl + tx;
                        const bf16x8 xv = *reinterpret_cast<const bf16x8*>(
                            &bx[pix * kConvPix + 8 * conv_slot(pix, slot)]);
#pragma unroll
                        for (int b = 0; b < NBP; ++b)
                            acc[p][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aw[b], xv,
                                                                                acc[p][b], 0, 0, 0);
                    }
                }
            }
            const int c0 = (s % chunks) * kConvKc;
            if (c0 + kConvKc >= a.cin) {                    // the pass's last chunk: store
                const int t = t_begin + s / per_tile;
                const int cb0 = ((s % per_tile) / chunks) * NBP * 32;
                const int n = t / row_tiles;
                const int y = (t % row_tiles) * kConvRows + wv;
                if (y < a.H) {
                    // D[co, pixel]: lane holds pixel pl, channels 8*(i/4) + 4*(lane/32) + i%4.
#pragma unroll
                    for (int p = 0; p < P; ++p) {
                        if (x0 + p * 32 >= a.W) continue;
                        __bf16* Y = EPI == kEpiApply ? nullptr
                                                     : a.y + ((int64_t)n * a.H * a.W +
                                                              (int64_t)y * a.W + x0 + p * 32 + pl) *
                                                                 a.ldy;
#pragma unroll
                        for (int b = 0; b < NBP; ++b) {
#pragma unroll
                            for (int g = 0; g < 4; ++g) {
                                const int co = cb0 + b * 32 + g * 8 + ((lane >> 5) << 2);
                                __bf16 out[4];
#pragma unroll
                                for (int i = 0; i < 4; ++i) {
                                    float v = acc[p][b][g * 4 + i];
                                    if (BIAS) v += a.bias[co + i];
                                    if (RELU) v = v > 0.0f ? v : 0.0f;
                                    out[i] = f2bf(v);
                                }
                                if constexpr (EPI == kEpiApply) {
                                    // This lane holds channels 0..3 of pixel x: the
                                    // apply kernel's arithmetic on the bf16 outputs.
                                    if (co == 0) {
                                        const int64_t o = n * a.pplane + (int64_t)y * a.ppitch +
                                                          x0 + p * 32 + pl;
                                        const float vcap =
                                            fmaxf((a.cmax - a.pphi[o]) / a.f, 0.0f);
                                        const float un = a.pu[o] + bf2f(out[0]) / a.su;
                                        const float vn = a.pv[o] + bf2f(out[1]) / a.sv;
                                        a.uo[o] = fminf(fmaxf(un, 0.0f), 1.0f);
                                        a.vo[o] = fminf(fmaxf(vn, 0.0f), vcap);
                                    }
                                } else if (co < a.cout_store) {
                                    uint2 pk;
                                    pk.x = (uint32_t)__builtin_bit_cast(uint16_t, out[0]) |
                                           ((uint32_t)__builtin_bit_cast(uint16_t, out[1]) << 16);
                                    pk.y = (uint32_t)__builtin_bit_cast(uint16_t, out[2]) |
                                           ((uint32_t)__builtin_bit_cast(uint16_t, out[3]) << 16);
                                    *reinterpret_cast<uint2*>(Y + co) = pk;
                                }
                            }
                        }
                    }
                }
#pragma unroll
                for (int p = 0; p < P; ++p)
#pragma unroll
                    for (int b = 0; b < NBP; ++b)
#pragma unroll
                        for (int i = 0; i < 16; ++i) acc[p][b][i] = 0.0f;
            }
        }
        __syncthreads();
    }
}

// dgrad weights: Wd[tap'][ci][co] = W[8 - tap'][co][ci] (bf16 from the fp32 master).
__global__ void k_flip_weights(const float* __restrict__ w, __bf16* __restrict__ wd, int cout,
                               int cin) {
    const int64_t total = 9LL * cout * cin;
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < total;
         j += (int64_t)gridDim.x * blockDim.x) {
        const int co = j % cout;
        const int64_t r = j / cout;
        const int ci = r % cin;
        const int tp = r / cin;
        wd[j] = f2bf(w[((int64_t)(8 - tp) * cout + co) * cin + ci]);
    }
}

// fp32 master weights -> bf16 copies used by the forward kernel.
__global__ void k_to_bf16(const float* __restrict__ s, __bf16* __restrict__ d, int64_t n) {
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * blockDim.x)
        d[j] = f2bf(s[j]);
}

// wgrad partials.  Block = one wave; grid.x = chunk of kChunkSegs 32-pixel row
// segments (a flat index over n, y, x0), grid.y = tap * (cout/32) + co tile,
// grid.z = ci tile (32).  Writes part[chunk][tap][co][ci] for its tile.  The
// centre-tap blocks of ci tile 0 also sum dY over the chunk's pixels (the bias
// gradient) into bpart[chunk][co] when bpart is given.
constexpr int kChunkSegs = 64;

__global__ __launch_bounds__(64) void k_conv3x3_wgrad(WgradArgs a) {
    // [co][pixel] and [ci][pixel] staging (padded rows); after the chunk
    // the same memory holds the per-lane bias sums.
    __shared__ float smem[1280];
    __bf16 (*sdy)[40] = reinterpret_cast<__bf16 (*)[40]>(smem);
    __bf16 (*sx)[40] = sdy + 32;
    float (*sb)[16] = reinterpret_cast<float (*)[16]>(smem);
    const int lane = threadIdx.x;
    const int co_tiles = a.cout >> 5;
    const int tap = blockIdx.y / co_tiles;
    const int co0 = (blockIdx.y % co_tiles) << 5;
    const int ci0 = blockIdx.z << 5;
    const int dy = tap / 3 - 1, dx = tap % 3 - 1;
    const bool do_bias = a.bpart != nullptr && tap == 4 && ci0 == 0;
    const int segs_per_row = a.W >> 5;
    const int64_t total_segs = (int64_t)a.N * a.H * segs_per_row;
    f32x16 acc;
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[i] = 0.0f;
    float bsum[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) bsum[i] = 0.0f;
    for (int s = 0; s < kChunkSegs; ++s) {
        const int64_t seg = (int64_t)blockIdx.x * kChunkSegs + s;
        if (seg >= total_segs) break;
        const int x0 = (int)(seg % segs_per_row) << 5;
        const int64_t row = seg / segs_per_row;        // n * H + y
        const int y = (int)(row % a.H);
        const int n = (int)(row / a.H);
        // Stage dY[32 px][co0..co0+31] and X[shifted 32 px][ci0..ci0+31],
        // transposed: lane loads 8 channels of pixel (lane & 31), half
        // (lane >> 5) picks channels 0-7 / 8-15, then 16-23 / 24-31.
        const int p = lane & 31;
        const int64_t pix = ((int64_t)n * a.H + y) * a.W + x0 + p;
        const int yy = y + dy, xx = x0 + p + dx;
        const bool in = yy >= 0 && yy < a.H && xx >= 0 && xx < a.W;
        const int64_t xpix = ((int64_t)n * a.H + (in ? yy : 0)) * a.W + (in ? xx : 0);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int c = ((lane >> 5) << 3) + h * 16;
            const bf16x8 gy = load8(a.dy + pix * a.lddy + co0 + c);
            const bf16x8 gx = in ? load8(a.x + xpix * a.ldx + ci0 + c) : zero8();
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                sdy[c + j][p] = gy[j];
                sx[c + j][p] = gx[j];
                if (do_bias) bsum[h * 8 + j] += bf2f(gy[j]);
            }
        }
        __syncthreads();
        // K = 32 pixels = two MFMA K-steps of 16.
#pragma unroll
        for (int k0 = 0; k0 < 32; k0 += 16) {
            const int kq = k0 + ((lane >> 5) << 3);
            bf16x8 av, bv;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                av[j] = sdy[lane & 31][kq + j];
                bv[j] = sx[lane & 31][kq + j];
            }
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc, 0, 0, 0);
        }
        __syncthreads();
    }
    // D[co][ci]: lane holds ci = lane & 31, co = 8*(i/4) + 4*(lane/32) + i%4.
    float* out = a.part + (((int64_t)blockIdx.x * 9 + tap) * a.cout + co0) * a.cin + ci0;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int co = (i >> 2) * 8 + ((lane >> 5) << 2) + (i & 3);
        out[(int64_t)co * a.cin + (lane & 31)] = acc[i];
    }
    if (do_bias) {
        // Lane L summed channels 16*h + 8*(L/32) + j over pixel L%32; channel
        // c is the sum over the 32 lanes of its half, in lane order.
#pragma unroll
        for (int i = 0; i < 16; ++i) sb[lane][i] = bsum[i];   // staging is done (barrier above)
        __syncthreads();
        if (lane < 32) {
            const int h = lane >> 4, half = (lane >> 3) & 1, j = lane & 7;
            float t = 0.0f;
            for (int l = 0; l < 32; ++l) t += sb[half * 32 + l][h * 8 + j];
            a.bpart[(int64_t)blockIdx.x * a.cout + co0 + lane] = t;
        }
    }
}

// Sum the wgrad partials over chunks in a fixed order: g[j] = sum_c part[c][j].
__global__ void k_sum_chunks(const float* __restrict__ part, float* __restrict__ g, int chunks,
                             int64_t n) {
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * blockDim.x) {
        float s = 0.0f;
        for (int c = 0; c < chunks; ++c) s += part[(int64_t)c * n + j];
        g[j] = s;
    }
}


// ------------------------------------------------------------------ element-wise

// dY := dY * (Y > 0) over a channel slice (pixels x c, strides ldg / ldy).
__global__ void k_relu_bwd(__bf16* g, int ldg, const __bf16* y, int ldy, int64_t pixels, int c) {
    const int64_t total = pixels * c;
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < total;
         j += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p = j / c;
        const int ch = j % c;
        if (!(bf2f(y[p * ldy + ch]) > 0.0f)) g[p * ldg + ch] = f2bf(0.0f);
    }
}

// 2x2 average pool: out[n, y, x, c] = mean of in[n, 2y..2y+1, 2x..2x+1, c].
__global__ void k_pool2(const __bf16* in, int ldi, __bf16* out, int ldo, int N, int Ho, int Wo,
                        int c) {
    const int64_t total = (int64_t)N * Ho * Wo * c;
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < total;
         j += (int64_t)gridDim.x * blockDim.x) {
        const int ch = j % c;
        const int64_t q = j / c;
        const int x = q % Wo;
        const int64_t r = q / Wo;
        const int y = r % Ho;
        const int n = r / Ho;
        const int Wi = 2 * Wo;
        const int64_t b = ((int64_t)n * 2 * Ho + 2 * y) * Wi + 2 * x;
        const float s = bf2f(in[b * ldi + ch]) + bf2f(in[(b + 1) * ldi + ch]) +
                        bf2f(in[(b + Wi) * ldi + ch]) + bf2f(in[(b + Wi + 1) * ldi + ch]);
        out[q * ldo + ch] = f2bf(0.25f * s);
    }
}

// Adjoint of the 2x2 average pool, accumulated: gin[...] (+)= 0.25 gout.
__global__ void k_pool2_bwd(const __bf16* gout, int ldo, __bf16* gin, int ldi, int N, int Ho,
                            int Wo, int c, int accumulate) {
    const int64_t total = (int64_t)N * Ho * Wo * c;
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < total;
         j += (int64_t)gridDim.x * blockDim.x) {
        const int ch = j % c;
        const int64_t q = j / c;
        const int x = q % Wo;
        const int64_t r = q / Wo;
        const int y = r % Ho;
        const int n = r / Ho;
        const int Wi = 2 * Wo;
        const float g = 0.25f * bf2f(gout[q * ldo + ch]);
        const int64_t b = ((int64_t)n * 2 * Ho + 2 * y) * Wi + 2 * x;
        const int64_t idx[4] = {b, b + 1, b + Wi, b + Wi + 1};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            __bf16* d = gin + idx[k] * ldi + ch;
            *d = f2bf(accumulate ? bf2f(*d) + g : g);
        }
    }
}

// Nearest 2x upsampling: out[n, y, x, c] = in[n, y/2, x/2, c].
__global__ void k_up2(const __bf16* in, int ldi, __bf16* out, int ldo, int N, int Ho, int Wo,
                      int c) {
    const int64_t total = (int64_t)N * Ho * Wo * c;
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < total;
         j += (int64_t)gridDim.x * blockDim.x) {
        const int ch = j % c;
        const int64_t q = j / c;
        const int x = q % Wo;
        const int64_t r = q / Wo;
        const int y = r % Ho;
        const int n = r / Ho;
        const int64_t s = ((int64_t)n * (Ho / 2) + y / 2) * (Wo / 2) + x / 2;
        out[q * ldo + ch] = in[s * ldi + ch];
    }
}

// Adjoint of nearest 2x upsampling: gin[n, y, x, c] = sum of the 2x2 block.
__global__ void k_up2_bwd(const __bf16* gout, int ldo, __bf16* gin, int ldi, int N, int Hi,
                          int Wi, int c) {
    const int64_t total = (int64_t)N * Hi * Wi * c;
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < total;
         j += (int64_t)gridDim.x * blockDim.x) {
        const int ch = j % c;
        const int64_t q = j / c;
        const int x = q % Wi;
        const int64_t r = q / Wi;
        const int y = r % Hi;
        const int n = r / Hi;
        const int Wo = 2 * Wi;
        const int64_t b = ((int64_t)n * 2 * Hi + 2 * y) * Wo + 2 * x;
        const float s = bf2f(gout[b * ldo + ch]) + bf2f(gout[(b + 1) * ldo + ch]) +
                        bf2f(gout[(b + Wo) * ldo + ch]) + bf2f(gout[(b + Wo + 1) * ldo + ch]);
        gin[q * ldi + ch] = f2bf(s);
    }
}

// 16-byte variants of the element-wise kernels above, used when the
// channel count, the pixel strides and the base addresses allow 8-channel
// (16-byte) accesses; item j = (pixel, 8-channel group), same arithmetic and
// summation order as the scalar kernels.
__device__ __forceinline__ void store8(__bf16* p, const bf16x8& v) {
    *reinterpret_cast<bf16x8*>(p) = v;
}

__global__ void k_relu_bwd8(__bf16* g, int ldg, const __bf16* y, int ldy, int64_t pixels,
                            int c8) {
    const int64_t total = pixels * c8;
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < total;
         j += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p = j / c8;
        const int q = (int)(j - p * c8) * 8;
        const bf16x8 yv = load8(y + p * ldy + q);
        bf16x8 gv = load8(g + p * ldg + q);
#pragma unroll
        for (int e = 0; e < 8; ++e)
            if (!(bf2f(yv[e]) > 0.0f)) gv[e] = f2bf(0.0f);
        store8(g + p * ldg + q, gv);
    }
}

__global__ void k_pool2_8(const __bf16* in, int ldi, __bf16* out, int ldo, int N, int Ho, int Wo,
                          int c8) {
    const int64_t total = (int64_t)N * Ho * Wo * c8;
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < total;
         j += (int64_t)gridDim.x * blockDim.x) {
        const int64_t q = j / c8;
        const int ch = (int)(j - q * c8) * 8;
        const int x = q % Wo;
        const int64_t r = q / Wo;
        const int y = r % Ho;
        const int n = r / Ho;
        const int Wi = 2 * Wo;
        const int64_t b = ((int64_t)n * 2 * Ho + 2 * y) * Wi + 2 * x;
        const bf16x8 a0 = load8(in + b * ldi + ch), a1 = load8(in + (b + 1) * ldi + ch);
        const bf16x8 a2 = load8(in + (b + Wi) * ldi + ch), a3 = load8(in + (b + Wi + 1) * ldi + ch);
        bf16x8 o;
#pragma unroll
        for (int e = 0; e < 8; ++e)
            o[e] = f2bf(0.25f * (bf2f(a0[e]) + bf2f(a1[e]) + bf2f(a2[e]) + bf2f(a3[e])));
        store8(out + q * ldo + ch, o);
    }
}

__global__ void k_pool2_bwd8(const __bf16* gout, int ldo, __bf16* gin, int ldi, int N, int Ho,
                             int Wo, int c8, int accumulate) {
    const int64_t total = (int64_t)N * Ho * Wo * c8;
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < total;
         j += (int64_t)gridDim.x * blockDim.x) {
        const int64_t q = j / c8;
        const int ch = (int)(j - q * c8) * 8;
        const int x = q % Wo;
        const int64_t r = q / Wo;
        const int y = r % Ho;
        const int n = r / Ho;
        const int Wi = 2 * Wo;
        const bf16x8 gv = load8(gout + q * ldo + ch);
        float g[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) g[e] = 0.25f * bf2f(gv[e]);
        const int64_t b = ((int64_t)n * 2 * Ho + 2 * y) * Wi + 2 * x;
        const int64_t idx[4] = {b, b + 1, b + Wi, b + Wi + 1};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            __bf16* d = gin + idx[k] * ldi + ch;
            bf16x8 o;
            if (accumulate) {
                const bf16x8 old = load8(d);
#pragma unroll
                for (int e = 0; e < 8; ++e) o[e] = f2bf(bf2f(old[e]) + g[e]);
            } else {
#pragma unroll
                for (int e = 0; e < 8; ++e) o[e] = f2bf(g[e]);
            }
            store8(d, o);
        }
    }
}

__global__ void k_up2_8(const __bf16* in, int ldi, __bf16* out, int ldo, int N, int Ho, int Wo,
                        int c8) {
    const int64_t total = (int64_t)N * Ho * Wo * c8;
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < total;
         j += (int64_t)gridDim.x * blockDim.x) {
        const int64_t q = j / c8;
        const int ch = (int)(j - q * c8) * 8;
        const int x = q % Wo;
        const int64_t r = q / Wo;
        const int y = r % Ho;
        const int n = r / Ho;
        const int64_t src = ((int64_t)n * (Ho / 2) + y / 2) * (Wo / 2) + x / 2;
        store8(out + q * ldo + ch, load8(in + src * ldi + ch));
    }
}

__global__ void k_up2_bwd8(const __bf16* gout, int ldo, __bf16* gin, int ldi, int N, int Hi,
                           int Wi, int c8) {
    const int64_t total = (int64_t)N * Hi * Wi * c8;
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < total;
         j += (int64_t)gridDim.x * blockDim.x) {
        const int64_t q = j / c8;
        const int ch = (int)(j - q * c8) * 8;
        const int x = q % Wi;
        const int64_t r = q / Wi;
        const int y = r % Hi;
        const int n = r / Hi;
        const int Wo = 2 * Wi;
        const int64_t b = ((int64_t)n * 2 * Hi + 2 * y) * Wo + 2 * x;
        const bf16x8 a0 = load8(gout + b * ldo + ch), a1 = load8(gout + (b + 1) * ldo + ch);
        const bf16x8 a2 = load8(gout + (b + Wo) * ldo + ch);
        const bf16x8 a3 = load8(gout + (b + Wo + 1) * ldo + ch);
        bf16x8 o;
#pragma unroll
        for (int e = 0; e < 8; ++e)
            o[e] = f2bf(bf2f(a0[e]) + bf2f(a1[e]) + bf2f(a2[e]) + bf2f(a3[e]));
        store8(gin + q * ldi + ch, o);
    }
}

// Network input, one pixel per item, written as c/8 16-byte groups.
__global__ void k_prep8(const float* u, const float* v, const float* phi, int64_t pitch,
                        int64_t plane_stride, __bf16* x, int c8, int N, int H, int W, float su,
                        float sv, float sp) {
    const int64_t total = (int64_t)N * H * W;
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < total;
         j += (int64_t)gridDim.x * blockDim.x) {
        const int xx = j % W;
        const int64_t r = j / W;
        const int yy = r % H;
        const int n = r / H;
        const int64_t o = n * plane_stride + (int64_t)yy * pitch + xx;
        bf16x8 first = zero8();
        first[0] = f2bf(su * u[o]);
        first[1] = f2bf(sv * v[o]);
        first[2] = f2bf(sp * phi[o]);
        __bf16* d = x + j * c8 * 8;
        store8(d, first);
        for (int k = 1; k < c8; ++k) store8(d + 8 * k, zero8());
    }
}

// Network input from the stepper planes (fp32, row pitch `pitch`) of image n:
// channels (u, v, phi) scaled by (su, sv, sp), the rest zero up to c.
__global__ void k_prep(const float* u, const float* v, const float* phi, int64_t pitch,
                       int64_t plane_stride, __bf16* x, int c, int N, int H, int W, float su,
                       float sv, float sp) {
    const int64_t total = (int64_t)N * H * W;
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < total;
         j += (int64_t)gridDim.x * blockDim.x) {
        const int xx = j % W;
        const int64_t r = j / W;
        const int yy = r % H;
        const int n = r / H;
        const int64_t o = n * plane_stride + (int64_t)yy * pitch + xx;
        __bf16* d = x + j * c;
        d[0] = f2bf(su * u[o]);
        d[1] = f2bf(sv * v[o]);
        d[2] = f2bf(sp * phi[o]);
        for (int k = 3; k < c; ++k) d[k] = f2bf(0.0f);
    }
}

// Prediction: (u, v)_out = (u, v)_in + (du, dv) / (su, sv) from the head's
// first two channels (fp32 planes, same layout as k_prep), projected onto the
// states the explicit stepper can continue from: 0 <= u <= 1 (invariant under
// the flow of Eq. (1)) and 0 <= v <= (cmax - phi) / f, which keeps one Euler
// step from any u >= 0 above the pole at u = -q (cmax is set by the caller
// from eps, q and dt).
__global__ void k_apply(const float* u, const float* v, const float* phi, const __bf16* head,
                        int ldh, int64_t pitch, int64_t plane_stride, float* uo, float* vo, int N,
                        int H, int W, float su, float sv, float f, float cmax) {
    const int64_t total = (int64_t)N * H * W;
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < total;
         j += (int64_t)gridDim.x * blockDim.x) {
        const int xx = j % W;
        const int64_t r = j / W;
        const int yy = r % H;
        const int n = r / H;
        const int64_t o = n * plane_stride + (int64_t)yy * pitch + xx;
        const float vcap = fmaxf((cmax - phi[o]) / f, 0.0f);
        uo[o] = fminf(fmaxf(u[o] + bf2f(head[j * ldh + 0]) / su, 0.0f), 1.0f);
        vo[o] = fminf(fmaxf(v[o] + bf2f(head[j * ldh + 1]) / sv, 0.0f), vcap);
    }
}

// Loss on the head (the scaled increments): per pixel
//   w (|du_pred - du_true|^2 + |dv_pred - dv_true|^2),  w = 1 + front_w [front]
// where du_true = su (u_target - u_in) and "front" marks cells where the input
// or the target crosses theta.  Writes the gradient d loss / d head (bf16,
// scaled by 1/pixels) into the first two channels of g (others zero) and
// per-block partial sums of the loss.
__global__ __launch_bounds__(256) void k_loss(const float* u, const float* v, const float* ut,
                                              const float* vt, int64_t pitch,
                                              int64_t plane_stride, const __bf16* head, int ldh,
                                              __bf16* g, int ldg, int N, int H, int W, float su,
                                              float sv, float theta, float front_w,
                                              float* partial) {
    __shared__ float red[256];
    const int64_t total = (int64_t)N * H * W;
    const float inv = 1.0f / (float)total;
    float s = 0.0f;
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < total;
         j += (int64_t)gridDim.x * blockDim.x) {
        const int xx = j % W;
        const int64_t r = j / W;
        const int yy = r % H;
        const int n = r / H;
        const int64_t o = n * plane_stride + (int64_t)yy * pitch + xx;
        const bool front = (u[o] >= theta) != (ut[o] >= theta);
        const float w = 1.0f + (front ? front_w : 0.0f);
        const float eu = bf2f(head[j * ldh + 0]) - su * (ut[o] - u[o]);
        const float ev = bf2f(head[j * ldh + 1]) - sv * (vt[o] - v[o]);
        s += w * (eu * eu + ev * ev);
        g[j * ldg + 0] = f2bf(2.0f * w * eu * inv);
        g[j * ldg + 1] = f2bf(2.0f * w * ev * inv);
        for (int k = 2; k < ldg; ++k) g[j * ldg + k] = f2bf(0.0f);
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w2 = 128; w2 > 0; w2 >>= 1) {
        if (threadIdx.x < w2) red[threadIdx.x] += red[threadIdx.x + w2];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0] * inv;
}

// Adam on fp32 master parameters (bias-corrected step sizes passed in).
__global__ void k_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr_t,
                       float b1, float b2, float eps, float clip) {
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * blockDim.x) {
        float gj = g[j];
        gj = gj > clip ? clip : (gj < -clip ? -clip : gj);
        const float mj = b1 * m[j] + (1.0f - b1) * gj;
        const float vj = b2 * v[j] + (1.0f - b2) * gj * gj;
        m[j] = mj;
        v[j] = vj;
        p[j] -= lr_t * mj / (sqrtf(vj) + eps);
    }
}

// Front check: counts cells where a >= theta but no cell of b's 3x3
// neighbourhood is, and vice versa (front error <= 1 cell iff 0).
__global__ __launch_bounds__(256) void k_front_check(const float* a, const float* b,
                                                     int64_t pitch, int nx, int ny, float theta,
                                                     unsigned int* count) {
    const int64_t total = (int64_t)nx * ny;
    unsigned int bad = 0;
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < total;
         j += (int64_t)gridDim.x * blockDim.x) {
        const int x = j % nx, y = j / nx;
        const bool ia = a[(int64_t)y * pitch + x] >= theta;
        const bool ib = b[(int64_t)y * pitch + x] >= theta;
        if (ia == ib) continue;
        bool na = false, nb = false;
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                const int yy = y + dy, xx = x + dx;
                if (yy < 0 || yy >= ny || xx < 0 || xx >= nx) continue;
                na |= a[(int64_t)yy * pitch + xx] >= theta;
                nb |= b[(int64_t)yy * pitch + xx] >= theta;
            }
        if ((ia && !nb) || (ib && !na)) ++bad;
    }
    if (bad) atomicAdd(count, bad);
}

// State check: counts cells the explicit stepper cannot continue from:
// u or v NaN, u outside [ulo, uhi], or f v + phi > cmax.
__global__ __launch_bounds__(256) void k_state_check(const float* u, const float* v,
                                                     const float* phi, int64_t pitch, int nx,
                                                     int ny, float ulo, float uhi, float f,
                                                     float cmax, unsigned int* count) {
    const int64_t total = (int64_t)nx * ny;
    unsigned int bad = 0;
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < total;
         j += (int64_t)gridDim.x * blockDim.x) {
        const int64_t o = (j / nx) * pitch + j % nx;
        const float uu = u[o];
        const float c = f * v[o] + phi[o];
        if (!(uu >= ulo && uu <= uhi && c <= cmax)) ++bad;
    }
    if (bad) atomicAdd(count, bad);
}

inline unsigned grid_for(int64_t n, int block = 256) {
    const int64_t g = (n + block - 1) / block;
    return (unsigned)(g < 16384 ? (g > 0 ? g : 1) : 16384);
}

template <int NB, bool RELU, bool BIAS, int SRC = kSrcX, int EPI = kEpiStore, int WCH = 0>
hipError_t conv_launch(const ConvArgs& a, hipStream_t s) {
    constexpr int P = conv_pixel_blocks<NB>();
    constexpr int NBP = conv_pass_blocks<NB>();
    const int strips = (a.W + 32 * P - 1) / (32 * P);
    const int row_tiles = (a.H + kConvRows - 1) / kConvRows;
    const int total_tiles = a.N * row_tiles;
    // Enough workgroups to fill the chip, each sweeping a contiguous run of
    // row tiles of its strip (consecutive tiles share two staged rows in L2).
    int cus = 256;
    int dev = 0;
    if (hipGetDevice(&dev) == hipSuccess) {
        int c = 0;
        if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
            c > 0)
            cus = c;
    }
    const int want = RDC_CONV_WG_PER_CU * cus;
    int runs = (want + strips - 1) / strips;
    runs = runs < 1 ? 1 : (runs > total_tiles ? total_tiles : runs);
    const int run_len = (total_tiles + runs - 1) / runs;
    runs = (total_tiles + run_len - 1) / run_len;
    if (WCH > 0 && (a.cin + kConvKc - 1) / kConvKc > WCH) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_conv3x3<NBP, NB / NBP, P, RELU, BIAS, SRC, EPI, WCH>), dim3(strips * runs),
                       dim3(kConvThreads), 0, s, a, row_tiles, runs, run_len);
    return hipGetLastError();
}

template <int NB>
hipError_t conv_nb(const ConvArgs& a, bool relu, bool bias, hipStream_t s) {
    // Layers whose one pass of weights fits the LDS the double buffer uses
    // (32 outputs: up to 3 chunks; 64 outputs: 2 chunks) keep them resident.
    const int chunks = (a.cin + kConvKc - 1) / kConvKc;
    if constexpr (NB == 1) {
        if (relu && bias && chunks >= 2 && chunks <= 3)
            return conv_launch<NB, true, true, kSrcX, kEpiStore, 3>(a, s);
    }
    if constexpr (NB == 2) {
        if (relu && bias && chunks == 2)
            return conv_launch<NB, true, true, kSrcX, kEpiStore, 2>(a, s);
    }
    if (relu && bias) return conv_launch<NB, true, true>(a, s);
    if (bias) return conv_launch<NB, false, true>(a, s);
    if (relu) return conv_launch<NB, true, false>(a, s);
    return conv_launch<NB, false, false>(a, s);
}

}  // namespace

hipError_t conv3x3(const ConvArgs& a, bool relu, bool bias, hipStream_t s) {
    switch (a.cout >> 5) {
        case 1: return conv_nb<1>(a, relu, bias, s);
        case 2: return conv_nb<2>(a, relu, bias, s);
        case 3: return conv_nb<3>(a, relu, bias, s);
        case 4: return conv_nb<4>(a, relu, bias, s);
        case 6: return conv_nb<6>(a, relu, bias, s);
        case 8: return conv_nb<8>(a, relu, bias, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t conv3x3_up(const ConvArgs& a, hipStream_t s) {
    switch (a.cout >> 5) {
        case 1:   // 32 outputs: up to three 18 KB weight chunks stay in LDS
            if (a.cin > kConvKc && a.cin <= 3 * kConvKc)
                return conv_launch<1, true, true, kSrcUp, kEpiStore, 3>(a, s);
            return conv_launch<1, true, true, kSrcUp>(a, s);
        case 2: return conv_launch<2, true, true, kSrcUp>(a, s);
        case 4: return conv_launch<4, true, true, kSrcUp>(a, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t conv3x3_planes(const ConvArgs& a, hipStream_t s) {
    switch (a.cout >> 5) {
        case 1: return conv_launch<1, true, true, kSrcPlanes>(a, s);
        case 2: return conv_launch<2, true, true, kSrcPlanes>(a, s);
        case 4: return conv_launch<4, true, true, kSrcPlanes>(a, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t conv3x3_apply(const ConvArgs& a, hipStream_t s) {
    if (a.cout != 32) return hipErrorInvalidValue;
    return conv_launch<1, false, true, kSrcX, kEpiApply>(a, s);
}

hipError_t flip_weights(const float* w, __bf16* wd, int cout, int cin, hipStream_t s) {
    hipLaunchKernelGGL(k_flip_weights, dim3(grid_for(9LL * cout * cin)), dim3(256), 0, s, w, wd,
                       cout, cin);
    return hipGetLastError();
}

hipError_t to_bf16(const float* src, __bf16* dst, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_to_bf16, dim3(grid_for(n)), dim3(256), 0, s, src, dst, n);
    return hipGetLastError();
}

int64_t wgrad_chunks(int N, int H, int W) {
    const int64_t segs = (int64_t)N * H * (W >> 5);
    return (segs + kChunkSegs - 1) / kChunkSegs;
}

hipError_t conv3x3_wgrad(const WgradArgs& a, float* grad, float* gbias, hipStream_t s) {
    const int64_t chunks = wgrad_chunks(a.N, a.H, a.W);
    const dim3 grid((unsigned)chunks, 9 * (a.cout >> 5), a.cin >> 5);
    hipLaunchKernelGGL(k_conv3x3_wgrad, grid, dim3(64), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t n = 9LL * a.cout * a.cin;
    hipLaunchKernelGGL(k_sum_chunks, dim3(grid_for(n)), dim3(256), 0, s, a.part, grad,
                       (int)chunks, n);
    e = hipGetLastError();
    if (e != hipSuccess || !gbias) return e;
    hipLaunchKernelGGL(k_sum_chunks, dim3(grid_for(a.cout)), dim3(256), 0, s, a.bpart, gbias,
                       (int)chunks, (int64_t)a.cout);
    return hipGetLastError();
}

// 16-byte accesses possible for c channels at these strides and bases.
inline bool vec8(int c, std::initializer_list<int> lds, std::initializer_list<const void*> ptrs) {
    if (c % 8) return false;
    for (int l : lds)
        if (l % 8) return false;
    for (const void* p : ptrs)
        if (reinterpret_cast<uintptr_t>(p) & 15u) return false;
    return true;
}

hipError_t relu_bwd(__bf16* g, int ldg, const __bf16* y, int ldy, int64_t pixels, int c,
                    hipStream_t s) {
    if (vec8(c, {ldg, ldy}, {g, y})) {
        hipLaunchKernelGGL(k_relu_bwd8, dim3(grid_for(pixels * (c / 8))), dim3(256), 0, s, g, ldg,
                           y, ldy, pixels, c / 8);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_relu_bwd, dim3(grid_for(pixels * c)), dim3(256), 0, s, g, ldg, y, ldy,
                       pixels, c);
    return hipGetLastError();
}

hipError_t pool2(const __bf16* in, int ldi, __bf16* out, int ldo, int N, int Ho, int Wo, int c,
                 hipStream_t s) {
    if (vec8(c, {ldi, ldo}, {in, out})) {
        hipLaunchKernelGGL(k_pool2_8, dim3(grid_for((int64_t)N * Ho * Wo * (c / 8))), dim3(256), 0,
                           s, in, ldi, out, ldo, N, Ho, Wo, c / 8);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_pool2, dim3(grid_for((int64_t)N * Ho * Wo * c)), dim3(256), 0, s, in,
                       ldi, out, ldo, N, Ho, Wo, c);
    return hipGetLastError();
}

hipError_t pool2_bwd(const __bf16* gout, int ldo, __bf16* gin, int ldi, int N, int Ho, int Wo,
                     int c, bool accumulate, hipStream_t s) {
    if (vec8(c, {ldo, ldi}, {gout, gin})) {
        hipLaunchKernelGGL(k_pool2_bwd8, dim3(grid_for((int64_t)N * Ho * Wo * (c / 8))),
                           dim3(256), 0, s, gout, ldo, gin, ldi, N, Ho, Wo, c / 8,
                           accumulate ? 1 : 0);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_pool2_bwd, dim3(grid_for((int64_t)N * Ho * Wo * c)), dim3(256), 0, s,
                       gout, ldo, gin, ldi, N, Ho, Wo, c, accumulate ? 1 : 0);
    return hipGetLastError();
}

hipError_t up2(const __bf16* in, int ldi, __bf16* out, int ldo, int N, int Ho, int Wo, int c,
               hipStream_t s) {
    if (vec8(c, {ldi, ldo}, {in, out})) {
        hipLaunchKernelGGL(k_up2_8, dim3(grid_for((int64_t)N * Ho * Wo * (c / 8))), dim3(256), 0,
                           s, in, ldi, out, ldo, N, Ho, Wo, c / 8);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_up2, dim3(grid_for((int64_t)N * Ho * Wo * c)), dim3(256), 0, s, in, ldi,
                       out, ldo, N, Ho, Wo, c);
    return hipGetLastError();
}

hipError_t up2_bwd(const __bf16* gout, int ldo, __bf16* gin, int ldi, int N, int Hi, int Wi,
                   int c, hipStream_t s) {
    if (vec8(c, {ldo, ldi}, {gout, gin})) {
        hipLaunchKernelGGL(k_up2_bwd8, dim3(grid_for((int64_t)N * Hi * Wi * (c / 8))), dim3(256),
                           0, s, gout, ldo, gin, ldi, N, Hi, Wi, c / 8);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_up2_bwd, dim3(grid_for((int64_t)N * Hi * Wi * c)), dim3(256), 0, s,
                       gout, ldo, gin, ldi, N, Hi, Wi, c);
    return hipGetLastError();
}

hipError_t prep(const float* u, const float* v, const float* phi, int64_t pitch,
                int64_t plane_stride, __bf16* x, int c, int N, int H, int W, float su, float sv,
                float sp, hipStream_t s) {
    if (c >= 8 && vec8(c, {}, {x})) {
        hipLaunchKernelGGL(k_prep8, dim3(grid_for((int64_t)N * H * W)), dim3(256), 0, s, u, v, phi,
                           pitch, plane_stride, x, c / 8, N, H, W, su, sv, sp);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_prep, dim3(grid_for((int64_t)N * H * W)), dim3(256), 0, s, u, v, phi,
                       pitch, plane_stride, x, c, N, H, W, su, sv, sp);
    return hipGetLastError();
}

hipError_t apply(const float* u, const float* v, const float* phi, const __bf16* head, int ldh,
                 int64_t pitch, int64_t plane_stride, float* uo, float* vo, int N, int H, int W,
                 float su, float sv, float f, float cmax, hipStream_t s) {
    hipLaunchKernelGGL(k_apply, dim3(grid_for((int64_t)N * H * W)), dim3(256), 0, s, u, v, phi,
                       head, ldh, pitch, plane_stride, uo, vo, N, H, W, su, sv, f, cmax);
    return hipGetLastError();
}

int loss_blocks(int64_t pixels) { return (int)grid_for(pixels); }

hipError_t loss(const float* u, const float* v, const float* ut, const float* vt, int64_t pitch,
                int64_t plane_stride, const __bf16* head, int ldh, __bf16* g, int ldg, int N,
                int H, int W, float su, float sv, float theta, float front_w, float* partial,
                hipStream_t s) {
    const int64_t px = (int64_t)N * H * W;
    const int nb = loss_blocks(px);
    hipLaunchKernelGGL(k_loss, dim3(nb), dim3(256), 0, s, u, v, ut, vt, pitch, plane_stride, head,
                       ldh, g, ldg, N, H, W, su, sv, theta, front_w, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // The loss itself: the block partials summed in a fixed order into partial[nb].
    hipLaunchKernelGGL(k_sum_chunks, dim3(1), dim3(256), 0, s, partial, partial + nb, nb,
                       (int64_t)1);
    return hipGetLastError();
}

hipError_t adam(float* p, const float* g, float* m, float* v, int64_t n, float lr_t, float b1,
                float b2, float eps, float clip, hipStream_t s) {
    hipLaunchKernelGGL(k_adam, dim3(grid_for(n)), dim3(256), 0, s, p, g, m, v, n, lr_t, b1, b2,
                       eps, clip);
    return hipGetLastError();
}

hipError_t front_check(const float* a, const float* b, int64_t pitch, int nx, int ny,
                       float theta, unsigned int* count, hipStream_t s) {
    hipLaunchKernelGGL(k_front_check, dim3(grid_for((int64_t)nx * ny)), dim3(256), 0, s, a, b,
                       pitch, nx, ny, theta, count);
    return hipGetLastError();
}

hipError_t state_check(const float* u, const float* v, const float* phi, int64_t pitch, int nx,
                       int ny, float ulo, float uhi, float f, float cmax, unsigned int* count,
                       hipStream_t s) {
    hipLaunchKernelGGL(k_state_check, dim3(grid_for((int64_t)nx * ny)), dim3(256), 0, s, u, v,
                       phi, pitch, nx, ny, ulo, uhi, f, cmax, count);
    return hipGetLastError();
}

}  // namespace nn
}  // namespace rdc
