// The search-window network of the learned-window form: four 3x3
// convolutions, 16 channels, zero padding, ReLU after the first three,
// bfloat16 weights and activations with float32 accumulation on the matrix
// cores, plus its hand-written training kernels (loss, input and weight
// gradients, Adam) and the window map that turns its output into per-pixel
// search windows.
//
// Implicit GEMM: a wave owns 16 consecutive pixels of one row (the M
// dimension) and all 16 output channels (N); the reduction runs over the 9
// taps x 16 input channels.  The forward passes (training forward and the
// one-launch inference) take two taps per v_mfma_f32_16x16x32_bf16 step
// (5 steps, the last one tap and zeros); the input gradient takes one tap
// per v_mfma_f32_16x16x16bf16_1k step.  Activations are NHWC [n][H][W][16]
// bfloat16, so a lane's 8 (4) input channels of one pixel are one 16-byte
// (8-byte) load.
//
// Operand layouts (lane l, g = l/16; checked on the device):
//   16x16x32: A[i][k]: i = l % 16, k = 8g .. 8g+7; B[k][j]: j = l % 16,
//             k = 8g .. 8g+7 (8 bf16 in four registers)
//   16x16x16: the same with k = 4g .. 4g+3 (4 bf16 in two registers)
//   D[i][j]:  j = l % 16, i = 4g + r for accumulator element r = 0..3.
//
// Weight-gradient sums run over pixels; each wave writes its partial sums
// and a second kernel adds the partials in wave order, so the gradient is
// bitwise reproducible.

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>

#include "../../include/sgm.h"
#include "sgm_internal.h"

namespace sgm {
namespace {

constexpr int CH = 16;
constexpr int LAYERS = 4;
constexpr int PER_LAYER = 9 * CH * CH + CH;
constexpr int NPARAMS = LAYERS * PER_LAYER;
constexpr int kWgradWaves = 1024;
constexpr int kOutCh = 2;  // output channels used: centre offset, confidence logit

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

// float -> bfloat16, round to nearest even
__device__ __forceinline__ uint16_t f2bf(float f)
{
    const uint32_t u = __float_as_uint(f);
    return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// 8 consecutive bfloat16 (16 bytes, 4-byte aligned at least)
__device__ __forceinline__ v8bf load8(const uint16_t *p)
{
    return __builtin_bit_cast(v8bf, *reinterpret_cast<const uint4 *>(p));
}
__device__ __forceinline__ v8bf zero8() { return __builtin_bit_cast(v8bf, make_uint4(0u, 0u, 0u, 0u)); }

__device__ __forceinline__ v4s load4(const uint16_t *p)
{
    const uint2 t = *reinterpret_cast<const uint2 *>(p);
    v4s r;
    r[0] = (short)(t.x & 0xFFFF);
    r[1] = (short)(t.x >> 16);
    r[2] = (short)(t.y & 0xFFFF);
    r[3] = (short)(t.y >> 16);
    return r;
}

// strip s of 16 pixels: image n, row y, first column x0
struct Strip {
    int n, y, x0;
};
__device__ __forceinline__ Strip strip_of(int s, int W, int H)
{
    const int sx = (W + 15) / 16;
    Strip t;
    t.x0 = (s % sx) * 16;
    const int r = s / sx;
    t.y = r % H;
    t.n = r / H;
    return t;
}

// ---------------------------------------------------------------------------
// convolution forward (and input gradient): D[pixel][co] over 9 taps

// MODE 0: hidden layer forward  (out = bf16(relu(conv + b)))
// MODE 1: last layer forward    (out32 = conv + b, float, only the two
//                                channels the window map reads: offset, logit)
// MODE 2: input gradient        (dx = conv^T(dy); out = bf16(dx * [mask > 0]))
//
// A wave takes kStripsPerWave consecutive strips: the 9 taps' weight
// operands stay in registers, and each strip's 9 input loads are issued
// before its 9 MFMAs.
constexpr int kStripsPerWave = 8;

template <int MODE>
__global__ __launch_bounds__(256) void k_conv(const uint16_t *__restrict__ x, const uint16_t *__restrict__ wt,
                                              const float *__restrict__ bias, const uint16_t *__restrict__ mask,
                                              int W, int H, int nstrips, uint16_t *__restrict__ out,
                                              float *__restrict__ out32)
{
    const int lane = threadIdx.x & 63;
    const int wave = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int s_first = wave * kStripsPerWave;
    if (s_first >= nstrips) return;
    const int i = lane & 15, g = lane >> 4;
    const float bi = MODE == 2 ? 0.0f : bias[i];
    const int s_end = min(s_first + kStripsPerWave, nstrips);
    // forward (MODE 0, 1): K = 32 per MFMA, two taps at a time — lane group
    // g holds tap 2m + g/2, channels 8 (g % 2) .. +7 of step m (the fifth
    // step carries tap 8 and zeros).  Input gradient (MODE 2): K = 16, one
    // tap per step, lane group g holds channels 4g .. 4g+3.
    v8bf b8[5];
    v4s b[9];
    if constexpr (MODE != 2) {
#pragma unroll
        for (int m = 0; m < 5; ++m) {
            const int t = 2 * m + (g >> 1);
            b8[m] = t < 9 ? load8(wt + (size_t)t * CH * CH + (size_t)i * CH + 8 * (g & 1)) : zero8();
        }
    } else {
#pragma unroll
        for (int t = 0; t < 9; ++t) b[t] = load4(wt + (size_t)t * CH * CH + (size_t)i * CH + 4 * g);
    }
    for (int s = s_first; s < s_end; ++s) {
        const Strip st = strip_of(s, W, H);
        v4f acc = {0.f, 0.f, 0.f, 0.f};
        if constexpr (MODE != 2) {
            v8bf a8[5];
#pragma unroll
            for (int m = 0; m < 5; ++m) {
                const int t = 2 * m + (g >> 1);
                const int yy = st.y + t / 3 - 1, xx = st.x0 + i + t % 3 - 1;
                a8[m] = zero8();
                if (t < 9 && yy >= 0 && yy < H && xx >= 0 && xx < W)
                    a8[m] = load8(x + (((size_t)st.n * H + yy) * W + xx) * CH + 8 * (g & 1));
            }
#pragma unroll
            for (int m = 0; m < 5; ++m) acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a8[m], b8[m], acc, 0, 0, 0);
        } else {
            v4s a[9];
#pragma unroll
            for (int t = 0; t < 9; ++t) {
                // transpose: the gradient flows back from p - offset
                const int yy = st.y - (t / 3 - 1), xx = st.x0 + i - (t % 3 - 1);
                a[t] = (v4s){0, 0, 0, 0};
                if (yy >= 0 && yy < H && xx >= 0 && xx < W)
                    a[t] = load4(x + (((size_t)st.n * H + yy) * W + xx) * CH + 4 * g);
            }
#pragma unroll
            for (int t = 0; t < 9; ++t) acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[t], b[t], acc, 0, 0, 0);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int xo = st.x0 + 4 * g + r;
            if (xo >= W) continue;
            const size_t o = (((size_t)st.n * H + st.y) * W + xo) * CH + i;
            if (MODE == 0) {
                out[o] = f2bf(fmaxf(acc[r] + bi, 0.0f));
            } else if (MODE == 1) {
                if (i < kOutCh) out32[(((size_t)st.n * H + st.y) * W + xo) * kOutCh + i] = acc[r] + bi;
            } else {
                out[o] = f2bf(bf2f(mask[o]) > 0.0f ? acc[r] : 0.0f);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// inference: all four layers for one output tile in one workgroup
//
// The tile's input with a halo of 4 pixels (one per layer) sits in LDS as
// bfloat16 [row][column][16]; each layer reads one LDS buffer and writes the
// other, shrinking the computed region by one pixel per side, so hidden
// activations never reach HBM.  A layer's output outside the image is
// written as 0 (the next layer's zero padding).  Positions beyond a
// layer's computed region are never read by a position inside the next
// layer's region, so their contents do not matter.
//
// The MFMA runs transposed with respect to k_conv (weights as the A
// operand, pixels as B): D[co][pixel], so each lane ends with 4 channels of
// one pixel, which is one 8-byte LDS write in the layout the next layer
// reads.  The products and their positions in each K = 32 step (two taps x
// 16 input channels) are those of k_conv's forward, and the steps
// accumulate in the same order, so the result equals the layer-by-layer
// forward bit for bit.  A wave runs two
// items' MFMA chains interleaved and loads the next two items' operands from
// LDS before them.

constexpr int kFTW = 24;           // output tile columns
constexpr int kFTH = 16;           // output tile rows
constexpr int kFR = kFTH + 8;      // tile rows with the halo
constexpr int kFCP = 40;           // tile columns with the halo (32) and slack for the last strip's reads
constexpr int kFPix = kFR * kFCP;  // pixels per LDS buffer

// LDS entry of channels 4q .. 4q+3 of tile pixel p: the four 8-byte groups
// of pixels with bit 3 set are stored in the order 2, 3, 0, 1, so that the
// 16 consecutive pixels x 2 groups of a half-wave's access fall on 32
// distinct bank pairs
__device__ __forceinline__ int fslot(int p, int q) { return p * 4 + (q ^ ((p >> 2) & 2)); }

__global__ __launch_bounds__(256) void k_cnn_infer(const uint16_t *__restrict__ x0, const uint16_t *__restrict__ wf,
                                                   const float *__restrict__ params, int W, int H,
                                                   float *__restrict__ out)
{
    __shared__ uint2 buf[2][kFPix * 4];  // 4 channels (8 bytes) per entry
    const int X0 = (int)blockIdx.x * kFTW - 4, Y0 = (int)blockIdx.y * kFTH - 4;
    const size_t img = (size_t)blockIdx.z * H;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));  // uniform: item loops without exec masks
    const int i = lane & 15, g = lane >> 4;
    // every global load of the launch is issued before the first wait: the
    // input tile, then all four layers' weight operands and biases
    constexpr int kLoads = kFPix * 4 / 256;
    static_assert(kFPix * 4 % 256 == 0, "tile loads must split evenly over 256 threads");
    uint2 tile[kLoads];
#pragma unroll
    for (int k = 0; k < kLoads; ++k) {
        const int q = (int)threadIdx.x + 256 * k;
        const int px = q >> 2, part = q & 3;
        const int r = px / kFCP, c = px - r * kFCP;
        const int yy = Y0 + r, xx = X0 + c;
        tile[k] = make_uint2(0u, 0u);
        if (yy >= 0 && yy < H && xx >= 0 && xx < W)
            tile[k] = *reinterpret_cast<const uint2 *>(x0 + ((img + yy) * W + xx) * CH + 4 * part);
    }
    v8bf wt[LAYERS][5];
    float bias[LAYERS][4];
#pragma unroll
    for (int l = 0; l < LAYERS; ++l) {
#pragma unroll
        for (int m = 0; m < 5; ++m) {
            const int t = 2 * m + (g >> 1);
            wt[l][m] = t < 9 ? load8(wf + ((size_t)l * 9 + t) * CH * CH + (size_t)i * CH + 8 * (g & 1)) : zero8();
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) bias[l][e] = params[(size_t)l * PER_LAYER + 9 * CH * CH + 4 * g + e];
    }
#pragma unroll
    for (int k = 0; k < kLoads; ++k) {
        const int q = (int)threadIdx.x + 256 * k;
        buf[0][fslot(q >> 2, q & 3)] = tile[k];
    }
    __syncthreads();
#pragma unroll
    for (int l = 0; l < LAYERS; ++l) {
        const uint2 *in = buf[l & 1];
        uint2 *ob = buf[(l + 1) & 1];
        // layer l computes rows [l + 1, kFR - l - 1) and columns
        // [l + 1, l + 33) of the tile: two strips of 16 pixels per row
        const int h = l + 1;
        const int nitems = 2 * (kFR - 2 * h);
        auto load_item = [&](int it, v8bf(&a)[5]) __attribute__((always_inline)) {
            const int r = h + (it >> 1), c0 = h + 16 * (it & 1);
#pragma unroll
            for (int m = 0; m < 5; ++m) {
                // tap 2m + g/2, channels 8 (g % 2) .. +7: two adjacent 8-byte groups
                const int t = 2 * m + (g >> 1);
                a[m] = zero8();
                if (t < 9) {
                    const uint2 *q = &in[fslot((r + t / 3 - 1) * kFCP + c0 + i + t % 3 - 1, 2 * (g & 1))];
                    a[m] = __builtin_bit_cast(v8bf, *reinterpret_cast<const uint4 *>(q));
                }
            }
        };
        // items it and it + 4 together: two independent MFMA chains
        auto compute = [&](int it, const v8bf(&a)[5], const v8bf(&b)[5]) __attribute__((always_inline)) {
            v4f acc[2] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
#pragma unroll
            for (int m = 0; m < 5; ++m) {
                acc[0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wt[l][m], a[m], acc[0], 0, 0, 0);
                acc[1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wt[l][m], b[m], acc[1], 0, 0, 0);
            }
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int iu = it + 4 * u;
                if (iu >= nitems) break;
                const int r = h + (iu >> 1), c = h + 16 * (iu & 1) + i;
                const int yy = Y0 + r, xx = X0 + c;
                // acc[u][e]: channel 4g + e of pixel (r, c)
                if (l < LAYERS - 1) {
                    const uint32_t inside = ((unsigned)yy < (unsigned)H) & ((unsigned)xx < (unsigned)W);
                    const uint32_t keep = 0u - inside;
                    uint32_t v[4];
#pragma unroll
                    for (int e = 0; e < 4; ++e) v[e] = f2bf(fmaxf(acc[u][e] + bias[l][e], 0.0f));
                    ob[fslot(r * kFCP + c, g)] =
                        make_uint2((v[0] | (v[1] << 16)) & keep, (v[2] | (v[3] << 16)) & keep);
                } else if (g == 0 && c < 4 + kFTW && yy < H && xx < W) {
                    *reinterpret_cast<float2 *>(out + ((img + yy) * W + xx) * kOutCh) =
                        make_float2(acc[u][0] + bias[l][0], acc[u][1] + bias[l][1]);
                }
            }
        };
        // a wave's items: wave, wave + 4, ...; pairs of them, the next pair's
        // operands loaded from LDS before the current pair's MFMAs
        v8bf p0[2][5], p1[2][5];
        auto load_pair = [&](int it, v8bf(&p)[2][5]) __attribute__((always_inline)) {
            if (it < nitems) load_item(it, p[0]);
            if (it + 4 < nitems) load_item(it + 4, p[1]);
        };
        int it = wave;
        load_pair(it, p0);
        while (it < nitems) {
            load_pair(it + 8, p1);
            compute(it, p0[0], p0[1]);
            it += 8;
            if (it >= nitems) break;
            load_pair(it + 8, p0);
            compute(it, p1[0], p1[1]);
            it += 8;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// weight gradient: per tap D[co][ci] = sum_p dy[p][co] x[p + offset][ci]

__global__ __launch_bounds__(64) void k_wgrad(const uint16_t *__restrict__ x, const uint16_t *__restrict__ dy, int W,
                                              int H, int nstrips, float *__restrict__ partial)
{
    const int lane = threadIdx.x;
    const int wave = blockIdx.x;
    const int i = lane & 15, g = lane >> 4;
    v4f acc[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) acc[t] = (v4f){0.f, 0.f, 0.f, 0.f};
    float dbias = 0.0f;
    for (int s = wave; s < nstrips; s += gridDim.x) {
        const Strip st = strip_of(s, W, H);
        // A[co][k]: dy of pixels x0 + 4g .. 4g+3, channel co = i
        v4s a;
        const size_t rowb = ((size_t)st.n * H + st.y) * W;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int xk = st.x0 + 4 * g + e;
            const uint16_t v = xk < W ? dy[(rowb + xk) * CH + i] : (uint16_t)0;
            a[e] = (short)v;
            dbias += bf2f(v);
        }
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            const int ddy = t / 3 - 1, ddx = t % 3 - 1;
            const int yy = st.y + ddy;
            v4s b;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int xk = st.x0 + 4 * g + e, xx = xk + ddx;
                uint16_t v = 0;
                if (xk < W && yy >= 0 && yy < H && xx >= 0 && xx < W)
                    v = x[(((size_t)st.n * H + yy) * W + xx) * CH + i];
                b[e] = (short)v;
            }
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[t], 0, 0, 0);
        }
    }
    // partial layout per wave: [tap][co][ci] then bias partials [group][co]
    float *p = partial + (size_t)wave * (9 * CH * CH + 4 * CH);
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) p[(size_t)t * CH * CH + (4 * g + r) * CH + i] = acc[t][r];
    p[9 * CH * CH + g * CH + i] = dbias;
}

// sum of the per-wave partials, in wave order
__global__ __launch_bounds__(256) void k_wgrad_reduce(const float *__restrict__ partial, int nwaves,
                                                      float *__restrict__ grad)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= PER_LAYER) return;
    const int stride = 9 * CH * CH + 4 * CH;
    float sum = 0.0f;
    if (k < 9 * CH * CH) {
        for (int wv = 0; wv < nwaves; ++wv) sum += partial[(size_t)wv * stride + k];
    } else {
        const int co = k - 9 * CH * CH;
        for (int wv = 0; wv < nwaves; ++wv)
            for (int g = 0; g < 4; ++g) sum += partial[(size_t)wv * stride + 9 * CH * CH + g * CH + co];
    }
    grad[k] = sum;
}

// ---------------------------------------------------------------------------
// input, loss, optimiser, window map

__global__ void k_prepare_input(const float *__restrict__ coarse, const uint8_t *__restrict__ left, int W, int npix,
                                uint16_t *__restrict__ x0)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= npix) return;
    const float cd = coarse[p];
    const float col = (float)(p % W);
    const uint16_t c0 = f2bf(__fdiv_rn(cd, 16.0f));
    const uint16_t c1 = f2bf(__fsub_rn(__fdiv_rn((float)left[p], 255.0f), 0.5f));
    // distance of the coarse match from the left border, saturated at 16
    const uint16_t c2 = f2bf(__fdiv_rn(fminf(__fsub_rn(col, cd), 16.0f), 16.0f));
    uint4 *o = reinterpret_cast<uint4 *>(x0 + (size_t)p * CH);
    o[0] = make_uint4(c0 | (uint32_t)c1 << 16, c2, 0u, 0u);
    o[1] = make_uint4(0u, 0u, 0u, 0u);
}

__global__ void k_loss(const float *__restrict__ out, const float *__restrict__ coarse, const float *__restrict__ label,
                       int npix, uint16_t *__restrict__ dy, float *__restrict__ loss_sum)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= npix) return;
    const float invn = 1.0f / (float)npix;
    const float off = out[(size_t)p * kOutCh], logit = out[(size_t)p * kOutCh + 1];
    const float e = off - (label[p] - coarse[p]);
    const float ae = fabsf(e);
    const float c = ae < 1.0f ? 1.0f : 0.0f;
    const float huber = ae <= 1.0f ? 0.5f * e * e : ae - 0.5f;
    const float bce = fmaxf(logit, 0.0f) - c * logit + log1pf(expf(-fabsf(logit)));
    uint16_t g[CH];
#pragma unroll
    for (int k = 0; k < CH; ++k) g[k] = 0;
    g[0] = f2bf(fminf(fmaxf(e, -1.0f), 1.0f) * invn);
    g[1] = f2bf((1.0f / (1.0f + expf(-logit)) - c) * invn);
    uint4 *o = reinterpret_cast<uint4 *>(dy + (size_t)p * CH);
    o[0] = make_uint4(g[0] | (uint32_t)g[1] << 16, 0u, 0u, 0u);
    o[1] = make_uint4(0u, 0u, 0u, 0u);
    if (loss_sum) {
        atomicAdd(loss_sum, huber * invn);
        atomicAdd(loss_sum + 1, bce * invn);
    }
}

// Adam on the float32 master parameters; also refreshes the bfloat16
// weights in the forward ([tap][co][ci]) and transposed ([tap][ci][co])
// layouts.
__global__ void k_adam(float *__restrict__ params, float *__restrict__ m, float *__restrict__ v,
                       const float *__restrict__ grad, float lr, float b1, float b2, float eps, float c1, float c2,
                       int update, uint16_t *__restrict__ wf, uint16_t *__restrict__ wb)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= NPARAMS) return;
    float p = params[k];
    if (update) {
        const float gk = grad[k];
        const float mk = b1 * m[k] + (1.0f - b1) * gk;
        const float vk = b2 * v[k] + (1.0f - b2) * gk * gk;
        m[k] = mk;
        v[k] = vk;
        p = p - lr * (mk / c1) / (sqrtf(vk / c2) + eps);
        params[k] = p;
    }
    const int l = k / PER_LAYER, r = k % PER_LAYER;
    if (r < 9 * CH * CH) {
        const int t = r / (CH * CH), co = (r / CH) % CH, ci = r % CH;
        const size_t base = (size_t)l * 9 * CH * CH + (size_t)t * CH * CH;
        wf[base + co * CH + ci] = f2bf(p);
        wb[base + ci * CH + co] = f2bf(p);
    }
}

__global__ void k_clear_stats(int32_t *__restrict__ row_stats, int H, int W, uint32_t *__restrict__ nfallback)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    // image blockIdx.z of a stack
    if (row_stats) row_stats += (size_t)blockIdx.z * 3 * H;
    if (nfallback) nfallback += blockIdx.z;
    if (row_stats && i < H) {
        row_stats[i] = 0;          // fallback pixels in the row
        row_stats[H + i] = W;      // leftmost fallback column
        row_stats[2 * H + i] = -1; // rightmost fallback column
    }
    if (nfallback && i == 0) *nfallback = 0u;
}

// One row of full-resolution pixels per grid row, four consecutive pixels
// per thread (one 16-byte store of window starts and one 4-byte store of
// fallback flags where the row offset allows).  The fallback count and
// column extent of the row segment are reduced over the workgroup (wave
// shuffles, then LDS) before one atomic per statistic.
constexpr int kMapPix = 4;

__global__ __launch_bounds__(256) void k_window_map(const float *__restrict__ coarse, const float *__restrict__ out,
                                                    int Wc, int Hc, int W, int H, int D, int w, float thr,
                                                    float fb_margin, int32_t *__restrict__ lo,
                                                    uint8_t *__restrict__ mask,
                                                    int32_t *__restrict__ row_stats, uint32_t *__restrict__ nfallback)
{
    const int x0 = (blockIdx.x * blockDim.x + threadIdx.x) * kMapPix, y = blockIdx.y;
    // image blockIdx.z of a stack: every buffer is packed per image
    {
        const size_t z = blockIdx.z;
        coarse += z * Wc * Hc;
        out += z * Wc * Hc * kOutCh;
        lo += z * W * H;
        if (mask) mask += z * W * H;
        if (row_stats) row_stats += z * 3 * H;
        if (nfallback) nfallback += z;
    }
    int cnt = 0, xmin = W, xmax = -1;
    int32_t lv[kMapPix];
    uint32_t mv = 0;
    const int cy = min(y / 4, Hc - 1);
#pragma unroll
    for (int e = 0; e < kMapPix; ++e) {
        const int x = x0 + e;
        lv[e] = 0;
        if (x < W) {
            const int cx = min(x / 4, Wc - 1);
            const size_t cp = (size_t)cy * Wc + cx;
            const float cd = coarse[cp];
            const bool conf = out[cp * kOutCh + 1] > thr;
            const float centre = 4.0f * (conf ? __fadd_rn(cd, out[cp * kOutCh]) : cd);
            int l = (int)floorf(__fadd_rn(centre, 0.5f)) - w / 2;
            lv[e] = min(max(l, 0), D - w);
            // a low-confidence pixel falls back to full range only while its
            // coarse match lies inside the right image (x - 4 coarse >=
            // margin); further left it sees a point outside the right
            // camera's view, which no disparity range can match
            if (!conf && __fsub_rn((float)x, 4.0f * cd) >= fb_margin) {
                mv |= 1u << (8 * e);
                ++cnt;
                xmin = min(xmin, x);
                xmax = max(xmax, x);
            }
        }
    }
    const size_t o = (size_t)y * W + x0;
    if (x0 + kMapPix <= W && (o % kMapPix) == 0) {
        *reinterpret_cast<int4 *>(lo + o) = make_int4(lv[0], lv[1], lv[2], lv[3]);
        if (mask) *reinterpret_cast<uint32_t *>(mask + o) = mv;
    } else {
        for (int e = 0; e < kMapPix && x0 + e < W; ++e) {
            lo[o + e] = lv[e];
            if (mask) mask[o + e] = (uint8_t)((mv >> (8 * e)) & 1u);
        }
    }
    if (!row_stats && !nfallback) return;
    // the workgroup's fallback count and column extent
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        cnt += __shfl_xor(cnt, d);
        xmin = min(xmin, __shfl_xor(xmin, d));
        xmax = max(xmax, __shfl_xor(xmax, d));
    }
    __shared__ int s_st[3][4];
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        s_st[0][wv] = cnt;
        s_st[1][wv] = xmin;
        s_st[2][wv] = xmax;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < (int)(blockDim.x >> 6); ++k) {
            cnt += s_st[0][k];
            xmin = min(xmin, s_st[1][k]);
            xmax = max(xmax, s_st[2][k]);
        }
        if (cnt > 0) {
            if (row_stats) {
                atomicAdd(row_stats + y, cnt);
                atomicMin(row_stats + H + y, xmin);
                atomicMax(row_stats + 2 * H + y, xmax);
            }
            if (nfallback) atomicAdd(nfallback, (uint32_t)cnt);
        }
    }
}

// Fallback pixels of the rectangle (rows y0.., columns x0..) take the
// rectangle's full-range result.
__global__ void k_merge_fallback(const uint8_t *__restrict__ mask, const int16_t *__restrict__ band_int,
                                 const float *__restrict__ band_sub, int W, int y0, int rows, int x0, int cols,
                                 int16_t *__restrict__ dint, float *__restrict__ dsub)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x, r = blockIdx.y;
    if (c >= cols || r >= rows) return;
    const size_t o = (size_t)(y0 + r) * W + x0 + c, b = (size_t)r * cols + c;
    if (!mask[o]) return;
    dint[o] = band_int[b];
    if (dsub && band_sub) dsub[o] = band_sub[b];
}

// Every fallback rectangle of a batch in one launch: rectangle z (grid z)
// = rects[6z .. 6z+5] = frame, y0, rows, x0, cols, offset of its first
// element in the band arrays.  Rectangles, or pixels of them, outside the
// frames or the band arrays are skipped (memory-safe for any table).
__global__ void k_merge_fallback_rects(const uint8_t *__restrict__ mask, const int32_t *__restrict__ rects, int W,
                                       int H, int nframes, const int16_t *__restrict__ band_int,
                                       const float *__restrict__ band_sub, long long band_len,
                                       int16_t *__restrict__ dint, float *__restrict__ dsub)
{
    const int32_t *R = rects + 6 * (size_t)blockIdx.z;
    const int f = R[0], y0 = R[1], rows = R[2], x0 = R[3], cols = R[4];
    const long long boff = R[5];
    const int c = blockIdx.x * blockDim.x + threadIdx.x, r = blockIdx.y;
    if (c >= cols || r >= rows || f < 0 || f >= nframes || y0 < 0 || x0 < 0 || y0 + r >= H || x0 + c >= W) return;
    const long long b = boff + (long long)r * cols + c;
    if (boff < 0 || b >= band_len) return;
    const size_t o = ((size_t)f * H + (size_t)(y0 + r)) * W + x0 + c;
    if (!mask[o]) return;
    dint[o] = band_int[b];
    if (dsub && band_sub) dsub[o] = band_sub[b];
}

__global__ void k_label_downsample4(const float *__restrict__ full, int W, int H, float *__restrict__ coarse)
{
    const int Wc = W / 4, Hc = H / 4;
    const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
    if (x >= Wc || y >= Hc) return;
    float s = 0.0f;
    for (int dy = 0; dy < 4; ++dy)
        for (int dx = 0; dx < 4; ++dx) s += full[(size_t)(4 * y + dy) * W + 4 * x + dx];
    coarse[(size_t)y * Wc + x] = s * (1.0f / 64.0f);  // mean of the block, in coarse pixels
}

sgm_status cfail(sgm_status st, const char *msg)
{
    snprintf(error_buffer(), kErrorBufferSize, "%s", msg);
    return st;
}

sgm_status launched(const char *what)
{
    const hipError_t e = hipGetLastError();
    if (e == hipSuccess) return SGM_OK;
    snprintf(error_buffer(), kErrorBufferSize, "%s: %s", what, hipGetErrorString(e));
    return SGM_ERR_HIP;
}

bool aligned(const void *p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

// n images of W x H: sizes >= 1, and every element index (16 channels per
// pixel) fits the kernels' 32-bit arithmetic
sgm_status check_images(int32_t width, int32_t height, int32_t nimg)
{
    if (width < 1 || height < 1 || nimg < 1) return cfail(SGM_ERR_INVALID, "sizes must be >= 1");
    if ((long long)width * height * nimg * CH >= (1ll << 31))
        return cfail(SGM_ERR_UNSUPPORTED, "nimg * height * width * 16 must be < 2^31");
    return SGM_OK;
}

}  // namespace
}  // namespace sgm

using namespace sgm;

extern "C" {

int32_t sgm_cnn_num_params(void) { return NPARAMS; }

size_t sgm_cnn_scratch_bytes(int32_t width, int32_t height, int32_t nimg)
{
    if (width < 1 || height < 1 || nimg < 1) return 0;
    const size_t act = (size_t)nimg * height * width * CH * 2;
    return 2 * ((act + 255) & ~(size_t)255) + (size_t)kWgradWaves * (9 * CH * CH + 4 * CH) * 4;
}

sgm_status sgm_cnn_pack_weights(const float *params, uint16_t *wf, uint16_t *wb, void *stream)
{
    if (!params || !wf || !wb) return cfail(SGM_ERR_INVALID, "params, wf and wb must not be NULL");
    if (fault_take(kFaultLaunch)) return cfail(SGM_ERR_HIP, "injected launch failure");
    hipLaunchKernelGGL(k_adam, dim3((NPARAMS + 255) / 256), dim3(256), 0, (hipStream_t)stream,
                       const_cast<float *>(params), nullptr, nullptr, nullptr, 0.f, 0.f, 0.f, 0.f, 1.f, 1.f, 0, wf,
                       wb);
    return launched("pack weights");
}

sgm_status sgm_cnn_prepare_input(const float *coarse_disp, const uint8_t *coarse_left, int32_t width, int32_t height,
                                 int32_t nimg, uint16_t *x0, void *stream)
{
    if (!coarse_disp || !coarse_left || !x0) return cfail(SGM_ERR_INVALID, "NULL buffer");
    if (sgm_status st = check_images(width, height, nimg)) return st;
    if (!aligned(x0, 16)) return cfail(SGM_ERR_INVALID, "x0 must be 16-byte aligned");
    const int npix = width * height * nimg;
    if (fault_take(kFaultLaunch)) return cfail(SGM_ERR_HIP, "injected launch failure");
    hipLaunchKernelGGL(k_prepare_input, dim3((npix + 255) / 256), dim3(256), 0, (hipStream_t)stream, coarse_disp,
                       coarse_left, width, npix, x0);
    return launched("prepare input");
}

sgm_status sgm_cnn_forward(const uint16_t *wf, const float *params, const uint16_t *x0, int32_t width, int32_t height,
                           int32_t nimg, uint16_t *acts, float *out, void *stream)
{
    if (!wf || !params || !x0 || !acts || !out) return cfail(SGM_ERR_INVALID, "NULL buffer");
    if (sgm_status st = check_images(width, height, nimg)) return st;
    if (!aligned(x0, 8) || !aligned(acts, 8) || !aligned(wf, 8)) return cfail(SGM_ERR_INVALID, "misaligned buffer");
    const size_t act = (size_t)nimg * height * width * CH;
    const int nstrips = nimg * height * ((width + 15) / 16);
    const int nwaves = (nstrips + kStripsPerWave - 1) / kStripsPerWave;
    dim3 grid((nwaves + 3) / 4), block(256);
    hipStream_t s = (hipStream_t)stream;
    const uint16_t *in = x0;
    if (fault_take(kFaultLaunch)) return cfail(SGM_ERR_HIP, "injected launch failure");
    for (int l = 0; l < LAYERS; ++l) {
        const uint16_t *wl = wf + (size_t)l * 9 * CH * CH;
        const float *bl = params + (size_t)l * PER_LAYER + 9 * CH * CH;
        if (l < LAYERS - 1) {
            uint16_t *o = acts + (size_t)l * act;
            hipLaunchKernelGGL(k_conv<0>, grid, block, 0, s, in, wl, bl, nullptr, width, height, nstrips, o, nullptr);
            in = o;
        } else {
            hipLaunchKernelGGL(k_conv<1>, grid, block, 0, s, in, wl, bl, nullptr, width, height, nstrips, nullptr,
                               out);
        }
    }
    return launched("cnn forward");
}

sgm_status sgm_cnn_infer(const uint16_t *wf, const float *params, const uint16_t *x0, int32_t width, int32_t height,
                         int32_t nimg, float *out, void *stream)
{
    if (!wf || !params || !x0 || !out) return cfail(SGM_ERR_INVALID, "NULL buffer");
    if (sgm_status st = check_images(width, height, nimg)) return st;
    if (!aligned(x0, 8) || !aligned(wf, 8)) return cfail(SGM_ERR_INVALID, "misaligned buffer");
    if (nimg > 65535) return cfail(SGM_ERR_UNSUPPORTED, "more than 65535 images");
    if (fault_take(kFaultLaunch)) return cfail(SGM_ERR_HIP, "injected launch failure");
    dim3 grid((width + kFTW - 1) / kFTW, (height + kFTH - 1) / kFTH, nimg), block(256);
    hipLaunchKernelGGL(k_cnn_infer, grid, block, 0, (hipStream_t)stream, x0, wf, params, width, height, out);
    return launched("cnn inference");
}

sgm_status sgm_cnn_loss(const float *out, const float *coarse_disp, const float *label, int32_t width, int32_t height,
                        int32_t nimg, uint16_t *dy, float *loss_sum, void *stream)
{
    if (!out || !coarse_disp || !label || !dy) return cfail(SGM_ERR_INVALID, "NULL buffer");
    if (sgm_status st = check_images(width, height, nimg)) return st;
    if (!aligned(dy, 16)) return cfail(SGM_ERR_INVALID, "dy must be 16-byte aligned");
    const int npix = width * height * nimg;
    if (fault_take(kFaultLaunch)) return cfail(SGM_ERR_HIP, "injected launch failure");
    hipLaunchKernelGGL(k_loss, dim3((npix + 255) / 256), dim3(256), 0, (hipStream_t)stream, out, coarse_disp, label,
                       npix, dy, loss_sum);
    return launched("cnn loss");
}

sgm_status sgm_cnn_backward(const uint16_t *wb, const uint16_t *x0, const uint16_t *acts, const uint16_t *dy_out,
                            int32_t width, int32_t height, int32_t nimg, float *grad, void *scratch,
                            size_t scratch_bytes, void *stream)
{
    if (!wb || !x0 || !acts || !dy_out || !grad || !scratch) return cfail(SGM_ERR_INVALID, "NULL buffer");
    if (sgm_status st = check_images(width, height, nimg)) return st;
    if (scratch_bytes < sgm_cnn_scratch_bytes(width, height, nimg))
        return cfail(SGM_ERR_WORKSPACE, "scratch smaller than sgm_cnn_scratch_bytes");
    if (!aligned(scratch, 256)) return cfail(SGM_ERR_INVALID, "scratch must be 256-byte aligned");
    const size_t act = (size_t)nimg * height * width * CH;
    const size_t act_bytes = (act * 2 + 255) & ~(size_t)255;
    uint16_t *dyA = static_cast<uint16_t *>(scratch);
    uint16_t *dyB = reinterpret_cast<uint16_t *>(static_cast<uint8_t *>(scratch) + act_bytes);
    float *partial = reinterpret_cast<float *>(static_cast<uint8_t *>(scratch) + 2 * act_bytes);
    const int nstrips = nimg * height * ((width + 15) / 16);
    const int nw = nstrips < kWgradWaves ? nstrips : kWgradWaves;
    hipStream_t s = (hipStream_t)stream;
    const uint16_t *dy = dy_out;
    if (fault_take(kFaultLaunch)) return cfail(SGM_ERR_HIP, "injected launch failure");
    for (int l = LAYERS - 1; l >= 0; --l) {
        const uint16_t *xin = l == 0 ? x0 : acts + (size_t)(l - 1) * act;
        hipLaunchKernelGGL(k_wgrad, dim3(nw), dim3(64), 0, s, xin, dy, width, height, nstrips, partial);
        hipLaunchKernelGGL(k_wgrad_reduce, dim3((PER_LAYER + 255) / 256), dim3(256), 0, s, partial, nw,
                           grad + (size_t)l * PER_LAYER);
        if (l > 0) {
            uint16_t *dnext = (l % 2) ? dyA : dyB;
            const int nwaves = (nstrips + kStripsPerWave - 1) / kStripsPerWave;
            hipLaunchKernelGGL(k_conv<2>, dim3((nwaves + 3) / 4), dim3(256), 0, s, dy, wb + (size_t)l * 9 * CH * CH,
                               nullptr, xin, width, height, nstrips, dnext, nullptr);
            dy = dnext;
        }
    }
    return launched("cnn backward");
}

sgm_status sgm_cnn_adam(float *params, float *m, float *v, const float *grad, int32_t step, float lr, float beta1,
                        float beta2, float eps, uint16_t *wf, uint16_t *wb, void *stream)
{
    if (!params || !m || !v || !grad || !wf || !wb) return cfail(SGM_ERR_INVALID, "NULL buffer");
    if (step < 1) return cfail(SGM_ERR_INVALID, "step must be >= 1");
    // bias corrections in double: 1 - beta2^t is small early on and would
    // lose most of its digits in float
    const float c1 = (float)(1.0 - pow((double)beta1, (double)step));
    const float c2 = (float)(1.0 - pow((double)beta2, (double)step));
    if (fault_take(kFaultLaunch)) return cfail(SGM_ERR_HIP, "injected launch failure");
    hipLaunchKernelGGL(k_adam, dim3((NPARAMS + 255) / 256), dim3(256), 0, (hipStream_t)stream, params, m, v, grad,
                       lr, beta1, beta2, eps, c1, c2, 1, wf, wb);
    return launched("cnn adam");
}

static sgm_status window_map_n(const float *coarse_disp, const float *cnn_out, int32_t coarse_width,
                               int32_t coarse_height, int32_t width, int32_t height, int32_t ndisp, int32_t w,
                               float conf_threshold, int32_t fallback_margin, int32_t nimg, int32_t *lo,
                               uint8_t *fallback_mask, int32_t *row_stats, uint32_t *nfallback, void *stream)
{
    if (!coarse_disp || !cnn_out || !lo) return cfail(SGM_ERR_INVALID, "NULL buffer");
    if (coarse_width < 1 || coarse_height < 1 || width < 1 || height < 1 || w < 1 || w > ndisp || ndisp > 256)
        return cfail(SGM_ERR_INVALID, "bad size");
    if (nimg < 1 || nimg > 65535) return cfail(SGM_ERR_INVALID, "nimg must be in [1, 65535]");
    if (height > 65535 || (long long)width * height * nimg >= (1ll << 31) ||
        (long long)coarse_width * coarse_height * CH * nimg >= (1ll << 31))
        return cfail(SGM_ERR_UNSUPPORTED, "image too large");
    if (conf_threshold != conf_threshold) return cfail(SGM_ERR_INVALID, "threshold is NaN");
    // confident iff sigmoid(logit) > tau  <=>  logit > log(tau / (1 - tau))
    float thr;
    if (conf_threshold <= 0.0f)
        thr = -INFINITY;
    else if (conf_threshold >= 1.0f)
        thr = INFINITY;
    else
        thr = (float)log((double)conf_threshold / (1.0 - (double)conf_threshold));
    hipStream_t s = (hipStream_t)stream;
    if (fault_take(kFaultLaunch)) return cfail(SGM_ERR_HIP, "injected launch failure");
    if (row_stats || nfallback)
        hipLaunchKernelGGL(k_clear_stats, dim3((height + 255) / 256, 1, nimg), dim3(256), 0, s, row_stats,
                           (int)height, (int)width, nfallback);
    dim3 grid((width + 256 * kMapPix - 1) / (256 * kMapPix), height, nimg), block(256);
    hipLaunchKernelGGL(k_window_map, grid, block, 0, s, coarse_disp, cnn_out, coarse_width, coarse_height, width,
                       height, ndisp, w, thr, (float)fallback_margin, lo, fallback_mask, row_stats, nfallback);
    return launched("window map");
}

sgm_status sgm_window_map(const float *coarse_disp, const float *cnn_out, int32_t coarse_width, int32_t coarse_height,
                          int32_t width, int32_t height, int32_t ndisp, int32_t w, float conf_threshold,
                          int32_t fallback_margin, int32_t *lo, uint8_t *fallback_mask, int32_t *row_stats,
                          uint32_t *nfallback, void *stream)
{
    return window_map_n(coarse_disp, cnn_out, coarse_width, coarse_height, width, height, ndisp, w, conf_threshold,
                        fallback_margin, 1, lo, fallback_mask, row_stats, nfallback, stream);
}

sgm_status sgm_window_map_batch(const float *coarse_disp, const float *cnn_out, int32_t coarse_width,
                                int32_t coarse_height, int32_t width, int32_t height, int32_t ndisp, int32_t w,
                                float conf_threshold, int32_t fallback_margin, int32_t nimg, int32_t *lo,
                                uint8_t *fallback_mask, int32_t *row_stats, uint32_t *nfallback, void *stream)
{
    return window_map_n(coarse_disp, cnn_out, coarse_width, coarse_height, width, height, ndisp, w, conf_threshold,
                        fallback_margin, nimg, lo, fallback_mask, row_stats, nfallback, stream);
}

sgm_status sgm_fallback_merge(const uint8_t *fallback_mask, const int16_t *band_int, const float *band_sub,
                              int32_t width, int32_t height, int32_t y0, int32_t rows, int32_t x0, int32_t cols,
                              int16_t *disp_int, float *disp_sub, void *stream)
{
    if (!fallback_mask || !band_int || !disp_int) return cfail(SGM_ERR_INVALID, "NULL buffer");
    if (width < 1 || height < 1 || y0 < 0 || rows < 0 || y0 + rows > height || x0 < 0 || cols < 0 ||
        x0 + cols > width)
        return cfail(SGM_ERR_INVALID, "rectangle outside the frame");
    if (rows == 0 || cols == 0) return SGM_OK;
    if (rows > 65535) return cfail(SGM_ERR_UNSUPPORTED, "more than 65535 rows");
    dim3 grid((cols + 255) / 256, rows), block(256);
    if (fault_take(kFaultLaunch)) return cfail(SGM_ERR_HIP, "injected launch failure");
    hipLaunchKernelGGL(k_merge_fallback, grid, block, 0, (hipStream_t)stream, fallback_mask, band_int, band_sub,
                       width, y0, rows, x0, cols, disp_int, disp_sub);
    return launched("fallback merge");
}

sgm_status sgm_fallback_merge_rects(const uint8_t *fallback_mask, const int32_t *rects, int32_t nrects,
                                    int32_t max_rows, int32_t max_cols, int32_t width, int32_t height,
                                    int32_t nframes, const int16_t *band_int, const float *band_sub,
                                    int64_t band_len, int16_t *disp_int, float *disp_sub, void *stream)
{
    if (!fallback_mask || !rects || !band_int || !disp_int) return cfail(SGM_ERR_INVALID, "NULL buffer");
    if (width < 1 || height < 1 || nframes < 1 || nrects < 0 || max_rows < 0 || max_cols < 0 || band_len < 0)
        return cfail(SGM_ERR_INVALID, "sizes must be >= 0 (frames >= 1)");
    if (nrects == 0 || max_rows == 0 || max_cols == 0) return SGM_OK;
    if (nrects > 65535 || max_rows > 65535) return cfail(SGM_ERR_UNSUPPORTED, "more than 65535 rectangles or rows");
    if ((long long)width * height * nframes >= (1ll << 40)) return cfail(SGM_ERR_UNSUPPORTED, "frames too large");
    dim3 grid((max_cols + 255) / 256, max_rows, nrects), block(256);
    if (fault_take(kFaultLaunch)) return cfail(SGM_ERR_HIP, "injected launch failure");
    hipLaunchKernelGGL(k_merge_fallback_rects, grid, block, 0, (hipStream_t)stream, fallback_mask, rects, width,
                       height, nframes, band_int, band_sub, (long long)band_len, disp_int, disp_sub);
    return launched("fallback merge of rectangles");
}

sgm_status sgm_label_downsample4(const float *label, int32_t width, int32_t height, float *coarse, void *stream)
{
    if (!label || !coarse) return cfail(SGM_ERR_INVALID, "NULL buffer");
    if (width < 4 || height < 4) return cfail(SGM_ERR_INVALID, "need width, height >= 4");
    if (height / 4 > 65535 || (long long)width * height >= (1ll << 31))
        return cfail(SGM_ERR_UNSUPPORTED, "image too large");
    dim3 grid((width / 4 + 255) / 256, height / 4), block(256);
    if (fault_take(kFaultLaunch)) return cfail(SGM_ERR_HIP, "injected launch failure");
    hipLaunchKernelGGL(k_label_downsample4, grid, block, 0, (hipStream_t)stream, label, width, height, coarse);
    return launched("label downsample");
}

}  // extern "C"
