// Kernels of the learned warm start X0 = f(C) (not in the paper: an
// extension of its initial guess X^0): a 3 x 3 convolution with zero
// padding 1 (cross-correlation convention)
//   y[n,o,h,w] = b[o] + sum_{c,i,j} W[o,c,i,j] x[n,c,h+i-1,w+j-1],
// its input gradient dx[n,c,h,w] = sum_{o,i,j} W[o,c,i,j] g[n,o,h-i+1,w-j+1]
// (the same kernel reading W transposed and flipped), its weight and bias
// gradients dW[o,c,i,j] = sum_{n,h,w} g[n,o,h,w] x[n,c,h+i-1,w+j-1],
// db[o] = sum g, the mean-squared-error loss and its gradient, and Adam.
//
// Storage: activations and their gradients in BF16 (round to nearest even),
// weights as FP32 holding BF16-rounded values (the optimiser keeps FP32
// master copies), every sum in FP32 (the loss in FP64). Layout: tensors with
// 3 channels (the image-shaped input, output and loss gradient) NCHW;
// tensors with 32 channels (hidden activations and their gradients) NHWC,
// so that the 32 channels of a pixel are 64 contiguous bytes (four 16-byte
// chunks of 8 channels, one MFMA k chunk each).
#include "internal.h"

#include <math.h>

namespace mek {

namespace {

constexpr int kCT = 16;                  // output tile edge (pixels)
constexpr int kHalo = kCT + 2;           // input tile edge with the halo
constexpr int kHaloPix = kHalo * kHalo;  // 324
constexpr int kChanStride = kHaloPix + 1;   // odd: 32 channels hit 32 LDS banks
constexpr int kCThreads = kCT * kCT;     // one thread per output pixel
constexpr int kMaxC = 32;                // channels of the network
constexpr int kGsStride = kCThreads + 1;  // odd: a wave's 32 channels of one pixel on 32 banks

__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float float4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint32_t pack2(uint16_t lo, uint16_t hi) {
    return (uint32_t)lo | ((uint32_t)hi << 16);
}

// Element (n, c, h, w) of a tensor with C channels: NHWC for 32 channels,
// NCHW otherwise.
__device__ __forceinline__ size_t tidx(int n, int c, int h, int w, int C, int H, int W) {
    return C == 32 ? (((size_t)n * H + h) * W + w) * 32 + c
                   : (((size_t)n * C + c) * H + h) * W + w;
}

// FP32 -> BF16, round to nearest, ties to even (NaN stays a quiet NaN).
__device__ __forceinline__ uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x7fffffu)) return 0x7fc0;
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// Stage channels [0, C) of the (kHalo x kHalo) input tile at (h0-1, w0-1)
// of image n into LDS as FP32, zero outside the image; with a mask, entries
// whose mask value is not > 0 read as zero (a ReLU's gradient gate). A
// thread issues kStageU loads before it stores any of them, each from an
// address clamped into the tensor (no branch around a load), so that their
// latencies overlap; entries outside the image or past the end are then
// replaced by zero.
constexpr int kStageU = 4;
__device__ __forceinline__ void stage_halo(float* xs, const uint16_t* __restrict__ x,
                                           const uint16_t* __restrict__ mask, int n, int C,
                                           int H, int W, int h0, int w0) {
    const int tot = C * kHaloPix;
    // Without a mask the gate loads re-read x (cache hits), so that no
    // branch sits between the loads.
    const uint16_t* __restrict__ mp = mask ? mask : x;
    for (int e0 = threadIdx.x; e0 < tot; e0 += kStageU * kCThreads) {
        uint16_t xv[kStageU], mv[kStageU];
        bool in[kStageU];
#pragma unroll
        for (int u = 0; u < kStageU; ++u) {
            const int e = min(e0 + u * kCThreads, tot - 1);
            const int c = e / kHaloPix, r = e - c * kHaloPix;
            const int hh = h0 - 1 + r / kHalo, ww = w0 - 1 + r % kHalo;
            in[u] = e0 + u * kCThreads < tot && hh >= 0 && hh < H && ww >= 0 && ww < W;
            const size_t idx = tidx(n, c, min(max(hh, 0), H - 1), min(max(ww, 0), W - 1), C, H, W);
            xv[u] = x[idx];
            mv[u] = mp[idx];
        }
#pragma unroll
        for (int u = 0; u < kStageU; ++u) {
            const int e = e0 + u * kCThreads;
            if (e < tot) {
                const int c = e / kHaloPix, r = e - c * kHaloPix;
                xs[c * kChanStride + r] =
                    (in[u] && (!mask || bf2f(mv[u]) > 0.0f)) ? bf2f(xv[u]) : 0.0f;
            }
        }
    }
}

// Forward (TRANS = false): CO output channels from kFewIn = 3 input
// channels with weights w (CO, 3, 3, 3). Input gradient (TRANS = true): the
// layer's weights W (3, CO, 3, 3) read as W[ci][co][2-i][2-j], no bias, no
// ReLU. Writes BF16 (yb) or FP64 (yd) outputs; an FP64 output may add a
// tensor of its shape. One thread per output pixel keeps its 27 inputs in
// registers; the weights are the same in every lane, so they are read from
// device memory with uniform addresses (the scalar unit, scalar registers
// as the multiply-add operands) rather than through LDS.
constexpr int kFewIn = 3;
template <int CO, bool TRANS>
__global__ void __launch_bounds__(kCThreads)
conv3x3_kernel(const uint16_t* __restrict__ x, const uint16_t* __restrict__ mask, int H, int W,
               const float* __restrict__ w, const float* __restrict__ bias, int relu,
               uint16_t* __restrict__ yb, double* __restrict__ yd, const double* __restrict__ add) {
    constexpr int KT = kFewIn * 9;
    __shared__ float xs[kFewIn * kChanStride];
    const int tiles_w = (W + kCT - 1) / kCT;
    const int th = blockIdx.x / tiles_w, tw = blockIdx.x - th * tiles_w;
    const int n = blockIdx.y;
    const int h0 = th * kCT, w0 = tw * kCT;
    stage_halo(xs, x, mask, n, kFewIn, H, W, h0, w0);
    __syncthreads();
    const int ty = threadIdx.x / kCT, tx = threadIdx.x % kCT;
    float xv[KT];
#pragma unroll
    for (int c = 0; c < kFewIn; ++c)
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) xv[(c * 3 + i) * 3 + j] = xs[c * kChanStride + (ty + i) * kHalo + tx + j];
    float acc[CO];
#pragma unroll
    for (int o = 0; o < CO; ++o) {
        float a = 0.0f;
#pragma unroll
        for (int c = 0; c < kFewIn; ++c)
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    const float wv = TRANS ? w[((c * CO + o) * 3 + (2 - i)) * 3 + (2 - j)]
                                           : w[((o * kFewIn + c) * 3 + i) * 3 + j];
                    a = fmaf(xv[(c * 3 + i) * 3 + j], wv, a);
                }
        acc[o] = a;
    }
    const int h = h0 + ty, wq = w0 + tx;
    if (h >= H || wq >= W) return;
    if (CO == 32 && yb) {
        // NHWC: the pixel's 32 outputs as four 16-byte stores.
        uint32_t pk[16];
#pragma unroll
        for (int o = 0; o < 32; o += 2) {
            float v0 = acc[o] + (bias ? bias[o] : 0.0f);
            float v1 = acc[o + 1] + (bias ? bias[o + 1] : 0.0f);
            if (relu) {
                v0 = fmaxf(v0, 0.0f);
                v1 = fmaxf(v1, 0.0f);
            }
            pk[o / 2] = pack2(f2bf(v0), f2bf(v1));
        }
        uint4* dst = reinterpret_cast<uint4*>(yb + (((size_t)n * H + h) * W + wq) * 32);
#pragma unroll
        for (int c4 = 0; c4 < 4; ++c4)
            dst[c4] = make_uint4(pk[4 * c4], pk[4 * c4 + 1], pk[4 * c4 + 2], pk[4 * c4 + 3]);
        return;
    }
#pragma unroll
    for (int o = 0; o < CO; ++o) {
        float v = acc[o] + (bias ? bias[o] : 0.0f);
        if (relu) v = fmaxf(v, 0.0f);
        const size_t idx = tidx(n, o, h, wq, CO, H, W);
        if (yb) yb[idx] = f2bf(v);
        else yd[idx] = (add ? add[idx] : 0.0) + (double)v;
    }
}

// Weight and bias gradient partial sums of one tile: thread (group, c)
// accumulates dW[o][c][i][j] for its CO/8 output channels o and the 9 taps
// over the tile's pixels in ascending order, and (c == 0) db[o].
template <int CO>
__global__ void __launch_bounds__(kCThreads)
conv3x3_wgrad_kernel(const uint16_t* __restrict__ x, int Cin, int H, int W,
                     const uint16_t* __restrict__ g, const uint16_t* __restrict__ gmask,
                     float* __restrict__ partial) {
    constexpr int OPER = (CO + 7) / 8;
    __shared__ float xs[kMaxC * kChanStride];
    __shared__ float gs[CO * kGsStride];
    const int tiles_w = (W + kCT - 1) / kCT;
    const int th = blockIdx.x / tiles_w, tw = blockIdx.x - th * tiles_w;
    const int n = blockIdx.y;
    const int h0 = th * kCT, w0 = tw * kCT;
    stage_halo(xs, x, nullptr, n, Cin, H, W, h0, w0);
    for (int e = threadIdx.x; e < CO * kCThreads; e += kCThreads) {
        // Channel fastest across lanes for NHWC gradients (coalesced reads),
        // pixel fastest for NCHW.
        const int o = CO == 32 ? e % CO : e / kCThreads;
        const int p = CO == 32 ? e / CO : e - o * kCThreads;
        const int hh = h0 + p / kCT, ww = w0 + p % kCT;
        float v = 0.0f;
        if (hh < H && ww < W) {
            const size_t idx = tidx(n, o, hh, ww, CO, H, W);
            v = bf2f(g[idx]);
            if (gmask && !(bf2f(gmask[idx]) > 0.0f)) v = 0.0f;
        }
        gs[o * kGsStride + p] = v;
    }
    __syncthreads();
    const int c = threadIdx.x % kMaxC, grp = threadIdx.x / kMaxC;
    const int o0 = grp * OPER;
    float acc[OPER][9], bacc[OPER];
#pragma unroll
    for (int k = 0; k < OPER; ++k) {
        bacc[k] = 0.0f;
#pragma unroll
        for (int t = 0; t < 9; ++t) acc[k][t] = 0.0f;
    }
    if (c < Cin) {
        const float* xc = xs + c * kChanStride;
        for (int p = 0; p < kCThreads; ++p) {
            const int py = p / kCT, px = p % kCT;
            float xv[9];
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) xv[i * 3 + j] = xc[(py + i) * kHalo + px + j];
#pragma unroll
            for (int k = 0; k < OPER; ++k) {
                const int o = o0 + k;
                const float gv = o < CO ? gs[o * kGsStride + p] : 0.0f;
                bacc[k] += gv;
#pragma unroll
                for (int t = 0; t < 9; ++t) acc[k][t] = fmaf(gv, xv[t], acc[k][t]);
            }
        }
    }
    const size_t E = (size_t)CO * Cin * 9 + CO;
    float* out = partial + ((size_t)n * gridDim.x + blockIdx.x) * E;
    if (c < Cin) {
#pragma unroll
        for (int k = 0; k < OPER; ++k) {
            const int o = o0 + k;
            if (o >= CO) continue;
#pragma unroll
            for (int t = 0; t < 9; ++t) out[((size_t)o * Cin + c) * 9 + t] = acc[k][t];
            if (c == 0) out[(size_t)CO * Cin * 9 + o] = bacc[k];
        }
    }
}

// Weight and bias gradient partial sums of one 16 x 16 tile for few input
// channels (Cin <= kFewC, the network's first layer) and 32 output
// channels: thread (o, part) takes output channel o and 32 of the tile's
// 256 pixels, every input channel and tap; the 8 parts are then added in
// part order through LDS. (One thread per (input channel, output group)
// would leave most of the block idle with 3 input channels.)
constexpr int kFewC = 4;
__global__ void __launch_bounds__(kCThreads)
conv3x3_wgrad_fewc_kernel(const uint16_t* __restrict__ x, int Cin, int H, int W,
                          const uint16_t* __restrict__ g, const uint16_t* __restrict__ gmask,
                          float* __restrict__ partial) {
    constexpr int CO = 32, NA = kFewC * 9 + 1, PARTS = kCThreads / CO;
    // The parts' sums reuse the tiles' LDS once every thread is done with
    // them (38 KB per block: four blocks fit a compute unit).
    constexpr int kTileF = kFewC * kChanStride + CO * kGsStride, kRedF = PARTS * CO * NA;
    __shared__ float smem[kTileF > kRedF ? kTileF : kRedF];
    float* const xs = smem;
    float* const gs = smem + kFewC * kChanStride;
    float* const red = smem;
    const int tiles_w = (W + kCT - 1) / kCT;
    const int th = blockIdx.x / tiles_w, tw = blockIdx.x - th * tiles_w;
    const int n = blockIdx.y;
    const int h0 = th * kCT, w0 = tw * kCT;
    stage_halo(xs, x, nullptr, n, Cin, H, W, h0, w0);
    // Gradient (channels-last): task e = (pixel, 8-channel chunk), one
    // 16-byte load (and one of the gate), 8 values to the channels' rows.
    // The four tasks of a thread load first (clamped addresses, no branch
    // between the loads; without a gate it re-reads g), then store.
    const uint16_t* __restrict__ gm = gmask ? gmask : g;
    uint4 gv4[4], gm4[4];
    bool gin[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int e = threadIdx.x + u * kCThreads;
        const int p = e >> 2, q = e & 3;
        const int hh = h0 + p / kCT, ww = w0 + p % kCT;
        gin[u] = hh < H && ww < W;
        const size_t off = (((size_t)n * H + min(hh, H - 1)) * W + min(ww, W - 1)) * CO + 8 * q;
        gv4[u] = *reinterpret_cast<const uint4*>(g + off);
        gm4[u] = *reinterpret_cast<const uint4*>(gm + off);
    }
#pragma unroll
    for (int u0 = 0; u0 < 4; ++u0) {
        const int e = threadIdx.x + u0 * kCThreads;
        const int p = e >> 2, q = e & 3;
        const uint4 v = gin[u0] ? gv4[u0] : make_uint4(0u, 0u, 0u, 0u);
        const uint4 mk = gm4[u0];
        const uint32_t vv[4] = {v.x, v.y, v.z, v.w}, mm[4] = {mk.x, mk.y, mk.z, mk.w};
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const uint32_t b = (u & 1) ? (vv[u >> 1] >> 16) : (vv[u >> 1] & 0xffff);
            float f = bf2f(b);
            if (gmask) {
                const uint32_t mb = (u & 1) ? (mm[u >> 1] >> 16) : (mm[u >> 1] & 0xffff);
                if (!(bf2f(mb) > 0.0f)) f = 0.0f;
            }
            gs[(8 * q + u) * kGsStride + p] = f;
        }
    }
    __syncthreads();
    const int o = threadIdx.x % CO, part = threadIdx.x / CO;
    float acc[kFewC][9], bacc = 0.0f;
#pragma unroll
    for (int c = 0; c < kFewC; ++c)
#pragma unroll
        for (int t = 0; t < 9; ++t) acc[c][t] = 0.0f;
    for (int pp = 0; pp < kCThreads / PARTS; ++pp) {
        const int p = part * (kCThreads / PARTS) + pp;
        const int py = p / kCT, px = p % kCT;
        const float gv = gs[o * kGsStride + p];
        bacc += gv;
#pragma unroll
        for (int c = 0; c < kFewC; ++c) {
            if (c < Cin) {
                const float* xc = xs + c * kChanStride + py * kHalo + px;
#pragma unroll
                for (int i = 0; i < 3; ++i)
#pragma unroll
                    for (int j = 0; j < 3; ++j) acc[c][i * 3 + j] = fmaf(gv, xc[i * kHalo + j], acc[c][i * 3 + j]);
            }
        }
    }
    __syncthreads();   // the tiles are read; their space takes the parts' sums
    float* rp = red + (part * CO + o) * NA;
#pragma unroll
    for (int c = 0; c < kFewC; ++c)
#pragma unroll
        for (int t = 0; t < 9; ++t) rp[c * 9 + t] = acc[c][t];
    rp[kFewC * 9] = bacc;
    __syncthreads();
    const size_t E = (size_t)CO * Cin * 9 + CO;
    float* out = partial + ((size_t)n * gridDim.x + blockIdx.x) * E;
    const int per_o = Cin * 9 + 1;
    for (int e = threadIdx.x; e < CO * per_o; e += kCThreads) {
        const int oo = e / per_o, r = e - oo * per_o;
        const int slot = r < Cin * 9 ? r : kFewC * 9;
        float sacc = 0.0f;
        for (int q = 0; q < PARTS; ++q) sacc += red[(q * CO + oo) * NA + slot];
        if (r < Cin * 9) out[((size_t)oo * Cin + r / 9) * 9 + r % 9] = sacc;
        else out[(size_t)CO * Cin * 9 + oo] = sacc;
    }
}

// Weight and bias gradient partial sums of one 16 x 16 pixel tile on the
// BF16 matrix cores, for 32 input channels: per tap t, D_t[o][c] =
// sum over the tile's pixels of g'[o][p] x[c][p + shift_t], the 256 pixels
// as 8 k steps of 32 (two 16-pixel rows each). The gradient tile sits in LDS
// as [o][pixel] (a k chunk is 8 consecutive pixels of a row); the input as
// three column-shifted copies x_j[c][halo row][16 columns] = x[c][h0 - 1 +
// row][w0 + col + j - 1], so that the chunk of tap (i, j) is one aligned
// 16-byte read. The 9 taps x output-channel tiles x input-channel tiles of
// the block's result are shared out over its 4 waves; the bias gradient is
// a plain sum. Partials are written in the layout of the VALU kernel, so the
// same fixed-order summation follows.
constexpr int kGStride = 33;   // 16-byte slots per output channel of the gradient tile (odd)
constexpr int kXStride = 37;   // slots per input channel of a shifted copy (18 rows x 2, + 1)
constexpr int kWgTiles = 2;    // pixel tiles per block of the matrix-core weight gradient

template <int CO>
__global__ void __launch_bounds__(256)
conv3x3_wgrad_mfma_kernel(const uint16_t* __restrict__ x, int H, int W,
                          const uint16_t* __restrict__ g, const uint16_t* __restrict__ gmask,
                          float* __restrict__ partial) {
    constexpr int CI = 32;
    constexpr int COP = (CO + 15) & ~15;
    constexpr int OT = COP / 16, CT = CI / 16;
    constexpr int TILES = 9 * OT * CT;            // 16 x 16 result tiles of the block
    constexpr int PER = (TILES + 3) / 4;          // per wave
    __shared__ uint4 gs[COP * kGStride];
    __shared__ uint16_t xsh[3 * CI * kXStride * 8];
    __shared__ float bsum[4][COP];
    const int tiles_w = (W + kCT - 1) / kCT, tiles = tiles_w * ((H + kCT - 1) / kCT);
    const int n = blockIdx.y;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int l16 = lane & 15, lq = lane >> 4;
    const uint4* xs4 = reinterpret_cast<const uint4*>(xsh);
    float4_t acc[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) acc[u] = (float4_t){0.f, 0.f, 0.f, 0.f};
    float bacc = 0.0f;
    // kWgTiles consecutive pixel tiles per block, accumulated in order.
    const int t_end = min(tiles, (int)(blockIdx.x + 1) * kWgTiles);
    for (int pt = blockIdx.x * kWgTiles; pt < t_end; ++pt) {
        const int th = pt / tiles_w, tw = pt - th * tiles_w;
        const int h0 = th * kCT, w0 = tw * kCT;
        // Gradient tile (gated), zero outside the image and in padded channels;
        // the bias gradient from the same values. 32 channels (channels-last):
        // task e = (pixel, 8-channel chunk), one 16-byte load (and one of the
        // mask), its 8 values stored to the 8 channels' pixel rows.
        if (CO == 32) {
            uint16_t* gs16 = reinterpret_cast<uint16_t*>(gs);
            for (int e = tid; e < 4 * kCT * kCT; e += 256) {
                const int px = e >> 2, q = e & 3;
                const int hh = h0 + (px >> 4), ww = w0 + (px & 15);
                uint4 v = make_uint4(0u, 0u, 0u, 0u);
                if (hh < H && ww < W) {
                    const size_t off = (((size_t)n * H + hh) * W + ww) * 32 + 8 * q;
                    v = *reinterpret_cast<const uint4*>(g + off);
                    if (gmask) {
                        const uint4 mk = *reinterpret_cast<const uint4*>(gmask + off);
                        const uint32_t mm[4] = {mk.x, mk.y, mk.z, mk.w};
                        uint32_t vv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            const uint32_t lo = (bf2f(mm[u] & 0xffff) > 0.0f) ? 0x0000ffffu : 0u;
                            const uint32_t hi = (bf2f(mm[u] >> 16) > 0.0f) ? 0xffff0000u : 0u;
                            vv[u] &= (lo | hi);
                        }
                        v = make_uint4(vv[0], vv[1], vv[2], vv[3]);
                    }
                }
                const uint32_t vv[4] = {v.x, v.y, v.z, v.w};
                const int chk = 2 * (px >> 4) + ((px & 15) >> 3), pos = px & 7;
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    gs16[((8 * q + u) * kGStride + chk) * 8 + pos] =
                        (uint16_t)((u & 1) ? (vv[u >> 1] >> 16) : (vv[u >> 1] & 0xffff));
            }
        } else
        for (int e = tid; e < COP * 32; e += 256) {
            const int o = e >> 5, chk = e & 31;          // 32 chunks of 8 pixels
            const int hh = h0 + (chk >> 1), ww0 = w0 + 8 * (chk & 1);
            uint16_t v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            if (o < CO && hh < H) {
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int ww = ww0 + u;
                    if (ww < W) {
                        const size_t idx = tidx(n, o, hh, ww, CO, H, W);
                        uint16_t b = g[idx];
                        if (gmask && !(bf2f(gmask[idx]) > 0.0f)) b = 0;
                        v[u] = b;
                    }
                }
            }
            gs[o * kGStride + chk] = make_uint4(pack2(v[0], v[1]), pack2(v[2], v[3]), pack2(v[4], v[5]),
                                                pack2(v[6], v[7]));
        }
        // Input (NHWC): task e = (halo pixel, 8-channel chunk), one 16-byte load;
        // each of its 8 values goes to the shifted copies that hold it.
        for (int e = tid; e < 4 * kHaloPix; e += 256) {
            const int r = e >> 2, ch = e & 3;
            const int hr = r / kHalo, hc = r % kHalo;
            const int hh = h0 - 1 + hr, ww = w0 - 1 + hc;
            uint4 v = make_uint4(0u, 0u, 0u, 0u);
            if (hh >= 0 && hh < H && ww >= 0 && ww < W)
                v = *reinterpret_cast<const uint4*>(x + (((size_t)n * H + hh) * W + ww) * CI + 8 * ch);
            const uint32_t vv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const int col = hc - j;
                if (col >= 0 && col < 16) {
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const int c = 8 * ch + u;
                        xsh[((j * CI + c) * kXStride + 2 * hr + (col >> 3)) * 8 + (col & 7)] =
                            (uint16_t)((u & 1) ? (vv[u >> 1] >> 16) : (vv[u >> 1] & 0xffff));
                    }
                }
            }
        }
        __syncthreads();
        // Bias gradient: thread (o, part) sums a quarter of the tile's pixels.
        if (tid < 4 * COP) {
            const int o = tid % COP, part = tid / COP;
            float sacc = 0.0f;
            for (int chk = 8 * part; chk < 8 * part + 8; ++chk) {
                const uint4 w4 = gs[o * kGStride + chk];
                const uint32_t ww[4] = {w4.x, w4.y, w4.z, w4.w};
#pragma unroll
                for (int u = 0; u < 4; ++u) sacc += bf2f(ww[u] & 0xffff) + bf2f(ww[u] >> 16);
            }
            bacc += sacc;
        }

#pragma unroll
        for (int ks = 0; ks < 8; ++ks) {
            // k chunk of this lane: pixel row 2 ks + lq / 2, columns 8 (lq & 1) ..
            const int prow = 2 * ks + (lq >> 1), half = lq & 1;
#pragma unroll
            for (int u = 0; u < PER; ++u) {
                const int tile = wave * PER + u;
                if (tile >= TILES) break;
                const int t = tile / (OT * CT), rem = tile % (OT * CT);
                const int ot = rem / CT, ct = rem % CT;
                const int i = t / 3, j = t % 3;
                const bf16x8_t fa =
                    __builtin_bit_cast(bf16x8_t, gs[(16 * ot + l16) * kGStride + 2 * prow + half]);
                const bf16x8_t fb = __builtin_bit_cast(
                    bf16x8_t, xs4[(j * CI + 16 * ct + l16) * kXStride + 2 * (prow + i) + half]);
                acc[u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa, fb, acc[u], 0, 0, 0);
            }
        }
        __syncthreads();   // the tile's LDS is read; the next tile may overwrite it
    }
    if (tid < 4 * COP) bsum[tid / COP][tid % COP] = bacc;
    __syncthreads();
    const size_t E = (size_t)CO * CI * 9 + CO;
    float* out = partial + ((size_t)n * gridDim.x + blockIdx.x) * E;
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int tile = wave * PER + u;
        if (tile >= TILES) break;
        const int t = tile / (OT * CT), rem = tile % (OT * CT);
        const int ot = rem / CT, ct = rem % CT;
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
            const int o = 16 * ot + 4 * lq + jj, c = 16 * ct + l16;
            if (o < CO) out[((size_t)o * CI + c) * 9 + t] = acc[u][jj];
        }
    }
    if (tid < CO) out[(size_t)CO * CI * 9 + tid] = bsum[0][tid] + bsum[1][tid] + bsum[2][tid] + bsum[3][tid];
}

// Two-level fixed-order sum of the T tile partials of each entry e: block
// (x, k) sums tiles [k T / S, (k + 1) T / S) in tile order into mid[k][e],
// then mid is summed over k in order.
__global__ void sum_partials_kernel(const float* __restrict__ partial, long long T, long long E,
                                    int S, float* __restrict__ mid) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= E) return;
    const long long k = blockIdx.y;
    const long long t0 = k * T / S, t1 = (k + 1) * T / S;
    float s = 0.0f;
#pragma unroll 8
    for (long long t = t0; t < t1; ++t) s += partial[t * E + e];
    mid[k * E + e] = s;
}

__global__ void sum_mid_kernel(const float* __restrict__ mid, int S, long long E,
                               float* __restrict__ dw, float* __restrict__ db, long long nw) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= E) return;
    float s = 0.0f;
#pragma unroll 8
    for (int k = 0; k < S; ++k) s += mid[(long long)k * E + e];
    if (e < nw) dw[e] = s;
    else db[e - nw] = s;
}

// g = BF16(scale (y - label)); per-block sums of (y - label)^2 in FP64.
__global__ void mse_grad_kernel(long long len, const double* __restrict__ y,
                                const double* __restrict__ label, double scale,
                                uint16_t* __restrict__ g, double* __restrict__ part) {
    __shared__ double red[256];
    double s = 0.0;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < len;
         e += (long long)gridDim.x * blockDim.x) {
        const double d = y[e] - label[e];
        s += d * d;
        if (g) g[e] = f2bf((float)(scale * d));
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = blockDim.x / 2; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void adam_kernel(long long n, float* __restrict__ w, float* __restrict__ wq,
                            const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, float lr, float b1, float b2, float eps,
                            float c1, float c2) {
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const float gk = g[k];
    const float mk = b1 * m[k] + (1.0f - b1) * gk;
    const float vk = b2 * v[k] + (1.0f - b2) * gk * gk;
    m[k] = mk;
    v[k] = vk;
    const float wk = w[k] - lr * (mk / c1) / (sqrtf(vk / c2) + eps);
    w[k] = wk;
    wq[k] = bf2f(f2bf(wk));
}

__global__ void to_bf16_kernel(long long n, const double* __restrict__ x, double scale,
                               uint16_t* __restrict__ y) {
    for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < n;
         k += (long long)gridDim.x * blockDim.x)
        y[k] = f2bf((float)(scale * x[k]));
}

__global__ void round_bf16_kernel(long long n, const float* __restrict__ x, float* __restrict__ y) {
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) y[k] = bf2f(f2bf(x[k]));
}

// ---------------------------------------------------------------------------
// The same convolution on the BF16 matrix cores (v_mfma_f32_16x16x32_bf16,
// FP32 accumulation) for 32 input channels: per 3 x 3 tap, a product of the
// tap's weights (output channels x 32 input channels) with the input tile
// (32 input channels x 16 pixels of a row), summed over the 9 taps. The 32
// input channels of a tap are one k step of the instruction, so an output
// value is the FP32 sum of 9 k steps of 32 exact bf16 x bf16 products.
//
// Operand layout (checked on gfx950): lane l supplies row l % 16 of the
// first operand and column l % 16 of the second, each as the 8 consecutive
// k values 8 (l / 16) .. 8 (l / 16) + 7; accumulator value j of lane l is
// D[4 (l / 16) + j][l % 16]. Here rows are output channels, columns pixels.
//
// LDS: the (kMT + 2) x 18 input tile, pixel-major with the 32 channels of a
// pixel in four 16-byte chunks and a pixel stride of five chunks (so any 8
// or 16 consecutive pixels of one chunk fall on distinct 16-byte bank
// groups); the weights as [tap][output channel][32 channels], the same
// padded stride.
constexpr int kMT = 16;                      // output rows per block (4 per wave)
constexpr int kMW = 16;                      // output columns per block
constexpr int kMHr = kMT + 2, kMHc = kMW + 2;
constexpr int kMPix = kMHr * kMHc;           // 324 halo pixels
constexpr int kSlot = 5;                     // 16-byte slots per pixel / per weight row

// The weights of a matrix-core convolution in MFMA order, BF16:
// wb[(t * COP + o) * 32 + c] = W[o][c][i][j] (forward) or W[c][o][2-i][2-j]
// (input gradient), t = 3 i + j, zero for padded output channels o >= CO.
template <int CO, bool TRANS>
__global__ void prep_weights_kernel(const float* __restrict__ w, uint16_t* __restrict__ wb) {
    constexpr int CI = 32;
    constexpr int COP = (CO + 15) & ~15;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= 9 * COP * CI) return;
    const int c = e % CI, o = (e / CI) % COP, t = e / (CI * COP);
    const int i = t / 3, j = t % 3;
    float f = 0.0f;
    if (o < CO)
        f = TRANS ? w[((c * CO + o) * 3 + (2 - i)) * 3 + (2 - j)] : w[((o * CI + c) * 3 + i) * 3 + j];
    wb[e] = f2bf(f);
}

// Input x: 32 channels, NHWC. mask (input gradient): the ReLU output of the
// layer whose gradient x is, same layout; entries whose mask is not > 0 read
// as zero. Output: NHWC BF16 for 32 channels, NCHW (BF16 or FP64 + add) for 3.
//
// Persistent over tiles: a block puts the weights in LDS once, then takes
// tiles blockIdx.x, blockIdx.x + gridDim.x, ... (tile = image, row band,
// column band); the next tile's input is fetched into registers while the
// current one's products run.
constexpr int kMPre = (4 * kMPix + 255) / 256;   // 16-byte input chunks per thread and tile

template <int CO, bool TRANS, bool MASK>
__global__ void __launch_bounds__(256)
conv3x3_mfma_kernel(const uint16_t* __restrict__ x, const uint16_t* __restrict__ mask, int N,
                    int H, int W, const uint16_t* __restrict__ wb, const float* __restrict__ bias,
                    int relu, uint16_t* __restrict__ yb, double* __restrict__ yd,
                    const double* __restrict__ add) {
    constexpr int CI = 32;
    constexpr int COP = (CO + 15) & ~15;     // output channels padded to MFMA rows
    constexpr int OT = COP / 16;
    __shared__ uint4 xs[kMPix * kSlot];
    __shared__ uint4 ws[9 * COP * kSlot];
    const int tiles_w = (W + kMW - 1) / kMW, tiles_h = (H + kMT - 1) / kMT;
    const int per_img = tiles_w * tiles_h, total = N * per_img;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

    // Weights, already in MFMA order: one 16-byte load per slot, once.
    for (int e = tid; e < 9 * COP * 4; e += 256)
        ws[(e >> 2) * kSlot + (e & 3)] = *reinterpret_cast<const uint4*>(wb + 8 * e);

    // Input tile: task e = (halo pixel, chunk of 8 channels), one 16-byte
    // load each (four lanes cover a pixel's 64 bytes); the mask, if any,
    // is fetched beside it and applied on the way into LDS.
    uint4 pre[kMPre], mpre[MASK ? kMPre : 1];
    auto fetch = [&](int tile) {
        const int n = tile / per_img, rest = tile - n * per_img;
        const int th = rest / tiles_w, tw = rest - th * tiles_w;
        const int h0 = th * kMT, w0 = tw * kMW;
#pragma unroll
        for (int u = 0; u < kMPre; ++u) {
            const int e = tid + 256 * u;
            const int px = e >> 2, ch = e & 3;
            const int hh = h0 - 1 + px / kMHc, ww = w0 - 1 + px % kMHc;
            pre[u] = make_uint4(0u, 0u, 0u, 0u);
            if (MASK) mpre[MASK ? u : 0] = make_uint4(0u, 0u, 0u, 0u);
            if (e < 4 * kMPix && hh >= 0 && hh < H && ww >= 0 && ww < W) {
                const size_t off = (((size_t)n * H + hh) * W + ww) * CI + 8 * ch;
                pre[u] = *reinterpret_cast<const uint4*>(x + off);
                if (MASK) mpre[MASK ? u : 0] = *reinterpret_cast<const uint4*>(mask + off);
            }
        }
    };
    // This lane's output channels 16 a + 4 lq + jj: their biases, once.
    float bv[OT][4];
#pragma unroll
    for (int a = 0; a < OT; ++a)
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
            const int o = 16 * a + 4 * (lane >> 4) + jj;
            bv[a][jj] = (bias && o < CO) ? bias[o] : 0.0f;
        }
    int tile = blockIdx.x;
    if (tile < total) fetch(tile);
    for (; tile < total; tile += gridDim.x) {
        __syncthreads();   // every wave is done with the previous tile's input
#pragma unroll
        for (int u = 0; u < kMPre; ++u) {
            const int e = tid + 256 * u;
            if (e >= 4 * kMPix) continue;
            uint4 v = pre[u];
            if (MASK) {
                const uint4 mk = mpre[MASK ? u : 0];
                uint32_t vv[4] = {v.x, v.y, v.z, v.w};
                const uint32_t mm[4] = {mk.x, mk.y, mk.z, mk.w};
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const uint32_t lo = (bf2f(mm[q] & 0xffff) > 0.0f) ? 0x0000ffffu : 0u;
                    const uint32_t hi = (bf2f(mm[q] >> 16) > 0.0f) ? 0xffff0000u : 0u;
                    vv[q] &= (lo | hi);
                }
                v = make_uint4(vv[0], vv[1], vv[2], vv[3]);
            }
            xs[(e >> 2) * kSlot + (e & 3)] = v;
        }
        __syncthreads();
        const int n = tile / per_img, rest = tile - n * per_img;
        const int th = rest / tiles_w, tw = rest - th * tiles_w;
        const int h0 = th * kMT, w0 = tw * kMW;
        if (tile + (int)gridDim.x < total) fetch(tile + gridDim.x);

        const int l16 = lane & 15, lq = lane >> 4;
        const int r0 = wave * 4;   // this wave's first output row in the tile
        float4_t acc[4][OT];
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int a = 0; a < OT; ++a) acc[r][a] = (float4_t){0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            const int i = t / 3, j = t % 3;
            bf16x8_t fa[OT];
#pragma unroll
            for (int a = 0; a < OT; ++a)
                fa[a] = __builtin_bit_cast(bf16x8_t, ws[(t * COP + 16 * a + l16) * kSlot + lq]);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const bf16x8_t fb =
                    __builtin_bit_cast(bf16x8_t, xs[((r0 + r + i) * kMHc + l16 + j) * kSlot + lq]);
#pragma unroll
                for (int a = 0; a < OT; ++a)
                    acc[r][a] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[a], fb, acc[r][a], 0, 0, 0);
            }
        }

        // Lane (l16, lq) holds output channels 16 a + 4 lq + jj of pixel l16.
        const int wq = w0 + l16;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int h = h0 + r0 + r;
            if (h >= H || wq >= W) continue;
#pragma unroll
            for (int a = 0; a < OT; ++a) {
                float v[4];
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) {
                    v[jj] = acc[r][a][jj] + bv[a][jj];
                    if (relu) v[jj] = fmaxf(v[jj], 0.0f);
                }
                if (CO == 32) {
                    // Four consecutive channels of one pixel: one 8-byte store.
                    const size_t off = (((size_t)n * H + h) * W + wq) * 32 + 16 * a + 4 * lq;
                    *reinterpret_cast<uint2*>(yb + off) =
                        make_uint2(pack2(f2bf(v[0]), f2bf(v[1])), pack2(f2bf(v[2]), f2bf(v[3])));
                } else {
#pragma unroll
                    for (int jj = 0; jj < 4; ++jj) {
                        const int o = 16 * a + 4 * lq + jj;
                        if (o >= CO) continue;
                        const size_t idx = (((size_t)n * CO + o) * H + h) * W + wq;
                        if (yb) yb[idx] = f2bf(v[jj]);
                        else yd[idx] = (add ? add[idx] : 0.0) + (double)v[jj];
                    }
                }
            }
        }
    }
}

// Work-groups of a persistent matrix-core convolution: at most per_cu per
// compute unit (3 with 32 output channels, 49 KB of LDS each; 4 with 3), as
// few as keep the same number of rounds of tiles, so that every work-group
// takes the same number of tiles.
static int conv_mfma_blocks(int tiles, int per_cu) {
    static int cus = 0;
    if (cus == 0) {
        int dev = 0, c = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && c > 0)
            cus = c;
        else
            cus = 256;
    }
    const int slots = per_cu * cus;
    const int rounds = (tiles + slots - 1) / slots;
    return (tiles + rounds - 1) / rounds;
}

template <bool TRANS>
hipError_t conv_dispatch(int N, int Cin, int H, int W, int Cout, const uint16_t* x,
                         const uint16_t* mask, const float* w, const float* b, int relu,
                         uint16_t* yb, double* yd, const double* add, uint16_t* wb,
                         hipStream_t s) {
    if (Cin == 32) {
        // 32 input channels: the matrix-core form, weights put in MFMA order
        // first.
        const int tiles = ((H + kMT - 1) / kMT) * ((W + kMW - 1) / kMW) * N;
        const dim3 grid(conv_mfma_blocks(tiles, Cout == 32 ? 3 : 4));
        if (Cout == 32) {
            hipLaunchKernelGGL((prep_weights_kernel<32, TRANS>), dim3((9 * 32 * 32 + 255) / 256),
                               dim3(256), 0, s, w, wb);
            if (mask)
                hipLaunchKernelGGL((conv3x3_mfma_kernel<32, TRANS, true>), grid, dim3(256), 0, s, x,
                                   mask, N, H, W, wb, b, relu, yb, yd, add);
            else
                hipLaunchKernelGGL((conv3x3_mfma_kernel<32, TRANS, false>), grid, dim3(256), 0, s, x,
                                   mask, N, H, W, wb, b, relu, yb, yd, add);
        } else if (Cout == 3) {
            hipLaunchKernelGGL((prep_weights_kernel<3, TRANS>), dim3((9 * 16 * 32 + 255) / 256),
                               dim3(256), 0, s, w, wb);
            if (mask)
                hipLaunchKernelGGL((conv3x3_mfma_kernel<3, TRANS, true>), grid, dim3(256), 0, s, x,
                                   mask, N, H, W, wb, b, relu, yb, yd, add);
            else
                hipLaunchKernelGGL((conv3x3_mfma_kernel<3, TRANS, false>), grid, dim3(256), 0, s, x,
                                   mask, N, H, W, wb, b, relu, yb, yd, add);
        } else {
            return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    const int tiles = ((H + kCT - 1) / kCT) * ((W + kCT - 1) / kCT);
    dim3 grid(tiles, N);
    if (Cin != kFewIn) return hipErrorInvalidValue;
    switch (Cout) {
        case 32:
            hipLaunchKernelGGL((conv3x3_kernel<32, TRANS>), grid, dim3(kCThreads), 0, s, x, mask, H, W,
                               w, b, relu, yb, yd, add);
            break;
        case 3:
            hipLaunchKernelGGL((conv3x3_kernel<3, TRANS>), grid, dim3(kCThreads), 0, s, x, mask, H, W,
                               w, b, relu, yb, yd, add);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

bool cnn_channels_ok(int64_t c) { return c == 3 || c == 32; }

constexpr int kSumSplits = 64;   // chunks of the first summation level

size_t cnn_wgrad_partial_floats(int N, int Cin, int H, int W, int Cout) {
    const size_t tiles = (size_t)((H + kCT - 1) / kCT) * ((W + kCT - 1) / kCT);
    return (tiles * N + kSumSplits) * ((size_t)Cout * Cin * 9 + Cout);
}

hipError_t cnn_conv3x3(int N, int Cin, int H, int W, int Cout, const uint16_t* x,
                       const uint16_t* mask, const float* w, const float* b, int relu,
                       uint16_t* yb, double* yd, const double* add, uint16_t* wb, hipStream_t s) {
    return conv_dispatch<false>(N, Cin, H, W, Cout, x, mask, w, b, relu, yb, yd, add, wb, s);
}

hipError_t cnn_conv3x3_grad_input(int N, int Cout, int H, int W, int Cin, const uint16_t* g,
                                  const uint16_t* gmask, const float* w, uint16_t* gx,
                                  uint16_t* wb, hipStream_t s) {
    // A convolution over g (Cout channels) producing Cin channels.
    return conv_dispatch<true>(N, Cout, H, W, Cin, g, gmask, w, nullptr, 0, gx, nullptr, nullptr,
                               wb, s);
}

hipError_t cnn_conv3x3_grad_weight(int N, int Cin, int H, int W, int Cout, const uint16_t* x,
                                   const uint16_t* g, const uint16_t* gmask, float* partial,
                                   float* dw, float* db, hipStream_t s) {
    const int tiles = ((H + kCT - 1) / kCT) * ((W + kCT - 1) / kCT);
    dim3 grid(tiles, N);
    const bool mm = Cin == 32;
    dim3 grid_mm((tiles + kWgTiles - 1) / kWgTiles, N);
    if (mm && Cout == 32)
        hipLaunchKernelGGL(conv3x3_wgrad_mfma_kernel<32>, grid_mm, dim3(256), 0, s, x, H, W, g,
                           gmask, partial);
    else if (mm && Cout == 3)
        hipLaunchKernelGGL(conv3x3_wgrad_mfma_kernel<3>, grid_mm, dim3(256), 0, s, x, H, W, g,
                           gmask, partial);
    else if (Cin <= kFewC && Cout == 32)
        hipLaunchKernelGGL(conv3x3_wgrad_fewc_kernel, grid, dim3(kCThreads), 0, s, x, Cin, H, W, g,
                           gmask, partial);
    else switch (Cout) {
        case 32:
            hipLaunchKernelGGL(conv3x3_wgrad_kernel<32>, grid, dim3(kCThreads), 0, s, x, Cin, H, W,
                               g, gmask, partial);
            break;
        case 3:
            hipLaunchKernelGGL(conv3x3_wgrad_kernel<3>, grid, dim3(kCThreads), 0, s, x, Cin, H, W,
                               g, gmask, partial);
            break;
        default: return hipErrorInvalidValue;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const long long nw = (long long)Cout * Cin * 9, E = nw + Cout;
    const long long T = (long long)(mm ? grid_mm.x : grid.x) * N;
    const int S = (int)std::min<long long>(T, kSumSplits);
    float* mid = partial + T * E;   // the buffer holds (T + kSumSplits) E floats
    hipLaunchKernelGGL(sum_partials_kernel, dim3((unsigned)((E + 255) / 256), S), dim3(256), 0, s,
                       partial, T, E, S, mid);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(sum_mid_kernel, dim3((unsigned)((E + 255) / 256)), dim3(256), 0, s, mid, S,
                       E, dw, db, nw);
    return hipGetLastError();
}

hipError_t cnn_mse_grad(long long len, const double* y, const double* label, double scale,
                        uint16_t* g, double* part, int nblocks, hipStream_t s) {
    hipLaunchKernelGGL(mse_grad_kernel, dim3(nblocks), dim3(256), 0, s, len, y, label, scale, g,
                       part);
    return hipGetLastError();
}

hipError_t cnn_adam(long long n, float* w, float* wq, const float* g, float* m, float* v, float lr,
                    float b1, float b2, float eps, int t, hipStream_t s) {
    const float c1 = 1.0f - powf(b1, (float)t), c2 = 1.0f - powf(b2, (float)t);
    hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, w, wq, g,
                       m, v, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t cnn_to_bf16(long long n, const double* x, double scale, uint16_t* y, hipStream_t s) {
    const long long blocks = std::min<long long>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(to_bf16_kernel, dim3((unsigned)std::max<long long>(blocks, 1)), dim3(256), 0,
                       s, n, x, scale, y);
    return hipGetLastError();
}

hipError_t cnn_round_bf16(long long n, const float* x, float* y, hipStream_t s) {
    hipLaunchKernelGGL(round_bf16_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, x,
                       y);
    return hipGetLastError();
}

}  // namespace mek
