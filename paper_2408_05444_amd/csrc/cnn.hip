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
// master copies), every sum in FP32 (the loss in FP64). Layout NCHW.
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

__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// FP32 -> BF16, round to nearest, ties to even (NaN stays a quiet NaN).
__device__ __forceinline__ uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x7fffffu)) return 0x7fc0;
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// Stage channels [0, C) of the (kHalo x kHalo) input tile at (h0-1, w0-1)
// of image n into LDS as FP32, zero outside the image; with a mask, entries
// whose mask value is not > 0 read as zero (a ReLU's gradient gate).
__device__ __forceinline__ void stage_halo(float* xs, const uint16_t* __restrict__ x,
                                           const uint16_t* __restrict__ mask, int n, int C,
                                           int H, int W, int h0, int w0) {
    const int tot = C * kHaloPix;
    for (int e = threadIdx.x; e < tot; e += kCThreads) {
        const int c = e / kHaloPix, r = e - c * kHaloPix;
        const int hh = h0 - 1 + r / kHalo, ww = w0 - 1 + r % kHalo;
        float v = 0.0f;
        if (hh >= 0 && hh < H && ww >= 0 && ww < W) {
            const size_t idx = (((size_t)n * C + c) * H + hh) * W + ww;
            v = bf2f(x[idx]);
            if (mask && !(bf2f(mask[idx]) > 0.0f)) v = 0.0f;
        }
        xs[c * kChanStride + r] = v;
    }
}

// Forward (TRANS = false): CO output channels from Cin inputs with weights
// w (CO, Cin, 3, 3). Input gradient (TRANS = true): the layer's weights W
// (Cin, CO, 3, 3) read as W[ci][co][2-i][2-j], no bias, no ReLU. Writes BF16
// (yb) or FP64 (yd) outputs; an FP64 output may add a tensor of its shape.
template <int CO, bool TRANS>
__global__ void __launch_bounds__(kCThreads)
conv3x3_kernel(const uint16_t* __restrict__ x, const uint16_t* __restrict__ mask, int Cin, int H,
               int W, const float* __restrict__ w, const float* __restrict__ bias, int relu,
               uint16_t* __restrict__ yb, double* __restrict__ yd, const double* __restrict__ add) {
    // Weights staged as ws[c][i][j][o] (o padded to a multiple of 4), so that
    // the CO weights of one input tap are one run of 16-byte LDS reads, the
    // same address in every lane.
    constexpr int COP = (CO + 3) & ~3;
    __shared__ float xs[kMaxC * kChanStride];
    __shared__ __align__(16) float ws[kMaxC * 9 * COP];
    const int tiles_w = (W + kCT - 1) / kCT;
    const int th = blockIdx.x / tiles_w, tw = blockIdx.x - th * tiles_w;
    const int n = blockIdx.y;
    const int h0 = th * kCT, w0 = tw * kCT;
    stage_halo(xs, x, mask, n, Cin, H, W, h0, w0);
    for (int e = threadIdx.x; e < Cin * 9 * COP; e += kCThreads) {
        const int o = e % COP, t = e / COP;
        const int c = t / 9, i = (t % 9) / 3, j = t % 3;
        float v = 0.0f;
        if (o < CO)
            v = TRANS ? w[((c * CO + o) * 3 + (2 - i)) * 3 + (2 - j)]
                      : w[((o * Cin + c) * 3 + i) * 3 + j];
        ws[e] = v;
    }
    __syncthreads();
    const int ty = threadIdx.x / kCT, tx = threadIdx.x % kCT;
    float acc[COP];
#pragma unroll
    for (int o = 0; o < COP; ++o) acc[o] = 0.0f;
    for (int c = 0; c < Cin; ++c) {
        const float* xc = xs + c * kChanStride + ty * kHalo + tx;
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const float xv = xc[i * kHalo + j];
                const float4* wp = reinterpret_cast<const float4*>(ws + ((c * 3 + i) * 3 + j) * COP);
#pragma unroll
                for (int o4 = 0; o4 < COP / 4; ++o4) {
                    const float4 w4 = wp[o4];
                    acc[4 * o4 + 0] = fmaf(xv, w4.x, acc[4 * o4 + 0]);
                    acc[4 * o4 + 1] = fmaf(xv, w4.y, acc[4 * o4 + 1]);
                    acc[4 * o4 + 2] = fmaf(xv, w4.z, acc[4 * o4 + 2]);
                    acc[4 * o4 + 3] = fmaf(xv, w4.w, acc[4 * o4 + 3]);
                }
            }
    }
    const int h = h0 + ty, wq = w0 + tx;
    if (h >= H || wq >= W) return;
#pragma unroll
    for (int o = 0; o < CO; ++o) {
        float v = acc[o] + (bias ? bias[o] : 0.0f);
        if (relu) v = fmaxf(v, 0.0f);
        const size_t idx = (((size_t)n * CO + o) * H + h) * W + wq;
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
    __shared__ float gs[CO * kCThreads];
    const int tiles_w = (W + kCT - 1) / kCT;
    const int th = blockIdx.x / tiles_w, tw = blockIdx.x - th * tiles_w;
    const int n = blockIdx.y;
    const int h0 = th * kCT, w0 = tw * kCT;
    stage_halo(xs, x, nullptr, n, Cin, H, W, h0, w0);
    for (int e = threadIdx.x; e < CO * kCThreads; e += kCThreads) {
        const int o = e / kCThreads, p = e - o * kCThreads;
        const int hh = h0 + p / kCT, ww = w0 + p % kCT;
        float v = 0.0f;
        if (hh < H && ww < W) {
            const size_t idx = (((size_t)n * CO + o) * H + hh) * W + ww;
            v = bf2f(g[idx]);
            if (gmask && !(bf2f(gmask[idx]) > 0.0f)) v = 0.0f;
        }
        gs[e] = v;
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
                const float gv = o < CO ? gs[o * kCThreads + p] : 0.0f;
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
    for (long long t = t0; t < t1; ++t) s += partial[t * E + e];
    mid[k * E + e] = s;
}

__global__ void sum_mid_kernel(const float* __restrict__ mid, int S, long long E,
                               float* __restrict__ dw, float* __restrict__ db, long long nw) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= E) return;
    float s = 0.0f;
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

template <bool TRANS>
hipError_t conv_dispatch(int N, int Cin, int H, int W, int Cout, const uint16_t* x,
                         const uint16_t* mask, const float* w, const float* b, int relu,
                         uint16_t* yb, double* yd, const double* add, hipStream_t s) {
    const int tiles = ((H + kCT - 1) / kCT) * ((W + kCT - 1) / kCT);
    dim3 grid(tiles, N);
    switch (Cout) {
        case 32:
            hipLaunchKernelGGL((conv3x3_kernel<32, TRANS>), grid, dim3(kCThreads), 0, s, x, mask,
                               Cin, H, W, w, b, relu, yb, yd, add);
            break;
        case 3:
            hipLaunchKernelGGL((conv3x3_kernel<3, TRANS>), grid, dim3(kCThreads), 0, s, x, mask,
                               Cin, H, W, w, b, relu, yb, yd, add);
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
                       uint16_t* yb, double* yd, const double* add, hipStream_t s) {
    return conv_dispatch<false>(N, Cin, H, W, Cout, x, mask, w, b, relu, yb, yd, add, s);
}

hipError_t cnn_conv3x3_grad_input(int N, int Cout, int H, int W, int Cin, const uint16_t* g,
                                  const uint16_t* gmask, const float* w, uint16_t* gx,
                                  hipStream_t s) {
    // A convolution over g (Cout channels) producing Cin channels.
    return conv_dispatch<true>(N, Cout, H, W, Cin, g, gmask, w, nullptr, 0, gx, nullptr, nullptr,
                               s);
}

hipError_t cnn_conv3x3_grad_weight(int N, int Cin, int H, int W, int Cout, const uint16_t* x,
                                   const uint16_t* g, const uint16_t* gmask, float* partial,
                                   float* dw, float* db, hipStream_t s) {
    const int tiles = ((H + kCT - 1) / kCT) * ((W + kCT - 1) / kCT);
    dim3 grid(tiles, N);
    switch (Cout) {
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
    const long long T = (long long)tiles * N;
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
