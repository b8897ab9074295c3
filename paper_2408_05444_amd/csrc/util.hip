// Small dense kernels around the solver: norms, transposes, conversions,
// the active-row list and the column pick of the repeated squaring for ||B||_2^2.
#include "internal.h"

#include <string.h>

#include <math.h>

namespace mek {

// ||A_i||^2 for every row: one wave per row, lanes stride over the columns.
__global__ void row_sq_norms_kernel(const double* __restrict__ A, int m, int p,
                                    double* __restrict__ out) {
    const int wave = (blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int lane = threadIdx.x & (kWave - 1);
    if (wave >= m) return;
    const double* row = A + (size_t)wave * p;
    double s = 0.0;
    for (int j = lane; j < p; j += kWave) s += row[j] * row[j];
    s = wave_sum(s);
    if (lane == 0) out[wave] = s;
}

hipError_t row_sq_norms(const double* A, int m, int p, double* out, hipStream_t s) {
    const int waves_per_block = 4;
    const int blocks = (m + waves_per_block - 1) / waves_per_block;
    hipLaunchKernelGGL(row_sq_norms_kernel, dim3(blocks), dim3(waves_per_block * kWave), 0, s, A,
                       m, p, out);
    return hipGetLastError();
}

// Reductions in two fixed-order stages: kReduceBlocks work-groups each sum
// a strided share into a partial, then one work-group adds the partials in
// block order. The result does not depend on scheduling.
// mode 0: sum x; 1: sum x^2; 2: sum (x - y)^2.
constexpr int kReduceBlocks = 256;

__global__ void __launch_bounds__(kThreads, 1)
reduce_partial_kernel(const double* __restrict__ x, const double* __restrict__ y, long long len,
                      int mode, double* partial) {
    __shared__ BlockScratch sc;
    double acc[1] = {0.0};
    const long long stride = (long long)gridDim.x * kThreads;
    for (long long e = (long long)blockIdx.x * kThreads + threadIdx.x; e < len; e += stride) {
        const double v = x[e];
        if (mode == 0) acc[0] += v;
        else if (mode == 1) acc[0] += v * v;
        else {
            const double d = v - y[e];
            acc[0] += d * d;
        }
    }
    block_sum<1>(acc, sc);
    if (threadIdx.x == 0) partial[blockIdx.x] = acc[0];
}

__global__ void __launch_bounds__(kThreads, 1)
reduce_final_kernel(const double* __restrict__ partial, int nparts, double* out) {
    __shared__ BlockScratch sc;
    double acc[1] = {threadIdx.x < nparts ? partial[threadIdx.x] : 0.0};
    block_sum<1>(acc, sc);
    if (threadIdx.x == 0) *out = acc[0];
}

static hipError_t reduce2(const double* x, const double* y, long long len, int mode, double* out,
                          double* scratch, hipStream_t s) {
    hipLaunchKernelGGL(reduce_partial_kernel, dim3(kReduceBlocks), dim3(kThreads), 0, s, x, y, len,
                       mode, scratch);
    hipLaunchKernelGGL(reduce_final_kernel, dim3(1), dim3(kThreads), 0, s, scratch, kReduceBlocks,
                       out);
    return hipGetLastError();
}

hipError_t sum_reduce(const double* x, long long len, double* out, double* scratch, hipStream_t s) {
    return reduce2(x, nullptr, len, 0, out, scratch, s);
}
hipError_t sq_norm(const double* x, long long len, double* out, double* scratch, hipStream_t s) {
    return reduce2(x, nullptr, len, 1, out, scratch, s);
}
hipError_t sq_diff_norm(const double* x, const double* y, long long len, double* out,
                        double* scratch, hipStream_t s) {
    return reduce2(x, y, len, 2, out, scratch, s);
}

__global__ void nonfinite_kernel(const double* __restrict__ x, long long len, int* out) {
    int bad = 0;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < len;
         e += (long long)gridDim.x * blockDim.x)
        bad |= !isfinite(x[e]);
    if (__any(bad) && (threadIdx.x & (kWave - 1)) == 0) atomicAdd(out, 1);
}

hipError_t nonfinite_count(const double* x, long long len, int* out, hipStream_t s) {
    hipError_t e = fill_zero_bytes(out, sizeof(int), s);
    if (e != hipSuccess) return e;
    long long blocks = (len + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(nonfinite_kernel, dim3((unsigned)blocks), dim3(256), 0, s, x, len, out);
    return hipGetLastError();
}

// List of rows with a_i > 0 in ascending order (chunk per thread + scan).
__global__ void __launch_bounds__(kThreads, 1)
active_rows_kernel(const double* __restrict__ a, int m, int* list, int* count) {
    __shared__ BlockScratch sc;
    const int cs = (m + kThreads - 1) / kThreads;
    const int b = min(m, (int)threadIdx.x * cs), e = min(m, b + cs);
    int cnt = 0;
    for (int i = b; i < e; ++i) cnt += (a[i] > 0.0);
    double pre_v, tot_v;
    int pre_c, tot_c;
    block_excl_scan(0.0, cnt, pre_v, pre_c, tot_v, tot_c, sc);
    int pos = pre_c;
    for (int i = b; i < e; ++i)
        if (a[i] > 0.0) list[pos++] = i;
    if (threadIdx.x == 0) *count = tot_c;
}

hipError_t active_rows(const double* a, int m, int* list, int* count, hipStream_t s) {
    hipLaunchKernelGGL(active_rows_kernel, dim3(1), dim3(kThreads), 0, s, a, m, list, count);
    return hipGetLastError();
}

// Xt (cols x rows, type T) = transpose of X (rows x cols, double); 32x32 LDS tiles.
template <typename T>
__global__ void transpose_to_kernel(const double* __restrict__ X, int rows, int cols,
                                    T* __restrict__ Xt) {
    __shared__ double tile[32][33];
    const int bi = blockIdx.y * 32, bj = blockIdx.x * 32;
    for (int y = threadIdx.y; y < 32; y += blockDim.y) {
        const int i = bi + y, j = bj + threadIdx.x;
        if (i < rows && j < cols) tile[y][threadIdx.x] = X[(size_t)i * cols + j];
    }
    __syncthreads();
    for (int y = threadIdx.y; y < 32; y += blockDim.y) {
        const int j = bj + y, i = bi + threadIdx.x;
        if (i < rows && j < cols) Xt[(size_t)j * rows + i] = (T)tile[threadIdx.x][y];
    }
}

template <typename T>
__global__ void transpose_from_kernel(const T* __restrict__ Xt, int rows, int cols,
                                      double* __restrict__ X) {
    __shared__ double tile[32][33];
    const int bi = blockIdx.y * 32, bj = blockIdx.x * 32;   // bi over rows of X, bj over cols
    for (int y = threadIdx.y; y < 32; y += blockDim.y) {
        const int j = bj + y, i = bi + threadIdx.x;
        if (i < rows && j < cols) tile[y][threadIdx.x] = (double)Xt[(size_t)j * rows + i];
    }
    __syncthreads();
    for (int y = threadIdx.y; y < 32; y += blockDim.y) {
        const int i = bi + y, j = bj + threadIdx.x;
        if (i < rows && j < cols) X[(size_t)i * cols + j] = tile[threadIdx.x][y];
    }
}

template <typename T>
hipError_t transpose_to(const double* X, int rows, int cols, T* Xt, hipStream_t s) {
    dim3 grid((cols + 31) / 32, (rows + 31) / 32), block(32, 8);
    hipLaunchKernelGGL(transpose_to_kernel<T>, grid, block, 0, s, X, rows, cols, Xt);
    return hipGetLastError();
}
template <typename T>
hipError_t transpose_from(const T* Xt, int rows, int cols, double* X, hipStream_t s) {
    dim3 grid((cols + 31) / 32, (rows + 31) / 32), block(32, 8);
    hipLaunchKernelGGL(transpose_from_kernel<T>, grid, block, 0, s, Xt, rows, cols, X);
    return hipGetLastError();
}
template hipError_t transpose_to<double>(const double*, int, int, double*, hipStream_t);
template hipError_t transpose_to<float>(const double*, int, int, float*, hipStream_t);
template hipError_t transpose_from<double>(const double*, int, int, double*, hipStream_t);
template hipError_t transpose_from<float>(const float*, int, int, double*, hipStream_t);

__global__ void convert_kernel(const double* __restrict__ x, long long len, float* __restrict__ y) {
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < len;
         e += (long long)gridDim.x * blockDim.x)
        y[e] = (float)x[e];
}
__global__ void widen_kernel(const float* __restrict__ x, long long len, double* __restrict__ y) {
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < len;
         e += (long long)gridDim.x * blockDim.x)
        y[e] = (double)x[e];
}
__global__ void copy_kernel(const double* __restrict__ x, long long len, double* __restrict__ y) {
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < len;
         e += (long long)gridDim.x * blockDim.x)
        y[e] = x[e];
}
// Zeroes exactly `bytes` bytes: 4-byte stores over the aligned body when the
// start is 4-byte aligned, single-byte stores for the rest (and for the whole
// buffer when the start is not aligned), so nothing past the end is written.
__global__ void zero_kernel(unsigned char* __restrict__ x, long long bytes, long long words) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    const long long t0 = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned int* xw = reinterpret_cast<unsigned int*>(x);
    for (long long e = t0; e < words; e += stride) xw[e] = 0u;
    for (long long e = words * 4 + t0; e < bytes; e += stride) x[e] = 0;
}
__global__ void lincomb_kernel(double a, const double* x, double b, const double* y,
                               long long len, double* out) {
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < len;
         e += (long long)gridDim.x * blockDim.x)
        out[e] = a * x[e] + b * y[e];
}

static dim3 ew_grid(long long len) {
    long long b = (len + 255) / 256;
    if (b > 2048) b = 2048;
    if (b < 1) b = 1;
    return dim3((unsigned)b);
}

hipError_t convert_f64_f32(const double* x, long long len, float* y, hipStream_t s) {
    hipLaunchKernelGGL(convert_kernel, ew_grid(len), dim3(256), 0, s, x, len, y);
    return hipGetLastError();
}
hipError_t convert_f32_f64(const float* x, long long len, double* y, hipStream_t s) {
    hipLaunchKernelGGL(widen_kernel, ew_grid(len), dim3(256), 0, s, x, len, y);
    return hipGetLastError();
}
hipError_t copy_f64(const double* x, long long len, double* y, hipStream_t s) {
    hipLaunchKernelGGL(copy_kernel, ew_grid(len), dim3(256), 0, s, x, len, y);
    return hipGetLastError();
}
// Zero a buffer of any size and alignment with a kernel (not a memset node,
// so the call is safe inside captured graphs).
hipError_t fill_zero_bytes(void* x, long long bytes, hipStream_t s) {
    if (bytes <= 0) return hipSuccess;
    const long long words = ((uintptr_t)x & 3) ? 0 : bytes / 4;
    const long long work = words + (bytes - words * 4);
    hipLaunchKernelGGL(zero_kernel, ew_grid(work), dim3(256), 0, s, (unsigned char*)x, bytes,
                       words);
    return hipGetLastError();
}
// Bytes carried in a launch's arguments and stored by the kernel: a host
// table reaches device memory through kernel nodes only (no copy node that
// would read host memory again when a captured graph is replayed).
struct ArgBlob {
    unsigned long long w[kBlobWords];
};
__global__ void store_blob_kernel(ArgBlob b, int words, unsigned long long* __restrict__ dst) {
    const int t = threadIdx.x;
    if (t < words) dst[t] = b.w[t];
}
hipError_t store_bytes(const void* src, size_t bytes, void* dst, hipStream_t s) {
    const unsigned char* in = (const unsigned char*)src;
    unsigned long long* out = (unsigned long long*)dst;
    for (size_t off = 0; off < bytes; off += kBlobWords * 8) {
        ArgBlob b;
        memset(&b, 0, sizeof(b));
        const size_t len = bytes - off < (size_t)kBlobWords * 8 ? bytes - off : (size_t)kBlobWords * 8;
        memcpy(&b, in + off, len);
        const int words = (int)((len + 7) / 8);
        hipLaunchKernelGGL(store_blob_kernel, dim3(1), dim3(kBlobWords), 0, s, b, words,
                           out + off / 8);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}
hipError_t lincomb_f64(double a, const double* x, double b, const double* y, long long len,
                       double* out, hipStream_t s) {
    hipLaunchKernelGGL(lincomb_kernel, ew_grid(len), dim3(256), 0, s, a, x, b, y, len, out);
    return hipGetLastError();
}

// Column of the q x q symmetric matrix G with the largest diagonal entry
// (lowest index on ties), copied to v; one work-group.
__global__ void __launch_bounds__(kThreads, 1)
diag_argmax_col_kernel(const double* __restrict__ G, int q, double* v) {
    __shared__ double bv[kWaves];
    __shared__ int bi[kWaves];
    __shared__ int best;
    double mv = -1.0;
    int mi = 0x7fffffff;
    for (int i = threadIdx.x; i < q; i += kThreads) {
        const double d = G[(size_t)i * q + i];
        if (d > mv) { mv = d; mi = i; }
    }
    // Wave, then block: largest value, lowest index among equal values.
    for (int off = 32; off > 0; off >>= 1) {
        const double ov = __shfl_xor(mv, off);
        const int oi = __shfl_xor(mi, off);
        if (ov > mv || (ov == mv && oi < mi)) { mv = ov; mi = oi; }
    }
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    if (lane == 0) { bv[wv] = mv; bi[wv] = mi; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double b = bv[0];
        int ib = bi[0];
        for (int w = 1; w < kWaves; ++w)
            if (bv[w] > b || (bv[w] == b && bi[w] < ib)) { b = bv[w]; ib = bi[w]; }
        best = ib < q ? ib : 0;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < q; i += kThreads) v[i] = G[(size_t)best * q + i];
}

hipError_t diag_argmax_col(const double* G, int q, double* v, hipStream_t s) {
    hipLaunchKernelGGL(diag_argmax_col_kernel, dim3(1), dim3(kThreads), 0, s, G, q, v);
    return hipGetLastError();
}

}  // namespace mek
