// FP64 GEMM on the CDNA matrix cores (v_mfma_f64_16x16x4f64), used for the
// residual engine R = C - (A X) B (initialisation of Alg. 3 and the
// refinement passes) and for the Gram matrices A A^T and B^T B that the
// residual update needs (the remark after Alg. 3).
//
// D = beta * C + alpha * A B with arbitrary element strides for A and B, so
// the same kernels serve A B, A B^T and A^T B. Small products: block tile
// 64 x 64, K tile 16,
// 256 threads = 4 waves in a 2 x 2 grid; each wave owns a 32 x 32 sub-tile
// made of 2 x 2 MFMA 16 x 16 tiles. Tiles of A and B are staged through LDS
// (k-major, padded against bank conflicts) with a register prefetch of the
// next K tile while the current one is multiplied.
//
// MFMA operand layout (16x16x4, f64; checked on gfx950 with a probe of unique
// input values): lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16];
// accumulator value j of lane l is D[l / 16 + 4 j][l % 16], j = 0..3.
#include "internal.h"

namespace mek {

typedef double double4_t __attribute__((ext_vector_type(4)));

constexpr int kGT = 64;      // block tile (M and N)
constexpr int kGK = 16;      // K tile
constexpr int kGThreads = 256;
constexpr int kPad = 2;      // LDS row padding (doubles)

__global__ void __launch_bounds__(kGThreads)
gemm_f64_kernel(int M, int N, int K, double alpha, const double* __restrict__ A, long long a_i,
                long long a_k, const double* __restrict__ B, long long b_k, long long b_j,
                double beta, const double* C, long long ldc, double* D, long long ldd) {
    __shared__ double As[kGK][kGT + kPad];   // As[k][i]
    __shared__ double Bs[kGK][kGT + kPad];   // Bs[k][j]

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1;
    const int tile_i = blockIdx.y * kGT, tile_j = blockIdx.x * kGT;

    // Global-load mapping: 1024 elements per tile, 4 per thread. Choose the
    // element order so that the unit-stride dimension is the fastest one.
    const bool a_k_fast = (a_k == 1);
    const bool b_j_fast = (b_j == 1);

    double ra[4], rb[4];
    auto load_tiles = [&](int k0) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int e = tid + s * kGThreads;
            int ii, kk;
            if (a_k_fast) { ii = e / kGK; kk = e % kGK; }
            else { kk = e / kGT; ii = e % kGT; }
            const int gi = tile_i + ii, gk = k0 + kk;
            ra[s] = (gi < M && gk < K) ? A[(long long)gi * a_i + (long long)gk * a_k] : 0.0;
            int jj, kb;
            if (b_j_fast) { kb = e / kGT; jj = e % kGT; }
            else { jj = e / kGK; kb = e % kGK; }
            const int gj = tile_j + jj, gkb = k0 + kb;
            rb[s] = (gj < N && gkb < K) ? B[(long long)gkb * b_k + (long long)gj * b_j] : 0.0;
        }
    };
    auto store_tiles = [&]() {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int e = tid + s * kGThreads;
            int ii, kk;
            if (a_k_fast) { ii = e / kGK; kk = e % kGK; }
            else { kk = e / kGT; ii = e % kGT; }
            As[kk][ii] = ra[s];
            int jj, kb;
            if (b_j_fast) { kb = e / kGT; jj = e % kGT; }
            else { jj = e / kGK; kb = e % kGK; }
            Bs[kb][jj] = rb[s];
        }
    };

    double4_t acc[2][2];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) acc[x][y] = (double4_t){0.0, 0.0, 0.0, 0.0};

    const int l16 = lane & 15, lq = lane >> 4;
    load_tiles(0);
    for (int k0 = 0; k0 < K; k0 += kGK) {
        __syncthreads();
        store_tiles();
        __syncthreads();
        if (k0 + kGK < K) load_tiles(k0 + kGK);
#pragma unroll
        for (int ks = 0; ks < kGK; ks += 4) {
            double af[2], bf[2];
#pragma unroll
            for (int x = 0; x < 2; ++x) af[x] = As[ks + lq][wr * 32 + x * 16 + l16];
#pragma unroll
            for (int y = 0; y < 2; ++y) bf[y] = Bs[ks + lq][wc * 32 + y * 16 + l16];
#pragma unroll
            for (int x = 0; x < 2; ++x)
#pragma unroll
                for (int y = 0; y < 2; ++y)
                    acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[x], bf[y], acc[x][y], 0, 0, 0);
        }
    }

#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int gi = tile_i + wr * 32 + x * 16 + lq + 4 * j;
                const int gj = tile_j + wc * 32 + y * 16 + l16;
                if (gi < M && gj < N) {
                    double v = alpha * acc[x][y][j];
                    if (beta != 0.0) v += beta * C[(long long)gi * ldc + gj];
                    D[(long long)gi * ldd + gj] = v;
                }
            }
}

// Large-tile variant for products that give every CU a tile: block tile
// 128 x 128, 8 waves in a 2 x 4 grid of 64 x 32 wave tiles (4 x 2 MFMA tiles,
// 8 accumulators per wave; two waves per SIMD, so one multiplies while the
// other waits on memory), K tile 16, two LDS buffers so that the next K tile
// is stored while the current one is multiplied (one barrier per K tile),
// and the K tile after that already in registers. LDS rows are padded by 16
// doubles so that the four k-rows a wave reads in one MFMA step fall on
// disjoint halves of the 64 banks.
constexpr int kBT = 128;
constexpr int kBPad = 16;
constexpr int kBThreads = 512;

__global__ void __launch_bounds__(kBThreads)
gemm_f64_big_kernel(int M, int N, int K, double alpha, const double* __restrict__ A, long long a_i,
                    long long a_k, const double* __restrict__ B, long long b_k, long long b_j,
                    double beta, const double* C, long long ldc, double* D, long long ldd) {
    __shared__ double As[2][kGK][kBT + kBPad];   // As[buf][k][i]
    __shared__ double Bs[2][kGK][kBT + kBPad];   // Bs[buf][k][j]

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wr = wave >> 2, wc = wave & 3;   // 64-row x 32-column wave tile
    const int tile_i = blockIdx.y * kBT, tile_j = blockIdx.x * kBT;
    const bool a_k_fast = (a_k == 1);
    const bool b_j_fast = (b_j == 1);

    // 2048 elements of each operand tile, 4 per thread, with the operand's
    // unit-stride dimension fastest across threads.
    double ra[4], rb[4];
    auto load_tiles = [&](int k0) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int e = tid + s * kBThreads;
            int ii, kk;
            if (a_k_fast) { ii = e / kGK; kk = e % kGK; }
            else { kk = e / kBT; ii = e % kBT; }
            const int gi = tile_i + ii, gk = k0 + kk;
            ra[s] = (gi < M && gk < K) ? A[(long long)gi * a_i + (long long)gk * a_k] : 0.0;
            int jj, kb;
            if (b_j_fast) { kb = e / kBT; jj = e % kBT; }
            else { jj = e / kGK; kb = e % kGK; }
            const int gj = tile_j + jj, gkb = k0 + kb;
            rb[s] = (gj < N && gkb < K) ? B[(long long)gkb * b_k + (long long)gj * b_j] : 0.0;
        }
    };
    auto store_tiles = [&](int buf) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int e = tid + s * kBThreads;
            int ii, kk;
            if (a_k_fast) { ii = e / kGK; kk = e % kGK; }
            else { kk = e / kBT; ii = e % kBT; }
            As[buf][kk][ii] = ra[s];
            int jj, kb;
            if (b_j_fast) { kb = e / kBT; jj = e % kBT; }
            else { jj = e / kGK; kb = e % kGK; }
            Bs[buf][kb][jj] = rb[s];
        }
    };

    double4_t acc[4][2];
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) acc[x][y] = (double4_t){0.0, 0.0, 0.0, 0.0};

    const int l16 = lane & 15, lq = lane >> 4;
    const int nk = (K + kGK - 1) / kGK;
    load_tiles(0);
    store_tiles(0);
    if (nk > 1) load_tiles(kGK);
    __syncthreads();
    for (int t = 0; t < nk; ++t) {
        const int cur = t & 1;
        // Multiply the current buffer.
#pragma unroll
        for (int ks = 0; ks < kGK; ks += 4) {
            double af[4], bf[2];
#pragma unroll
            for (int x = 0; x < 4; ++x) af[x] = As[cur][ks + lq][wr * 64 + x * 16 + l16];
#pragma unroll
            for (int y = 0; y < 2; ++y) bf[y] = Bs[cur][ks + lq][wc * 32 + y * 16 + l16];
#pragma unroll
            for (int x = 0; x < 4; ++x)
#pragma unroll
                for (int y = 0; y < 2; ++y)
                    acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[x], bf[y], acc[x][y], 0, 0, 0);
        }
        // Store the next tile into the other buffer (last read one K tile
        // ago, before the barrier that ended that step), fetch the one after.
        if (t + 1 < nk) {
            store_tiles(cur ^ 1);
            if (t + 2 < nk) load_tiles((t + 2) * kGK);
        }
        __syncthreads();
    }

#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int gi = tile_i + wr * 64 + x * 16 + lq + 4 * j;
                const int gj = tile_j + wc * 32 + y * 16 + l16;
                if (gi < M && gj < N) {
                    double v = alpha * acc[x][y][j];
                    if (beta != 0.0) v += beta * C[(long long)gi * ldc + gj];
                    D[(long long)gi * ldd + gj] = v;
                }
            }
}

hipError_t gemm_f64(int M, int N, int K, double alpha, const double* A, long long a_i,
                    long long a_k, const double* B, long long b_k, long long b_j, double beta,
                    const double* C, long long ldc, double* D, long long ldd, hipStream_t s) {
    if (M <= 0 || N <= 0) return hipSuccess;
    int dev = 0, cus = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const long long big_tiles = (long long)((M + kBT - 1) / kBT) * ((N + kBT - 1) / kBT);
    if (big_tiles >= cus) {
        dim3 grid((N + kBT - 1) / kBT, (M + kBT - 1) / kBT);
        hipLaunchKernelGGL(gemm_f64_big_kernel, grid, dim3(kBThreads), 0, s, M, N, K, alpha, A,
                           a_i, a_k, B, b_k, b_j, beta, C, ldc, D, ldd);
        return hipGetLastError();
    }
    dim3 grid((N + kGT - 1) / kGT, (M + kGT - 1) / kGT);
    hipLaunchKernelGGL(gemm_f64_kernel, grid, dim3(kGThreads), 0, s, M, N, K, alpha, A, a_i, a_k,
                       B, b_k, b_j, beta, C, ldc, D, ldd);
    return hipGetLastError();
}

}  // namespace mek
