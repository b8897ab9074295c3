// FP64 GEMM on the CDNA matrix cores (v_mfma_f64_16x16x4f64), used for the
// residual engine R = C - (A X) B (initialisation of Alg. 3 and the
// refinement passes) and for the Gram matrices A A^T and B^T B that the
// residual update needs (the remark after Alg. 3).
//
// D_b = beta * C_b + alpha * A_b B_b for b < nb (strided batch; a stride of 0
// shares an operand), with arbitrary element strides for A and B, so the
// same kernel serves A B, A B^T and A^T B. One templated tile kernel: block
// tile 128 x 128 with 8 waves of 64 x 32 when the product gives every CU a
// tile, else 64 x 64 with 8 waves of 32 x 16.
//
// MFMA operand layout (16x16x4, f64; checked on gfx950 with a probe of unique
// input values): lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16];
// accumulator value j of lane l is D[l / 16 + 4 j][l % 16], j = 0..3.
#include "internal.h"

namespace mek {

typedef double double4_t __attribute__((ext_vector_type(4)));

// Tiled kernel: block tile BM x BN, waves in a (BM/WM) x (BN/WN) grid of WM x WN wave tiles
// ((WM/16) x (WN/16) MFMA tiles each), K tile 32. Per K tile: one barrier;
// the next K tile, already in registers, is stored to the other LDS buffer
// and the one after it is fetched; the MFMA fragments of step ks+4 are read
// from LDS while step ks multiplies.
//
// LDS layout: element (k, i) of a K tile sits at k * BM + (i ^ swz(k)). The
// XOR keeps i inside its aligned 32-column group, moves it to the other
// 16-column half when k is odd and permutes its low 4 bits by a value that
// differs for any 16 consecutive k (and, with the half bit, for any 32).
// With 8-byte words this makes three access sets conflict free whether LDS
// serves 16 lanes over 16 word slots or 32 lanes over 32 slots per cycle:
// the MFMA read (4 consecutive k x 16 consecutive i), the store of a
// unit-stride-in-i operand (64 consecutive i, one k) and the store of a
// unit-stride-in-k operand (32 consecutive k x 2 i).
constexpr int kTK = 32;

__device__ __forceinline__ int swz(int k) { return ((k & 1) << 4) | ((k & 15) ^ ((k >> 4) & 1)); }

// AK: A has unit stride along k (else along i); BJ: B has unit stride along
// j (else along k). The loads put the unit-stride dimension fastest across
// threads; the other strides are general.
template <int BM, int BN, int WM, int WN, bool AK, bool BJ>
__global__ void __launch_bounds__(64 * (BM / WM) * (BN / WN))
gemm_f64_tile_kernel(int M, int N, int K, double alpha, const double* __restrict__ A,
                     long long a_i, long long a_k, const double* __restrict__ B, long long b_k,
                     long long b_j, double beta, const double* C, long long ldc, double* D,
                     long long ldd, int tiles_m, int tiles_n, int nb, long long sA, long long sB,
                     long long sC, long long sD) {
    constexpr int WAVES_N = BN / WN;
    constexpr int THREADS = 64 * (BM / WM) * WAVES_N;
    constexpr int TM = WM / 16, TN = WN / 16;
    constexpr int LA = BM * kTK / THREADS, LB = BN * kTK / THREADS;
    constexpr int KS = kTK / 4;
    static_assert(LA * THREADS == BM * kTK && LB * THREADS == BN * kTK, "tile split");
    static_assert(THREADS % kTK == 0 && THREADS % BM == 0 && THREADS % BN == 0, "load map");
    static_assert(BM % 32 == 0 && BN % 32 == 0 && WM % 16 == 0 && WN % 16 == 0, "tile shape");
    __shared__ double As[2][kTK * BM];
    __shared__ double Bs[2][kTK * BN];

    // Instances stack along the tile rows of the grouped order.
    int bti, tj;
    tile_coords(blockIdx.x, nb * tiles_m, tiles_n, bti, tj);
    const int inst = bti / tiles_m, ti = bti - inst * tiles_m;
    A += inst * sA;
    B += inst * sB;
    if (beta != 0.0) C += inst * sC;
    D += inst * sD;
    const int tile_i = ti * BM, tile_j = tj * BN;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave / WAVES_N, wn = wave % WAVES_N;
    const int l16 = lane & 15, lq = lane >> 4;

    // Load s of a thread covers element e = tid + s * THREADS of the tile in
    // the order (row, k) for a unit-stride-in-k operand (k fastest) and
    // (k, row) otherwise. Rows (columns) past the matrix edge are clamped to
    // the last one: they feed only outputs that are never stored. Only the
    // K tail is zeroed.
    const int ak0 = AK ? tid % kTK : tid / BM, ai0 = AK ? tid / kTK : tid % BM;
    const int bk0 = BJ ? tid / BN : tid % kTK, bj0 = BJ ? tid % BN : tid / kTK;
    constexpr int ARS = AK ? THREADS / kTK : 0, AKS = AK ? 0 : THREADS / BM;
    constexpr int BCS = BJ ? 0 : THREADS / kTK, BKS = BJ ? THREADS / BN : 0;
    auto a_at = [&](int s, int k) -> const double* {
        const long long r = min(tile_i + ai0 + s * ARS, M - 1);
        return A + r * a_i + (long long)k * a_k;
    };
    auto b_at = [&](int s, int k) -> const double* {
        const long long c = min(tile_j + bj0 + s * BCS, N - 1);
        return B + (long long)k * b_k + c * b_j;
    };
    // Small tiles (short K steps) keep two register sets, so that the tile
    // two steps ahead is in flight while the next one is stored to LDS; the
    // large tiles have the registers for one set only.
    constexpr bool DEEP = BM * BN <= 64 * 64;
    constexpr int NS = DEEP ? 2 : 1;
    double ra[NS][LA], rb[NS][LB];
    auto load = [&](int k0, double (&xa)[LA], double (&xb)[LB]) {
        if (k0 + kTK <= K) {
#pragma unroll
            for (int s = 0; s < LA; ++s) xa[s] = *a_at(s, k0 + ak0 + s * AKS);
#pragma unroll
            for (int s = 0; s < LB; ++s) xb[s] = *b_at(s, k0 + bk0 + s * BKS);
        } else {
#pragma unroll
            for (int s = 0; s < LA; ++s) {
                const int k = k0 + ak0 + s * AKS;
                const double v = *a_at(s, min(k, K - 1));
                xa[s] = k < K ? v : 0.0;
            }
#pragma unroll
            for (int s = 0; s < LB; ++s) {
                const int k = k0 + bk0 + s * BKS;
                const double v = *b_at(s, min(k, K - 1));
                xb[s] = k < K ? v : 0.0;
            }
        }
    };
    auto store = [&](int buf, const double (&xa)[LA], const double (&xb)[LB]) {
#pragma unroll
        for (int s = 0; s < LA; ++s) {
            const int k = ak0 + s * AKS, i = ai0 + s * ARS;
            As[buf][k * BM + (i ^ swz(k))] = xa[s];
        }
#pragma unroll
        for (int s = 0; s < LB; ++s) {
            const int k = bk0 + s * BKS, j = bj0 + s * BCS;
            Bs[buf][k * BN + (j ^ swz(k))] = xb[s];
        }
    };

    double4_t acc[TM][TN];
#pragma unroll
    for (int x = 0; x < TM; ++x)
#pragma unroll
        for (int y = 0; y < TN; ++y) acc[x][y] = (double4_t){0.0, 0.0, 0.0, 0.0};

    // Fragment reads: lane (l16, lq) takes row i = wave base + 16 x + l16 of
    // k = ks + lq.
    const int ia = wm * WM, jb = wn * WN;
    double fa[2][TM], fb[2][TN];
    auto frag = [&](int buf, int ks, int slot) {
        const int k = ks + lq, h = swz(k);
#pragma unroll
        for (int x = 0; x < TM; ++x) fa[slot][x] = As[buf][k * BM + ((ia + x * 16 + l16) ^ h)];
#pragma unroll
        for (int y = 0; y < TN; ++y) fb[slot][y] = Bs[buf][k * BN + ((jb + y * 16 + l16) ^ h)];
    };

    const int nk = (K + kTK - 1) / kTK;   // K = 0 leaves acc at zero
    if (nk > 0) {
        load(0, ra[0], rb[0]);
        store(0, ra[0], rb[0]);
    }
    if (nk > 1) load(kTK, ra[NS - 1], rb[NS - 1]);
    if (DEEP && nk > 2) load(2 * kTK, ra[0], rb[0]);
    // Step t: tile t multiplies from buffer t & 1; after its first MFMA
    // steps tile t + 1 (register set (t + 1) % NS) goes to the other buffer
    // and that set fetches tile t + 1 + NS.
    auto step = [&](int t, double (&xa)[LA], double (&xb)[LB]) {
        const int cur = t & 1;
        __syncthreads();   // tile t is in buffer cur; nobody reads cur ^ 1 any more
        frag(cur, 0, 0);
#pragma unroll
        for (int q = 0; q < KS; ++q) {
            if (q + 1 < KS) frag(cur, 4 * (q + 1), (q + 1) & 1);
            if (q == 1 && t + 1 < nk) {
                store(cur ^ 1, xa, xb);
                if (t + 1 + NS < nk) load((t + 1 + NS) * kTK, xa, xb);
            }
#pragma unroll
            for (int x = 0; x < TM; ++x)
#pragma unroll
                for (int y = 0; y < TN; ++y)
                    acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[q & 1][x], fb[q & 1][y],
                                                                     acc[x][y], 0, 0, 0);
        }
    };
    if constexpr (DEEP) {
        for (int t = 0; t < nk; t += 2) {
            step(t, ra[NS - 1], rb[NS - 1]);
            if (t + 1 < nk) step(t + 1, ra[0], rb[0]);
        }
    } else {
        for (int t = 0; t < nk; ++t) {
            const int cur = t & 1;
            __syncthreads();   // tile t is in buffer cur; nobody reads cur ^ 1 any more
            frag(cur, 0, 0);
#pragma unroll
            for (int q = 0; q < KS; ++q) {
                if (q + 1 < KS) frag(cur, 4 * (q + 1), (q + 1) & 1);
                // Hand the next tile to LDS and fetch the one after while the
                // MFMAs of the first steps run.
                if (q == 1 && t + 1 < nk) {
                    store(cur ^ 1, ra[0], rb[0]);
                    if (t + 2 < nk) load((t + 2) * kTK, ra[0], rb[0]);
                }
#pragma unroll
                for (int x = 0; x < TM; ++x)
#pragma unroll
                    for (int y = 0; y < TN; ++y)
                        acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(
                            fa[q & 1][x], fb[q & 1][y], acc[x][y], 0, 0, 0);
            }
        }
    }

    // Epilogue: all loads of C first (clamped into the matrix, so always in
    // bounds), then the guarded stores; no load waits behind a store.
    double cv[TM][TN][4];
    if (beta != 0.0) {
#pragma unroll
        for (int x = 0; x < TM; ++x)
#pragma unroll
            for (int y = 0; y < TN; ++y)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const long long gi = min(tile_i + ia + x * 16 + lq + 4 * j, M - 1);
                    const long long gj = min(tile_j + jb + y * 16 + l16, N - 1);
                    cv[x][y][j] = C[gi * ldc + gj];
                }
    }
#pragma unroll
    for (int x = 0; x < TM; ++x)
#pragma unroll
        for (int y = 0; y < TN; ++y)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int gi = tile_i + ia + x * 16 + lq + 4 * j;
                const int gj = tile_j + jb + y * 16 + l16;
                double v = alpha * acc[x][y][j];
                if (beta != 0.0) v += beta * cv[x][y][j];
                if (gi < M && gj < N) D[(long long)gi * ldd + gj] = v;
            }
}

template <int BM, int BN, int WM, int WN>
static hipError_t launch_tiles(int M, int N, int K, double alpha, const double* A, long long a_i,
                               long long a_k, const double* B, long long b_k, long long b_j,
                               double beta, const double* C, long long ldc, double* D,
                               long long ldd, int nb, long long sA, long long sB, long long sC,
                               long long sD, hipStream_t s) {
    const int tm = (M + BM - 1) / BM, tn = (N + BN - 1) / BN;
    const bool ak = (a_k == 1), bj = (b_j == 1);
    auto kern = ak ? (bj ? gemm_f64_tile_kernel<BM, BN, WM, WN, true, true>
                         : gemm_f64_tile_kernel<BM, BN, WM, WN, true, false>)
                   : (bj ? gemm_f64_tile_kernel<BM, BN, WM, WN, false, true>
                         : gemm_f64_tile_kernel<BM, BN, WM, WN, false, false>);
    hipLaunchKernelGGL(kern, dim3((unsigned)((long long)nb * tm * tn)),
                       dim3(64 * (BM / WM) * (BN / WN)), 0, s, M, N, K, alpha, A, a_i, a_k, B,
                       b_k, b_j, beta, C, ldc, D, ldd, tm, tn, nb, sA, sB, sC, sD);
    return hipGetLastError();
}

hipError_t gemm_f64_batched(int nb, int M, int N, int K, double alpha, const double* A,
                            long long a_i, long long a_k, long long sA, const double* B,
                            long long b_k, long long b_j, long long sB, double beta,
                            const double* C, long long ldc, long long sC, double* D,
                            long long ldd, long long sD, hipStream_t s) {
    if (M <= 0 || N <= 0 || nb <= 0) return hipSuccess;
    int dev = 0, cus = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const long long big = (long long)nb * ((M + 127) / 128) * ((N + 127) / 128);
    if (big >= cus)
        return launch_tiles<128, 128, 64, 32>(M, N, K, alpha, A, a_i, a_k, B, b_k, b_j, beta, C,
                                              ldc, D, ldd, nb, sA, sB, sC, sD, s);
    return launch_tiles<64, 64, 32, 16>(M, N, K, alpha, A, a_i, a_k, B, b_k, b_j, beta, C, ldc, D,
                                        ldd, nb, sA, sB, sC, sD, s);
}

hipError_t gemm_f64(int M, int N, int K, double alpha, const double* A, long long a_i,
                    long long a_k, const double* B, long long b_k, long long b_j, double beta,
                    const double* C, long long ldc, double* D, long long ldd, hipStream_t s) {
    return gemm_f64_batched(1, M, N, K, alpha, A, a_i, a_k, 0, B, b_k, b_j, 0, beta, C, ldc, 0, D,
                            ldd, 0, s);
}

}  // namespace mek
