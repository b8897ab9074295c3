// Split-BF16 GEMM on the CDNA4 matrix cores (v_mfma_f32_16x16x32_bf16, FP32
// accumulation), the residual engine of the FP32 and mixed iterations:
// R = C - (A X) B recomputed from the current iterate (the initialisation of
// Alg. 3, repeated so that the incrementally updated residual does not drift).
//
// D_b = beta * C_b + alpha * A_b B_b for b < nb, A and B in FP32, C in FP64
// (the caller's right-hand side or a true FP64 residual), D in FP32.
//
// Each FP32 operand value x is split into P bf16 terms on its way into LDS:
// h = rn(x), m = rn(x - h), l = rn(x - h - m); every difference is exact in
// FP32, and h + m + l carries all 24 significand bits of x. A product of two
// split values is the sum of P^2 cross products; term (a_u, b_v) is of order
// 2^(-8 (u + v)) of the product, and the kernel keeps the terms with u + v < P
// (P = 1: h h, about bf16 accuracy, 2^-9; P = 2: + h m, m h, about 2^-17;
// P = 3: + h l, l h, m m, about FP32 accuracy). The kept terms of one k step
// are summed into the same FP32 accumulator, smallest order first.
//
// MFMA operand layout (16x16x32, bf16 -> f32): lane l supplies row l % 16 of
// the A block and column l % 16 of the B block, each as 8 consecutive k
// values (k = 8 (l / 16) .. 8 (l / 16) + 7, the same k set on both sides);
// accumulator value j of lane l is D[4 (l / 16) + j][l % 16], j = 0..3.
#include "internal.h"

namespace mek {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float float4_t __attribute__((ext_vector_type(4)));

namespace {

constexpr int kKT = 32;   // K tile: one MFMA k step

// Round-to-nearest-even of an FP32 value to bf16 (finite inputs), as raw bits.
__device__ __forceinline__ uint32_t bf16_rn_bits(float x) {
    uint32_t u = __float_as_uint(x);
    u += 0x7fffu + ((u >> 16) & 1u);
    return u >> 16;
}
__device__ __forceinline__ float bf16_bits_value(uint32_t b) { return __uint_as_float(b << 16); }

// The 16-byte slot of (row r, k chunk c) in an operand tile: chunk c of a row
// sits at position c ^ swz(r) of the row's four slots. The XOR makes both
// the fragment reads (16 rows, one chunk) and the stores of either load
// mapping conflict free whether LDS serves 8 lanes x 16 bytes or 16 lanes x
// 16 bytes per cycle.
__device__ __forceinline__ int chunk_slot(int r, int c) {
    return r * 4 + (c ^ (((r >> 1) & 3) ^ ((r >> 3) & 1)));
}

// Loads one 8-value chunk of an operand tile (row `row` of the tile, k values
// k0 + 8 c .. k0 + 8 c + 7) from FP32 memory with row stride rs and k stride
// ks; k values at or past K read as zero. KC: the operand is contiguous along
// k (then VEC allows two 16-byte loads, used when rs and the base are
// 16-byte aligned).
template <bool KC>
__device__ __forceinline__ void load_chunk(const float* __restrict__ base, long long rs,
                                           long long ks, int row, int k0, int K, bool vec,
                                           float (&v)[8]) {
    const float* p = base + (long long)row * rs;
    if (k0 + 8 <= K) {
        if (KC && vec) {
            const float4 a = *reinterpret_cast<const float4*>(p + k0);
            const float4 b = *reinterpret_cast<const float4*>(p + k0 + 4);
            v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
            v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
        } else {
#pragma unroll
            for (int e = 0; e < 8; ++e) v[e] = p[(long long)(k0 + e) * ks];
        }
    } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int k = k0 + e;
            const float x = p[(long long)min(k, K - 1) * ks];
            v[e] = k < K ? x : 0.0f;
        }
    }
}

// Splits 8 values into P bf16 terms each and writes one 16-byte slot per
// term: term t of the tile sits at t * rows * 4 slots from the tile start.
template <int P>
__device__ __forceinline__ void store_split(uint4* __restrict__ tile, int rows, int slot,
                                            const float (&v)[8]) {
    uint32_t pk[P][4];
#pragma unroll
    for (int e = 0; e < 8; e += 2) {
        float x0 = v[e], x1 = v[e + 1];
#pragma unroll
        for (int t = 0; t < P; ++t) {
            const uint32_t b0 = bf16_rn_bits(x0), b1 = bf16_rn_bits(x1);
            pk[t][e / 2] = b0 | (b1 << 16);
            x0 -= bf16_bits_value(b0);
            x1 -= bf16_bits_value(b1);
        }
    }
#pragma unroll
    for (int t = 0; t < P; ++t)
        tile[t * rows * 4 + slot] = make_uint4(pk[t][0], pk[t][1], pk[t][2], pk[t][3]);
}

// Block tile BM x BN, waves in a (BM/WM) x (BN/WN) grid of WM x WN wave tiles,
// one 8-value chunk per thread and operand per K tile (so THREADS = 4 BM =
// 4 BN). Per K tile: one barrier; fragments of the current buffer read; the
// next K tile (in registers) split into the other buffer and the one after
// it fetched; then the MFMAs.
template <int BM, int BN, int WM, int WN, int P, bool AK, bool BJ>
__global__ void __launch_bounds__(64 * (BM / WM) * (BN / WN))
gemm_bf16s_kernel(int M, int N, int K, double alpha, const float* __restrict__ A, long long a_i,
                  long long a_k, const float* __restrict__ B, long long b_k, long long b_j,
                  double beta, const double* __restrict__ C, long long ldc,
                  float* __restrict__ D, long long ldd, int tiles_m, int tiles_n, long long sA,
                  long long sB, long long sC, long long sD, int vec_a, int vec_b) {
    constexpr int WAVES_N = BN / WN;
    constexpr int THREADS = 64 * (BM / WM) * WAVES_N;
    constexpr int TM = WM / 16, TN = WN / 16;
    static_assert(THREADS == 4 * BM && THREADS == 4 * BN, "one chunk per thread and operand");
    static_assert(WM % 16 == 0 && WN % 16 == 0 && P >= 1 && P <= 3, "tile shape");
    constexpr int SA = BM * 4 * P, SB = BN * 4 * P;   // 16-byte slots per buffer
    __shared__ uint4 lds[2][SA + SB];

    int bti, tj;
    tile_coords(blockIdx.x, gridDim.x / tiles_n, tiles_n, bti, tj);
    const int inst = bti / tiles_m, ti = bti - inst * tiles_m;
    A += inst * sA;
    B += inst * sB;
    if (beta != 0.0) C += inst * sC;
    D += inst * sD;
    const int tile_i = ti * BM, tile_j = tj * BN;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave / WAVES_N, wn = wave % WAVES_N;

    // Chunk of this thread: contiguous-in-k operands take (row tid / 4,
    // chunk tid % 4), so four lanes read one row's 32 k values; the others
    // take (row tid % rows, chunk tid / rows), so a wave reads 64 consecutive
    // rows of one k. Rows past the edge are clamped (their outputs are never
    // stored).
    const int ar = AK ? tid / 4 : tid % BM, ac = AK ? tid % 4 : tid / BM;
    const int br = BJ ? tid % BN : tid / 4, bc = BJ ? tid / BN : tid % 4;
    const float* a_row = A + (long long)min(tile_i + ar, M - 1) * a_i;
    const float* b_col = B + (long long)min(tile_j + br, N - 1) * b_j;
    const int a_slot = chunk_slot(ar, ac), b_slot = chunk_slot(br, bc);
    // Two register sets: the tile two steps ahead is in flight while the
    // next one is split into LDS.
    float va[2][8], vb[2][8];
    auto load = [&](int k0, float (&ra)[8], float (&rb)[8]) {
        load_chunk<AK>(a_row, 0, a_k, 0, k0 + 8 * ac, K, vec_a != 0, ra);
        load_chunk<!BJ>(b_col, 0, b_k, 0, k0 + 8 * bc, K, vec_b != 0, rb);
    };
    auto store = [&](int buf, const float (&ra)[8], const float (&rb)[8]) {
        store_split<P>(&lds[buf][0], BM, a_slot, ra);
        store_split<P>(&lds[buf][SA], BN, b_slot, rb);
    };

    float4_t acc[TM][TN];
#pragma unroll
    for (int x = 0; x < TM; ++x)
#pragma unroll
        for (int y = 0; y < TN; ++y) acc[x][y] = (float4_t){0.f, 0.f, 0.f, 0.f};

    const int l16 = lane & 15, lq = lane >> 4;
    const int ia = wm * WM, jb = wn * WN;
    const int nk = (K + kKT - 1) / kKT;   // K = 0 leaves acc at zero
    if (nk > 0) {
        load(0, va[0], vb[0]);
        store(0, va[0], vb[0]);
    }
    if (nk > 1) load(kKT, va[1], vb[1]);
    if (nk > 2) load(2 * kKT, va[0], vb[0]);
    // Step t: tile t multiplies from LDS buffer t & 1; tile t + 1 (register
    // set (t + 1) & 1) is split into the other buffer, and that set then
    // fetches tile t + 3.
    auto step = [&](int t, float (&ra)[8], float (&rb)[8]) {
        const int cur = t & 1;
        __syncthreads();   // tile t is in buffer cur; nobody reads cur ^ 1 any more
        bf16x8_t fa[P][TM], fb[P][TN];
#pragma unroll
        for (int u = 0; u < P; ++u) {
#pragma unroll
            for (int x = 0; x < TM; ++x) {
                const uint4 w = lds[cur][u * BM * 4 + chunk_slot(ia + 16 * x + l16, lq)];
                fa[u][x] = __builtin_bit_cast(bf16x8_t, w);
            }
#pragma unroll
            for (int y = 0; y < TN; ++y) {
                const uint4 w = lds[cur][SA + u * BN * 4 + chunk_slot(jb + 16 * y + l16, lq)];
                fb[u][y] = __builtin_bit_cast(bf16x8_t, w);
            }
        }
        if (t + 1 < nk) {
            store(cur ^ 1, ra, rb);
            if (t + 3 < nk) load((t + 3) * kKT, ra, rb);
        }
        // Cross products with u + v < P, highest order (smallest) first.
#pragma unroll
        for (int ord = P - 1; ord >= 0; --ord)
#pragma unroll
            for (int u = 0; u <= ord; ++u)
#pragma unroll
                for (int x = 0; x < TM; ++x)
#pragma unroll
                    for (int y = 0; y < TN; ++y)
                        acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                            fa[u][x], fb[ord - u][y], acc[x][y], 0, 0, 0);
    };
    for (int t = 0; t < nk; t += 2) {
        step(t, va[1], vb[1]);
        if (t + 1 < nk) step(t + 1, va[0], vb[0]);
    }

    // Epilogue: C loads first (clamped, always in bounds), then guarded
    // stores; alpha acc + beta C formed in FP64, rounded once to FP32.
    double cv[TM][TN][4];
    if (beta != 0.0) {
#pragma unroll
        for (int x = 0; x < TM; ++x)
#pragma unroll
            for (int y = 0; y < TN; ++y)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const long long gi = min(tile_i + ia + 16 * x + 4 * lq + j, M - 1);
                    const long long gj = min(tile_j + jb + 16 * y + l16, N - 1);
                    cv[x][y][j] = C[gi * ldc + gj];
                }
    }
#pragma unroll
    for (int x = 0; x < TM; ++x)
#pragma unroll
        for (int y = 0; y < TN; ++y)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int gi = tile_i + ia + 16 * x + 4 * lq + j;
                const int gj = tile_j + jb + 16 * y + l16;
                double v = alpha * (double)acc[x][y][j];
                if (beta != 0.0) v += beta * cv[x][y][j];
                if (gi < M && gj < N) D[(long long)gi * ldd + gj] = (float)v;
            }
}

template <int BM, int BN, int WM, int WN, int P>
hipError_t launch_bf16s(int nb, int M, int N, int K, double alpha, const float* A, long long a_i,
                        long long a_k, long long sA, const float* B, long long b_k, long long b_j,
                        long long sB, double beta, const double* C, long long ldc, long long sC,
                        float* D, long long ldd, long long sD, hipStream_t s) {
    const int tm = (M + BM - 1) / BM, tn = (N + BN - 1) / BN;
    const bool ak = (a_k == 1), bj = (b_j == 1);
    // Two 16-byte loads per chunk when every chunk start is 16-byte aligned.
    auto aligned = [](const float* p, long long rs, long long ss) {
        return ((uintptr_t)p % 16 == 0) && rs % 4 == 0 && ss % 4 == 0;
    };
    const int va = ak && aligned(A, a_i, sA), vb = (b_k == 1) && aligned(B, b_j, sB);
    auto kern = ak ? (bj ? gemm_bf16s_kernel<BM, BN, WM, WN, P, true, true>
                         : gemm_bf16s_kernel<BM, BN, WM, WN, P, true, false>)
                   : (bj ? gemm_bf16s_kernel<BM, BN, WM, WN, P, false, true>
                         : gemm_bf16s_kernel<BM, BN, WM, WN, P, false, false>);
    hipLaunchKernelGGL(kern, dim3((unsigned)((long long)nb * tm * tn)),
                       dim3(64 * (BM / WM) * (BN / WN)), 0, s, M, N, K, alpha, A, a_i, a_k, B,
                       b_k, b_j, beta, C, ldc, D, ldd, tm, tn, sA, sB, sC, sD, va, vb);
    return hipGetLastError();
}

template <int P>
hipError_t gemm_bf16s_pieces(int nb, int M, int N, int K, double alpha, const float* A,
                             long long a_i, long long a_k, long long sA, const float* B,
                             long long b_k, long long b_j, long long sB, double beta,
                             const double* C, long long ldc, long long sC, float* D,
                             long long ldd, long long sD, int cus, hipStream_t s) {
    const long long big = (long long)nb * ((M + 127) / 128) * ((N + 127) / 128);
    if (big >= cus)
        return launch_bf16s<128, 128, 64, 32, P>(nb, M, N, K, alpha, A, a_i, a_k, sA, B, b_k, b_j,
                                                 sB, beta, C, ldc, sC, D, ldd, sD, s);
    return launch_bf16s<64, 64, 32, 32, P>(nb, M, N, K, alpha, A, a_i, a_k, sA, B, b_k, b_j, sB,
                                           beta, C, ldc, sC, D, ldd, sD, s);
}

}  // namespace

hipError_t gemm_bf16s_batched(int pieces, int nb, int M, int N, int K, double alpha,
                              const float* A, long long a_i, long long a_k, long long sA,
                              const float* B, long long b_k, long long b_j, long long sB,
                              double beta, const double* C, long long ldc, long long sC, float* D,
                              long long ldd, long long sD, hipStream_t s) {
    if (M <= 0 || N <= 0 || nb <= 0) return hipSuccess;
    if (pieces < 1 || pieces > 3) return hipErrorInvalidValue;
    int dev = 0, cus = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    switch (pieces) {
        case 1:
            return gemm_bf16s_pieces<1>(nb, M, N, K, alpha, A, a_i, a_k, sA, B, b_k, b_j, sB, beta,
                                        C, ldc, sC, D, ldd, sD, cus, s);
        case 2:
            return gemm_bf16s_pieces<2>(nb, M, N, K, alpha, A, a_i, a_k, sA, B, b_k, b_j, sB, beta,
                                        C, ldc, sC, D, ldd, sD, cus, s);
        default:
            return gemm_bf16s_pieces<3>(nb, M, N, K, alpha, A, a_i, a_k, sA, B, b_k, b_j, sB, beta,
                                        C, ldc, sC, D, ldd, sD, cus, s);
    }
}

}  // namespace mek
