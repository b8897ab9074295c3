// Persistent solver kernel for the two-sided greedy block projection on
// gfx950: the entry-wise extension of the greedy criterion of Algs. 3/4 with
// an exact projection onto a block of equations A_I X B_J = C_IJ.
//
// Step k, with omega_ij = R_ij^2 / (||A_i||^2 ||B_j||^2) (B_j the j-th column
// of B), Omega = max omega, S = ||R||_F^2:
//   eps = min(Omega, theta Omega + (1 - theta) S / (||A||_F^2 ||B||_F^2));
//   candidate rows: max_j omega_ij >= eps, ranked by that maximum (ties:
//   lower index first); I = the first s of them, less those dependent on
//   higher-ranked kept rows (Cholesky pivot of A_I A_I^T at most tau times
//   its diagonal); J likewise from the columns with B^T B, at most t;
//   W = (A_I A_I^T)^{-1} R_IJ (B_J^T B_J)^{-1};
//   X += A_I^T W B_J^T;  R -= (A A^T)_{:,I} W (B^T B)_{J,:}.
//
// Team layout as in the row solver: W co-resident work-groups; work-group g
// owns rows [g*rpw, ...) of R (in LDS when they fit) and rows [g*xpw, ...)
// of X^T. Per step four tagged exchanges (exchange.h):
//   A. each work-group publishes, for its rows, ||R_i||^2 and max_j omega_ij,
//      its column maxima of omega over its rows (one word per column) and
//      its error partial;
//   B. each work-group reads every row word and the error partials, reduces
//      a slice of the columns over the work-groups and publishes that slice
//      of the column maxima;
//   C. each work-group reads all column maxima, then (redundantly, in a fixed
//      order, so every work-group gets the same result) selects I and J and
//      factors A_I A_I^T and B_J^T B_J (one wave per factor, rows held in
//      registers);
//   D. the owners of the rows in I publish R_IJ; with it every work-group
//      forms W (one wave, columns then rows of W in registers), updates its
//      columns of X, then its rows of R together with the next step's row
//      words and column maxima (A of step k + 1).
// Reading every row word before publishing its column slice (B) makes every
// rewrite of a buffer causally after all reads of its previous contents,
// so one buffer per kind suffices.
#include "exchange.h"
#include "internal.h"

#include <math.h>

namespace mek {

namespace {

constexpr int kChunk = 8;   // rows of R per pass of the fused update/score loop
constexpr int kXRows = 8;   // rows of X^T per pass of the X update
constexpr int kInvWaves = 2;   // waves that invert the Gram blocks while the others exchange R_IJ
static_assert(kBlkCap * kBlkCap == 2 * kThreads, "W products: two entries per thread");
static_assert(kChunk == 8 && kXRows == 8, "block2_fac_doubles sizes the factor region for 8-row passes");
static_assert(kChunk * kBlkCap <= kThreads && 2 * kXRows * kBlkCap <= kThreads,
              "one thread per entry of (A A^T)_{i, I}, c and B_{l, J}");

// Optional phase timing (work-group 0, thread 0): wall-clock ticks per phase
// of a step, summed over the solve.
enum { kB2Rows, kB2Cols, kB2Select, kB2Gram, kB2Chol, kB2Factor, kB2E, kB2W, kB2X, kB2RUpd, kB2R,
       kB2Count };

// Orders a wave's LDS accesses around an exchange between its own lanes. A
// wave's LDS instructions are performed in issue order, so a store by one
// lane is seen by a later load of another lane of the same wave; the fences
// and the wave barrier keep the compiler from moving accesses across.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Order-preserving key of a non-negative double; 0 is reserved for "not a
// candidate".
__device__ __forceinline__ unsigned long long score_key(double v) {
    return (unsigned long long)__double_as_longlong(v) + 1ull;
}

struct Blk2Smem {
    BlockScratch sc;
    double red[kWaves][2 * kChunk];      // per-wave partials of the chunk reductions
    double err_w[kWaves];
    double diag[2][kBlkCap];             // diagonals of the candidate Gram blocks
    double dpiv[2][kBlkCap];             // pivots of the kept candidates
    double rd[2][kBlkCap];               // 1 / diagonal of the compacted factors
    unsigned long long ukey[2][kBlkCap]; // selected candidates, index order
    int uidx[2][kBlkCap];
    unsigned long long skey[2][kBlkCap]; // the same, rank order
    int sidx[2][kBlkCap];
    int keep[2][kBlkCap];                // 1 if the ranked candidate is kept
    int I[kBlkCap], J[kBlkCap];
    unsigned long long prefix[2];
    int need[2];
    int bincnt[2];                       // keys in the radix bin that holds the threshold
    int gcnt[2];                         // keys of that bin gathered (early exit)
    int nsel[2];
    int nI, nJ;
    int fail;
    // Phase timing (thread 0 of work-group 0 only): the clock at the last
    // mark and the ticks per phase, in LDS rather than in registers.
    unsigned long long t_last;
    unsigned long long ph[kB2Count];
};

// Sum (first NS values) and max (next NM values) over the block, results in
// sm.red row 0 for thread use after the call (fixed wave order).
template <int NS, int NM>
__device__ __forceinline__ void block_sums_maxes(double (&v)[NS + NM], Blk2Smem& sm) {
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
#pragma unroll
    for (int j = 0; j < NS; ++j) v[j] = wave_sum(v[j]);
#pragma unroll
    for (int j = NS; j < NS + NM; ++j) v[j] = wave_max(v[j]);
    if (lane == 0) {
#pragma unroll
        for (int j = 0; j < NS + NM; ++j) sm.red[wv][j] = v[j];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < NS; ++j) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) t += sm.red[w][j];
        v[j] = t;
    }
#pragma unroll
    for (int j = NS; j < NS + NM; ++j) {
        double t = sm.red[0][j];
#pragma unroll
        for (int w = 1; w < kWaves; ++w) t = fmax(t, sm.red[w][j]);
        v[j] = t;
    }
    __syncthreads();
}

// Block totals of 16 values per thread, the first 8 summed and the last 8
// maximised, returned to thread t < 16 (the total of value t). Within a
// wave the values are reduced and scattered by halving exchanges (lane
// partner l ^ 32, 16, 8, 4 keeps one half of the remaining values, then
// l ^ 2 and l ^ 1 complete the single value each lane holds), 34 lane
// exchanges in place of 16 separate wave reductions; the wave totals are
// then combined in wave order. Fixed order: identical inputs give identical
// results in every work-group.
__device__ __forceinline__ double block_reduce_scatter16(double (&v)[16], Blk2Smem& sm) {
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    const bool mx = (lane & 32) != 0;   // this lane ends with one of the maxima
    double a[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const double send = mx ? v[i] : v[i + 8];
        const double mine = mx ? v[i + 8] : v[i];
        const double r = __shfl_xor(send, 32);
        a[i] = mx ? fmax(mine, r) : mine + r;
    }
#pragma unroll
    for (int half = 4, mask = 16; half >= 1; half >>= 1, mask >>= 1) {
        const bool up = (lane & mask) != 0;
#pragma unroll
        for (int i = 0; i < half; ++i) {
            const double send = up ? a[i] : a[i + half];
            const double mine = up ? a[i + half] : a[i];
            const double r = __shfl_xor(send, mask);
            a[i] = mx ? fmax(mine, r) : mine + r;
        }
    }
#pragma unroll
    for (int mask = 2; mask >= 1; mask >>= 1) {
        const double r = __shfl_xor(a[0], mask);
        a[0] = mx ? fmax(a[0], r) : a[0] + r;
    }
    const int idx = (mx ? 8 : 0) + ((lane & 16) ? 4 : 0) + ((lane & 8) ? 2 : 0) + ((lane & 4) ? 1 : 0);
    if ((lane & 3) == 0) sm.red[wv][idx] = a[0];
    __syncthreads();
    double t = 0.0;
    const int tid = threadIdx.x;
    if (tid < 16) {
        t = sm.red[0][tid];
#pragma unroll
        for (int w = 1; w < kWaves; ++w) t = (tid < 8) ? t + sm.red[w][tid] : fmax(t, sm.red[w][tid]);
    }
    __syncthreads();
    return t;
}

// Radix selection of the largest keys, run by the whole block for two key
// sets at once (kind 0: rows, kind 1: columns). Thread t holds keys
// kr[0..rc) for indices rb.. and kc[0..cc) for indices cb.. (contiguous
// chunks in thread order). Writes the chosen candidates, at most cap of
// each kind, in rank order (key descending, index ascending) to sm.sidx /
// sm.skey and their count to sm.nsel. hist: 1024 ints of LDS.
template <int SR>
__device__ __forceinline__ void select_top(const unsigned long long (&kr)[SR], int rb, int rc,
                                           const unsigned long long (&kc)[SR], int cb, int cc,
                                           int capR, int capC, int* hist, Blk2Smem& sm) {
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
    // Candidates of each kind.
    int nr = 0, nc = 0;
#pragma unroll
    for (int j = 0; j < SR; ++j) {
        nr += (j < rc && kr[j] != 0ull);
        nc += (j < cc && kc[j] != 0ull);
    }
    double pv, tv;
    int pc, tc;
    block_excl_scan((double)nc, nr, pv, pc, tv, tc, sm.sc);
    const int totR = tc, totC = (int)tv;
    const bool radR = totR > capR, radC = totC > capC;
    // Threshold key T and the number of keys equal to T to take: every key
    // above T is taken, then keys equal to T in index order.
    unsigned long long thR = 0ull, thC = 0ull;
    int eqR = 0, eqC = 0;
    if (radR || radC) {
        // Smallest and largest candidate key of each kind: the radix passes
        // start at the highest byte where they differ (the bytes above are
        // common to every candidate), which also keeps the first histogram
        // from piling every key into one bin.
        double mm[4] = {-1.0, -INFINITY, -1.0, -INFINITY};
#pragma unroll
        for (int j = 0; j < SR; ++j) {
            if (j < rc && kr[j] != 0ull) {
                const double h = __longlong_as_double((long long)(kr[j] - 1ull));
                mm[0] = fmax(mm[0], h);
                mm[1] = fmax(mm[1], -h);
            }
            if (j < cc && kc[j] != 0ull) {
                const double h = __longlong_as_double((long long)(kc[j] - 1ull));
                mm[2] = fmax(mm[2], h);
                mm[3] = fmax(mm[3], -h);
            }
        }
        block_sums_maxes<0, 4>(mm, sm);
        int startR = -1, startC = -1;
        unsigned long long preR = 0ull, preC = 0ull;
        if (radR) {
            const unsigned long long kmax = score_key(mm[0]), kmin = score_key(-mm[1]);
            for (int d = 7; d >= 0 && startR < 0; --d)
                if ((kmax >> (8 * d)) != (kmin >> (8 * d))) startR = d;
            preR = startR >= 7 ? 0ull : (kmax >> (8 * (startR + 1))) << (8 * (startR + 1));
            if (startR < 0) preR = kmax;   // all candidate keys equal
        }
        if (radC) {
            const unsigned long long kmax = score_key(mm[2]), kmin = score_key(-mm[3]);
            for (int d = 7; d >= 0 && startC < 0; --d)
                if ((kmax >> (8 * d)) != (kmin >> (8 * d))) startC = d;
            preC = startC >= 7 ? 0ull : (kmax >> (8 * (startC + 1))) << (8 * (startC + 1));
            if (startC < 0) preC = kmax;
        }
        for (int e = tid; e < 1024; e += kThreads) hist[e] = 0;
        if (tid == 0) {
            sm.prefix[0] = preR;
            sm.prefix[1] = preC;
            sm.need[0] = min(capR, totR);
            sm.need[1] = min(capC, totC);
        }
        __syncthreads();
        // Radix passes, most significant byte first. A kind leaves the passes
        // early once the bin that holds its threshold has at most kBinMax
        // keys: those are gathered and ranked directly, which gives the same
        // threshold key and count of equal keys to take.
        constexpr int kBinMax = kWave;
        unsigned long long* bink = reinterpret_cast<unsigned long long*>(hist + 1024);
        bool doneR = !radR || startR < 0, doneC = !radC || startC < 0;
        const int dstart = max(startR, startC);
        for (int d = dstart; d >= 0 && !(doneR && doneC); --d) {
            int* H = hist + (d & 1) * 512;
            const int sh = 8 * d;
            const unsigned long long pR = sm.prefix[0], pC = sm.prefix[1];
            const bool inR = !doneR && d <= startR, inC = !doneC && d <= startC;
#pragma unroll
            for (int j = 0; j < SR; ++j) {
                if (inR && j < rc && kr[j] != 0ull &&
                    (d == 7 || (kr[j] >> (sh + 8)) == (pR >> (sh + 8))))
                    atomicAdd(&H[(int)((kr[j] >> sh) & 255ull)], 1);
                if (inC && j < cc && kc[j] != 0ull &&
                    (d == 7 || (kc[j] >> (sh + 8)) == (pC >> (sh + 8))))
                    atomicAdd(&H[256 + (int)((kc[j] >> sh) & 255ull)], 1);
            }
            __syncthreads();
            if (wv < 2 && (wv == 0 ? inR : inC)) {
                // Lane l holds bins 255-4l .. 252-4l (descending); find the bin
                // where the count of keys from the top reaches `need`.
                const int* h = H + wv * 256;
                int c4[4], s = 0;
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    c4[u] = h[255 - 4 * lane - u];
                    s += c4[u];
                }
                const int incl = wave_incl_scan_int(s);
                int run = incl - s;
                const int need = sm.need[wv];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    if (run < need && run + c4[u] >= need) {
                        const unsigned long long bin = (unsigned long long)(255 - 4 * lane - u);
                        sm.prefix[wv] |= bin << sh;
                        sm.need[wv] = need - run;
                        sm.bincnt[wv] = c4[u];
                        sm.gcnt[wv] = 0;
                    }
                    run += c4[u];
                }
            } else if (wv == 2) {
                int* Hn = hist + ((d + 1) & 1) * 512;
                for (int e = lane; e < 512; e += kWave) Hn[e] = 0;
            }
            __syncthreads();
            const bool exR = inR && d > 0 && sm.bincnt[0] <= kBinMax;
            const bool exC = inC && d > 0 && sm.bincnt[1] <= kBinMax;
            if (exR || exC) {
                const unsigned long long qR = sm.prefix[0], qC = sm.prefix[1];
#pragma unroll
                for (int j = 0; j < SR; ++j) {
                    if (exR && j < rc && kr[j] != 0ull && (kr[j] >> sh) == (qR >> sh))
                        bink[atomicAdd(&sm.gcnt[0], 1)] = kr[j];
                    if (exC && j < cc && kc[j] != 0ull && (kc[j] >> sh) == (qC >> sh))
                        bink[kBinMax + atomicAdd(&sm.gcnt[1], 1)] = kc[j];
                }
                __syncthreads();
                if (wv < 2 && (wv == 0 ? exR : exC)) {
                    // The need-th largest key of the bin (with multiplicity)
                    // and how many keys equal to it are taken: lane l holds
                    // key l and compares it with every other lane's.
                    const int cnt = sm.gcnt[wv], need = sm.need[wv];
                    const unsigned long long key = lane < cnt ? bink[wv * kBinMax + lane] : 0ull;
                    int gt = 0, eq = 0;
#pragma unroll
                    for (int u = 0; u < kBinMax; ++u) {
                        if (u < cnt) {
                            const unsigned long long ku =
                                ((unsigned long long)(unsigned int)__builtin_amdgcn_readlane((int)(key >> 32), u)
                                 << 32) |
                                (unsigned int)__builtin_amdgcn_readlane((int)key, u);
                            gt += ku > key;
                            eq += ku == key;
                        }
                    }
                    if (lane < cnt && gt < need && need <= gt + eq) {
                        sm.prefix[wv] = key;
                        sm.need[wv] = need - gt;
                    }
                }
                __syncthreads();
                doneR = doneR || exR;
                doneC = doneC || exC;
            }
        }
        thR = sm.prefix[0];
        thC = sm.prefix[1];
        eqR = sm.need[0];
        eqC = sm.need[1];
    }
    // Membership: key > T, or key == T among the first eq such keys.
    int er = 0, ec = 0;
#pragma unroll
    for (int j = 0; j < SR; ++j) {
        er += (radR && j < rc && kr[j] == thR);
        ec += (radC && j < cc && kc[j] == thC);
    }
    block_excl_scan((double)ec, er, pv, pc, tv, tc, sm.sc);
    int preR = pc, preC = (int)pv;
    bool selR[SR], selC[SR];
    int sr = 0, scn = 0;
#pragma unroll
    for (int j = 0; j < SR; ++j) {
        bool a = false, b = false;
        if (j < rc && kr[j] != 0ull) {
            if (!radR || kr[j] > thR) a = true;
            else if (kr[j] == thR) a = (preR++ < eqR);
        }
        if (j < cc && kc[j] != 0ull) {
            if (!radC || kc[j] > thC) b = true;
            else if (kc[j] == thC) b = (preC++ < eqC);
        }
        selR[j] = a;
        selC[j] = b;
        sr += a;
        scn += b;
    }
    block_excl_scan((double)scn, sr, pv, pc, tv, tc, sm.sc);
    int posR = pc, posC = (int)pv;
    // At most cap of each kind are selected by construction; the bounds
    // checks keep the lists in place whatever the keys are.
#pragma unroll
    for (int j = 0; j < SR; ++j) {
        if (selR[j] && posR < capR) {
            sm.uidx[0][posR] = rb + j;
            sm.ukey[0][posR] = kr[j];
            ++posR;
        }
        if (selC[j] && posC < capC) {
            sm.uidx[1][posC] = cb + j;
            sm.ukey[1][posC] = kc[j];
            ++posC;
        }
    }
    if (tid == 0) {
        sm.nsel[0] = min(tc, capR);
        sm.nsel[1] = min((int)tv, capC);
    }
    __syncthreads();
    // Rank order: count the keys above (and equal keys at lower indices).
    // Each lane compares its key with the others' taken from registers.
    if (wv < 2) {
        const int ns = sm.nsel[wv];
        const unsigned long long key = lane < ns ? sm.ukey[wv][lane] : 0ull;
        const int idx = lane < ns ? sm.uidx[wv][lane] : 0;
        int rank = 0;
#pragma unroll
        for (int u = 0; u < kBlkCap; ++u) {
            if (u < ns) {
                const unsigned long long ku =
                    ((unsigned long long)(unsigned int)__builtin_amdgcn_readlane((int)(key >> 32), u) << 32) |
                    (unsigned int)__builtin_amdgcn_readlane((int)key, u);
                const int iu = __builtin_amdgcn_readlane(idx, u);
                rank += (ku > key) || (ku == key && iu < idx);
            }
        }
        if (lane < ns) {
            sm.sidx[wv][rank] = idx;
            sm.skey[wv][rank] = key;
        }
    }
    __syncthreads();
}

}  // namespace

// One right-looking triangular sweep over a vector held in registers:
// forward, pivots x = 0, 1, ..., n - 2 subtract Mt[x][r] e[x] from e[r] for
// r > x; backward, pivots x = n - 1, ..., 1 subtract it for r < x. Mt holds
// the pivots' factors as rows of kBlkCap, zero past n, in `cap` >= n rows.
// One pivot at a time, its factor row in registers: pivots taken in pairs
// (two rows at once, one LDS round trip per pair) held so many registers
// that the kernel spilled around the sweeps; the pair form took 5.6 us more
// per step of the two-sided solve. The (uniform) branch per pivot keeps
// the compiler from fetching further ahead.
template <bool kFwd>
__device__ __forceinline__ void tri_sweep(double (&e)[kBlkCap], const double* Mt, int n, int cap) {
#pragma unroll
    for (int st = 0; st < kBlkCap - 1; ++st) {
        const int x = kFwd ? st : kBlkCap - 1 - st;
        if (x < n) {
            const double* m1 = Mt + min(x, cap - 1) * kBlkCap;
            double a1[kBlkCap];
#pragma unroll
            for (int r = 0; r < kBlkCap; ++r)
                if (kFwd ? r > x : r < x) a1[r] = m1[r];
            const double e1 = e[x];
#pragma unroll
            for (int r = 0; r < kBlkCap; ++r)
                if (kFwd ? r > x : r < x) e[r] -= a1[r] * e1;
        }
    }
}

template <int SR, bool LDS>
__global__ void __launch_bounds__(kThreads, 1) block2_kernel(Block2Params P) {
    extern __shared__ __align__(16) unsigned char dyn_smem[];
    __shared__ Blk2Smem sm;
    // The thread's indices are re-derived at the start of every phase of a
    // step through an opaque copy, so that the compiler recomputes the many
    // per-thread addresses of a phase inside it instead of keeping them in
    // registers across the whole loop.
    int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
    auto fresh_ids = [&]() {
        int t = threadIdx.x;
        asm volatile("; thread index, opaque to code motion" : "+v"(t));
        tid = t;
        lane = t & (kWave - 1);
        wv = t / kWave;
    };
    if (tid == 0) sm.fail = 0;

    const int W = P.W, g = blockIdx.x;
    const int m = P.m, n = P.n, p = P.p, q = P.q;
    const int scap = P.s_cap, tcap = P.t_cap;
    constexpr int ldE = kBlkCap + 1;
    const int row0 = g * P.rpw;
    const int nrow = max(0, min(P.rpw, m - row0));
    const int xc0 = g * P.xpw;
    const int nx = max(0, min(P.xpw, q - xc0));
    const int ncs = (n + W - 1) / W;                 // columns per slice (exchange B)
    const int cs0 = g * ncs;
    const int nslice = max(0, min(ncs, n - cs0));
    xword* const hx = reinterpret_cast<xword*>(P.hbuf);
    xword* const rx = reinterpret_cast<xword*>(P.rbuf);
    xword* const cx = reinterpret_cast<xword*>(P.cpart);
    xword* const gx = reinterpret_cast<xword*>(P.gcol);
    xword* const ex = reinterpret_cast<xword*>(P.ebuf);
    xword* const px = reinterpret_cast<xword*>(P.errpart);

    // LDS: [own rows of R] [E / W (kBlkCap x ldE), also the radix histograms,
    // the column slice and the factorisations' column buffers] [factors:
    // L_I (s_cap rows), L_J (t_cap rows), each row kBlkCap wide and zero
    // outside the block] [(A A^T)_{i, I}: kChunk x kBlkCap]. After W is
    // formed the factors' space holds the X update's c and B_{l, J}, then
    // the R update's z.
    const size_t r_bytes = LDS ? (((size_t)P.rpw * n * 8 + 15) & ~(size_t)15) : 0;
    const size_t e_bytes = block2_ereg_bytes(ncs);
    const int fac = block2_fac_doubles(scap, tcap);
    double *Rl, *E, *colbuf, *LI, *LJ, *gaI, *cX, *bX, *zT, *Rown;
    int* hist;
    unsigned long long* slice;
    // The region addresses are re-derived with the thread indices (below)
    // from an opaque zero offset, for the same reason.
    auto fresh_lds = [&]() {
        unsigned int z = 0;
        asm volatile("; LDS base, opaque to code motion" : "+s"(z));
        unsigned char* base = dyn_smem + z;
        Rl = reinterpret_cast<double*>(base);
        unsigned char* ereg = base + r_bytes;
        E = reinterpret_cast<double*>(ereg);
        hist = reinterpret_cast<int*>(ereg);
        slice = reinterpret_cast<unsigned long long*>(ereg);
        colbuf = reinterpret_cast<double*>(ereg);  // 4 x kBlkCap, during the factorisations
        LI = reinterpret_cast<double*>(ereg + e_bytes);
        LJ = LI + scap * kBlkCap;
        gaI = LI + fac;                            // kChunk x kBlkCap
        cX = LI;                                   // kXRows x kBlkCap (after W)
        bX = LI + kXRows * kBlkCap;                // kXRows x kBlkCap (after W)
        zT = LI;                                   // kBlkCap x kChunk (after the X update)
        // Own rows of R: LDS or device memory, fixed at compile time so that
        // every access is a plain LDS or global instruction.
        Rown = LDS ? Rl : P.R + (size_t)row0 * n;
    };
    fresh_lds();
    auto fresh = [&]() {
        fresh_ids();
        fresh_lds();
    };
    const bool timing = P.phase != nullptr && g == 0 && tid == 0;
    if (timing) {
        for (int i = 0; i < kB2Count; ++i) sm.ph[i] = 0;
        sm.t_last = wall_clock64();
    }
#define B2_PHASE(id)                                                    \
    do {                                                                \
        if (timing) {                                                   \
            const unsigned long long now_ = wall_clock64();             \
            sm.ph[id] += now_ - sm.t_last;                              \
            sm.t_last = now_;                                           \
        }                                                               \
    } while (0)

    if (LDS) {
        const double* src = P.R + (size_t)row0 * n;
        const size_t tot = (size_t)nrow * n;
        for (size_t e = tid; e < tot; e += kThreads) Rl[e] = src[e];
        __syncthreads();
    }

    // (A A^T)_{i, I} of rows c0 .. c0 + kChunk of this work-group, as the
    // value thread tid < kChunk * kBlkCap stores to gaI[tid] (zero outside
    // the rows and the block).
    auto fetch_gaI = [&](int c0, int nI, int e) -> double {
        const int ii = e / kBlkCap, x = e - ii * kBlkCap;
        if (e < kChunk * kBlkCap && c0 + ii < nrow && x < nI)
            return P.GA[(size_t)(row0 + c0 + ii) * m + sm.I[x]];
        return 0.0;
    };

    // Fused pass over own rows: optional update R_i -= z_i (B^T B)_{J,:}, then
    // ||R_i||^2, max_j omega_ij and this work-group's column maxima; publishes
    // the row words and column maxima with `tag`. Thread t handles columns
    // t, t + kThreads, ... (coalesced), kChunk rows at a time. With `upd`,
    // gaI holds the first chunk's (A A^T)_{i, I} on entry and E holds W,
    // zero outside nI x nJ.
    auto update_and_score = [&](bool upd, int nI, int nJ, unsigned int tag) {
        for (int c0 = 0; upd && c0 < nrow; c0 += kChunk) {
            const int cr = min(kChunk, nrow - c0);
            {
                if (c0 > 0) {
                    const double gv = fetch_gaI(c0, nI, tid);
                    __syncthreads();   // every thread is done with the previous chunk
                    if (tid < kChunk * kBlkCap) gaI[tid] = gv;
                    __syncthreads();
                }
                // z_i = (A A^T)_{i, I} W, stored transposed (zT[y][i]); the
                // terms past nI are exact zeros.
                if (tid < kChunk * kBlkCap) {
                    const int ii = tid & (kChunk - 1), y = tid / kChunk;
                    double a0 = 0.0, a1 = 0.0;
#pragma unroll
                    for (int x = 0; x < kBlkCap; x += 2) {
                        a0 += gaI[ii * kBlkCap + x] * E[x * ldE + y];
                        a1 += gaI[ii * kBlkCap + x + 1] * E[(x + 1) * ldE + y];
                    }
                    zT[y * kChunk + ii] = a0 + a1;
                }
                __syncthreads();
                // R_i -= z_i (B^T B)_{J,:}: columns in groups of 4 per thread,
                // so each z value read from LDS serves four columns.
#pragma unroll
                for (int u0 = 0; u0 < SR; u0 += 4) {
                    double acc[4][kChunk];
#pragma unroll
                    for (int u = 0; u < 4; ++u)
#pragma unroll
                        for (int ii = 0; ii < kChunk; ++ii) acc[u][ii] = 0.0;
                    // Rows J_y of B^T B, 8 at a time with every load issued
                    // before the multiply-adds that use them (row index made
                    // uniform, column clamped: the loads need no branch).
                    unsigned int jc[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) jc[u] = (unsigned int)min(tid + (u0 + u) * kThreads, n - 1);
                    for (int y0 = 0; y0 < nJ; y0 += 8) {
                        double gb[8][4];
#pragma unroll
                        for (int yy = 0; yy < 8; ++yy) {
                            const int Jy = __builtin_amdgcn_readfirstlane(sm.J[min(y0 + yy, nJ - 1)]);
                            const double* gbr = P.GB + (size_t)Jy * n;
#pragma unroll
                            for (int u = 0; u < 4; ++u) gb[yy][u] = (u0 + u < SR) ? gbr[jc[u]] : 0.0;
                        }
#pragma unroll
                        for (int yy = 0; yy < 8; ++yy) {
                            if (y0 + yy < nJ) {
                                double zv[kChunk];
#pragma unroll
                                for (int ii = 0; ii < kChunk; ++ii) zv[ii] = zT[(y0 + yy) * kChunk + ii];
#pragma unroll
                                for (int ii = 0; ii < kChunk; ++ii)
#pragma unroll
                                    for (int u = 0; u < 4; ++u) acc[u][ii] += zv[ii] * gb[yy][u];
                            }
                        }
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int j = tid + (u0 + u) * kThreads;
                        if (u0 + u < SR && j < n) {
#pragma unroll
                            for (int ii = 0; ii < kChunk; ++ii)
                                if (ii < cr) Rown[(size_t)(c0 + ii) * n + j] -= acc[u][ii];
                        }
                    }
                }
            }
        }
        if (upd) B2_PHASE(kB2RUpd);
        fresh();
        // Norms, row maxima and column maxima of omega, kChunk rows at a time
        // (every thread reads its own columns, so no barrier after the
        // update). With one chunk a column's maximum over the work-group's
        // rows is final once its rows are scored and is published at once;
        // with several it is carried over the chunks in cm.
        // Every global load of the pass is issued before its first store: a
        // wave's vector memory operations are counted in issue order, so a
        // load behind a store would also wait for the store.
        auto score = [&](int c0, int cr, double (&cm)[SR], bool carry) {
            double aa[kChunk];
#pragma unroll
            for (int ii = 0; ii < kChunk; ++ii) aa[ii] = (ii < cr) ? P.a[row0 + c0 + ii] : 0.0;
            double bv[SR];
#pragma unroll
            for (int u = 0; u < SR; ++u) bv[u] = P.b[min(tid + u * kThreads, n - 1)];
            double v[2 * kChunk];
#pragma unroll
            for (int ii = 0; ii < kChunk; ++ii) {
                v[ii] = 0.0;            // ||R_i||^2 partial
                v[kChunk + ii] = 0.0;   // max_j omega_ij partial
            }
            double cmo[SR];
#pragma unroll
            for (int u = 0; u < SR; ++u) {
                const int j = tid + u * kThreads;
                cmo[u] = 0.0;
                if (j < n) {
                    const double bj = bv[u];
                    double cmu = carry ? cm[u] : 0.0;
#pragma unroll
                    for (int ii = 0; ii < kChunk; ++ii) {
                        if (ii < cr) {
                            const double val = Rown[(size_t)(c0 + ii) * n + j];
                            const double sq = val * val;
                            v[ii] += sq;
                            if (aa[ii] > 0.0 && bj > 0.0) {
                                const double w = sq / (aa[ii] * bj);
                                v[kChunk + ii] = fmax(v[kChunk + ii], w);
                                cmu = fmax(cmu, w);
                            }
                        }
                    }
                    if (carry) cm[u] = cmu;
                    cmo[u] = cmu;
                }
            }
            if (!carry) {
#pragma unroll
                for (int u = 0; u < SR; ++u) {
                    const int j = tid + u * kThreads;
                    if (j < n) xstore(&cx[(size_t)g * n + j], pack_word(cmo[u], tag));
                }
            }
            static_assert(2 * kChunk == 16, "the scoring reduction takes 8 sums and 8 maxima");
            const double tot = block_reduce_scatter16(v, sm);
            if (tid < cr) xstore(&rx[row0 + c0 + tid], pack_word(tot, tag));
            else if (tid >= kChunk && tid - kChunk < cr) xstore(&hx[row0 + c0 + tid - kChunk], pack_word(tot, tag));
        };
        if (nrow <= kChunk) {
            double none[SR];
            score(0, nrow, none, false);
        } else {
            double cm[SR];
#pragma unroll
            for (int u = 0; u < SR; ++u) cm[u] = 0.0;
            for (int c0 = 0; c0 < nrow; c0 += kChunk) score(c0, min(kChunk, nrow - c0), cm, true);
#pragma unroll
            for (int u = 0; u < SR; ++u) {
                const int j = tid + u * kThreads;
                if (j < n) xstore(&cx[(size_t)g * n + j], pack_word(cm[u], tag));
            }
        }
    };

    // B_{l, J_y} for rows l0 .. l0 + kXRows of this work-group's X^T, as the
    // value thread kThreads - kXRows * kBlkCap + e stores to bX[e].
    constexpr int kBxT0 = kThreads - kXRows * kBlkCap;
    auto fetch_bX = [&](int l0, int nJ) -> double {
        const int e = tid - kBxT0, l = e / kBlkCap, y = e - l * kBlkCap;
        if (e >= 0 && l0 + l < nx && y < nJ) return P.B[(size_t)(xc0 + l0 + l) * n + sm.J[y]];
        return 0.0;
    };

    // X^T rows of this work-group, kXRows at a time:
    //   c[l][x] = sum_y W[x][y] B[l][J_y] (LDS, stored as cX[x][l]), then
    //   X^T[l, s] += sum_x c[l][x] A[I_x][s], a thread per column s,
    // with the column's entries of A loaded before c is formed, all in
    // flight together. bpre: this thread's fetch_bX(0) value. W (in E) and
    // c are zero outside the block, so the sums run over kBlkCap terms.
    // Leaves the squared-error partial of the updated rows in sm.err_w.
    auto update_x = [&](int nI, int nJ, double bpre) {
        double ep = 0.0;
        constexpr int kXH = kBlkCap / 2;   // A's entries in two halves of the block
        for (int l0 = 0; l0 < nx; l0 += kXRows) {
            const int lc = min(kXRows, nx - l0);
            for (int s0 = 0; s0 < p; s0 += kThreads) {
                const int s2 = s0 + tid, s2c = min(s2, p - 1);
                double acc[kXRows];
#pragma unroll
                for (int l = 0; l < kXRows; ++l) acc[l] = 0.0;
#pragma unroll
                for (int hf = 0; hf < 2; ++hf) {
                    double av[kXH];
#pragma unroll
                    for (int x = 0; x < kXH; ++x) {
                        const int xx = hf * kXH + x;
                        const int Ix = __builtin_amdgcn_readfirstlane(sm.I[xx < nI ? xx : 0]);
                        av[x] = P.A[(size_t)Ix * p + (unsigned int)s2c];
                    }
                    if (hf == 0 && s0 == 0) {
                        const double bv = (l0 == 0) ? bpre : fetch_bX(l0, nJ);
                        if (tid >= kBxT0) bX[tid - kBxT0] = bv;
                        __syncthreads();
                        if (tid < kXRows * kBlkCap) {
                            const int x = tid / kXRows, l = tid - x * kXRows;
                            double a0 = 0.0, a1 = 0.0;
#pragma unroll 4
                            for (int y = 0; y < kBlkCap; y += 2) {
                                a0 += E[x * ldE + y] * bX[l * kBlkCap + y];
                                a1 += E[x * ldE + y + 1] * bX[l * kBlkCap + y + 1];
                            }
                            cX[x * kXRows + l] = a0 + a1;
                        }
                        __syncthreads();
                    }
                    // The chunk's rows (terms in x order, first half then
                    // second), A's entries of this half in registers.
#pragma unroll
                    for (int l = 0; l < kXRows; ++l)
                        if (l < lc) {
#pragma unroll
                            for (int x = 0; x < kXH; ++x)
                                acc[l] += cX[(hf * kXH + x) * kXRows + l] * av[x];
                        }
                }
                if (s2 < p) {
#pragma unroll
                    for (int l = 0; l < kXRows; ++l) {
                        if (l < lc) {
                            const size_t off = (size_t)(xc0 + l0 + l) * p + s2;
                            const double nv = P.Xt[off] + acc[l];
                            P.Xt[off] = nv;
                            if (P.Xref_t) {
                                const double d = nv - P.Xref_t[off];
                                ep += d * d;
                            }
                        }
                    }
                }
            }
            __syncthreads();   // before the next chunk rewrites bX and cX
        }
        ep = wave_sum(ep);
        if (lane == 0) sm.err_w[wv] = ep;
    };

    // ---- Set-up: the first row words, column maxima and error partial.
    update_and_score(false, 0, 0, seq_tag(0));
    {
        double ep = 0.0;
        if (P.Xref_t) {
            const size_t base = (size_t)xc0 * p, total = (size_t)nx * p;
            for (size_t e = tid; e < total; e += kThreads) {
                const double d = P.Xt[base + e] - P.Xref_t[base + e];
                ep += d * d;
            }
        }
        double v[1] = {ep};
        block_sum<1>(v, sm.sc);
        if (tid == 0) xstore(&px[g], pack_word(v[0], seq_tag(0)));
    }

    const int cs = (max(m, n) + kThreads - 1) / kThreads;   // chunk per thread (<= SR)
    int rb, rcnt, cb, ccnt;
    double S0 = -1.0, S = 0.0, err = NAN;
    long long k = 0;
    int status = kMaxIter, last_nI = 0;
    bool ok = true;
    const bool has_ref = P.Xref_t != nullptr;
    if (timing) sm.t_last = wall_clock64();
    while (ok) {
        {
            fresh();
            rb = min(m, tid * cs);
            rcnt = min(m, rb + cs) - rb;
            cb = min(n, tid * cs);
            ccnt = min(n, cb + cs) - cb;
        }
        const unsigned int tag = seq_tag(k);
        // ---- B. Row words, error partials, and a slice of the column maxima.
        for (int c = tid; c < ncs; c += kThreads) slice[c] = 0ull;
        __syncthreads();
        double rr[SR], hh[SR];
        if (!poll_words<double, SR>(rx + rb, rcnt, tag, rr, P.sync, P.poll_sleep)) sm.fail = 1;
        if (!poll_words<double, SR>(hx + rb, rcnt, tag, hh, P.sync, P.poll_sleep)) sm.fail = 1;
        double Ep = 0.0;
        if (tid < W) {
            double e1[1];
            if (!poll_words<double, 1>(px + tid, 1, tag, e1, P.sync, P.poll_sleep)) sm.fail = 1;
            Ep = e1[0];
        }
        {
            const int tot = nslice * W;
            for (int f0 = tid; f0 < tot; f0 += kThreads * 4) {
                const xword* ptr[4];
                int cnt = 0;
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int f = f0 + u * kThreads;
                    const int c = (f < tot) ? f / W : 0, w2 = (f < tot) ? f - c * W : 0;
                    ptr[u] = cx + (size_t)w2 * n + cs0 + c;
                    cnt += (f < tot);
                }
                double vals[4];
                if (!poll_gather<double, 4>(ptr, cnt, tag, vals, P.sync, P.poll_sleep)) sm.fail = 1;
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int f = f0 + u * kThreads;
                    if (u < cnt)
                        atomicMax(&slice[f / W], (unsigned long long)__double_as_longlong(vals[u]));
                }
            }
        }
        __syncthreads();
        for (int c = tid; c < nslice; c += kThreads)
            xstore(&gx[cs0 + c], pack_word(__longlong_as_double((long long)slice[c]), tag));
        // ||R||_F^2, Omega and the error.
        double Sp = 0.0, Mp = 0.0;
#pragma unroll
        for (int j = 0; j < SR; ++j) {
            if (j < rcnt) {
                Sp += rr[j];
                if (P.a[rb + j] > 0.0) Mp = fmax(Mp, hh[j]);
            }
        }
        block_sum_max_sum(Sp, Mp, Ep, sm.sc);
        if (sm.fail) { ok = false; break; }
        S = Sp;
        const double Om = Mp;
        if (S0 < 0.0) S0 = S;
        err = has_ref ? sqrt(Ep / P.ref2) : NAN;
        if (g == 0 && tid == 0 && k < P.hist_cap) {
            if (P.resid_hist) P.resid_hist[k] = S;
            if (P.err_hist) P.err_hist[k] = err;
        }
        // Stop tests, in a fixed order (every work-group decides the same).
        if (P.stop == kStopRelErr && err <= P.tol) { status = kOK; break; }
        if (P.stop == kStopRelResid && sqrt(S) <= P.tol * sqrt(P.C2)) { status = kOK; break; }
        if (S == 0.0) { status = kExact; break; }
        if (!isfinite(S) || (P.diverge > 0.0 && S > P.diverge * S0)) { status = kEDiverged; break; }
        if (k >= P.max_iters) { status = kMaxIter; break; }
        B2_PHASE(kB2Rows);

        fresh();
        // ---- C. Column maxima; selection of I and J.
        double gg[SR];
        if (!poll_words<double, SR>(gx + cb, ccnt, tag, gg, P.sync, P.poll_sleep)) sm.fail = 1;
        double eps;
        {
#pragma clang fp contract(off)
            eps = P.theta * Om + (1.0 - P.theta) * (S / (P.F_A * P.F_B));
            if (eps > Om) eps = Om;
        }
        unsigned long long kr[SR], kc[SR];
#pragma unroll
        for (int j = 0; j < SR; ++j) {
            kr[j] = (j < rcnt && P.a[rb + j] > 0.0 && hh[j] >= eps) ? score_key(hh[j]) : 0ull;
            kc[j] = (j < ccnt && P.b[cb + j] > 0.0 && gg[j] >= eps) ? score_key(gg[j]) : 0ull;
        }
        __syncthreads();   // every thread is past its use of `slice` (same LDS as hist)
        if (sm.fail) { ok = false; break; }
        B2_PHASE(kB2Cols);
        fresh();
        select_top<SR>(kr, rb, rcnt, kc, cb, ccnt, scap, tcap, hist, sm);
        B2_PHASE(kB2Select);
        const int nsR = sm.nsel[0], nsC = sm.nsel[1];
        fresh();
        // Gram blocks of the ranked candidates (lower triangles, zero
        // elsewhere), then an in-place right-looking Cholesky in rank order
        // that skips dependent candidates.
        for (int e = tid; e < scap * kBlkCap; e += kThreads) {
            const int x = e / kBlkCap, y = e - x * kBlkCap;
            LI[e] = (x < nsR && y <= x) ? P.GA[(size_t)sm.sidx[0][x] * m + sm.sidx[0][y]] : 0.0;
        }
        for (int e = tid; e < tcap * kBlkCap; e += kThreads) {
            const int x = e / kBlkCap, y = e - x * kBlkCap;
            LJ[e] = (x < nsC && y <= x) ? P.GB[(size_t)sm.sidx[1][x] * n + sm.sidx[1][y]] : 0.0;
        }
        if (tid < nsR) sm.diag[0][tid] = P.GA[(size_t)sm.sidx[0][tid] * (m + 1)];
        else if (tid >= kWave && tid < kWave + nsC)
            sm.diag[1][tid - kWave] = P.GB[(size_t)sm.sidx[1][tid - kWave] * (n + 1)];
        __syncthreads();
        B2_PHASE(kB2Gram);
        // One wave per Gram block (wave 0: A_I A_I^T, wave 1: B_J^T B_J), no
        // block barrier per pivot. Lane l holds row r = l / 2 of the block,
        // the entries of columns of parity h = l % 2, in registers.
        // Trailing update of pivot c: G[r][q] -= G[r][c] G[q][c] / d_c for
        // c < q <= r (d_c the pivot, kept or skipped as above). Pivots go in
        // pairs (c, c + 1), whose columns sit in the same register of the
        // two parities: both columns go to LDS at once, and every lane forms
        // column c + 1 after pivot c's update itself (the same expression
        // the owning lanes evaluate), so the second pivot needs no second
        // round trip; each entry then takes the two terms in pivot order.
        if (wv < 2) {
            const int side = wv, ns = side ? nsC : nsR;
            double* G = side ? LJ : LI;
            double* ca = colbuf + side * 2 * kBlkCap;   // column c
            double* cb = ca + kBlkCap;                  // column c + 1
            const int r = lane >> 1, h = lane & 1;
            double gr[kBlkCap / 2];
#pragma unroll
            for (int i = 0; i < kBlkCap / 2; ++i) gr[i] = (r < ns) ? G[r * kBlkCap + 2 * i + h] : 0.0;
            const double tau = P.tau;
#pragma unroll
            for (int c = 0; c < kBlkCap; c += 2) {
                if (c < ns) {
                    (h ? cb : ca)[r] = gr[c >> 1];
                    wave_lds_sync();
                    const bool two = c + 1 < ns;
                    const double d0 = ca[c];
                    const bool k0 = d0 > tau * sm.diag[side][c];
                    const double f0 = k0 ? 1.0 / d0 : 0.0;
                    // Column c + 1 after pivot c (exact zero term if skipped).
                    const double g10 = ca[c + 1];
                    auto col1 = [&](int q) { return __builtin_fma(-(ca[q] * g10), f0, cb[q]); };
                    const double d1 = col1(c + 1);
                    const bool k1 = two && d1 > tau * sm.diag[side][two ? c + 1 : c];
                    const double f1 = k1 ? 1.0 / d1 : 0.0;
                    if (lane == 0) {
                        sm.keep[side][c] = k0;
                        sm.dpiv[side][c] = d0;
                        if (two) {
                            sm.keep[side][c + 1] = k1;
                            sm.dpiv[side][c + 1] = d1;
                        }
                    }
                    // Entries outside c < q <= r < ns (c + 1 < q for the
                    // second pivot) take a zero factor: exact zero terms.
                    const double grc = ca[r];
                    const double grc1 = col1(r);
                    if (h == 1 && c + 1 <= r && r < ns) gr[c >> 1] = grc1;
#pragma unroll
                    for (int i = (c >> 1) + 1; i < kBlkCap / 2; ++i) {
                        const int qq = 2 * i + h;
                        const bool in = qq <= r && r < ns;
                        const double a0 = in ? f0 : 0.0, a1 = in ? f1 : 0.0;
                        gr[i] = __builtin_fma(-(grc * ca[qq]), a0, gr[i]);
                        gr[i] = __builtin_fma(-(grc1 * col1(qq)), a1, gr[i]);
                    }
                    wave_lds_sync();
                }
            }
            if (r < ns) {
#pragma unroll
                for (int i = 0; i < kBlkCap / 2; ++i) G[r * kBlkCap + 2 * i + h] = gr[i];
            }
        }
        __syncthreads();
        B2_PHASE(kB2Chol);
        // Compact the kept candidates into I, J and their Cholesky factors.
        if (tid == 0) {
            int r = 0;
            for (int c = 0; c < nsR; ++c)
                if (sm.keep[0][c]) sm.I[r++] = c;   // positions for now
            sm.nI = r;
            r = 0;
            for (int c = 0; c < nsC; ++c)
                if (sm.keep[1][c]) sm.J[r++] = c;
            sm.nJ = r;
        }
        __syncthreads();
        const int nI = sm.nI, nJ = sm.nJ;
        {
            // The factors L (L[x][y] = G[px][py] / sqrt(d_py) for y < x, with
            // L[x][x] = sqrt(d_px)) enter the solves only through the products
            // L[x][y] / L[y][y] (forward) and L[x][y] / L[x][x] (backward),
            // which are formed here: M[a][b] = L[max(a, b)][min(a, b)] / L[b][b]
            // for a != b, zero on the diagonal and outside the block, stored
            // transposed (row b holds column b of M, the factors of pivot b);
            // rd[x] = 1 / L[x][x] (zero past the block).
            double mv[2][2];
#pragma unroll
            for (int side = 0; side < 2; ++side) {
                const double* G = side ? LJ : LI;
                const int* pos = side ? sm.J : sm.I;
                const int nk = side ? nJ : nI;
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    const int e = tid + u * kThreads, b = e / kBlkCap, a = e - b * kBlkCap;
                    double v = 0.0;
                    if (a < nk && b < nk && a != b) {
                        const int ph = pos[max(a, b)], pl = pos[min(a, b)];
                        const double l = G[ph * kBlkCap + pl] / sqrt(sm.dpiv[side][pl]);
                        v = l * (1.0 / sqrt(sm.dpiv[side][pos[b]]));
                    }
                    mv[side][u] = v;
                }
            }
            __syncthreads();
#pragma unroll
            for (int side = 0; side < 2; ++side) {
                double* G = side ? LJ : LI;
                const int ne = (side ? tcap : scap) * kBlkCap;
#pragma unroll
                for (int u = 0; u < 2; ++u)
                    if (tid + u * kThreads < ne) G[tid + u * kThreads] = mv[side][u];
            }
            if (tid < kBlkCap) {
                sm.rd[0][tid] = tid < nI ? 1.0 / sqrt(sm.dpiv[0][sm.I[tid]]) : 0.0;
                if (tid < nI) sm.I[tid] = sm.sidx[0][sm.I[tid]];
            } else if (tid >= kWave && tid < kWave + kBlkCap) {
                const int y = tid - kWave;
                sm.rd[1][y] = y < nJ ? 1.0 / sqrt(sm.dpiv[1][sm.J[y]]) : 0.0;
                if (y < nJ) sm.J[y] = sm.sidx[1][sm.J[y]];
            }
            __syncthreads();
        }
        last_nI = nI;
        if (g == 0 && k < P.hist_cap) {
            if (P.rows_hist && tid < scap) P.rows_hist[k * scap + tid] = (tid < nI) ? sm.I[tid] : -1;
            if (P.cols_hist && tid >= kWave && tid < kWave + tcap) {
                const int y = tid - kWave;
                P.cols_hist[k * tcap + y] = (y < nJ) ? sm.J[y] : -1;
            }
        }
        if (nI == 0 || nJ == 0) { status = kEInval; break; }
        B2_PHASE(kB2Factor);

        fresh();
        double bX0 = 0.0;   // fetch_bX(0) of this thread (zero below kBxT0)
        static_assert(kBxT0 >= kInvWaves * kWave, "the inverting waves hold no B entries");
        if (wv < kInvWaves) {
            // ---- The inverses of the Gram blocks, G_I^{-1} by wave 0 and
            // G_J^{-1} by wave 1, while the other waves exchange R_IJ: lane y
            // < 32 solves G e = e_y with the factor (forward sweep over L,
            // pivots ascending, scaling by 1 / L[x][x], backward sweep over
            // L^T, pivots descending, scaling again). Right-looking: pivot x
            // subtracts M[r][x] e[x] from every later entry r, independent
            // multiply-adds whose factors are one contiguous row of the
            // stored M^T. Column y is written over column y of the factor's
            // own LDS rows once the whole wave is past its last factor read
            // (the lanes run in lockstep and every read was consumed); it is
            // zero outside the block (the unit entry of y past the block
            // meets only zero factors and a zero scale), and the rows past
            // the factor's capacity are zero, so they are not stored.
            const int side = __builtin_amdgcn_readfirstlane(wv);   // uniform: scalar branches
            double* const Mt = side ? LJ : LI;
            const int nk = side ? nJ : nI, cap = side ? tcap : scap;
            if (lane < kBlkCap) {
                double ev[kBlkCap];
#pragma unroll
                for (int x = 0; x < kBlkCap; ++x) ev[x] = (x == lane) ? 1.0 : 0.0;
                tri_sweep<true>(ev, Mt, nk, cap);
#pragma unroll
                for (int r = 0; r < kBlkCap; ++r) ev[r] *= sm.rd[side][r];
                tri_sweep<false>(ev, Mt, nk, cap);
#pragma unroll
                for (int r = 0; r < kBlkCap; ++r) ev[r] *= sm.rd[side][r];
                wave_lds_sync();
#pragma unroll
                for (int x = 0; x < kBlkCap; ++x)
                    if (x < cap) Mt[x * kBlkCap + lane] = ev[x];
            }
        } else {
            const int xt = tid - kInvWaves * kWave;
            constexpr int kXT = kThreads - kInvWaves * kWave;
            static_assert(kXT >= kChunk * kBlkCap, "one (A A^T)_{i, I} entry per exchanging thread");
            // Operands of the X and R updates that need only I and J, fetched
            // first (ahead of the stores below) and in flight while R_IJ is.
            const double gaI0 = fetch_gaI(0, nI, xt);
            bX0 = fetch_bX(0, nJ);
            // ---- D. R_IJ from the owners of the rows in I. Every word of the
            // s_cap x t_cap block is rewritten every step (zeros outside I x J;
            // work-group 0 writes the rows past nI), so no word can keep a value
            // from four steps back that carries the current 2-bit tag.
            for (int e = xt; e < scap * tcap; e += kXT) {
                const int x = e / tcap, y = e - x * tcap;
                if (x < nI) {
                    const int i = sm.I[x];
                    if (i >= row0 && i < row0 + nrow) {
                        const double v = (y < nJ) ? Rown[(size_t)(i - row0) * n + sm.J[y]] : 0.0;
                        xstore(&ex[x * kBlkCap + y], pack_word(v, tag));
                    }
                } else if (g == 0) {
                    xstore(&ex[x * kBlkCap + y], pack_word(0.0, tag));
                }
            }
            for (int e0 = xt; e0 < nI * nJ; e0 += kXT * 2) {
                const xword* ptr[2];
                int cnt = 0;
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    const int e = e0 + u * kXT;
                    const int x = (e < nI * nJ) ? e / nJ : 0, y = (e < nI * nJ) ? e - x * nJ : 0;
                    ptr[u] = ex + x * kBlkCap + y;
                    cnt += (e < nI * nJ);
                }
                double vals[2];
                if (!poll_gather<double, 2>(ptr, cnt, tag, vals, P.sync, P.poll_sleep)) sm.fail = 1;
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    const int e = e0 + u * kXT;
                    if (u < cnt) E[(e / nJ) * ldE + (e % nJ)] = vals[u];
                }
            }
            if (xt < kChunk * kBlkCap) gaI[xt] = gaI0;
        }
        __syncthreads();
        if (sm.fail) { ok = false; break; }
        B2_PHASE(kB2E);
        fresh();
        // W = (A_I A_I^T)^{-1} R_IJ (B_J^T B_J)^{-1} from the two inverses
        // (GI = G_I^{-1} over the factor L_I's rows, GJ = G_J^{-1} over
        // L_J's, row-major): W1 = G_I^{-1} R_IJ, then W = W1 G_J^{-1}, each
        // entry a sum over the block in index order by one thread, two
        // entries per thread (a wave: two rows x, 32 consecutive y), written
        // over E once every thread has read it. W is zero outside nI x nJ.
        {
            const double* GI = LI;
            const double* GJ = LJ;
            double wv2[2];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int e = tid + u * kThreads, x = e / kBlkCap, y = e - x * kBlkCap;
                double acc = 0.0;
                if (x < nI && y < nJ)
                    for (int z = 0; z < nI; ++z) acc += GI[x * kBlkCap + z] * E[z * ldE + y];
                wv2[u] = acc;
            }
            __syncthreads();
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int e = tid + u * kThreads, x = e / kBlkCap, y = e - x * kBlkCap;
                E[x * ldE + y] = wv2[u];
            }
            __syncthreads();
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int e = tid + u * kThreads, x = e / kBlkCap, y = e - x * kBlkCap;
                double acc = 0.0;
                if (x < nI && y < nJ)
                    for (int z = 0; z < nJ; ++z) acc += E[x * ldE + z] * GJ[z * kBlkCap + y];
                wv2[u] = acc;
            }
            __syncthreads();
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int e = tid + u * kThreads, x = e / kBlkCap, y = e - x * kBlkCap;
                E[x * ldE + y] = wv2[u];
            }
        }
        __syncthreads();
        fresh();
        // ---- X and R updates; A of step k + 1.
        B2_PHASE(kB2W);
        update_x(nI, nJ, bX0);
        B2_PHASE(kB2X);
        const unsigned int ntag = seq_tag(k + 1);
        fresh();
        update_and_score(true, nI, nJ, ntag);
        if (tid == 0) {
            double e = 0.0;
            for (int w2 = 0; w2 < kWaves; ++w2) e += sm.err_w[w2];
            xstore(&px[g], pack_word(e, ntag));
        }
        __syncthreads();
        B2_PHASE(kB2R);
        ++k;
    }
#undef B2_PHASE
    if (sm.fail) status = kETimeout;
    if (timing)
        for (int i = 0; i < kB2Count; ++i) P.phase[i] += sm.ph[i];
    if (g == 0 && tid == 0) {
        P.report->iters = k;
        P.report->status = status;
        P.report->last_set = last_nI;
        P.report->S = S;
        P.report->err = err;
    }
}

size_t block2_lds_bytes(int rpw, int n, int W, int s_cap, int t_cap, bool r_in_lds) {
    const int ncs = (n + W - 1) / W;
    size_t b = r_in_lds ? (((size_t)rpw * n * 8 + 15) & ~(size_t)15) : 0;
    b += block2_ereg_bytes(ncs);
    b += ((size_t)block2_fac_doubles(s_cap, t_cap) + (size_t)kChunk * kBlkCap) * 8;
    return b;
}

size_t block2_lds_budget() { return 160 * 1024 - sizeof(Blk2Smem) - 256; }

template <int SR, bool LDS>
static hipError_t launch_b2(const Block2Params& P, size_t lds_bytes, hipStream_t s) {
    auto kern = block2_kernel<SR, LDS>;
    if (hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds_bytes) != hipSuccess)
        (void)hipGetLastError();
    Block2Params copy = P;
    void* args[] = {&copy};
    if (P.W == 1)
        return hipLaunchKernel((const void*)kern, dim3(1), dim3(kThreads), args, lds_bytes, s);
    return hipLaunchCooperativeKernel((const void*)kern, dim3(P.W), dim3(kThreads), args,
                                      (unsigned int)lds_bytes, s);
}

template <bool LDS>
static hipError_t launch_b2_sr(const Block2Params& P, size_t lds_bytes, hipStream_t s) {
    switch (sel_rows_for(P.m > P.n ? P.m : P.n)) {
        case 1: return launch_b2<1, LDS>(P, lds_bytes, s);
        case 2: return launch_b2<2, LDS>(P, lds_bytes, s);
        case 4: return launch_b2<4, LDS>(P, lds_bytes, s);
        case 8: return launch_b2<8, LDS>(P, lds_bytes, s);
        default: return launch_b2<16, LDS>(P, lds_bytes, s);
    }
}

hipError_t launch_block2(const Block2Params& P, size_t lds_bytes, hipStream_t s) {
    return P.r_in_lds ? launch_b2_sr<true>(P, lds_bytes, s) : launch_b2_sr<false>(P, lds_bytes, s);
}

}  // namespace mek
