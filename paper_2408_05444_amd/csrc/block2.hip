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
//      factors A_I A_I^T and B_J^T B_J;
//   D. the owners of the rows in I publish R_IJ; with it every work-group
//      forms W, updates its columns of X, then its rows of R together with
//      the next step's row words and column maxima (A of step k + 1).
// Reading every row word before publishing its column slice (B) makes every
// rewrite of a buffer causally after all reads of its previous contents,
// so one buffer per kind suffices.
#include "exchange.h"
#include "internal.h"

#include <math.h>

namespace mek {

namespace {

constexpr int kChunk = 4;   // rows of R per pass of the fused update/score loop
constexpr int kXRows = 8;   // rows of X^T per pass of the X update

// Optional phase timing (work-group 0, thread 0): wall-clock ticks per phase
// of a step, summed over the solve.
enum { kB2Rows, kB2Cols, kB2Select, kB2Factor, kB2E, kB2W, kB2X, kB2R, kB2Count };

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
    int nsel[2];
    int nI, nJ;
    int fail;
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
        const int dstart = max(startR, startC);
        for (int d = dstart; d >= 0; --d) {
            int* H = hist + (d & 1) * 512;
            const int sh = 8 * d;
            const unsigned long long pR = sm.prefix[0], pC = sm.prefix[1];
            const bool inR = radR && d <= startR, inC = radC && d <= startC;
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
                    }
                    run += c4[u];
                }
            } else if (wv == 2) {
                int* Hn = hist + ((d + 1) & 1) * 512;
                for (int e = lane; e < 512; e += kWave) Hn[e] = 0;
            }
            __syncthreads();
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
    if (wv < 2) {
        const int ns = sm.nsel[wv];
        if (lane < ns) {
            const unsigned long long key = sm.ukey[wv][lane];
            const int idx = sm.uidx[wv][lane];
            int rank = 0;
            for (int u = 0; u < ns; ++u) {
                const unsigned long long ku = sm.ukey[wv][u];
                rank += (ku > key) || (ku == key && sm.uidx[wv][u] < idx);
            }
            sm.sidx[wv][rank] = idx;
            sm.skey[wv][rank] = key;
        }
    }
    __syncthreads();
}

}  // namespace

template <int SR, bool LDS>
__global__ void __launch_bounds__(kThreads, 1) block2_kernel(Block2Params P) {
    extern __shared__ __align__(16) unsigned char dyn_smem[];
    __shared__ Blk2Smem sm;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
    if (tid == 0) sm.fail = 0;

    const int W = P.W, g = blockIdx.x;
    const int m = P.m, n = P.n, p = P.p, q = P.q;
    const int scap = P.s_cap, tcap = P.t_cap, ldE = tcap + 1;
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

    // LDS: [own rows of R] [E / W, also radix histograms and the column
    // slice] [L_I] [L_J] [z: kChunk x tcap] [(A A^T)_{i, I}: kChunk x kBlkCap]
    // [c of the X update: kXRows x kBlkCap].
    const size_t r_bytes = LDS ? (((size_t)P.rpw * n * 8 + 15) & ~(size_t)15) : 0;
    double* Rl = reinterpret_cast<double*>(dyn_smem);
    unsigned char* ereg = dyn_smem + r_bytes;
    double* E = reinterpret_cast<double*>(ereg);
    int* hist = reinterpret_cast<int*>(ereg);
    unsigned long long* slice = reinterpret_cast<unsigned long long*>(ereg);
    const size_t e_bytes = block2_ereg_bytes(scap, tcap, ncs);
    double* LI = reinterpret_cast<double*>(ereg + e_bytes);
    double* LJ = LI + scap * scap;
    double* z = LJ + tcap * tcap;
    double* gaI = z + kChunk * tcap;                   // kChunk x kBlkCap
    double* cX = gaI + kChunk * kBlkCap;               // kXRows x kBlkCap
    // Own rows of R: LDS or device memory, fixed at compile time so that
    // every access is a plain LDS or global instruction.
    double* Rown = LDS ? Rl : P.R + (size_t)row0 * n;

    if (LDS) {
        const double* src = P.R + (size_t)row0 * n;
        const size_t tot = (size_t)nrow * n;
        for (size_t e = tid; e < tot; e += kThreads) Rl[e] = src[e];
        __syncthreads();
    }

    // Fused pass over own rows: optional update R_i -= z_i (B^T B)_{J,:}, then
    // ||R_i||^2, max_j omega_ij and this work-group's column maxima; publishes
    // the row words and column maxima with `tag`. Thread t handles columns
    // t, t + kThreads, ... (coalesced), kChunk rows at a time.
    auto update_and_score = [&](bool upd, int nJ, unsigned int tag) {
        double cm[SR];
#pragma unroll
        for (int u = 0; u < SR; ++u) cm[u] = 0.0;
        for (int c0 = 0; c0 < nrow; c0 += kChunk) {
            const int cr = min(kChunk, nrow - c0);
            if (upd) {
                // z_i = (A A^T)_{i, I} W for the chunk's rows: the entries
                // (A A^T)_{i, I} are loaded once, all in flight together.
                const int nI = sm.nI;
                for (int e = tid; e < cr * nI; e += kThreads) {
                    const int ii = e / nI, x = e - ii * nI;
                    gaI[ii * kBlkCap + x] = P.GA[(size_t)(row0 + c0 + ii) * m + sm.I[x]];
                }
                __syncthreads();
                for (int e = tid; e < cr * nJ; e += kThreads) {
                    const int ii = e / nJ, y = e - ii * nJ;
                    double a0 = 0.0, a1 = 0.0;
                    int x = 0;
                    for (; x + 1 < nI; x += 2) {
                        a0 += gaI[ii * kBlkCap + x] * E[x * ldE + y];
                        a1 += gaI[ii * kBlkCap + x + 1] * E[(x + 1) * ldE + y];
                    }
                    if (x < nI) a0 += gaI[ii * kBlkCap + x] * E[x * ldE + y];
                    z[ii * tcap + y] = a0 + a1;
                }
                __syncthreads();
            }
            if (upd) {
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
                    // before the multiply-adds that use them.
                    for (int y0 = 0; y0 < nJ; y0 += 8) {
                        double gb[8][4];
#pragma unroll
                        for (int yy = 0; yy < 8; ++yy) {
                            const int y = y0 + yy;
                            const double* gbr = P.GB + (size_t)sm.J[y < nJ ? y : 0] * n;
#pragma unroll
                            for (int u = 0; u < 4; ++u) {
                                const int j = tid + (u0 + u) * kThreads;
                                gb[yy][u] = (y < nJ && u0 + u < SR && j < n) ? gbr[j] : 0.0;
                            }
                        }
#pragma unroll
                        for (int yy = 0; yy < 8; ++yy) {
                            if (y0 + yy < nJ) {
#pragma unroll
                                for (int ii = 0; ii < kChunk; ++ii) {
                                    const double zv = z[ii * tcap + y0 + yy];
#pragma unroll
                                    for (int u = 0; u < 4; ++u) acc[u][ii] += zv * gb[yy][u];
                                }
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
            // Norms, row maxima and column maxima of omega over the chunk's
            // rows (the same thread's columns, so no barrier is needed).
            double aa[kChunk];
#pragma unroll
            for (int ii = 0; ii < kChunk; ++ii) aa[ii] = (ii < cr) ? P.a[row0 + c0 + ii] : 0.0;
            double v[2 * kChunk];
#pragma unroll
            for (int ii = 0; ii < kChunk; ++ii) {
                v[ii] = 0.0;            // ||R_i||^2 partial
                v[kChunk + ii] = 0.0;   // max_j omega_ij partial
            }
#pragma unroll
            for (int u = 0; u < SR; ++u) {
                const int j = tid + u * kThreads;
                if (j < n) {
                    const double bj = P.b[j];
                    double cmu = cm[u];
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
                    cm[u] = cmu;
                }
            }
            block_sums_maxes<kChunk, kChunk>(v, sm);
#pragma unroll
            for (int ii = 0; ii < kChunk; ++ii) {
                if (ii < cr && tid == ii) xstore(&rx[row0 + c0 + ii], pack_word(v[ii], tag));
                if (ii < cr && tid == kChunk + ii)
                    xstore(&hx[row0 + c0 + ii], pack_word(v[kChunk + ii], tag));
            }
        }
#pragma unroll
        for (int u = 0; u < SR; ++u) {
            const int j = tid + u * kThreads;
            if (j < n) xstore(&cx[(size_t)g * n + j], pack_word(cm[u], tag));
        }
    };

    // X^T rows of this work-group, kXRows at a time:
    //   c[l][x] = sum_y W[x][y] B[l][J_y] (LDS), then
    //   X^T[l, s] += sum_x c[l][x] A[I_x][s], a thread per column s,
    // with the entries of A loaded 8 at a time, all in flight together.
    // Leaves the squared-error partial of the updated rows in sm.err_w.
    auto update_x = [&](int nI, int nJ) {
        double ep = 0.0;
        for (int l0 = 0; l0 < nx; l0 += kXRows) {
            const int lc = min(kXRows, nx - l0);
            for (int e = tid; e < lc * nI; e += kThreads) {
                const int l = e / nI, x = e - l * nI;
                const double* brow = P.B + (size_t)(xc0 + l0 + l) * n;
                double a0 = 0.0, a1 = 0.0;
                for (int y0 = 0; y0 < nJ; y0 += 8) {
                    double bv[8];
#pragma unroll
                    for (int yy = 0; yy < 8; ++yy)
                        bv[yy] = (y0 + yy < nJ) ? brow[sm.J[y0 + yy]] : 0.0;
#pragma unroll
                    for (int yy = 0; yy < 8; yy += 2) {
                        if (y0 + yy < nJ) a0 += E[x * ldE + y0 + yy] * bv[yy];
                        if (y0 + yy + 1 < nJ) a1 += E[x * ldE + y0 + yy + 1] * bv[yy + 1];
                    }
                }
                cX[l * kBlkCap + x] = a0 + a1;
            }
            __syncthreads();
            for (int s2 = tid; s2 < p; s2 += kThreads) {
                double acc[kXRows];
#pragma unroll
                for (int l = 0; l < kXRows; ++l) acc[l] = 0.0;
                for (int x0 = 0; x0 < nI; x0 += 8) {
                    double av[8];
#pragma unroll
                    for (int xx = 0; xx < 8; ++xx)
                        av[xx] = (x0 + xx < nI) ? P.A[(size_t)sm.I[x0 + xx] * p + s2] : 0.0;
#pragma unroll
                    for (int xx = 0; xx < 8; ++xx) {
                        if (x0 + xx < nI) {
#pragma unroll
                            for (int l = 0; l < kXRows; ++l) acc[l] += cX[l * kBlkCap + x0 + xx] * av[xx];
                        }
                    }
                }
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
            __syncthreads();
        }
        ep = wave_sum(ep);
        if (lane == 0) sm.err_w[wv] = ep;
    };

    // ---- Set-up: the first row words, column maxima and error partial.
    update_and_score(false, 0, seq_tag(0));
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

    const bool timing = P.phase != nullptr && g == 0 && tid == 0;
    unsigned long long ph[kB2Count] = {0, 0, 0, 0, 0, 0, 0, 0};
    unsigned long long t_last = timing ? wall_clock64() : 0;
#define B2_PHASE(id)                                                    \
    do {                                                                \
        if (timing) {                                                   \
            const unsigned long long now_ = wall_clock64();             \
            ph[id] += now_ - t_last;                                    \
            t_last = now_;                                              \
        }                                                               \
    } while (0)
    const int cs = (max(m, n) + kThreads - 1) / kThreads;   // chunk per thread (<= SR)
    const int rb = min(m, tid * cs), rcnt = min(m, rb + cs) - rb;
    const int cb = min(n, tid * cs), ccnt = min(n, cb + cs) - cb;
    double S0 = -1.0, S = 0.0, err = NAN;
    long long k = 0;
    int status = kMaxIter, last_nI = 0;
    bool ok = true;
    const bool has_ref = P.Xref_t != nullptr;
    while (ok) {
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
        select_top<SR>(kr, rb, rcnt, kc, cb, ccnt, scap, tcap, hist, sm);
        B2_PHASE(kB2Select);
        const int nsR = sm.nsel[0], nsC = sm.nsel[1];
        // Gram blocks of the ranked candidates, then an in-place right-looking
        // Cholesky in rank order that skips dependent candidates.
        for (int e = tid; e < nsR * nsR; e += kThreads) {
            const int x = e / nsR, y = e - x * nsR;
            LI[x * scap + y] = P.GA[(size_t)sm.sidx[0][x] * m + sm.sidx[0][y]];
        }
        for (int e = tid; e < nsC * nsC; e += kThreads) {
            const int x = e / nsC, y = e - x * nsC;
            LJ[x * tcap + y] = P.GB[(size_t)sm.sidx[1][x] * n + sm.sidx[1][y]];
        }
        if (tid < nsR) sm.diag[0][tid] = P.GA[(size_t)sm.sidx[0][tid] * (m + 1)];
        else if (tid >= kWave && tid < kWave + nsC)
            sm.diag[1][tid - kWave] = P.GB[(size_t)sm.sidx[1][tid - kWave] * (n + 1)];
        __syncthreads();
        const int npiv = max(nsR, nsC);
        // Thread t owns entries (t / 32 + 16 h, t % 32), h = 0, 1, of both
        // Gram blocks (at most 32 x 32 each).
        const int er0 = tid >> 5, ec = tid & 31;
        for (int c = 0; c < npiv; ++c) {
            // Every thread reads the pivot and takes the same decision.
            const bool doR = c < nsR, doC = c < nsC;
            const double dR = doR ? LI[c * scap + c] : 0.0;
            const double dC = doC ? LJ[c * tcap + c] : 0.0;
            const bool keepR = doR && dR > P.tau * sm.diag[0][c];
            const bool keepC = doC && dC > P.tau * sm.diag[1][c];
            if (tid == 0) {
                if (doR) { sm.keep[0][c] = keepR; sm.dpiv[0][c] = dR; }
                if (doC) { sm.keep[1][c] = keepC; sm.dpiv[1][c] = dC; }
            }
            // Trailing update of the lower triangle below the pivot:
            // G[r][q] -= G[r][c] G[q][c] / d for c < q <= r.
            if (keepR) {
                const double rdR = 1.0 / dR;
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int r = er0 + 16 * h;
                    if (r < nsR && ec > c && ec <= r)
                        LI[r * scap + ec] -= LI[r * scap + c] * LI[ec * scap + c] * rdR;
                }
            }
            if (keepC) {
                const double rdC = 1.0 / dC;
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int r = er0 + 16 * h;
                    if (r < nsC && ec > c && ec <= r)
                        LJ[r * tcap + ec] -= LJ[r * tcap + c] * LJ[ec * tcap + c] * rdC;
                }
            }
            __syncthreads();
        }
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
            // L[x][y] = G[px][py] / sqrt(d_py) (y < x), sqrt(d_px) on the diagonal.
            double lv[2], lw[2];
            int cntI = 0, cntJ = 0;
            for (int e = tid, u = 0; e < nI * nI && u < 2; e += kThreads, ++u) {
                const int x = e / nI, y = e - x * nI;
                const int px_ = sm.I[x], py_ = sm.I[y];
                lv[u] = (y > x) ? 0.0
                        : (y == x) ? sqrt(sm.dpiv[0][px_])
                                   : LI[px_ * scap + py_] / sqrt(sm.dpiv[0][py_]);
                ++cntI;
            }
            for (int e = tid, u = 0; e < nJ * nJ && u < 2; e += kThreads, ++u) {
                const int x = e / nJ, y = e - x * nJ;
                const int px_ = sm.J[x], py_ = sm.J[y];
                lw[u] = (y > x) ? 0.0
                        : (y == x) ? sqrt(sm.dpiv[1][px_])
                                   : LJ[px_ * tcap + py_] / sqrt(sm.dpiv[1][py_]);
                ++cntJ;
            }
            __syncthreads();
            for (int u = 0; u < cntI; ++u) {
                const int e = tid + u * kThreads, x = e / nI, y = e - x * nI;
                LI[x * scap + y] = lv[u];
            }
            for (int u = 0; u < cntJ; ++u) {
                const int e = tid + u * kThreads, x = e / nJ, y = e - x * nJ;
                LJ[x * tcap + y] = lw[u];
            }
            __syncthreads();
            if (tid < nI) {
                sm.I[tid] = sm.sidx[0][sm.I[tid]];
                sm.rd[0][tid] = 1.0 / LI[tid * scap + tid];
            } else if (tid >= kWave && tid < kWave + nJ) {
                const int y = tid - kWave;
                sm.J[y] = sm.sidx[1][sm.J[y]];
                sm.rd[1][y] = 1.0 / LJ[y * tcap + y];
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

        // ---- D. R_IJ from the owners of the rows in I. Every word of the
        // s_cap x t_cap block is rewritten every step (zeros outside I x J;
        // work-group 0 writes the rows past nI), so no word can keep a value
        // from four steps back that carries the current 2-bit tag.
        for (int e = tid; e < scap * tcap; e += kThreads) {
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
        for (int e0 = tid; e0 < nI * nJ; e0 += kThreads * 2) {
            const xword* ptr[2];
            int cnt = 0;
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int e = e0 + u * kThreads;
                const int x = (e < nI * nJ) ? e / nJ : 0, y = (e < nI * nJ) ? e - x * nJ : 0;
                ptr[u] = ex + x * kBlkCap + y;
                cnt += (e < nI * nJ);
            }
            double vals[2];
            if (!poll_gather<double, 2>(ptr, cnt, tag, vals, P.sync, P.poll_sleep)) sm.fail = 1;
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int e = e0 + u * kThreads;
                if (u < cnt) E[(e / nJ) * ldE + (e % nJ)] = vals[u];
            }
        }
        __syncthreads();
        if (sm.fail) { ok = false; break; }
        B2_PHASE(kB2E);
        // W = (A_I A_I^T)^{-1} R_IJ (B_J^T B_J)^{-1}, in place in E, by
        // right-looking triangular solves over the whole block (one barrier
        // per pivot): first L_I and L_I^T on the columns of E, then L_J and
        // L_J^T on its rows. Entry (x, y) of E belongs to thread
        // (x / 16 + ...), see below; rows are kept unscaled until the end of
        // each sweep.
        {
            // Thread t handles entries (t / 32 + 16 h, t % 32) of E, h = 0, 1.
            const int ex0 = tid >> 5, ey = tid & 31;
            // L_I: forward (E[x'] -= L[x'][x] / L[x][x] * E[x] for x' > x).
            for (int x = 0; x + 1 < nI; ++x) {
                const double rx = sm.rd[0][x];
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int r = ex0 + 16 * h;
                    if (r > x && r < nI && ey < nJ)
                        E[r * ldE + ey] -= LI[r * scap + x] * rx * E[x * ldE + ey];
                }
                __syncthreads();
            }
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int r = ex0 + 16 * h;
                if (r < nI && ey < nJ) E[r * ldE + ey] *= sm.rd[0][r];
            }
            __syncthreads();
            // L_I^T: backward (E[x'] -= L[x][x'] / L[x][x] * E[x] for x' < x).
            for (int x = nI - 1; x > 0; --x) {
                const double rx = sm.rd[0][x];
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int r = ex0 + 16 * h;
                    if (r < x && ey < nJ) E[r * ldE + ey] -= LI[x * scap + r] * rx * E[x * ldE + ey];
                }
                __syncthreads();
            }
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int r = ex0 + 16 * h;
                if (r < nI && ey < nJ) E[r * ldE + ey] *= sm.rd[0][r];
            }
            __syncthreads();
            // L_J on the rows: column y plays the role of row x above.
            for (int y = 0; y + 1 < nJ; ++y) {
                const double ry = sm.rd[1][y];
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int r = ex0 + 16 * h;
                    if (r < nI && ey > y && ey < nJ)
                        E[r * ldE + ey] -= LJ[ey * tcap + y] * ry * E[r * ldE + y];
                }
                __syncthreads();
            }
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int r = ex0 + 16 * h;
                if (r < nI && ey < nJ) E[r * ldE + ey] *= sm.rd[1][ey];
            }
            __syncthreads();
            for (int y = nJ - 1; y > 0; --y) {
                const double ry = sm.rd[1][y];
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int r = ex0 + 16 * h;
                    if (r < nI && ey < y) E[r * ldE + ey] -= LJ[y * tcap + ey] * ry * E[r * ldE + y];
                }
                __syncthreads();
            }
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int r = ex0 + 16 * h;
                if (r < nI && ey < nJ) E[r * ldE + ey] *= sm.rd[1][ey];
            }
            __syncthreads();
        }
        // ---- X and R updates; A of step k + 1.
        B2_PHASE(kB2W);
        update_x(nI, nJ);
        B2_PHASE(kB2X);
        const unsigned int ntag = seq_tag(k + 1);
        update_and_score(true, nJ, ntag);
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
        for (int i = 0; i < kB2Count; ++i) P.phase[i] += ph[i];
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
    b += block2_ereg_bytes(s_cap, t_cap, ncs);
    b += ((size_t)s_cap * s_cap + (size_t)t_cap * t_cap + (size_t)kChunk * t_cap +
          (size_t)kChunk * kBlkCap + (size_t)kXRows * kBlkCap) * 8;
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
