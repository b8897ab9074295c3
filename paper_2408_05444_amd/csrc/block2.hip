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
        for (int e = tid; e < 1024; e += kThreads) hist[e] = 0;
        if (tid == 0) {
            sm.prefix[0] = sm.prefix[1] = 0ull;
            sm.need[0] = min(capR, totR);
            sm.need[1] = min(capC, totC);
        }
        __syncthreads();
        for (int d = 7; d >= 0; --d) {
            int* H = hist + (d & 1) * 512;
            const int sh = 8 * d;
            const unsigned long long pR = sm.prefix[0], pC = sm.prefix[1];
#pragma unroll
            for (int j = 0; j < SR; ++j) {
                if (radR && j < rc && kr[j] != 0ull &&
                    (d == 7 || (kr[j] >> (sh + 8)) == (pR >> (sh + 8))))
                    atomicAdd(&H[(int)((kr[j] >> sh) & 255ull)], 1);
                if (radC && j < cc && kc[j] != 0ull &&
                    (d == 7 || (kc[j] >> (sh + 8)) == (pC >> (sh + 8))))
                    atomicAdd(&H[256 + (int)((kc[j] >> sh) & 255ull)], 1);
            }
            __syncthreads();
            if (wv < 2 && (wv == 0 ? radR : radC)) {
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

template <int SR>
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
    // slice] [L_I] [L_J] [z: kChunk x tcap].
    const size_t r_bytes = P.r_in_lds ? (((size_t)P.rpw * n * 8 + 15) & ~(size_t)15) : 0;
    double* Rl = reinterpret_cast<double*>(dyn_smem);
    unsigned char* ereg = dyn_smem + r_bytes;
    double* E = reinterpret_cast<double*>(ereg);
    int* hist = reinterpret_cast<int*>(ereg);
    unsigned long long* slice = reinterpret_cast<unsigned long long*>(ereg);
    const size_t e_bytes = block2_ereg_bytes(scap, tcap, ncs);
    double* LI = reinterpret_cast<double*>(ereg + e_bytes);
    double* LJ = LI + scap * scap;
    double* z = LJ + tcap * tcap;
    double* Rown = P.r_in_lds ? Rl : P.R + (size_t)row0 * n;

    if (P.r_in_lds) {
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
                // z_i = (A A^T)_{i, I} W for the chunk's rows.
                for (int e = tid; e < cr * nJ; e += kThreads) {
                    const int ii = e / nJ, y = e - ii * nJ;
                    const double* ga = P.GA + (size_t)(row0 + c0 + ii) * m;
                    double acc = 0.0;
                    for (int x = 0; x < sm.nI; ++x) acc += ga[sm.I[x]] * E[x * ldE + y];
                    z[ii * tcap + y] = acc;
                }
                __syncthreads();
            }
            double aa[kChunk];
#pragma unroll
            for (int ii = 0; ii < kChunk; ++ii) aa[ii] = (ii < cr) ? P.a[row0 + c0 + ii] : 0.0;
            double v[2 * kChunk];
#pragma unroll
            for (int ii = 0; ii < kChunk; ++ii) {
                v[ii] = 0.0;            // ||R_i||^2 partial
                v[kChunk + ii] = 0.0;   // max_j omega_ij partial
            }
            // Columns in groups of 4 per thread: each z value read from LDS
            // serves the group's four columns.
#pragma unroll
            for (int u0 = 0; u0 < SR; u0 += 4) {
                double acc[4][kChunk];
#pragma unroll
                for (int u = 0; u < 4; ++u)
#pragma unroll
                    for (int ii = 0; ii < kChunk; ++ii) acc[u][ii] = 0.0;
                if (upd) {
#pragma unroll 2
                    for (int y = 0; y < nJ; ++y) {
                        const double* gbr = P.GB + (size_t)sm.J[y] * n;
                        double gb[4];
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            const int j = tid + (u0 + u) * kThreads;
                            gb[u] = (u0 + u < SR && j < n) ? gbr[j] : 0.0;
                        }
#pragma unroll
                        for (int ii = 0; ii < kChunk; ++ii) {
                            const double zv = z[ii * tcap + y];
#pragma unroll
                            for (int u = 0; u < 4; ++u) acc[u][ii] += zv * gb[u];
                        }
                    }
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int j = tid + (u0 + u) * kThreads;
                    if (u0 + u < SR && j < n) {
                        const double bj = P.b[j];
                        double cmu = cm[u0 + u < SR ? u0 + u : 0];
#pragma unroll
                        for (int ii = 0; ii < kChunk; ++ii) {
                            if (ii < cr) {
                                double* rp = Rown + (size_t)(c0 + ii) * n + j;
                                double val = *rp;
                                if (upd) {
                                    val -= acc[u][ii];
                                    *rp = val;
                                }
                                const double sq = val * val;
                                v[ii] += sq;
                                if (aa[ii] > 0.0 && bj > 0.0) {
                                    const double w = sq / (aa[ii] * bj);
                                    v[kChunk + ii] = fmax(v[kChunk + ii], w);
                                    cmu = fmax(cmu, w);
                                }
                            }
                        }
                        if (u0 + u < SR) cm[u0 + u] = cmu;
                    }
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

    // X^T rows of this work-group: X^T[l, :] += sum_x c_x A_{I_x, :} with
    // c_x = sum_y W[x][y] B[l][J_y]; returns nothing, leaves the error
    // partial of the updated rows in sm.err_w (one per wave).
    auto update_x = [&](int nI, int nJ) {
        double ep = 0.0;
        for (int l = wv; l < nx; l += kWaves) {
            const int lr = xc0 + l;
            double cx_ = 0.0;
            if (lane < nI) {
                for (int y = 0; y < nJ; ++y) cx_ += E[lane * ldE + y] * P.B[(size_t)lr * n + sm.J[y]];
            }
            double* xr = P.Xt + (size_t)lr * p;
            const double* xref = P.Xref_t ? P.Xref_t + (size_t)lr * p : nullptr;
            for (int s0 = 0; s0 < p; s0 += kWave) {
                const int s = s0 + lane;
                double acc = 0.0;
                for (int x = 0; x < nI; ++x) {
                    const double c = readlane_d(cx_, x);
                    if (s < p) acc += c * P.A[(size_t)sm.I[x] * p + s];
                }
                if (s < p) {
                    const double nv = xr[s] + acc;
                    xr[s] = nv;
                    if (xref) {
                        const double d = nv - xref[s];
                        ep += d * d;
                    }
                }
            }
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
        select_top<SR>(kr, rb, rcnt, kc, cb, ccnt, scap, tcap, hist, sm);
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
            // G[c1][c2] -= G[c1][c] G[c2][c] / d for c < c2 <= c1.
            const int lr = keepR ? nsR - c - 1 : 0, lc = keepC ? nsC - c - 1 : 0;
            const int tr = lr * (lr + 1) / 2, tcn = lc * (lc + 1) / 2;
            for (int e = tid; e < tr + tcn; e += kThreads) {
                const bool isR = e < tr;
                const int f = isR ? e : e - tr;
                // f -> (r1, r2) with 0 <= r2 <= r1 in a lower triangle.
                int r1 = (int)((sqrt(8.0 * f + 1.0) - 1.0) * 0.5);
                while ((r1 + 1) * (r1 + 2) / 2 <= f) ++r1;
                while (r1 * (r1 + 1) / 2 > f) --r1;
                const int r2 = f - r1 * (r1 + 1) / 2;
                const int c1 = c + 1 + r1, c2 = c + 1 + r2;
                double* L = isR ? LI : LJ;
                const int ld = isR ? scap : tcap;
                const double d = isR ? dR : dC;
                L[c1 * ld + c2] -= L[c1 * ld + c] * L[c2 * ld + c] / d;
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
            if (tid < nI) sm.I[tid] = sm.sidx[0][sm.I[tid]];
            else if (tid >= kWave && tid < kWave + nJ) sm.J[tid - kWave] = sm.sidx[1][sm.J[tid - kWave]];
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

        // ---- D. R_IJ from the owners of the rows in I.
        for (int e = tid; e < nI * nJ; e += kThreads) {
            const int x = e / nJ, y = e - x * nJ;
            const int i = sm.I[x];
            if (i >= row0 && i < row0 + nrow)
                xstore(&ex[x * kBlkCap + y], pack_word(Rown[(size_t)(i - row0) * n + sm.J[y]], tag));
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
        // W = (A_I A_I^T)^{-1} R_IJ (B_J^T B_J)^{-1}, in place in E: first the
        // columns (lane y solves with L_I), then the rows (lane x with L_J).
        if (wv == 0 && lane < nJ) {
            const int y = lane;
            for (int x = 0; x < nI; ++x) {
                double v = E[x * ldE + y];
                for (int x2 = 0; x2 < x; ++x2) v -= LI[x * scap + x2] * E[x2 * ldE + y];
                E[x * ldE + y] = v / LI[x * scap + x];
            }
            for (int x = nI - 1; x >= 0; --x) {
                double v = E[x * ldE + y];
                for (int x2 = x + 1; x2 < nI; ++x2) v -= LI[x2 * scap + x] * E[x2 * ldE + y];
                E[x * ldE + y] = v / LI[x * scap + x];
            }
        }
        __syncthreads();
        if (wv == 0 && lane < nI) {
            const int x = lane;
            for (int y = 0; y < nJ; ++y) {
                double v = E[x * ldE + y];
                for (int y2 = 0; y2 < y; ++y2) v -= LJ[y * tcap + y2] * E[x * ldE + y2];
                E[x * ldE + y] = v / LJ[y * tcap + y];
            }
            for (int y = nJ - 1; y >= 0; --y) {
                double v = E[x * ldE + y];
                for (int y2 = y + 1; y2 < nJ; ++y2) v -= LJ[y2 * tcap + y] * E[x * ldE + y2];
                E[x * ldE + y] = v / LJ[y * tcap + y];
            }
        }
        __syncthreads();
        // ---- X and R updates; A of step k + 1.
        update_x(nI, nJ);
        const unsigned int ntag = seq_tag(k + 1);
        update_and_score(true, nJ, ntag);
        if (tid == 0) {
            double e = 0.0;
            for (int w2 = 0; w2 < kWaves; ++w2) e += sm.err_w[w2];
            xstore(&px[g], pack_word(e, ntag));
        }
        __syncthreads();
        ++k;
    }
    if (sm.fail) status = kETimeout;
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
    b += ((size_t)s_cap * s_cap + (size_t)t_cap * t_cap + (size_t)kChunk * t_cap) * 8;
    return b;
}

size_t block2_lds_budget() { return 160 * 1024 - sizeof(Blk2Smem) - 256; }

template <int SR>
static hipError_t launch_b2(const Block2Params& P, size_t lds_bytes, hipStream_t s) {
    auto kern = block2_kernel<SR>;
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

hipError_t launch_block2(const Block2Params& P, size_t lds_bytes, hipStream_t s) {
    switch (sel_rows_for(P.m > P.n ? P.m : P.n)) {
        case 1: return launch_b2<1>(P, lds_bytes, s);
        case 2: return launch_b2<2>(P, lds_bytes, s);
        case 4: return launch_b2<4>(P, lds_bytes, s);
        case 8: return launch_b2<8>(P, lds_bytes, s);
        default: return launch_b2<16>(P, lds_bytes, s);
    }
}

}  // namespace mek
