// Persistent solver kernel for the greedy block Kaczmarz family (Algs. 1-5 of
// the paper) on gfx950.
//
// One launch runs the whole iteration for one instance (or, batched, one
// team per instance). The instance is split over a *team* of W co-resident
// work-groups (a cooperative launch):
//   - work-group g owns rows [g*rpw, (g+1)*rpw) of the residual R. When they
//     fit, those rows live in LDS for the whole solve, so R never travels to
//     HBM inside the loop; otherwise they stay in device memory.
//   - it owns rows [g*xpw, ...) of X^T (columns of X; in LDS when there is
//     room) and entries [g*wpw, ...) of the vector w = (R_{i_k} B^T) B.
// Per update k every work-group
//   1. reads all row norms r_i = ||R_i||^2 and computes ||R||_F^2, the
//      maximum ratio max_i r_i/||A_i||^2 and the stop test, then runs the
//      selection rule itself (redundantly, in a fixed reduction order, so all
//      work-groups pick the same i_k without another exchange);
//   2. takes the selected row R_{i_k} (published by its owner), computes its
//      entries of v = R_{i_k} B^T and publishes them, updates its columns of
//      X (Alg. 3's X^{k+1}) while the rest of v arrives, then computes and
//      publishes its entries of w = v B (R_{i_k} B^T B in factored form);
//   3. with all of w, updates its own rows
//      R_i -= alpha/||A_i_k||^2 (A A^T)_{i,i_k} w (Alg. 3's R^{k+1}) and
//      publishes their new norms, which start update k + 1.
// The hand-overs go through tagged exchange words (exchange.h), with no
// team-wide barrier.
#include "exchange.h"
#include "internal.h"
#include "select.h"

#include <float.h>
#include <limits.h>
#include <math.h>

namespace mek {

// Sum over each row of 16 lanes (DPP): every lane of a row gets the row total.
__device__ __forceinline__ double row16_sum(double v) {
    v += dpp_d<kDppSwap1>(v);
    v += dpp_d<kDppSwap2>(v);
    v += dpp_d<kDppHalfMirror>(v);
    v += dpp_d<kDppMirror>(v);
    return v;
}

// D dot products sink(d, sum_j x[j] * row(d)[j]) over len entries, x in LDS,
// the rows in device memory, run by the whole work-group. Short vectors
// (len <= 16 * kDotUnroll) take 16 lanes per dot, four dots per wave;
// longer ones are cut into segments of kDotSeg entries, one wave task per
// (dot, segment), with kDotUnroll loads in flight per lane. A wave takes TG
// of its tasks (or groups of four short dots) at a time, all their loads
// issued before the first sum, so that small work-groups that run many
// tasks each keep TG times the bytes in flight. Partial sums go to `part`
// (LDS) and are added in segment order; a task's sum does not depend on TG
// or on scheduling. Ends with a barrier.
template <typename T, int TG = 1, typename RowFn, typename SinkFn>
__device__ __forceinline__ void block_dots(const T* x, int len, int D, RowFn row_of, SinkFn sink,
                                           double* part) {
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
    int nseg = 1;
    if (len <= 16 * kDotUnroll) {
        const int sub = lane >> 4, l16 = lane & 15;
        for (int d0 = wv * 4; d0 < D; d0 += kWaves * 4 * TG) {
            T yv[TG][kDotUnroll];
#pragma unroll
            for (int g = 0; g < TG; ++g) {
                // Dots past D read a valid row (the last) and are not kept.
                const int d = min(d0 + g * kWaves * 4 + sub, D - 1);
                if (g == 0 || d0 + g * kWaves * 4 < D) {
                    const T* mr = row_of(d);
#pragma unroll
                    for (int u = 0; u < kDotUnroll; ++u) {
                        const int j = l16 + 16 * u;
                        yv[g][u] = (j < len) ? mr[j] : (T)0;
                    }
                }
            }
#pragma unroll
            for (int g = 0; g < TG; ++g) {
                const int d = d0 + g * kWaves * 4 + sub;
                if (g == 0 || d0 + g * kWaves * 4 < D) {
                    double acc = 0.0;
                    if (d < D) {
#pragma unroll
                        for (int u = 0; u < kDotUnroll; ++u) {
                            const int j = l16 + 16 * u;
                            if (j < len) acc += (double)x[j] * (double)yv[g][u];
                        }
                    }
                    acc = row16_sum(acc);
                    if (l16 == 0 && d < D) part[d] = acc;
                }
            }
        }
    } else {
        nseg = (len + kDotSeg - 1) / kDotSeg;
        const int ntask = D * nseg;
        for (int t0 = wv; t0 < ntask; t0 += kWaves * TG) {
            T yv[TG][kDotUnroll];
#pragma unroll
            for (int g = 0; g < TG; ++g) {
                const int task = t0 + g * kWaves;
                if (task < ntask) {   // uniform in the wave
                    const int d = task / nseg, sg = task - d * nseg;
                    const T* mr = row_of(d);
                    const int j0 = sg * kDotSeg + lane;
#pragma unroll
                    for (int u = 0; u < kDotUnroll; ++u) {
                        const int j = j0 + u * kWave;
                        yv[g][u] = (j < len) ? mr[j] : (T)0;
                    }
                }
            }
#pragma unroll
            for (int g = 0; g < TG; ++g) {
                const int task = t0 + g * kWaves;
                if (task < ntask) {
                    const int sg = task % nseg;
                    const int j0 = sg * kDotSeg + lane;
                    double acc = 0.0;
#pragma unroll
                    for (int u = 0; u < kDotUnroll; ++u) {
                        const int j = j0 + u * kWave;
                        if (j < len) acc += (double)x[j] * (double)yv[g][u];
                    }
                    acc = wave_sum(acc);
                    if (lane == 0) part[task] = acc;
                }
            }
        }
    }
    __syncthreads();
    for (int d = tid; d < D; d += kThreads) {
        double acc = 0.0;
        for (int sg = 0; sg < nseg; ++sg) acc += part[d * nseg + sg];
        sink(d, acc);
    }
    __syncthreads();
}

// Optional phase timing (work-group 0, thread 0): ticks of the constant-rate
// wall clock spent in each phase of an update, summed over the solve. The
// clocks live in LDS (ph[kPhCount] holds the last mark), not in registers
// that the untimed solves would carry too.
enum { kPhReduce, kPhSelect, kPhRow, kPhDots, kPhWait, kPhX, kPhUpdate, kPhEnd, kPhCount };
#define MEK_PHASE(id)                                                   \
    do {                                                                \
        if (timing) {                                                   \
            const unsigned long long now_ = wall_clock64();             \
            ph[id] += now_ - ph[kPhCount];                              \
            ph[kPhCount] = now_;                                        \
        }                                                               \
    } while (0)

// Point the per-instance fields of P at instance slot b of a batch.
template <typename T>
__device__ __forceinline__ void bind_instance(SolveParams<T>& P, int b) {
    const InstSlot sl = P.slots[b];
    const size_t id = (size_t)sl.id;
    const size_t mn = (size_t)P.m * P.n, pq = (size_t)P.p * P.q;
    P.R += id * mn;
    P.Xt += id * pq;
    if (P.Xref_t) P.Xref_t += id * pq;
    P.r += id * P.m;
    // Exchange buffers hold one 64-bit word per entry whatever T is.
    P.rowbuf = reinterpret_cast<T*>(reinterpret_cast<char*>(P.rowbuf) + id * P.n * 8);
    P.vbuf = reinterpret_cast<T*>(reinterpret_cast<char*>(P.vbuf) + id * P.q * 8);
    P.wbuf = reinterpret_cast<T*>(reinterpret_cast<char*>(P.wbuf) + id * P.n * 8);
    P.errpart += id * kErrStride;
    P.sync += id;
    P.report += id;
    const size_t hc = (size_t)P.hist_cap;
    if (P.resid_hist) P.resid_hist += id * hc;
    if (P.err_hist) P.err_hist += id * hc;
    if (P.idx_hist) P.idx_hist += id * hc;
    if (P.set_hist) P.set_hist += id * hc;
    if (b != 0) P.phase = nullptr;
    P.C2 = sl.C2;
    P.ref2 = sl.ref2;
    P.S_target = sl.S_target;
    P.max_iters = sl.max_iters;
    P.k_offset = sl.k_offset;
    P.hist_offset = sl.hist_offset;
    P.inst = sl.inst;
}

template <typename T, bool LDS, int SR, bool MULTI = false>
__global__ void __launch_bounds__(kThreads, 1) solve_kernel(SolveParams<T> P) {
    extern __shared__ __align__(16) unsigned char dyn_smem[];
    __shared__ BlockScratch sc;
    __shared__ int s_fail;   // set once a cross-work-group wait gives up
    __shared__ double s_err[kWaves];
    if (threadIdx.x == 0) s_fail = 0;
    // Dot tasks per wave in flight: with R in device memory the work-groups
    // are few per instance and run many dot tasks each; the registers allow
    // four FP32 or two FP64 tasks when the selection holds few rows.
    constexpr int kDotTG = (!LDS && SR <= 4) ? (sizeof(T) == 4 ? 4 : 2) : 1;

    int g = blockIdx.x;
    if (MULTI) {
        // Ragged batch: instance b owns work-groups [multi_start[b],
        // multi_start[b + 1]) and brings its own sizes, operands, state and
        // team layout.
        int lo = 0, hi = P.multi_n - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (P.multi_start[mid] <= g) lo = mid;
            else hi = mid - 1;
        }
        g -= P.multi_start[lo];
        P = P.multi[lo];
    } else if (P.slots) {
        const int b = g / P.W;
        g -= b * P.W;
        bind_instance(P, b);
    }
    if (P.norms) {   // stream-ordered solves: the norms were computed on the device
        P.C2 = P.norms[0];
        P.ref2 = P.norms[1] > 0.0 ? P.norms[1] : 1.0;
    }
    const int W = P.W;
    const bool team = W > 1;
    // Re-derived at the top of every update through an opaque copy, so that
    // the compiler recomputes per-thread addresses inside the update instead
    // of carrying them in registers across the loop.
    int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
    const int m = P.m, n = P.n, p = P.p, q = P.q;
    const int row0 = g * P.rpw;
    const int nrow = max(0, min(P.rpw, m - row0));
    const int xc0 = g * P.xpw;
    const int nx = max(0, min(P.xpw, q - xc0));
    const int wc0 = g * P.wpw;
    const int nw = max(0, min(P.wpw, n - wc0));
    xword* const r_x = reinterpret_cast<xword*>(P.r);
    xword* const e_x = reinterpret_cast<xword*>(P.errpart);
    xword* const row_x = reinterpret_cast<xword*>(P.rowbuf);
    xword* const w_x = reinterpret_cast<xword*>(P.wbuf);

    // LDS: [own rows of R (LDS mode)] [n-vector staging] [v for own X rows]
    // [dot-product partial sums (+ w when the team is one work-group)]
    // [row norms when the team is one work-group] [Philox draws of the next
    // kUTable updates] [||A_i||^2, when P.a_in_lds] [own rows of X^T, when
    // P.x_in_lds].
    const size_t r_bytes = LDS ? (((size_t)P.rpw * n * sizeof(T) + 15) & ~(size_t)15) : 0;
    const size_t v_bytes = ((size_t)max(n, q) * sizeof(T) + 15) & ~(size_t)15;
    T* Rl = reinterpret_cast<T*>(dyn_smem);
    T* vec = reinterpret_cast<T*>(dyn_smem + r_bytes);
    double* vl = reinterpret_cast<double*>(dyn_smem + r_bytes + v_bytes);
    double* part = vl + P.xpw;
    const int wslot = dot_parts(P.xpw, n, P.wpw, q, false);
    double* r_local = part + dot_parts(P.xpw, n, P.wpw, q, !team);
    double* u_tab = r_local + P.rpw;
    double* a_lds = u_tab + kUTable;
    T* Xl = P.x_in_lds ? reinterpret_cast<T*>(a_lds + (P.a_in_lds ? m : 0)) : nullptr;
    // B and B^T (the rows of the two dot-product phases) in LDS, after X^T.
    T* Bl = P.b_in_lds ? reinterpret_cast<T*>(a_lds + (P.a_in_lds ? m : 0)) +
                             (P.x_in_lds ? (size_t)P.xpw * p : 0)
                       : nullptr;
    T* BTl = Bl ? Bl + (size_t)q * n : nullptr;
    const T* Bsrc = Bl ? Bl : P.B;
    const T* BTsrc = BTl ? BTl : P.BT;
    T* Rown = LDS ? Rl : P.R + (size_t)row0 * n;
    if (P.a_in_lds)
        for (int i = tid; i < m; i += kThreads) a_lds[i] = P.a[i];
    const double* asrc = P.a_in_lds ? a_lds : P.a;

    // ---- Set-up: own rows into LDS, their norms, the first error partial.
    if (LDS) {
        const T* src = P.R + (size_t)row0 * n;
        const size_t tot = (size_t)nrow * n;
        for (size_t e = tid; e < tot; e += kThreads) Rl[e] = src[e];
    }
    if (Xl) {
        const T* src = P.Xt + (size_t)xc0 * p;
        const size_t tot = (size_t)nx * p;
        for (size_t e = tid; e < tot; e += kThreads) Xl[e] = src[e];
    }
    if (Bl) {
        const size_t tot = (size_t)q * n;
        for (size_t e = tid; e < tot; e += kThreads) {
            Bl[e] = P.B[e];
            BTl[e] = P.BT[e];
        }
    }
    __syncthreads();
    for (int ii = wv; ii < nrow; ii += kWaves) {
        const T* rp = Rown + (size_t)ii * n;
        double acc = 0.0;
        for (int j = lane; j < n; j += kWave) {
            const double v = (double)rp[j];
            acc += v * v;
        }
        acc = wave_sum(acc);
        if (lane == 0) {
            if (team) xstore(&r_x[row0 + ii], pack_word(acc, seq_tag(0)));
            else r_local[ii] = acc;
        }
    }
    {
        double ep = 0.0;
        if (P.Xref_t) {
            const size_t base = (size_t)xc0 * p, total = (size_t)nx * p;
            for (size_t e = tid; e < total; e += kThreads) {
                const double d = (double)(Xl ? Xl[e] : P.Xt[base + e]) - P.Xref_t[base + e];
                ep += d * d;
            }
        }
        double v[1] = {ep};
        block_sum<1>(v, sc);
        if (tid == 0) {
            if (team) xstore(&e_x[g], pack_word(v[0], seq_tag(0)));
            else s_err[0] = v[0];
        }
    }
    __syncthreads();

    // Timed work-groups: the first, the middle and the last of the team.
    const int tslot = (g == 0) ? 0 : (g == W / 2) ? 1 : (g == W - 1) ? 2 : -1;
    const bool timing = P.phase != nullptr && tslot >= 0 && threadIdx.x == 0;
    __shared__ unsigned long long ph[kPhCount + 1];
    if (timing) {
        for (int i = 0; i < kPhCount; ++i) ph[i] = 0;
        ph[kPhCount] = wall_clock64();
    }
    const int cs = (m + kThreads - 1) / kThreads;
    int sb, scnt;
    double S0 = -1.0, S = 0.0, err = NAN;
    long long k = 0;
    int status = kMaxIter, last_set = 0;
    bool ok = true;
    const bool has_ref = P.Xref_t != nullptr;
    // When every wave owns at most one row of X^T and p <= kAPre * 64, the
    // X update's operands from device memory (A_{i_k} and the wave's row of
    // X_ref) are loaded right after the selection, into registers.
    const bool ref_regs = has_ref && nx <= kWaves && p <= kAPre * kWave;
    while (ok) {
        {
            int t = threadIdx.x;
            asm volatile("; thread index, opaque to code motion" : "+v"(t));
            tid = t;
            lane = t & (kWave - 1);
            wv = t / kWave;
            sb = min(m, tid * cs);
            scnt = min(m, sb + cs) - sb;
        }
        const unsigned int tag = seq_tag(k);
        // Draws depend only on (seed, instance, k): every kUTable updates the
        // threads compute the next kUTable of them in parallel (one each), so
        // the ten dependent Philox rounds stay off the per-update path.
        if ((k % kUTable) == 0) {
            if (tid < kUTable) u_tab[tid] = philox_uniform(P.seed, P.inst, P.k_offset + k + tid);
            __syncthreads();
        }
        const double u_k = u_tab[k % kUTable];
        // ---- 1. Global quantities: this thread's chunk of r (polled until
        // current), its chunk of ||A_i||^2, and one error partial.
        double rr[SR], aa[SR], rho[SR];
#pragma unroll
        for (int j = 0; j < SR; ++j) aa[j] = (j < scnt) ? asrc[sb + j] : 0.0;
        double Ep = 0.0;
        if (team) {
            if (!poll_words<double, SR>(r_x + sb, scnt, tag, rr, P.sync, P.poll_sleep)) s_fail = 1;
            double e1[1];
            if (tid < W && !poll_words<double, 1>(e_x + tid, 1, tag, e1, P.sync, P.poll_sleep)) s_fail = 1;
            if (tid < W) Ep = e1[0];
        } else {
#pragma unroll
            for (int j = 0; j < SR; ++j) rr[j] = (j < scnt) ? r_local[sb + j] : 0.0;
            if (tid == 0) Ep = s_err[0];
        }
        double Sp = 0.0, Mp = -1.0;
#pragma unroll
        for (int j = 0; j < SR; ++j) {
            if (j >= scnt) rr[j] = 0.0;
            // rho_i = ||R_i||^2 / ||A_i||^2, computed once per update and row.
            rho[j] = (j < scnt && aa[j] > 0.0) ? rr[j] / aa[j] : -1.0;
            Sp += rr[j];
            Mp = fmax(Mp, rho[j]);
        }
        block_sum_max_sum(Sp, Mp, Ep, sc);
        if (s_fail) { ok = false; break; }
        MEK_PHASE(kPhReduce);
        S = Sp;
        const double M = Mp;
        if (S0 < 0.0) S0 = S;
        err = has_ref ? sqrt(Ep / P.ref2) : NAN;
        const long long hk = P.hist_offset + k;
        if (g == 0 && tid == 0 && hk < P.hist_cap) {
            if (P.resid_hist) P.resid_hist[hk] = S;
            if (P.err_hist) P.err_hist[hk] = err;
        }
        // Stop tests, in a fixed order (every work-group decides the same).
        if (P.stop == kStopRelErr && err <= P.tol) { status = kOK; break; }
        if (P.stop == kStopRelResid && sqrt(S) <= P.tol * sqrt(P.C2)) { status = kOK; break; }
        if (P.S_target > 0.0 && S <= P.S_target) { status = kOK; break; }
        if (S == 0.0) { status = kExact; break; }
        if (!isfinite(S) || (P.diverge > 0.0 && S > P.diverge * S0)) { status = kEDiverged; break; }
        if (k >= P.max_iters) { status = kMaxIter; break; }

        // ---- Selection.
        int ik;
        if (P.replay && P.k_offset + k < P.replay_len) {
            ik = P.replay[P.k_offset + k];
            last_set = 0;
        } else {
            const SelectOut so = select_rows<SR>(P.variant, sb, scnt, rr, aa, rho, S, M, P.F_A,
                                                 P.theta, u_k, P.k_offset + k, P.active,
                                                 P.n_active, sc, nullptr, nullptr);
            ik = so.idx;
            last_set = so.setsize;
        }
        if (g == 0 && tid == 0 && hk < P.hist_cap) {
            if (P.idx_hist) P.idx_hist[hk] = ik;
            if (P.set_hist) P.set_hist[hk] = last_set;
        }
        const double c = P.alpha / asrc[ik];
        // A_{i_k} for the X update, loaded now so that its latency hides
        // behind the exchange of the row.
        T apre[kAPre];
        if (wv < nx) {
            const T* arow = P.A + (size_t)ik * p;
#pragma unroll
            for (int u = 0; u < kAPre; ++u) {
                const int s2 = lane + u * kWave;
                apre[u] = (s2 < p) ? arow[s2] : (T)0;
            }
        }
        double xref_r[kAPre];
#pragma unroll
        for (int u = 0; u < kAPre; ++u) {
            const int s2 = lane + u * kWave;
            xref_r[u] = (ref_regs && wv < nx && s2 < p) ? P.Xref_t[(size_t)(xc0 + wv) * p + s2] : 0.0;
        }
        // (A A^T)_{i_k, i} of the first row i each wave updates, likewise.
        // (A A^T)_{i_k, i} of the rows this wave updates (row wv + 8 u in
        // lane u), likewise.
        const int ga_row = wv + kWaves * lane;
        const T ga_lane = (ga_row < nrow) ? P.GA[(size_t)ik * m + row0 + ga_row] : (T)0;
        MEK_PHASE(kPhSelect);

        // ---- 2. The selected row: its owner publishes it, the others poll
        // their part of it into the LDS staging vector.
        const T* rowsrc;
        if (!team) {
            rowsrc = Rown + (size_t)(ik - row0) * n;
        } else {
            if (ik / P.rpw == g) {
                const T* src = Rown + (size_t)(ik - row0) * n;
                for (int j = tid; j < n; j += kThreads) xstore(&row_x[j], pack_word(src[j], tag));
            }
            T rv[kVecRegs];
            const int nreg = max(0, min(kVecRegs, (n - tid + kThreads - 1) / kThreads));
            if (!poll_strided<T, kVecRegs>(row_x + tid, kThreads, nreg, tag, rv, P.sync, P.poll_sleep)) s_fail = 1;
#pragma unroll
            for (int u = 0; u < kVecRegs; ++u)
                if (u < nreg) vec[tid + u * kThreads] = rv[u];
            for (int j = tid + kVecRegs * kThreads; j < n; j += kThreads) {
                T one[1];
                if (!poll_words<T, 1>(row_x + j, 1, tag, one, P.sync, P.poll_sleep)) s_fail = 1;
                vec[j] = one[0];
            }
            __syncthreads();
            if (s_fail) { ok = false; break; }
            rowsrc = vec;
        }
        MEK_PHASE(kPhRow);
        // v = R_{i_k} B^T: this work-group's entries (rows xc0.. of B), into
        // LDS and, in a team, published for the others.
        xword* const v_x = reinterpret_cast<xword*>(P.vbuf);
        block_dots<T, kDotTG>(rowsrc, n, nx, [&](int d) { return Bsrc + (size_t)(xc0 + d) * n; },
                      [&](int d, double val) {
                          vl[d] = val;
                          if (team) xstore(&v_x[xc0 + d], pack_word((T)val, tag));
                      },
                      part);
        MEK_PHASE(kPhDots);
        // X^T rows l: X^T[l, :] += (c A_{i_k, :}) v_l, one wave per row (in
        // LDS when there is room), with the squared error against the
        // reference in the same pass. In a team this runs while the other
        // slices of v are on their way.
        {
            const T* arow = P.A + (size_t)ik * p;
            double ep = 0.0;
            for (int l = wv; l < nx; l += kWaves) {
                T* xr = Xl ? Xl + (size_t)l * p : P.Xt + (size_t)(xc0 + l) * p;
                const double* rr_ = has_ref ? P.Xref_t + (size_t)(xc0 + l) * p : nullptr;
                const T vlT = (T)vl[l];
#pragma unroll
                for (int u = 0; u < kAPre; ++u) {
                    const int s2 = lane + u * kWave;
                    if (s2 < p) {
                        const T nv = xr[s2] + (T)(c * (double)apre[u]) * vlT;
                        xr[s2] = nv;
                        if (has_ref) {
                            const double d = (double)nv - (ref_regs ? xref_r[u] : rr_[s2]);
                            ep += d * d;
                        }
                    }
                }
                for (int s2 = lane + kAPre * kWave; s2 < p; s2 += kWave) {
                    const T nv = xr[s2] + (T)(c * (double)arow[s2]) * vlT;
                    xr[s2] = nv;
                    if (has_ref) {
                        const double d = (double)nv - rr_[s2];
                        ep += d * d;
                    }
                }
            }
            ep = wave_sum(ep);
            if (lane == 0) s_err[wv] = ep;
        }
        MEK_PHASE(kPhX);
        // All of v, as the left factor of w = v B.
        const T* vfull;
        if (team) {
            for (int l0 = 0; l0 < q; l0 += kThreads * kVecRegs) {
                T tv[kVecRegs];
                const int cnt = max(0, min(kVecRegs, (q - l0 - tid + kThreads - 1) / kThreads));
                if (!poll_strided<T, kVecRegs>(v_x + l0 + tid, kThreads, cnt, tag, tv, P.sync, P.poll_sleep)) s_fail = 1;
#pragma unroll
                for (int u = 0; u < kVecRegs; ++u)
                    if (u < cnt) vec[l0 + tid + u * kThreads] = tv[u];
            }
            __syncthreads();
            if (s_fail) { ok = false; break; }
            vfull = vec;
        } else {
            for (int l = tid; l < q; l += kThreads) vec[l] = (T)vl[l];
            __syncthreads();
            vfull = vec;
        }
        // w = v B for this work-group's entries (rows wc0.. of B^T).
        block_dots<T, kDotTG>(vfull, q, nw, [&](int d) { return BTsrc + (size_t)(wc0 + d) * q; },
                      [&](int d, double val) {
                          if (team) xstore(&w_x[wc0 + d], pack_word((T)val, tag));
                          else part[wslot + d] = val;
                      },
                      part);
        // w into the staging vector.
        if (team) {
            for (int j0 = 0; j0 < n; j0 += kThreads * kVecRegs) {
                T tw[kVecRegs];
                const int cnt = max(0, min(kVecRegs, (n - j0 - tid + kThreads - 1) / kThreads));
                if (!poll_strided<T, kVecRegs>(w_x + j0 + tid, kThreads, cnt, tag, tw, P.sync, P.poll_sleep)) s_fail = 1;
#pragma unroll
                for (int u = 0; u < kVecRegs; ++u)
                    if (u < cnt) vec[j0 + tid + u * kThreads] = tw[u];
            }
        } else {
            for (int j = tid; j < n; j += kThreads) vec[j] = (T)part[wslot + j];
        }
        __syncthreads();
        if (s_fail) { ok = false; break; }
        MEK_PHASE(kPhWait);
        // ---- 3. Own rows: R_i -= (c (A A^T)_{i_k, i}) w and r_i = ||R_i||^2,
        // one wave per row; publish the norms and the error partial with the
        // next update's tag.
        {
            const unsigned int ntag = seq_tag(k + 1);
            const T* garow = P.GA + (size_t)ik * m + row0;
            // (A A^T)_{i_k, i} of row ii = wv + 8 u: from lane u's register
            // (ii is the same in the whole wave), past 64 rows from memory.
            auto ga_of = [&](int ii) -> T {
                const int u = (ii - wv) / kWaves;
                return u < kWave ? __shfl(ga_lane, u) : garow[ii];
            };
            auto publish = [&](int ii, double acc) {
                acc = wave_sum(acc);
                if (lane == 0) {
                    if (team) xstore(&r_x[row0 + ii], pack_word(acc, ntag));
                    else r_local[ii] = acc;
                }
            };
            if (LDS) {
                for (int ii = wv; ii < nrow; ii += kWaves) {
                    const T sc_i = (T)(c * (double)ga_of(ii));
                    T* rp = Rown + (size_t)ii * n;
                    double acc = 0.0;
                    for (int j = lane; j < n; j += kWave) {
                        const T v = rp[j] - sc_i * vec[j];
                        rp[j] = v;
                        acc += (double)v * (double)v;
                    }
                    publish(ii, acc);
                }
            } else {
                // R in device memory: two rows per wave at a time and
                // kRowBatch loads in flight per lane and row (each row's
                // elements in the same order as above, so the same sums).
                for (int ii = wv; ii < nrow; ii += 2 * kWaves) {
                    const int i2 = ii + kWaves;
                    const bool two = i2 < nrow;
                    const T sa = (T)(c * (double)ga_of(ii));
                    const T gb = ga_of(two ? i2 : ii);
                    const T sb = two ? (T)(c * (double)gb) : T(0);
                    T* ra = Rown + (size_t)ii * n;
                    T* rb = Rown + (size_t)(two ? i2 : ii) * n;
                    double acc_a = 0.0, acc_b = 0.0;
                    for (int j0 = 0; j0 < n; j0 += kRowBatch * kWave) {
                        T xa[kRowBatch], xb[kRowBatch];
#pragma unroll
                        for (int u = 0; u < kRowBatch; ++u) {
                            const int j = j0 + u * kWave + lane;
                            xa[u] = j < n ? ra[j] : T(0);
                            xb[u] = (two && j < n) ? rb[j] : T(0);
                        }
#pragma unroll
                        for (int u = 0; u < kRowBatch; ++u) {
                            const int j = j0 + u * kWave + lane;
                            if (j < n) {
                                const T wj = vec[j];
                                const T va = xa[u] - sa * wj;
                                ra[j] = va;
                                acc_a += (double)va * (double)va;
                                if (two) {
                                    const T vb = xb[u] - sb * wj;
                                    rb[j] = vb;
                                    acc_b += (double)vb * (double)vb;
                                }
                            }
                        }
                    }
                    publish(ii, acc_a);
                    if (two) publish(i2, acc_b);
                }
            }
            if (tid == 0) {
                double e = 0.0;
                for (int w2 = 0; w2 < kWaves; ++w2) e += s_err[w2];
                if (team) xstore(&e_x[g], pack_word(e, ntag));
                else s_err[0] = e;
            }
        }
        __syncthreads();
        MEK_PHASE(kPhUpdate);
        ++k;
    }
    if (s_fail) status = kETimeout;
    if (Xl) {
        T* dst = P.Xt + (size_t)xc0 * p;
        const size_t tot = (size_t)nx * p;
        for (size_t e = tid; e < tot; e += kThreads) dst[e] = Xl[e];
    }
    if (timing)
        for (int i = 0; i < kPhCount; ++i) P.phase[tslot * kPhCount + i] += ph[i];
    if (g == 0 && tid == 0) {
        P.report->iters = k;
        P.report->status = status;
        P.report->last_set = last_set;
        P.report->S = S;
        P.report->err = err;
    }
}

// ---------------------------------------------------------------------------
// Small instances (m, n, p, q <= kThreads): one work-group holds R, B and
// X^T in LDS; the selection sees one row per thread (thread t holds row t's
// norm). The two dot-product phases (v_l = R_{i_k} . B_l for l < q, then
// w_j = sum_l v_l B_lj for j < n) and the R update with the new row norms
// give each dot or row to a group of G lanes (G a power of two, G times the
// count at most kThreads): lane g of a group takes entries g, g + G, ...,
// and the group adds its partial sums by lane exchanges (fixed order). The
// operands the update reads from device memory (A_{i_k}, the column i_k of
// A A^T) are fetched right after the selection and used after the dot
// products; X_ref's entries of the first kSmallXr passes of the X update
// stay in registers. R and B rows are padded to n + 1 entries. Uniform
// batches: work-group b runs instance b. Same options, stop rules,
// histories and report as the team kernel.
constexpr int kSmallXr = 4;   // X update passes whose X_ref entries stay in registers

// Lanes per group for `count` dots or rows: the largest power of two G <= 64
// with G * count <= kThreads.
__device__ __forceinline__ int small_group(int count) {
    int g = 1;
    while (g < kWave && 2 * g * count <= kThreads) g *= 2;
    return g;
}

// Sum over aligned groups of G lanes (G a power of two <= 64): every lane
// of a group gets the group's total, added in butterfly order.
__device__ __forceinline__ double group_sum(double v, int G) {
    for (int off = G >> 1; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// The selection step of Algs. 1-5 by one wave for at most 2 kWave rows:
// lane l holds rows 2 l and 2 l + 1 (r: ||R_i||^2, a: ||A_i||^2, h: r / a,
// or -1 without a row or with a = 0), S and M the block totals. The same
// rules as select_rows on a block: the greedy set {a > 0, h >= t} with
// t = min(M, theta M + (1 - theta) S / F_A) and weights r (Algs. 3/4),
// every row with a > 0 and weight a (Alg. 1), the first row of largest h
// (Alg. 5), the cyclic order over the active rows (Alg. 2); the draw takes
// the first member whose running weight exceeds u T, else the last member.
// Returns the row | (set size << 16), the same in every lane.
__device__ __forceinline__ int small_select(int variant, int lane, int m, double r0, double r1,
                                            double a0, double a1, double h0, double h1, double S,
                                            double M, double F_A, double theta, double u,
                                            long long k, const int* __restrict__ active,
                                            int n_active) {
    const double r[2] = {r0, r1}, a[2] = {a0, a1}, h[2] = {h0, h1};
    if (variant == kBK) return active[k % n_active];
    if (variant == kMWRBK) {
        int cand = INT_MAX;
#pragma unroll
        for (int j = 0; j < 2; ++j)
            if (2 * lane + j < m && a[j] > 0.0 && h[j] == M) cand = min(cand, 2 * lane + j);
        return wave_min_int(cand) | (1 << 16);
    }
    const bool greedy = variant == kGRBK || variant == kRGRBK;
    double t = 0.0;
    if (greedy) {
#pragma clang fp contract(off)
        const double th = (variant == kGRBK) ? 0.5 : theta;
        t = th * M + (1.0 - th) * (S / F_A);
        if (t > M) t = M;
    }
    bool mem[2];
    double w[2];
    double ws = 0.0;
    int c = 0, lastm = -1;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        mem[j] = 2 * lane + j < m && a[j] > 0.0 && (!greedy || h[j] >= t);
        w[j] = greedy ? r[j] : a[j];
        if (mem[j]) {
            ws += w[j];
            ++c;
            lastm = 2 * lane + j;
        }
    }
    const double iv = wave_incl_scan(ws);
    const int ic = wave_incl_scan_int(c);
    const double T = readlane_d(iv, kWave - 1);
    const int tot = __builtin_amdgcn_readlane(ic, kWave - 1);
    const double target = u * T;
    double run = iv - ws;
    int cand = INT_MAX;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        if (mem[j]) {
            run += w[j];
            if (cand == INT_MAX && run > target) cand = 2 * lane + j;
        }
    }
    cand = wave_min_int(cand);
    lastm = wave_max_int(lastm);
    return (cand != INT_MAX ? cand : lastm) | (tot << 16);
}

template <typename T>
__global__ void __launch_bounds__(kThreads, 1) solve_small_kernel(SolveParams<T> P) {
    extern __shared__ __align__(16) unsigned char dyn_smem[];
    __shared__ BlockScratch sc;
    __shared__ double s_c;
    if (P.slots) bind_instance(P, blockIdx.x);
    if (P.norms) {
        P.C2 = P.norms[0];
        P.ref2 = P.norms[1] > 0.0 ? P.norms[1] : 1.0;
    }
    const int m = P.m, n = P.n, p = P.p, q = P.q, ld = n + 1;
    const int tid = threadIdx.x;
    // LDS: R (m x ld), B (q x ld), X^T (q x p), v (q), w (n), A_{i_k} (p),
    // Philox draws (kUTable).
    T* Rl = reinterpret_cast<T*>(dyn_smem);
    T* Bl = Rl + (size_t)m * ld;
    T* Xl = Bl + (size_t)q * ld;
    T* vl = Xl + (size_t)q * p;
    T* wl = vl + q;
    T* al = wl + n;
    double* u_tab = reinterpret_cast<double*>(
        reinterpret_cast<unsigned char*>(dyn_smem) +
        ((((size_t)m * ld + (size_t)q * ld + (size_t)q * p + q + n + p) * sizeof(T) + 15) & ~(size_t)15));
    double* rn = u_tab + kUTable;   // new row norms, m
    double* epart = rn + m;         // error partials of the waves, kWaves
    const int G1 = small_group(q), G2 = small_group(n), G3 = small_group(m);
    for (int e = tid; e < m * n; e += kThreads) Rl[(e / n) * ld + e % n] = P.R[e];
    for (int e = tid; e < q * n; e += kThreads) Bl[(e / n) * ld + e % n] = P.B[e];
    for (int e = tid; e < q * p; e += kThreads) Xl[e] = P.Xt[e];
    const bool has_ref = P.Xref_t != nullptr;
    const double ai = tid < m ? P.a[tid] : 0.0;
    __syncthreads();
    // Own row's norm and the first error partial.
    double ri = 0.0;
    if (tid < m) {
        const T* rp = Rl + (size_t)tid * ld;
        for (int j = 0; j < n; ++j) ri += (double)rp[j] * (double)rp[j];
    }
    double ep = 0.0;
    if (has_ref)
        for (int e = tid; e < q * p; e += kThreads) {
            const double d = (double)Xl[e] - P.Xref_t[e];
            ep += d * d;
        }
    double xr[kSmallXr];
#pragma unroll
    for (int u = 0; u < kSmallXr; ++u) {
        const int e = tid + u * kThreads;
        xr[u] = (has_ref && e < q * p) ? P.Xref_t[e] : 0.0;
    }
    double S0 = -1.0, S = 0.0, err = NAN;
    long long k = 0;
    int status = kMaxIter, last_set = 0;
    const int sb = min(m, tid), scnt = tid < m ? 1 : 0;
    // Up to 2 kWave rows, wave 0 alone reduces the norms and error partials
    // and runs the selection (lane l: rows 2 l and 2 l + 1), with no block
    // barrier until it hands the results over through LDS.
    const bool wsel = m <= 2 * kWave;
    const int lane = tid & (kWave - 1), wv = tid / kWave;
    const double a_lo = (wsel && wv == 0 && 2 * lane < m) ? P.a[2 * lane] : 0.0;
    const double a_hi = (wsel && wv == 0 && 2 * lane + 1 < m) ? P.a[2 * lane + 1] : 0.0;
    __shared__ double s_wd[3];
    __shared__ int s_wi[2];
    if (tid < m) rn[tid] = ri;
    {
        const double ew = wave_sum(ep);
        if (lane == 0) epart[wv] = ew;
    }
    __syncthreads();
    const bool timing = P.phase != nullptr && blockIdx.x == 0 && tid == 0;
    __shared__ unsigned long long ph[kPhCount + 1];
    if (timing) {
        for (int i = 0; i < kPhCount; ++i) ph[i] = 0;
        ph[kPhCount] = wall_clock64();
    }
    for (;;) {
        if ((k % kUTable) == 0) {
            if (tid < kUTable) u_tab[tid] = philox_uniform(P.seed, P.inst, P.k_offset + k + tid);
            __syncthreads();
        }
        const double u_k = u_tab[k % kUTable];
        double rr[1] = {scnt ? ri : 0.0}, aa[1] = {ai};
        double rho[1] = {(scnt && ai > 0.0) ? ri / ai : -1.0};
        double Sp = rr[0], Mp = rho[0], Ep = ep;
        if (wsel) {
            if (wv == 0) {
                double r2[2], h2[2];
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    const int row = 2 * lane + u;
                    const double au = u ? a_hi : a_lo;
                    r2[u] = row < m ? rn[row] : 0.0;
                    h2[u] = (row < m && au > 0.0) ? r2[u] / au : -1.0;
                }
                const double Sw = wave_sum(r2[0] + r2[1]);
                const double Mw = wave_max(fmax(h2[0], h2[1]));
                const double Ew = wave_sum(lane < kWaves ? epart[lane] : 0.0);
                const int sel = small_select(P.variant, lane, m, r2[0], r2[1], a_lo, a_hi, h2[0],
                                             h2[1], Sw, Mw, P.F_A, P.theta, u_k, P.k_offset + k,
                                             P.active, P.n_active);
                if (lane == 0) {
                    s_wd[0] = Sw;
                    s_wd[1] = Mw;
                    s_wd[2] = Ew;
                    s_wi[0] = sel & 0xffff;
                    s_wi[1] = sel >> 16;
                }
            }
            __syncthreads();
            Sp = s_wd[0];
            Mp = s_wd[1];
            Ep = s_wd[2];
        } else {
            block_sum_max_sum(Sp, Mp, Ep, sc);
        }
        MEK_PHASE(kPhReduce);
        S = Sp;
        const double M = Mp;
        if (S0 < 0.0) S0 = S;
        err = has_ref ? sqrt(Ep / P.ref2) : NAN;
        const long long hk = P.hist_offset + k;
        if (tid == 0 && hk < P.hist_cap) {
            if (P.resid_hist) P.resid_hist[hk] = S;
            if (P.err_hist) P.err_hist[hk] = err;
        }
        if (P.stop == kStopRelErr && err <= P.tol) { status = kOK; break; }
        if (P.stop == kStopRelResid && sqrt(S) <= P.tol * sqrt(P.C2)) { status = kOK; break; }
        if (P.S_target > 0.0 && S <= P.S_target) { status = kOK; break; }
        if (S == 0.0) { status = kExact; break; }
        if (!isfinite(S) || (P.diverge > 0.0 && S > P.diverge * S0)) { status = kEDiverged; break; }
        if (k >= P.max_iters) { status = kMaxIter; break; }
        int ik;
        if (P.replay && P.k_offset + k < P.replay_len) {
            ik = P.replay[P.k_offset + k];
            last_set = 0;
        } else if (wsel) {
            ik = s_wi[0];
            last_set = s_wi[1];
        } else {
            const SelectOut so = select_rows<1>(P.variant, sb, scnt, rr, aa, rho, S, M, P.F_A,
                                                P.theta, u_k, P.k_offset + k, P.active,
                                                P.n_active, sc, nullptr, nullptr);
            ik = so.idx;
            last_set = so.setsize;
        }
        if (tid == 0 && hk < P.hist_cap) {
            if (P.idx_hist) P.idx_hist[hk] = ik;
            if (P.set_hist) P.set_hist[hk] = last_set;
        }
        MEK_PHASE(kPhSelect);
        // Operands of the update from device memory, fetched now and used
        // after the dot products: A_{i_k} (into LDS then) and the entry of
        // column i_k of A A^T for the row this lane updates.
        if (tid == ik) s_c = P.alpha / ai;
        const T aval = tid < p ? P.A[(size_t)ik * p + tid] : (T)0;
        const int h3 = tid / G3, g3 = tid - h3 * G3;
        const T ga = h3 < m ? P.GA[(size_t)ik * m + h3] : (T)0;
        // v_l = R_{i_k} . B_l (pre-update row), G1 lanes per dot.
        {
            const int l = tid / G1, g1 = tid - l * G1;
            const T* rrow = Rl + (size_t)ik * ld;
            double acc = 0.0;
            if (l < q) {
                const T* brow = Bl + (size_t)l * ld;
                for (int j = g1; j < n; j += G1) acc += (double)rrow[j] * (double)brow[j];
            }
            acc = group_sum(acc, G1);
            if (l < q && g1 == 0) vl[l] = (T)acc;
        }
        if (tid < p) al[tid] = aval;
        __syncthreads();
        MEK_PHASE(kPhDots);
        const double c = s_c;
        // X^T[l][s] += c A_{i_k, s} v_l, with the error partial; then
        // w_j = sum_l v_l B_lj, G2 lanes per entry.
        ep = 0.0;
#pragma unroll
        for (int u = 0; u < kSmallXr; ++u) {
            const int e = tid + u * kThreads;
            if (e < q * p) {
                const int l = e / p, s2 = e - l * p;
                const T nv = Xl[e] + (T)(c * (double)al[s2]) * vl[l];
                Xl[e] = nv;
                if (has_ref) {
                    const double d = (double)nv - xr[u];
                    ep += d * d;
                }
            }
        }
        for (int e = tid + kSmallXr * kThreads; e < q * p; e += kThreads) {
            const int l = e / p, s2 = e - l * p;
            const T nv = Xl[e] + (T)(c * (double)al[s2]) * vl[l];
            Xl[e] = nv;
            if (has_ref) {
                const double d = (double)nv - P.Xref_t[e];
                ep += d * d;
            }
        }
        {
            const int j = tid / G2, g2 = tid - j * G2;
            double acc = 0.0;
            if (j < n)
                for (int l = g2; l < q; l += G2) acc += (double)vl[l] * (double)Bl[(size_t)l * ld + j];
            acc = group_sum(acc, G2);
            if (j < n && g2 == 0) wl[j] = (T)acc;
        }
        {
            const double ew = wave_sum(ep);
            if (lane == 0) epart[wv] = ew;
        }
        __syncthreads();
        MEK_PHASE(kPhX);
        // R_h -= (c (A A^T)_{i_k, h}) w and the new norm of row h, G3 lanes
        // per row; the norms go through LDS to the lane that owns the row in
        // the selection.
        {
            double acc = 0.0;
            if (h3 < m) {
                const T sc_h = (T)(c * (double)ga);
                T* rp = Rl + (size_t)h3 * ld;
                for (int j = g3; j < n; j += G3) {
                    const T v = rp[j] - sc_h * wl[j];
                    rp[j] = v;
                    acc += (double)v * (double)v;
                }
            }
            acc = group_sum(acc, G3);
            if (h3 < m && g3 == 0) rn[h3] = acc;
        }
        __syncthreads();
        ri = tid < m ? rn[tid] : 0.0;
        MEK_PHASE(kPhUpdate);
        ++k;
    }
    if (timing)
        for (int i2 = 0; i2 < kPhCount; ++i2) P.phase[i2] += ph[i2];
    for (int e = tid; e < q * p; e += kThreads) P.Xt[e] = Xl[e];
    if (tid == 0) {
        P.report->iters = k;
        P.report->status = status;
        P.report->last_set = last_set;
        P.report->S = S;
        P.report->err = err;
    }
}

size_t solve_small_lds_bytes(int m, int p, int q, int n, size_t elem) {
    const size_t ld = (size_t)n + 1;
    return (((size_t)m * ld + (size_t)q * ld + (size_t)q * p + q + n + p) * elem + 15) / 16 * 16 +
           (kUTable + (size_t)m + kWaves) * sizeof(double);
}

template <typename T>
static hipError_t launch_small(const SolveParams<T>& P, size_t lds_bytes, hipStream_t s) {
    auto kern = solve_small_kernel<T>;
    if (hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds_bytes) != hipSuccess)
        (void)hipGetLastError();
    SolveParams<T> copy = P;
    void* args[] = {&copy};
    const int blocks = P.slots ? P.nb : 1;
    return hipLaunchKernel((const void*)kern, dim3(blocks), dim3(kThreads), args, lds_bytes, s);
}

size_t solve_lds_budget() { return 160 * 1024 - 1024; }

size_t solve_lds_bytes(int rpw, int n, int q, int xpw, int wpw, size_t elem, bool r_in_lds,
                       bool single) {
    size_t b = r_in_lds ? (((size_t)rpw * n * elem + 15) & ~(size_t)15) : 0;
    b += ((size_t)(n > q ? n : q) * elem + 15) & ~(size_t)15;
    b += (size_t)xpw * sizeof(double) + (size_t)dot_parts(xpw, n, wpw, q, single) * sizeof(double);
    b += (size_t)rpw * sizeof(double);   // row norms of a one-work-group team
    return b + kUTable * sizeof(double); // Philox draws of the coming updates
}

size_t solve_lds_bytes_a(int m) { return (size_t)m * sizeof(double); }

template <typename T, bool LDS, int SR, bool MULTI = false>
static hipError_t launch_one(const SolveParams<T>& P, size_t lds_bytes, hipStream_t s) {
    auto kern = solve_kernel<T, LDS, SR, MULTI>;
    // Raise the dynamic LDS cap for this kernel; if the runtime refuses, the
    // launch below reports the error.
    if (hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds_bytes) != hipSuccess)
        (void)hipGetLastError();
    SolveParams<T> copy = P;
    void* args[] = {&copy};
    const int blocks = MULTI ? P.multi_wgs : P.W * (P.slots ? P.nb : 1);
    if (blocks == 1)
        return hipLaunchKernel((const void*)kern, dim3(1), dim3(kThreads), args, lds_bytes, s);
    // Teams wait on each other's words, so every work-group of the grid must
    // be resident at once: a cooperative launch guarantees it (or fails).
    return hipLaunchCooperativeKernel((const void*)kern, dim3(blocks), dim3(kThreads), args,
                                      (unsigned int)lds_bytes, s);
}

// Rows of the selection chunk per thread, rounded up to a power of two.
int sel_rows_for(int m) {
    const int cs = (m + kThreads - 1) / kThreads;
    return cs <= 1 ? 1 : cs <= 2 ? 2 : cs <= 4 ? 4 : cs <= 8 ? 8 : 16;
}

template <typename T, bool LDS>
static hipError_t launch_sr(const SolveParams<T>& P, size_t lds_bytes, hipStream_t s) {
    switch (sel_rows_for(P.m)) {
        case 1: return launch_one<T, LDS, 1>(P, lds_bytes, s);
        case 2: return launch_one<T, LDS, 2>(P, lds_bytes, s);
        case 4: return launch_one<T, LDS, 4>(P, lds_bytes, s);
        case 8: return launch_one<T, LDS, 8>(P, lds_bytes, s);
        default: return launch_one<T, LDS, 16>(P, lds_bytes, s);
    }
}

template <typename T>
static hipError_t launch_multi_sr(const SolveParams<T>& P, int max_m, size_t lds_bytes,
                                  hipStream_t s) {
    switch (sel_rows_for(max_m)) {
        case 1: return launch_one<T, false, 1, true>(P, lds_bytes, s);
        case 2: return launch_one<T, false, 2, true>(P, lds_bytes, s);
        case 4: return launch_one<T, false, 4, true>(P, lds_bytes, s);
        case 8: return launch_one<T, false, 8, true>(P, lds_bytes, s);
        default: return launch_one<T, false, 16, true>(P, lds_bytes, s);
    }
}

hipError_t launch_solve_multi(const SolveParams<double>& P, int max_m, size_t lds_bytes,
                              hipStream_t s) {
    return launch_multi_sr(P, max_m, lds_bytes, s);
}
hipError_t launch_solve_multi(const SolveParams<float>& P, int max_m, size_t lds_bytes,
                              hipStream_t s) {
    return launch_multi_sr(P, max_m, lds_bytes, s);
}

hipError_t launch_solve(const SolveParams<double>& P, bool r_in_lds, size_t lds_bytes,
                        hipStream_t s) {
    if (P.small) return launch_small<double>(P, lds_bytes, s);
    return r_in_lds ? launch_sr<double, true>(P, lds_bytes, s)
                    : launch_sr<double, false>(P, lds_bytes, s);
}
hipError_t launch_solve(const SolveParams<float>& P, bool r_in_lds, size_t lds_bytes,
                        hipStream_t s) {
    if (P.small) return launch_small<float>(P, lds_bytes, s);
    return r_in_lds ? launch_sr<float, true>(P, lds_bytes, s)
                    : launch_sr<float, false>(P, lds_bytes, s);
}

// ---------------------------------------------------------------------------
// Unit kernels: the selection step and the Philox draws on their own.
// ---------------------------------------------------------------------------
template <int SR>
__global__ void __launch_bounds__(kThreads, 1)
select_kernel(int variant, int m, const double* r, const double* a, double F_A, double theta,
              uint64_t seed, uint64_t inst, long long k0, long long count, int32_t* idx,
              uint8_t* in_set, int32_t* set_list, double* stats, const int* active,
              int n_active) {
    __shared__ BlockScratch sc;
    const int cs = (m + kThreads - 1) / kThreads;
    const int b = min(m, (int)threadIdx.x * cs);
    const int cnt = min(m, b + cs) - b;
    double rr[SR], aa[SR], rho[SR];
    double Sp = 0.0, Mp = -1.0, dummy = 0.0;
#pragma unroll
    for (int j = 0; j < SR; ++j) {
        rr[j] = (j < cnt) ? r[b + j] : 0.0;
        aa[j] = (j < cnt) ? a[b + j] : 0.0;
        rho[j] = (j < cnt && aa[j] > 0.0) ? rr[j] / aa[j] : -1.0;
        Sp += rr[j];
        Mp = fmax(Mp, rho[j]);
    }
    block_sum_max_sum(Sp, Mp, dummy, sc);
    for (long long j = 0; j < count; ++j) {
        const bool first = (j == 0);
        const SelectOut o = select_rows<SR>(variant, b, cnt, rr, aa, rho, Sp, Mp, F_A, theta,
                                            philox_uniform(seed, inst, k0 + j), k0 + j, active,
                                            n_active, sc, first ? set_list : nullptr,
                                            first ? in_set : nullptr);
        if (threadIdx.x == 0) {
            idx[j] = o.idx;
            if (first && stats) {
                stats[0] = o.t;
                stats[1] = (variant == kMWRBK) ? r[o.idx] : o.T;
                stats[2] = Sp;
                stats[3] = (double)o.setsize;
            }
        }
        __syncthreads();
    }
}

hipError_t launch_select(int variant, int m, const double* r, const double* a, double F_A,
                         double theta, uint64_t seed, uint64_t inst, long long k0,
                         long long count, int32_t* idx, uint8_t* in_set, int32_t* set_list,
                         double* stats, const int* active, int n_active, hipStream_t s) {
    auto go = [&](auto kern) {
        hipLaunchKernelGGL(kern, dim3(1), dim3(kThreads), 0, s, variant, m, r, a, F_A, theta,
                           seed, inst, k0, count, idx, in_set, set_list, stats, active, n_active);
        return hipGetLastError();
    };
    switch (sel_rows_for(m)) {
        case 1: return go(select_kernel<1>);
        case 2: return go(select_kernel<2>);
        case 4: return go(select_kernel<4>);
        case 8: return go(select_kernel<8>);
        default: return go(select_kernel<16>);
    }
}

__global__ void philox_kernel(uint64_t seed, uint64_t inst, long long k0, long long count,
                              double* out) {
    const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < count) out[j] = philox_uniform(seed, inst, k0 + j);
}

hipError_t launch_philox(uint64_t seed, uint64_t inst, long long k0, long long count,
                         double* out, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    const long long blocks = (count + 255) / 256;
    hipLaunchKernelGGL(philox_kernel, dim3((unsigned)blocks), dim3(256), 0, s, seed, inst, k0,
                       count, out);
    return hipGetLastError();
}

}  // namespace mek
