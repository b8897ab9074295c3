// Sparse-aware update for Algs. 1-5: the same iteration as the persistent
// solver, with every term that the structure of A and B makes zero left out.
//
// The update of Alg. 3 changes
//   X^{k+1} = X^k + c A_{i_k}^T v,         v = R_{i_k} B^T  (q entries)
//   R^{k+1} = R^k - c (A A^T)_{:, i_k} w,   w = v B          (n entries)
// with c = alpha / ||A_{i_k}||^2. When A and B are sparse (a blur: a few taps
// per row), only the rows of X where A_{i_k} is nonzero and the rows of R
// where column i_k of A A^T is nonzero change, and each entry of v and w is
// a short sum over the nonzeros of one row / column of B. So one update
// touches nnz(A_{i_k}) rows of X and nnz((A A^T)_{:, i_k}) rows of R instead
// of all p and m, and one work-group per instance does the whole solve with
// block barriers only: no cross-work-group exchange, any number of
// instances per launch.
//
// The row norms ||R_i||^2 and the per-row errors ||X_x - X_ref,x||^2 stay in
// LDS; only the changed rows are recomputed. The selection is the dense
// solver's (select.h) over the norms in LDS, with the same Philox draws, so
// a sparse and a dense solve of the same instance pick the same rows up to
// rounding in the norms.
//
// The structure is kept in ELL form (a fixed number of slots per row,
// padded with index -1): the nonzeros of each row of A (row-major: one row
// is read per update), of each row and each column of B (slot-major, so
// that neighbouring threads read neighbouring entries), and of each column
// of A A^T (row-major). Entries within a row are in ascending index order.
#include "internal.h"
#include "select.h"

#include <math.h>

namespace mek {

// ---------------------------------------------------------------------------
// Structure extraction (plan set-up): line i of M holds M[i*rs + j*cs] for
// j < cols; one wave per line.
// ---------------------------------------------------------------------------
__global__ void ell_count_kernel(const double* __restrict__ M, int rows, int cols, long long rs,
                                 long long cs, int* __restrict__ width) {
    const int lane = threadIdx.x & (kWave - 1);
    const int line = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (line >= rows) return;
    const double* base = M + (size_t)line * rs;
    int c = 0;
    for (int j = lane; j < cols; j += kWave) c += base[(size_t)j * cs] != 0.0;
    for (int o = kWave / 2; o > 0; o >>= 1) c += __shfl_xor(c, o);
    if (lane == 0) atomicMax(width, c);
}

template <typename T>
__global__ void ell_fill_kernel(const double* __restrict__ M, int rows, int cols, long long rs,
                                long long cs, int width, int slot_major, int* __restrict__ idx,
                                T* __restrict__ val) {
    const int lane = threadIdx.x & (kWave - 1);
    const int line = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (line >= rows) return;
    const double* base = M + (size_t)line * rs;
    auto slot = [&](int t) -> size_t {
        return slot_major ? (size_t)t * rows + line : (size_t)line * width + t;
    };
    int pos = 0;
    for (int j0 = 0; j0 < cols; j0 += kWave) {
        const int j = j0 + lane;
        const double v = j < cols ? base[(size_t)j * cs] : 0.0;
        const bool nz = v != 0.0;
        const unsigned long long mask = __ballot(nz);
        const int before = __popcll(mask & ((1ull << lane) - 1ull));
        if (nz && pos + before < width) {
            idx[slot(pos + before)] = j;
            val[slot(pos + before)] = (T)v;
        }
        pos += __popcll(mask);
    }
    for (int t = pos + lane; t < width; t += kWave) {
        idx[slot(t)] = -1;
        val[slot(t)] = (T)0;
    }
}

hipError_t ell_width(const double* M, int rows, int cols, long long rs, long long cs,
                     int* width_dev, hipStream_t s) {
    const int per = 256 / kWave;
    ell_count_kernel<<<(rows + per - 1) / per, 256, 0, s>>>(M, rows, cols, rs, cs, width_dev);
    return hipGetLastError();
}

template <typename T>
hipError_t ell_fill(const double* M, int rows, int cols, long long rs, long long cs, int width,
                    bool slot_major, int* idx, T* val, hipStream_t s) {
    const int per = 256 / kWave;
    ell_fill_kernel<T><<<(rows + per - 1) / per, 256, 0, s>>>(M, rows, cols, rs, cs, width,
                                                               slot_major ? 1 : 0, idx, val);
    return hipGetLastError();
}
template hipError_t ell_fill<double>(const double*, int, int, long long, long long, int, bool,
                                     int*, double*, hipStream_t);
template hipError_t ell_fill<float>(const double*, int, int, long long, long long, int, bool,
                                    int*, float*, hipStream_t);

// ---------------------------------------------------------------------------
// The solver: one work-group per instance.
// ---------------------------------------------------------------------------
// Rows of R and of X per wave held in registers for an update, and entries
// per lane of such a row: rows up to 512 long, or (the narrow shape, for
// n, q <= 64) one entry per lane and more rows, so that the whole update's
// rows are loaded at once. Entries and rows past these go through device
// memory in the same per-lane order, so both shapes give the same sums.
constexpr int kSpRows = 3, kSpX = 2, kSpE = 8;
constexpr int kSpRowsNarrow = 11, kSpXNarrow = 4, kSpENarrow = 1;

// Sum over the ELL slots of line j (slot t at idx[t * stride + j]) of
// val * x[idx], in slot order. Padded slots (index -1, value 0) add zero;
// the loads of four slots go out before their products are summed.
template <typename T>
__device__ __forceinline__ double ell_dot(const int* idx, const T* val, int slots, int stride,
                                          int j, const T* x) {
    double acc = 0.0;
    int t = 0;
    for (; t + 4 <= slots; t += 4) {
        int i4[4];
        T v4[4], x4[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            i4[u] = idx[(t + u) * stride + j];
            v4[u] = val[(t + u) * stride + j];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) x4[u] = x[max(i4[u], 0)];
#pragma unroll
        for (int u = 0; u < 4; ++u) acc += (double)v4[u] * (double)x4[u];
    }
    for (; t < slots; ++t)
        acc += (double)val[t * stride + j] * (double)x[max(idx[t * stride + j], 0)];
    return acc;
}

constexpr int kMemBatch = 24;   // rows loaded per batch in the device-memory selection

// Rows [b, b + cnt) of the {r_i, rho_i} pairs (rho_i = r_i / ||A_i||^2, -1
// for rows with A_i = 0) in batches of kMemBatch 16-byte loads, visited in
// ascending order; fn(i, r_i, rho_i) returns true to stop.
template <typename Fn>
__device__ __forceinline__ void visit_rows(const double2* __restrict__ r2, int b, int cnt, Fn fn) {
    for (int j0 = 0; j0 < cnt; j0 += kMemBatch) {
        double2 v[kMemBatch];
#pragma unroll
        for (int u = 0; u < kMemBatch; ++u) {
            const int j = j0 + u;
            v[u] = j < cnt ? r2[b + j] : make_double2(0.0, -1.0);
        }
#pragma unroll
        for (int u = 0; u < kMemBatch; ++u)
            if (j0 + u < cnt && fn(b + j0 + u, v[u].x, v[u].y)) return;
    }
}

// The same over ||A_i||^2 alone (the weights of Alg. 1).
template <typename Fn>
__device__ __forceinline__ void visit_norms(const double* __restrict__ a, int b, int cnt, Fn fn) {
    for (int j0 = 0; j0 < cnt; j0 += kMemBatch) {
        double v[kMemBatch];
#pragma unroll
        for (int u = 0; u < kMemBatch; ++u) {
            const int j = j0 + u;
            v[u] = j < cnt ? a[b + j] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kMemBatch; ++u)
            if (j0 + u < cnt && fn(b + j0 + u, v[u])) return;
    }
}

// The selection step of Algs. 1-5 over norms held in device memory (an
// instance whose row norms do not fit in LDS): thread t reads its rows
// [b, b + cnt) where select_rows would hold them in registers, and every
// decision, sum and scan follows select_rows in the same order, so the two
// forms pick the same rows with the same arithmetic. rho_i >= 0 exactly for
// the rows with ||A_i|| > 0. cmax = max of rho over the thread's rows: a
// chunk whose maximum is below the threshold (or below M for MWRBK) holds
// no member and is not read.
__device__ SelectOut select_rows_mem(int variant, int b, int cnt, const double2* __restrict__ r2,
                                     const double* __restrict__ a, double cmax, double S, double M,
                                     double F_A,
                                     double theta, double u, long long k,
                                     const int* __restrict__ active, int n_active,
                                     BlockScratch& sc) {
    SelectOut o;
    o.setsize = 0;
    o.t = 0.0;
    o.T = 0.0;
    if (variant == kBK) {
        o.idx = active[k % n_active];
        return o;
    }
    if (variant == kMWRBK) {
        int cand = INT_MAX;
        if (cmax >= M)
            visit_rows(r2, b, cnt, [&](int i, double, double rho) {
                if (rho >= 0.0 && rho == M) {
                    cand = i;
                    return true;
                }
                return false;
            });
        if (threadIdx.x == 0) sc.out_i[2] = INT_MAX;
        cand = wave_min_int(cand);
        __syncthreads();
        if ((threadIdx.x & (kWave - 1)) == 0 && cand != INT_MAX) atomicMin(&sc.out_i[2], cand);
        __syncthreads();
        o.idx = sc.out_i[2];
        __syncthreads();
        o.setsize = 1;
        o.t = M;
        return o;
    }
    const bool greedy = variant == kGRBK || variant == kRGRBK;
    double t = 0.0;
    if (greedy) {
#pragma clang fp contract(off)
        const double th = (variant == kGRBK) ? 0.5 : theta;
        t = th * M + (1.0 - th) * (S / F_A);
        if (t > M) t = M;
    }
    // Members: a_i > 0 and, greedy, r_i / a_i >= t; weights r_i (greedy) or
    // a_i (Alg. 1).
    double ws = 0.0;
    int c = 0, lastm = -1;
    if (greedy) {
        if (cmax >= t)
            visit_rows(r2, b, cnt, [&](int i, double ri, double rho) {
                if (rho >= 0.0 && rho >= t) {
                    ws += ri;
                    ++c;
                    lastm = i;
                }
                return false;
            });
    }
    else
        visit_norms(a, b, cnt, [&](int i, double ai) {
            if (ai > 0.0) {
                ws += ai;
                ++c;
                lastm = i;
            }
            return false;
        });
    if (threadIdx.x == 0) {
        sc.out_i[2] = INT_MAX;
        sc.out_i[3] = -1;
    }
    double pre_w, T;
    int pre_c, tot_c;
    block_excl_scan(ws, c, pre_w, pre_c, T, tot_c, sc);
    const double target = u * T;
    int cand = INT_MAX;
    if (c > 0) {
        double run = pre_w;
        if (greedy)
            visit_rows(r2, b, cnt, [&](int i, double ri, double rho) {
                if (rho >= 0.0 && rho >= t) {
                    run += ri;
                    if (run > target) {
                        cand = i;
                        return true;
                    }
                }
                return false;
            });
        else
            visit_norms(a, b, cnt, [&](int i, double ai) {
                if (ai > 0.0) {
                    run += ai;
                    if (run > target) {
                        cand = i;
                        return true;
                    }
                }
                return false;
            });
    }
    cand = wave_min_int(cand);
    lastm = wave_max_int(lastm);
    if ((threadIdx.x & (kWave - 1)) == 0) {
        if (cand != INT_MAX) atomicMin(&sc.out_i[2], cand);
        if (lastm >= 0) atomicMax(&sc.out_i[3], lastm);
    }
    __syncthreads();
    o.idx = (sc.out_i[2] != INT_MAX) ? sc.out_i[2] : sc.out_i[3];
    o.setsize = tot_c;
    o.t = t;
    o.T = T;
    __syncthreads();
    return o;
}

// Optional phase timing (work-group 0, thread 0): wall-clock ticks per phase
// of an update, summed over the solve.
enum { kSpPhReduce, kSpPhSelect, kSpPhLoad, kSpPhV, kSpPhWX, kSpPhR, kSpPhCount };
#define MEK_SP_PHASE(id)                                                \
    do {                                                                \
        if (timing) {                                                   \
            const unsigned long long now_ = wall_clock64();             \
            ph[id] += now_ - t_last;                                    \
            t_last = now_;                                              \
        }                                                               \
    } while (0)

template <typename T, int SR, bool NARROW>
__global__ void __launch_bounds__(kThreads, 1) sparse_kernel(SparseParams<T> P) {
    constexpr int kRows = NARROW ? kSpRowsNarrow : kSpRows;
    constexpr int kXr = NARROW ? kSpXNarrow : kSpX;
    constexpr int kE = NARROW ? kSpENarrow : kSpE;
    extern __shared__ __align__(16) unsigned char dyn_smem[];
    __shared__ BlockScratch sc;
    // Memory form: bit t set when a row of thread t's chunk of norms (of row
    // errors of X) changed since the thread last summed the chunk.
    __shared__ unsigned int dirty[kThreads / 32];
    __shared__ unsigned int edirty[kThreads / 32];
    // Ragged batch: work-group b runs instance b with its own parameters
    // (own plan, sizes, state and slot).
    const bool ragged = P.multi != nullptr;
    if (ragged) P = P.multi[blockIdx.x];
    InstSlot sl = P.slots[ragged ? 0 : blockIdx.x];
    if (P.norms) {   // stream-ordered solves: the norms were computed on the device
        sl.C2 = P.norms[0];
        sl.ref2 = P.norms[1] > 0.0 ? P.norms[1] : 1.0;
    }
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
    const int m = P.m, n = P.n, p = P.p, q = P.q;
    T* const R = P.R + (size_t)sl.id * P.sR;
    T* const X = P.X + (size_t)sl.id * P.sX;
    const double* const Xref = P.Xref ? P.Xref + (size_t)sl.id * P.sX : nullptr;
    const bool has_ref = Xref != nullptr;
    const long long hbase = (long long)sl.id * P.hist_cap;

    // LDS: [r: m row norms] [e: p row errors] [Philox draws] [||A_i||^2 when
    // P.a_in_lds] [R_{i_k}: n] [v: q] [w: n] [the ELL slots of B's rows and
    // columns, indices then values, when P.b_in_lds] [those of A A^T and A,
    // when P.g_in_lds]. SR = 0: r and e stay in device memory (instances
    // whose norms do not fit in LDS) and the selection reads them there.
    constexpr bool kNormsLds = SR > 0;
    constexpr int kSR = SR > 0 ? SR : 1;
    double* const lds_d = reinterpret_cast<double*>(dyn_smem);
    double* r_l = lds_d;   // LDS form
    double2* const r2g = reinterpret_cast<double2*>(P.r_glob) + (size_t)sl.id * m;   // memory form
    double* e_l = kNormsLds ? lds_d + m : P.e_glob + (size_t)sl.id * P.sX;
    double* u_tab = kNormsLds ? lds_d + m + p : lds_d;
    double* a_l = u_tab + kUTable;
    T* rowv = reinterpret_cast<T*>(a_l + (P.a_in_lds ? m : 0));
    T* vv = rowv + ((n + 1) & ~1);
    T* ww = vv + ((q + 1) & ~1);
    int* bl_idx = reinterpret_cast<int*>(ww + ((n + 1) & ~1));
    int* btl_idx = bl_idx + ((P.kb * q + 1) & ~1);
    T* bl_val = reinterpret_cast<T*>(btl_idx + ((P.kbt * n + 1) & ~1));
    T* btl_val = bl_val + P.kb * q;
    unsigned char* after_b = reinterpret_cast<unsigned char*>(btl_val + P.kbt * n);
    if (!P.b_in_lds) after_b = reinterpret_cast<unsigned char*>(bl_idx);
    int* gl_idx = reinterpret_cast<int*>(after_b);
    int* al_idx = gl_idx + ((m * P.kg + 1) & ~1);
    T* gl_val = reinterpret_cast<T*>(al_idx + ((m * P.ka + 1) & ~1));
    T* al_val = gl_val + m * P.kg;
    const double* asrc = P.a_in_lds ? a_l : P.a;
    const int* b_idx = P.b_in_lds ? bl_idx : P.b_idx;
    const T* b_val = P.b_in_lds ? bl_val : P.b_val;
    const int* bt_idx = P.b_in_lds ? btl_idx : P.bt_idx;
    const T* bt_val = P.b_in_lds ? btl_val : P.bt_val;
    const int* g_idx = P.g_in_lds ? gl_idx : P.g_idx;
    const T* g_val = P.g_in_lds ? gl_val : P.g_val;
    const int* a_idx = P.g_in_lds ? al_idx : P.a_idx;
    const T* a_val = P.g_in_lds ? al_val : P.a_val;

    // ---- Set-up: all row norms of R and row errors of X, the cached data.
    if (P.a_in_lds)
        for (int i = tid; i < m; i += kThreads) a_l[i] = P.a[i];
    if (P.b_in_lds) {
        for (int e = tid; e < P.kb * q; e += kThreads) {
            bl_idx[e] = P.b_idx[e];
            bl_val[e] = P.b_val[e];
        }
        for (int e = tid; e < P.kbt * n; e += kThreads) {
            btl_idx[e] = P.bt_idx[e];
            btl_val[e] = P.bt_val[e];
        }
    }
    if (P.g_in_lds) {
        for (int e = tid; e < m * P.kg; e += kThreads) {
            gl_idx[e] = P.g_idx[e];
            gl_val[e] = P.g_val[e];
        }
        for (int e = tid; e < m * P.ka; e += kThreads) {
            al_idx[e] = P.a_idx[e];
            al_val[e] = P.a_val[e];
        }
    }
    for (int i = wv; i < m; i += kWaves) {
        const T* rp = R + (size_t)i * n;
        double acc = 0.0;
        for (int j = lane; j < n; j += kWave) {
            const double v = (double)rp[j];
            acc += v * v;
        }
        acc = wave_sum(acc);
        if (lane == 0) {
            if constexpr (kNormsLds) r_l[i] = acc;
            else r2g[i] = make_double2(acc, asrc[i] > 0.0 ? acc / asrc[i] : -1.0);
        }
    }
    for (int x = wv; x < p; x += kWaves) {
        double acc = 0.0;
        if (has_ref) {
            for (int j = lane; j < q; j += kWave) {
                const double d = (double)X[(size_t)x * q + j] - Xref[(size_t)x * q + j];
                acc += d * d;
            }
            acc = wave_sum(acc);
        }
        if (lane == 0) e_l[x] = acc;
    }
    if (tid < kThreads / 32) {
        dirty[tid] = ~0u;
        edirty[tid] = ~0u;
    }
    __syncthreads();

    const int cs = (m + kThreads - 1) / kThreads;
    const int sb = min(m, tid * cs);
    const int scnt = min(m, sb + cs) - sb;
    const int ecs = (p + kThreads - 1) / kThreads;
    const int eb = min(p, tid * ecs);
    const int ecnt = min(p, eb + ecs) - eb;
    double S0 = -1.0, S = 0.0, err = NAN;
    // Memory form: this thread's chunk sums of r and of the row errors, and
    // the chunk's maximum of rho.
    double chunk_S = 0.0, chunk_M = -1.0, chunk_E = 0.0;
    long long k = 0;
    int status = kMaxIter, last_set = 0;
    const bool timing = P.phase != nullptr && blockIdx.x == 0 && tid == 0;
    unsigned long long ph[kSpPhCount] = {0, 0, 0, 0, 0, 0};
    unsigned long long t_last = timing ? wall_clock64() : 0;
    for (;;) {
        if ((k % kUTable) == 0) {
            if (tid < kUTable) u_tab[tid] = philox_uniform(P.seed, sl.inst, k + tid);
            __syncthreads();
        }
        const double u_k = u_tab[k % kUTable];
        // ---- Global quantities and the stop test.
        double rr[kSR], aa[kSR], rho[kSR];
        double Sp = 0.0, Mp = -1.0, Ep = 0.0;
        if constexpr (kNormsLds) {
#pragma unroll
            for (int j = 0; j < SR; ++j) {
                rr[j] = (j < scnt) ? r_l[sb + j] : 0.0;
                aa[j] = (j < scnt) ? asrc[sb + j] : 0.0;
                rho[j] = (j < scnt && aa[j] > 0.0) ? rr[j] / aa[j] : -1.0;
                Sp += rr[j];
                Mp = fmax(Mp, rho[j]);
            }
        } else {
            // The same sums and maximum; the register form's padding adds
            // +0 and -1, which change neither. Only a chunk with a changed
            // row is read again; the others keep their last sums.
            const unsigned int bit = 1u << (tid & 31);
            if (dirty[tid >> 5] & bit) {
                visit_rows(r2g, sb, scnt, [&](int, double rj, double rho) {
                    Sp += rj;
                    Mp = fmax(Mp, rho);
                    return false;
                });
                chunk_S = Sp;
                chunk_M = Mp;
                atomicAnd(&dirty[tid >> 5], ~bit);
            } else {
                Sp = chunk_S;
                Mp = chunk_M;
            }
        }
        if constexpr (kNormsLds) {
#pragma unroll 8
            for (int j = 0; j < ecnt; ++j) Ep += e_l[eb + j];
        } else {
            const unsigned int bit = 1u << (tid & 31);
            if (edirty[tid >> 5] & bit) {
#pragma unroll 8
                for (int j = 0; j < ecnt; ++j) Ep += e_l[eb + j];
                chunk_E = Ep;
                atomicAnd(&edirty[tid >> 5], ~bit);
            } else {
                Ep = chunk_E;
            }
        }
        block_sum_max_sum(Sp, Mp, Ep, sc);
        S = Sp;
        const double M = Mp;
        if (S0 < 0.0) S0 = S;
        err = has_ref ? sqrt(Ep / sl.ref2) : NAN;
        const long long hk = sl.hist_offset + k;
        if (tid == 0 && hk < P.hist_cap) {
            if (P.resid_hist) P.resid_hist[hbase + hk] = S;
            if (P.err_hist) P.err_hist[hbase + hk] = err;
        }
        if (P.stop == kStopRelErr && err <= P.tol) { status = kOK; break; }
        if (P.stop == kStopRelResid && sqrt(S) <= P.tol * sqrt(sl.C2)) { status = kOK; break; }
        if (sl.S_target > 0.0 && S <= sl.S_target) { status = kOK; break; }
        if (S == 0.0) { status = kExact; break; }
        if (!isfinite(S) || (P.diverge > 0.0 && S > P.diverge * S0)) { status = kEDiverged; break; }
        if (k >= sl.max_iters) { status = kMaxIter; break; }
        MEK_SP_PHASE(kSpPhReduce);

        // ---- Selection.
        int ik;
        if (P.replay && k < P.replay_len) {
            ik = P.replay[k];
            last_set = 0;
        } else {
            SelectOut so;
            if constexpr (kNormsLds)
                so = select_rows<kSR>(P.variant, sb, scnt, rr, aa, rho, S, M, P.F_A, P.theta, u_k, k,
                                      P.active, P.n_active, sc, nullptr, nullptr);
            else
                so = select_rows_mem(P.variant, sb, scnt, r2g, asrc, chunk_M, S, M, P.F_A, P.theta,
                                     u_k, k, P.active, P.n_active, sc);
            ik = so.idx;
            last_set = so.setsize;
        }
        if (tid == 0 && hk < P.hist_cap) {
            if (P.idx_hist) P.idx_hist[hbase + hk] = ik;
            if (P.set_hist) P.set_hist[hbase + hk] = last_set;
        }
        const double c = P.alpha / asrc[ik];
        MEK_SP_PHASE(kSpPhSelect);

        // ---- Loads of the whole update, issued now so that they travel
        // while v and w are formed: R_{i_k} into LDS, and into registers
        // this wave's rows of R (column i_k of A A^T, slots wv + u kWaves)
        // and of X and X_ref (row i_k of A, likewise).
        int ri[kRows], xi[kXr];
        double gv[kRows], av[kXr];
        T rreg[kRows][kE], xreg[kXr][kE];
        double xrf[kXr][kE];
#pragma unroll
        for (int u = 0; u < kRows; ++u) {
            const int t = wv + u * kWaves;
            ri[u] = t < P.kg ? g_idx[(size_t)ik * P.kg + t] : -1;
            gv[u] = ri[u] >= 0 ? (double)g_val[(size_t)ik * P.kg + t] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kXr; ++u) {
            const int t = wv + u * kWaves;
            xi[u] = t < P.ka ? a_idx[(size_t)ik * P.ka + t] : -1;
            av[u] = xi[u] >= 0 ? (double)a_val[(size_t)ik * P.ka + t] : 0.0;
        }
        for (int j = tid; j < n; j += kThreads) rowv[j] = R[(size_t)ik * n + j];
#pragma unroll
        for (int u = 0; u < kRows; ++u)
#pragma unroll
            for (int e = 0; e < kE; ++e) {
                const int l = lane + e * kWave;
                rreg[u][e] = (ri[u] >= 0 && l < n) ? R[(size_t)ri[u] * n + l] : (T)0;
            }
#pragma unroll
        for (int u = 0; u < kXr; ++u)
#pragma unroll
            for (int e = 0; e < kE; ++e) {
                const int j = lane + e * kWave;
                const bool in = xi[u] >= 0 && j < q;
                xreg[u][e] = in ? X[(size_t)xi[u] * q + j] : (T)0;
                xrf[u][e] = (in && has_ref) ? Xref[(size_t)xi[u] * q + j] : 0.0;
            }
        __syncthreads();
        MEK_SP_PHASE(kSpPhLoad);
        // ---- v = R_{i_k} B^T over the nonzeros of each row of B.
        for (int j = tid; j < q; j += kThreads) vv[j] = (T)ell_dot(b_idx, b_val, P.kb, q, j, rowv);
        __syncthreads();
        MEK_SP_PHASE(kSpPhV);
        // ---- w = v B over the nonzeros of each column of B; the rows of X
        // where A_{i_k} is nonzero, with their errors.
        for (int l = tid; l < n; l += kThreads) ww[l] = (T)ell_dot(bt_idx, bt_val, P.kbt, n, l, vv);
        // A row of X or R updated from device memory (rows past the ones
        // held in registers, entries past kE per lane).
        auto x_tail = [&](int x, T ca, int j0, double acc) {
            T* xr = X + (size_t)x * q;
            for (int j = j0; j < q; j += kWave) {
                const T nv = xr[j] + ca * vv[j];
                xr[j] = nv;
                if (has_ref) {
                    const double d = (double)nv - Xref[(size_t)x * q + j];
                    acc += d * d;
                }
            }
            if (has_ref) acc = wave_sum(acc);
            if (lane == 0) {
                e_l[x] = acc;
                if constexpr (!kNormsLds) {
                    const int owner = x / ecs;
                    atomicOr(&edirty[owner >> 5], 1u << (owner & 31));
                }
            }
        };
        auto r_tail = [&](int i, T cg, int l0, double acc) {
            T* rp = R + (size_t)i * n;
            for (int l = l0; l < n; l += kWave) {
                const T nv = rp[l] - cg * ww[l];
                rp[l] = nv;
                acc += (double)nv * (double)nv;
            }
            acc = wave_sum(acc);
            if (lane == 0) {
                if constexpr (kNormsLds) {
                    r_l[i] = acc;
                } else {
                    r2g[i] = make_double2(acc, asrc[i] > 0.0 ? acc / asrc[i] : -1.0);
                    const int owner = i / cs;
                    atomicOr(&dirty[owner >> 5], 1u << (owner & 31));
                }
            }
        };
#pragma unroll
        for (int u = 0; u < kXr; ++u) {
            if (xi[u] < 0) continue;
            const T ca = (T)(c * av[u]);
            T* xr = X + (size_t)xi[u] * q;
            double acc = 0.0;
#pragma unroll
            for (int e = 0; e < kE; ++e) {
                const int j = lane + e * kWave;
                if (j < q) {
                    const T nv = xreg[u][e] + ca * vv[j];
                    xr[j] = nv;
                    if (has_ref) {
                        const double d = (double)nv - xrf[u][e];
                        acc += d * d;
                    }
                }
            }
            x_tail(xi[u], ca, lane + kE * kWave, acc);
        }
        for (int t = wv + kXr * kWaves; t < P.ka; t += kWaves) {
            const int x = a_idx[(size_t)ik * P.ka + t];
            if (x < 0) break;
            x_tail(x, (T)(c * (double)a_val[(size_t)ik * P.ka + t]), lane, 0.0);
        }
        __syncthreads();
        MEK_SP_PHASE(kSpPhWX);
        // ---- The rows of R where column i_k of A A^T is nonzero, with their
        // new norms.
#pragma unroll
        for (int u = 0; u < kRows; ++u) {
            if (ri[u] < 0) continue;
            const T cg = (T)(c * gv[u]);
            T* rp = R + (size_t)ri[u] * n;
            double acc = 0.0;
#pragma unroll
            for (int e = 0; e < kE; ++e) {
                const int l = lane + e * kWave;
                if (l < n) {
                    const T nv = rreg[u][e] - cg * ww[l];
                    rp[l] = nv;
                    acc += (double)nv * (double)nv;
                }
            }
            r_tail(ri[u], cg, lane + kE * kWave, acc);
        }
        for (int t = wv + kRows * kWaves; t < P.kg; t += kWaves) {
            const int i = g_idx[(size_t)ik * P.kg + t];
            if (i < 0) break;
            r_tail(i, (T)(c * (double)g_val[(size_t)ik * P.kg + t]), lane, 0.0);
        }
        __syncthreads();
        MEK_SP_PHASE(kSpPhR);
        ++k;
    }
    if (timing)
        for (int i = 0; i < kSpPhCount; ++i) P.phase[i] += ph[i];
    if (tid == 0) {
        DevReport* rep = P.report + sl.id;
        rep->iters = k;
        rep->status = status;
        rep->last_set = last_set;
        rep->S = S;
        rep->err = err;
    }
}

size_t sparse_lds_bytes(int m, int p, int q, int n, size_t elem, bool norms_in_lds,
                        bool a_in_lds, int kb, int kbt, int ka, int kg) {
    size_t b = (size_t)((norms_in_lds ? m + p : 0) + kUTable + (a_in_lds ? m : 0)) * sizeof(double);
    b += (size_t)(2 * ((n + 1) & ~1) + ((q + 1) & ~1)) * elem;
    if (kb > 0)   // the ELL slots of B cached in LDS
        b += (size_t)(((kb * q + 1) & ~1) + ((kbt * n + 1) & ~1)) * sizeof(int) +
             (size_t)(kb * q + kbt * n) * elem;
    if (kg > 0)   // the ELL slots of A A^T and A cached in LDS
        b += (size_t)(((m * kg + 1) & ~1) + ((m * ka + 1) & ~1)) * sizeof(int) +
             (size_t)(m * kg + m * ka) * elem;
    return b;
}

template <typename T, int SR>
static hipError_t launch_sparse_sr(const SparseParams<T>& P, size_t lds_bytes, hipStream_t s) {
    // The narrow shape for instances of at most 64 columns of R and X (the
    // first instance's sizes decide for a ragged table; either shape is
    // correct for any size).
    auto kern = (P.n <= kWave && P.q <= kWave) ? sparse_kernel<T, SR, true>
                                               : sparse_kernel<T, SR, false>;
    if (hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds_bytes) != hipSuccess)
        (void)hipGetLastError();
    kern<<<P.nb, kThreads, lds_bytes, s>>>(P);
    return hipGetLastError();
}

template <typename T>
static hipError_t launch_sparse_t(const SparseParams<T>& P, size_t lds_bytes, hipStream_t s) {
    if (!P.norms_in_lds) return launch_sparse_sr<T, 0>(P, lds_bytes, s);
    switch (sel_rows_for(P.m)) {
        case 1: return launch_sparse_sr<T, 1>(P, lds_bytes, s);
        case 2: return launch_sparse_sr<T, 2>(P, lds_bytes, s);
        case 4: return launch_sparse_sr<T, 4>(P, lds_bytes, s);
        case 8: return launch_sparse_sr<T, 8>(P, lds_bytes, s);
        default: return launch_sparse_sr<T, 16>(P, lds_bytes, s);
    }
}

hipError_t launch_sparse(const SparseParams<double>& P, size_t lds_bytes, hipStream_t s) {
    return launch_sparse_t(P, lds_bytes, s);
}
hipError_t launch_sparse(const SparseParams<float>& P, size_t lds_bytes, hipStream_t s) {
    return launch_sparse_t(P, lds_bytes, s);
}

}  // namespace mek
