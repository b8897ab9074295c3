/*
 * Plain FP64 CPU oracle for the block Kaczmarz family that solves AXB = C.
 *
 * TEST INFRASTRUCTURE ONLY. This file is the slow, obviously-correct
 * reference that the GPU library is checked against. Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it.
 * It shares no code, header, table or helper with the GPU library.
 *
 * Paper: "Greedy randomized block Kaczmarz method for matrix equation
 * AXB = C and its applications in color image restoration" (arXiv 2408.05444).
 *
 *   Alg. 1 (ME-RBK, Sec. 2):  i_k drawn with probability ||A_i||^2 / ||A||_F^2,
 *       X += alpha/||A_i||^2 * A_i^T (C_i - A_i X B) B^T.
 *   Alg. 2 (ME-BK, Sec. 3):   i_k = (k mod m) + 1, same update.
 *   Alg. 3 (ME-GRBK, Sec. 4): threshold zeta_k, index set J_k, sample i in J_k
 *       with probability ||R_i||^2 / sum_{J_k} ||R_j||^2, update X, and keep
 *       the residual R = C - A X B up to date with the Gram matrices A A^T and
 *       B^T B (the remark right after Alg. 3).
 *   Alg. 4 (ME-RGRBK):        the same with the relaxed threshold xi_k(theta);
 *       theta = 1/2 is Alg. 3 (Remark 4.4).
 *   Alg. 5 (ME-MWRBK):        i_k = an index maximising ||R_i||^2 / ||A_i||^2.
 *
 * Readings of points the paper leaves open (each one is listed in the
 * design notes):
 *   - B is q x n (eq. 1.1); the theorems' "n x q" is a typo.
 *   - Rows with ||A_i|| = 0 are never selected (they would divide by zero).
 *   - The threshold tests of Algs. 3/4 are evaluated in the equivalent
 *     ratio form ||R_i||^2/||A_i||^2 >= t with
 *         t = min(M, theta*M + (1-theta)*||R||_F^2/||A||_F^2),
 *     M = max_i ||R_i||^2/||A_i||^2. Multiplying the paper's
 *     inequality through by 1/(||A_i||^2 ||R||_F^2) gives this form exactly;
 *     the min() keeps the maximiser in the set under rounding, as Remark 4.1
 *     proves it is in exact arithmetic.
 *   - Sampling "with probability ||R~_i||^2/||R~||_F^2" is done by inverse
 *     CDF in ascending row order: u in [0,1), target = u * T,
 *     T = sum over the set of ||R_i||^2 (ascending), choose the first row whose
 *     running sum exceeds the target, else the last row of the set.
 *   - u for iteration k is (w0 >> 11) * 2^-53, w0 the first 64-bit word of
 *     Philox4x64-10 (Salmon et al., SC'11) with key (seed, instance) and
 *     counter (k+1, 0, 0, 0).
 *   - MWRBK ties (Remark after Alg. 5: "any one") go to the lowest index.
 *   - ME-BK cycles over the rows with nonzero norm, in ascending order.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define MO_BK 0
#define MO_RBK 1
#define MO_GRBK 2
#define MO_RGRBK 3
#define MO_MWRBK 4

#define MO_STOP_NONE 0
#define MO_STOP_REL_ERR 1
#define MO_STOP_REL_RESID 2

#define MO_OK 0
#define MO_MAXITER 1
#define MO_EXACT 2
#define MO_EINVAL -1
#define MO_ENOMEM -2
#define MO_EDIVERGED -5

/* ---------------------------------------------------------------------- */
/* Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as  */
/* easy as 1, 2, 3", SC'11): 10 rounds of a multiply-xor network on four    */
/* 64-bit words, with a Weyl-sequence key schedule between rounds.          */
/* ---------------------------------------------------------------------- */
static const uint64_t PH_MUL0 = 0xD2E7470EE14C6C93ULL;
static const uint64_t PH_MUL1 = 0xCA5A826395121157ULL;
static const uint64_t PH_WEYL0 = 0x9E3779B97F4A7C15ULL; /* golden ratio */
static const uint64_t PH_WEYL1 = 0xBB67AE8584CAA73BULL; /* sqrt(3) - 1 */

static void mul_wide(uint64_t a, uint64_t b, uint64_t* hi, uint64_t* lo) {
    unsigned __int128 prod = (unsigned __int128)a * (unsigned __int128)b;
    *hi = (uint64_t)(prod >> 64);
    *lo = (uint64_t)prod;
}

void mo_philox4x64_10(const uint64_t ctr_in[4], const uint64_t key_in[2], uint64_t out[4]) {
    uint64_t x0 = ctr_in[0], x1 = ctr_in[1], x2 = ctr_in[2], x3 = ctr_in[3];
    uint64_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += PH_WEYL0;
            k1 += PH_WEYL1;
        }
        uint64_t hi0, lo0, hi1, lo1;
        mul_wide(PH_MUL0, x0, &hi0, &lo0);
        mul_wide(PH_MUL1, x2, &hi1, &lo1);
        uint64_t y0 = hi1 ^ x1 ^ k0;
        uint64_t y1 = lo1;
        uint64_t y2 = hi0 ^ x3 ^ k1;
        uint64_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Threads the row loops use: 1 in the plain build. */
int mo_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Uniform draw in [0, 1) for iteration k of instance `inst`. */
double mo_uniform(uint64_t seed, uint64_t inst, int64_t k) {
    uint64_t ctr[4] = {(uint64_t)k + 1u, 0u, 0u, 0u};
    uint64_t key[2] = {seed, inst};
    uint64_t out[4];
    mo_philox4x64_10(ctr, key, out);
    return (double)(out[0] >> 11) * (1.0 / 9007199254740992.0); /* 2^-53 */
}

/* ---------------------------------------------------------------------- */
/* Index selection (Algs. 1-5). r[i] = ||R_i||^2, a[i] = ||A_i||^2,          */
/* F_A = ||A||_F^2. Returns the chosen row (0-based), or -1 if no row of A  */
/* is nonzero. For the greedy variants, in_set (optional, m bytes) receives */
/* the index set, *t_out the ratio threshold and *T_out the set's weight.   */
/* ---------------------------------------------------------------------- */
int64_t mo_select(int variant, int64_t m, const double* r, const double* a, double F_A,
                  double theta, uint64_t seed, uint64_t inst, int64_t k,
                  unsigned char* in_set, double* t_out, double* T_out) {
    int64_t n_active = 0;
    for (int64_t i = 0; i < m; ++i)
        if (a[i] > 0.0) ++n_active;
    if (in_set && m > 0) memset(in_set, 0, (size_t)m);
    if (n_active == 0) return -1;

    if (variant == MO_BK) {
        /* Alg. 2: cyclic sweep, here over the rows that can be projected on. */
        int64_t want = k % n_active, seen = 0;
        for (int64_t i = 0; i < m; ++i) {
            if (a[i] > 0.0) {
                if (seen == want) return i;
                ++seen;
            }
        }
        return -1;
    }

    if (variant == MO_RBK) {
        /* Alg. 1: row i with probability ||A_i||^2 / ||A||_F^2. */
        double target = mo_uniform(seed, inst, k) * F_A;
        double run = 0.0;
        int64_t last = -1;
        for (int64_t i = 0; i < m; ++i) {
            if (!(a[i] > 0.0)) continue;
            run += a[i];
            last = i;
            if (run > target) return i;
        }
        return last;
    }

    /* The greedy variants all need M = max_i ||R_i||^2/||A_i||^2. */
    double M = 0.0;
    int64_t argmax = -1;
    for (int64_t i = 0; i < m; ++i) {
        if (!(a[i] > 0.0)) continue;
        double rho = r[i] / a[i];
        if (argmax < 0 || rho > M) {
            M = rho;
            argmax = i;
        }
    }

    if (variant == MO_MWRBK) {
        /* Alg. 5: the (lowest) maximiser of ||R_i||^2 / ||A_i||^2. */
        if (in_set) in_set[argmax] = 1;
        if (t_out) *t_out = M;
        if (T_out) *T_out = r[argmax];
        return argmax;
    }

    /* Algs. 3 and 4. GRBK is theta = 1/2 (Remark 4.4). */
    if (variant == MO_GRBK) theta = 0.5;
    double S = 0.0;
    for (int64_t i = 0; i < m; ++i) S += r[i];
    double mean_ratio = S / F_A;
    double t = theta * M + (1.0 - theta) * mean_ratio;
    if (t > M) t = M;

    double T = 0.0;
    for (int64_t i = 0; i < m; ++i) {
        if (a[i] > 0.0 && r[i] / a[i] >= t) {
            if (in_set) in_set[i] = 1;
            T += r[i];
        }
    }
    if (t_out) *t_out = t;
    if (T_out) *T_out = T;

    double target = mo_uniform(seed, inst, k) * T;
    double run = 0.0;
    int64_t last = -1;
    for (int64_t i = 0; i < m; ++i) {
        if (a[i] > 0.0 && r[i] / a[i] >= t) {
            run += r[i];
            last = i;
            if (run > target) return i;
        }
    }
    return last;
}

/* ---------------------------------------------------------------------- */
/* Dense helpers (row-major, plain triple loops).                          */
/* ---------------------------------------------------------------------- */

/* R = C - A X B, A m x p, X p x q, B q x n (the residual of eq. 1.1). */
void mo_residual(int64_t m, int64_t p, int64_t q, int64_t n, const double* A, const double* X,
                 const double* B, const double* C, double* R) {
    double* AX = (double*)malloc(sizeof(double) * (size_t)(m * q > 0 ? m * q : 1));
    for (int64_t i = 0; i < m; ++i)
        for (int64_t l = 0; l < q; ++l) {
            double s = 0.0;
            for (int64_t j = 0; j < p; ++j) s += A[i * p + j] * X[j * q + l];
            AX[i * q + l] = s;
        }
    for (int64_t i = 0; i < m; ++i)
        for (int64_t j = 0; j < n; ++j) {
            double s = 0.0;
            for (int64_t l = 0; l < q; ++l) s += AX[i * q + l] * B[l * n + j];
            R[i * n + j] = C[i * n + j] - s;
        }
    free(AX);
}

/* G = M M^T for M rows x cols (row-major). */
void mo_gram_rows(int64_t rows, int64_t cols, const double* M, double* G) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < rows; ++i)
        for (int64_t l = 0; l < rows; ++l) {
            double s = 0.0;
            for (int64_t j = 0; j < cols; ++j) s += M[i * cols + j] * M[l * cols + j];
            G[i * rows + l] = s;
        }
}

/* G = M^T M for M rows x cols (row-major). */
void mo_gram_cols(int64_t rows, int64_t cols, const double* M, double* G) {
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < cols; ++j)
        for (int64_t l = 0; l < cols; ++l) {
            double s = 0.0;
            for (int64_t i = 0; i < rows; ++i) s += M[i * cols + j] * M[i * cols + l];
            G[j * cols + l] = s;
        }
}

static double frob_diff2(int64_t len, const double* X, const double* Y) {
    double s = 0.0;
    for (int64_t i = 0; i < len; ++i) {
        double d = X[i] - Y[i];
        s += d * d;
    }
    return s;
}

/* ---------------------------------------------------------------------- */
/* The iteration.                                                          */
/*                                                                          */
/* Inputs: A (m x p), B (q x n), C (m x n), X0 (p x q, NULL = zero).       */
/* variant, theta (RGRBK only), alpha (step), stop rule + tol, Xref         */
/* (p x q, needed for the REL_ERR rule and for err_hist), max_iters,        */
/* seed/inst for the Philox draws, forced (optional index sequence that     */
/* replaces the selection rule, length n_forced), literal (0: keep R up to  */
/* date with the Gram matrices as in Alg. 3; 1: recompute the selected       */
/* residual row as C_i - A_i X B and all row norms from scratch each step,   */
/* as written in Algs. 1, 2 and 5), diverge (stop with EDIVERGED once        */
/* ||R||_F^2 exceeds diverge * ||R^0||_F^2; <= 0 disables).                   */
/*                                                                          */
/* Outputs: X (p x q), *iters = number of updates made, *status, and the    */
/* optional histories: s_hist[k] = ||R^k||_F^2 and e_hist[k] =              */
/* ||X^k - Xref||_F / ||Xref||_F for k = 0..iters (capacity hist_cap), and   */
/* idx_hist[k] = i_k for k = 0..iters-1, set_hist[k] = |index set|.          */
/*                                                                          */
/* Stop tests are evaluated before every update, so 0 updates are made when */
/* X0 already meets the tolerance; the iteration count is the number of     */
/* updates (Sec. 5's IT).                                                   */
/* ---------------------------------------------------------------------- */
int mo_solve(int64_t m, int64_t p, int64_t q, int64_t n, const double* A, const double* B,
             const double* C, const double* X0, int variant, double theta, double alpha,
             int stop, double tol, const double* Xref, int64_t max_iters, uint64_t seed,
             uint64_t inst, const int64_t* forced, int64_t n_forced, int literal, double diverge,
             double* X, int64_t* iters, int* status, double* s_hist, double* e_hist,
             int64_t* idx_hist, int64_t* set_hist, int64_t hist_cap) {
    if (m <= 0 || p <= 0 || q <= 0 || n <= 0 || !A || !B || !C || !X || !iters || !status)
        return MO_EINVAL;
    if (variant < MO_BK || variant > MO_MWRBK) return MO_EINVAL;
    if (stop == MO_STOP_REL_ERR && !Xref) return MO_EINVAL;
    if (!(alpha > 0.0)) return MO_EINVAL;

    size_t mn = (size_t)(m * n), pq = (size_t)(p * q);
    double* a = (double*)calloc((size_t)m, sizeof(double));
    double* r = (double*)calloc((size_t)m, sizeof(double));
    double* R = (double*)malloc(sizeof(double) * mn);
    double* GA = literal ? NULL : (double*)malloc(sizeof(double) * (size_t)(m * m));
    double* GB = literal ? NULL : (double*)malloc(sizeof(double) * (size_t)(n * n));
    double* v = (double*)malloc(sizeof(double) * (size_t)q);
    double* w = (double*)malloc(sizeof(double) * (size_t)n);
    double* Ri = (double*)malloc(sizeof(double) * (size_t)n);
    unsigned char* in_set = (unsigned char*)malloc((size_t)m);
    if (!a || !r || !R || (!literal && (!GA || !GB)) || !v || !w || !Ri || !in_set) {
        free(a); free(r); free(R); free(GA); free(GB); free(v); free(w); free(Ri); free(in_set);
        return MO_ENOMEM;
    }

    /* ||A_i||^2 and ||A||_F^2. */
    double F_A = 0.0;
    for (int64_t i = 0; i < m; ++i) {
        double s = 0.0;
        for (int64_t j = 0; j < p; ++j) s += A[i * p + j] * A[i * p + j];
        a[i] = s;
        F_A += s;
    }
    /* Gram matrices A A^T and B^T B, computed once (remark after Alg. 3). */
    if (!literal) {
        mo_gram_rows(m, p, A, GA);
        mo_gram_cols(q, n, B, GB);
    }
    /* X^0 and R^0 = C - A X^0 B (initialisation of Alg. 3). */
    if (X0) memcpy(X, X0, sizeof(double) * pq);
    else memset(X, 0, sizeof(double) * pq);
    if (X0) mo_residual(m, p, q, n, A, X, B, C, R);
    else memcpy(R, C, sizeof(double) * mn);

    double ref2 = 0.0, C2 = 0.0;
    if (Xref)
        for (size_t i = 0; i < pq; ++i) ref2 += Xref[i] * Xref[i];
    for (size_t i = 0; i < mn; ++i) C2 += C[i] * C[i];

    double S0 = -1.0;
    int64_t k = 0;
    int st = MO_MAXITER;
    for (;;) {
        if (literal) mo_residual(m, p, q, n, A, X, B, C, R);
        double S = 0.0;
        /* Row-parallel in the OpenMP build (each row's sum in the same
         * order; the total below in ascending row order, as in the plain
         * build). */
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < m; ++i) {
            double s = 0.0;
            for (int64_t j = 0; j < n; ++j) s += R[i * n + j] * R[i * n + j];
            r[i] = s;
        }
        for (int64_t i = 0; i < m; ++i) S += r[i];
        if (S0 < 0.0) S0 = S;
        double err = Xref ? sqrt(frob_diff2((int64_t)pq, X, Xref) / (ref2 > 0.0 ? ref2 : 1.0)) : NAN;
        if (k < hist_cap) {
            if (s_hist) s_hist[k] = S;
            if (e_hist) e_hist[k] = err;
        }
        if (stop == MO_STOP_REL_ERR && err <= tol) { st = MO_OK; break; }
        if (stop == MO_STOP_REL_RESID && sqrt(S) <= tol * sqrt(C2)) { st = MO_OK; break; }
        if (S == 0.0) { st = MO_EXACT; break; }
        if (!isfinite(S) || (diverge > 0.0 && S > diverge * S0)) { st = MO_EDIVERGED; break; }
        if (k >= max_iters) { st = MO_MAXITER; break; }

        int64_t ik;
        if (forced && k < n_forced) {
            ik = forced[k];
            if (ik < 0 || ik >= m || !(a[ik] > 0.0)) { st = MO_EINVAL; break; }
            if (set_hist && k < hist_cap) set_hist[k] = 0;
        } else {
            ik = mo_select(variant, m, r, a, F_A, theta, seed, inst, k, in_set, NULL, NULL);
            if (ik < 0) { st = MO_EINVAL; break; }
            if (set_hist && k < hist_cap) {
                int64_t cnt = 0;
                for (int64_t i = 0; i < m; ++i) cnt += in_set[i];
                set_hist[k] = (variant == MO_GRBK || variant == MO_RGRBK || variant == MO_MWRBK) ? cnt : 0;
            }
        }
        if (idx_hist && k < hist_cap) idx_hist[k] = ik;

        double c = alpha / a[ik];
        /* The selected residual row (from the pre-update iterate). */
        memcpy(Ri, R + ik * n, sizeof(double) * (size_t)n);
        /* v = R_i B^T (q-vector). */
#pragma omp parallel for schedule(static)
        for (int64_t l = 0; l < q; ++l) {
            double s = 0.0;
            for (int64_t j = 0; j < n; ++j) s += Ri[j] * B[l * n + j];
            v[l] = s;
        }
        /* X^{k+1} = X^k + alpha/||A_i||^2 A_i^T (R_i B^T). */
#pragma omp parallel for schedule(static)
        for (int64_t s_ = 0; s_ < p; ++s_) {
            double cas = c * A[ik * p + s_];
            for (int64_t l = 0; l < q; ++l) X[s_ * q + l] += cas * v[l];
        }
        if (!literal) {
            /* w = R_i (B^T B) (n-vector). */
#pragma omp parallel for schedule(static)
            for (int64_t j = 0; j < n; ++j) {
                double s = 0.0;
                for (int64_t l = 0; l < n; ++l) s += Ri[l] * GB[l * n + j];
                w[j] = s;
            }
            /* R^{k+1} = R^k - alpha/||A_i||^2 (A A^T)_{:,i} (R_i B^T B). */
#pragma omp parallel for schedule(static)
            for (int64_t h = 0; h < m; ++h) {
                double cg = c * GA[h * m + ik];
                for (int64_t j = 0; j < n; ++j) R[h * n + j] -= cg * w[j];
            }
        }
        ++k;
    }
    *iters = k;
    *status = st;
    free(a); free(r); free(R); free(GA); free(GB); free(v); free(w); free(Ri); free(in_set);
    return st;
}
