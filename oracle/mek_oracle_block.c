/*
 * Plain FP64 CPU oracle for the two-sided greedy block projection: the
 * extension of the greedy row criterion of Algs. 3/4 to single entries of the
 * residual, with an exact projection onto the selected block of equations.
 *
 * TEST INFRASTRUCTURE ONLY (see mek_oracle.c): loaded by the test suite, the
 * smoke check and the benchmark's CPU-baseline leg, never by the library.
 *
 * The paper's iteration (Algs. 3/4) projects onto one row of equations,
 * A_i X B = C_i, with the step alpha B^T standing in for the inverse of
 * B B^T. The extension keeps its structure but works on entries: equation
 * (i, j) of A X B = C reads A_i X B_j = C_ij (B_j the j-th column of B), and
 * the single-entry projection of X onto it lowers ||X - X*||_F^2 by
 * R_ij^2 / (||A_i||^2 ||B_j||^2) for every solution X*. With
 *     omega_ij = R_ij^2 / (a_i b_j),  a_i = ||A_i||^2,  b_j = ||B_j||^2,
 *     Omega = max omega_ij,  S = ||R||_F^2,  F_A = ||A||_F^2,  F_B = ||B||_F^2,
 * the threshold is the relaxed one of Alg. 4 carried over to entries,
 *     eps = min(Omega, theta Omega + (1 - theta) S / (F_A F_B)),
 * where S / (F_A F_B) is the mean of omega weighted by a_i b_j, so the
 * largest entry always passes (the argument of Remark 4.1). A row (column)
 * is a candidate when its largest omega passes; rows are ranked by that
 * largest omega (ties: lower index first); of the first s ranked rows, a row
 * is dropped when the part of A_i orthogonal to the higher-ranked rows kept
 * has squared norm at most tau * a_i (the pivot of a Cholesky factorisation
 * of A_I A_I^T in rank order), so at most s rows are kept; columns likewise
 * with B^T B, of the first t ranked columns. The step projects X onto {X : A_I X B_J = C_IJ}:
 *     W = (A_I A_I^T)^{-1} R_IJ (B_J^T B_J)^{-1},
 *     X += A_I^T W B_J^T,
 *     R -= (A A^T)_{:,I} W (B^T B)_{J,:},
 * the residual update in the Gram form of the remark after Alg. 3.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define MO_STOP_REL_ERR 1
#define MO_STOP_REL_RESID 2

#define MO_OK 0
#define MO_MAXITER 1
#define MO_EXACT 2
#define MO_EINVAL -1
#define MO_ENOMEM -2
#define MO_EDIVERGED -5

/* Rank candidates: indices with score >= eps, by score descending, then index
 * ascending (a plain insertion sort). Returns the number of candidates. */
static int64_t rank_candidates(int64_t len, const double* score, const unsigned char* usable,
                               double eps, int64_t* order) {
    int64_t cnt = 0;
    for (int64_t i = 0; i < len; ++i) {
        if (!usable[i] || !(score[i] >= eps)) continue;
        int64_t pos = cnt;
        while (pos > 0 && score[order[pos - 1]] < score[i]) {
            order[pos] = order[pos - 1];
            --pos;
        }
        order[pos] = i;
        ++cnt;
    }
    return cnt;
}

/* Pivoted Cholesky over the first cap ranked candidates: keep candidate c
 * when G_cc - sum_x L[r][x]^2 > tau * G_cc, with L the factor of G restricted
 * to the kept indices (row-major, ld = cap). G is len x len row-major. */
static int64_t take_independent(int64_t cnt, const int64_t* order, const double* G, int64_t len,
                                double tau, int64_t cap, int64_t* taken, double* L) {
    int64_t r = 0;
    for (int64_t c = 0; c < cnt && c < cap; ++c) {
        const int64_t i = order[c];
        double* Lr = L + r * cap;
        for (int64_t x = 0; x < r; ++x) {
            double s = G[i * len + taken[x]];
            for (int64_t y = 0; y < x; ++y) s -= Lr[y] * L[x * cap + y];
            Lr[x] = s / L[x * cap + x];
        }
        double d = G[i * len + i];
        for (int64_t x = 0; x < r; ++x) d -= Lr[x] * Lr[x];
        if (d > tau * G[i * len + i]) {
            Lr[r] = sqrt(d);
            taken[r] = i;
            ++r;
        }
    }
    return r;
}

/* Selection of one step. R (m x n), a (m), b (n), GA (m x m), GB (n x n).
 * Outputs I (s_max), J (t_max) in the order taken, their sizes, eps and
 * Omega. Returns 0, or -1 when no entry has a_i > 0 and b_j > 0. */
int mo_select_2s(int64_t m, int64_t n, const double* R, const double* a, const double* b,
                 double F_A, double F_B, double theta, int64_t s_max, int64_t t_max,
                 const double* GA, const double* GB, double tau, int64_t* I, int64_t* nI,
                 int64_t* J, int64_t* nJ, double* eps_out, double* Omega_out) {
    double* h = (double*)malloc(sizeof(double) * (size_t)m);
    double* g = (double*)malloc(sizeof(double) * (size_t)n);
    unsigned char* ua = (unsigned char*)malloc((size_t)m);
    unsigned char* ub = (unsigned char*)malloc((size_t)n);
    int64_t* ordr = (int64_t*)malloc(sizeof(int64_t) * (size_t)m);
    int64_t* ordc = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    double* LI = (double*)calloc((size_t)(s_max * s_max), sizeof(double));
    double* LJ = (double*)calloc((size_t)(t_max * t_max), sizeof(double));
    int ret = -1;
    if (!h || !g || !ua || !ub || !ordr || !ordc || !LI || !LJ) goto done;
    double S = 0.0;
    for (int64_t i = 0; i < m; ++i)
        for (int64_t j = 0; j < n; ++j) S += R[i * n + j] * R[i * n + j];
    for (int64_t i = 0; i < m; ++i) { h[i] = -1.0; ua[i] = a[i] > 0.0; }
    for (int64_t j = 0; j < n; ++j) { g[j] = -1.0; ub[j] = b[j] > 0.0; }
    double Omega = -1.0;
    for (int64_t i = 0; i < m; ++i) {
        if (!ua[i]) continue;
        for (int64_t j = 0; j < n; ++j) {
            if (!ub[j]) continue;
            const double w = (R[i * n + j] * R[i * n + j]) / (a[i] * b[j]);
            if (w > h[i]) h[i] = w;
            if (w > g[j]) g[j] = w;
            if (w > Omega) Omega = w;
        }
    }
    if (Omega < 0.0) goto done;
    double eps = theta * Omega + (1.0 - theta) * (S / (F_A * F_B));
    if (eps > Omega) eps = Omega;
    const int64_t cr = rank_candidates(m, h, ua, eps, ordr);
    const int64_t cc = rank_candidates(n, g, ub, eps, ordc);
    *nI = take_independent(cr, ordr, GA, m, tau, s_max, I, LI);
    *nJ = take_independent(cc, ordc, GB, n, tau, t_max, J, LJ);
    if (eps_out) *eps_out = eps;
    if (Omega_out) *Omega_out = Omega;
    ret = 0;
done:
    free(h); free(g); free(ua); free(ub); free(ordr); free(ordc); free(LI); free(LJ);
    return ret;
}

/* Solve G Y = E for Y (r x c) in place, G = L L^T with L r x r (ld = cap). */
static void chol_solve_cols(int64_t r, int64_t c, const double* L, int64_t cap, double* E,
                            int64_t lde) {
    for (int64_t col = 0; col < c; ++col) {
        for (int64_t x = 0; x < r; ++x) {          /* L z = e */
            double s = E[x * lde + col];
            for (int64_t y = 0; y < x; ++y) s -= L[x * cap + y] * E[y * lde + col];
            E[x * lde + col] = s / L[x * cap + x];
        }
        for (int64_t x = r - 1; x >= 0; --x) {     /* L^T y = z */
            double s = E[x * lde + col];
            for (int64_t y = x + 1; y < r; ++y) s -= L[y * cap + x] * E[y * lde + col];
            E[x * lde + col] = s / L[x * cap + x];
        }
    }
}

/* Cholesky factor of G restricted to idx (in that order): L (r x r, ld cap). */
static void chol_sub(int64_t r, const int64_t* idx, const double* G, int64_t len, double* L,
                     int64_t cap) {
    for (int64_t x = 0; x < r; ++x) {
        for (int64_t y = 0; y <= x; ++y) {
            double s = G[idx[x] * len + idx[y]];
            for (int64_t z = 0; z < y; ++z) s -= L[x * cap + z] * L[y * cap + z];
            if (y == x) L[x * cap + x] = sqrt(s);
            else L[x * cap + y] = s / L[y * cap + y];
        }
    }
}

static double frob_diff2_2s(int64_t len, const double* X, const double* Y) {
    double s = 0.0;
    for (int64_t i = 0; i < len; ++i) {
        const double d = X[i] - Y[i];
        s += d * d;
    }
    return s;
}

/* The iteration. Inputs as mo_solve (mek_oracle.c) plus theta, the block
 * caps s_max (rows) and t_max (columns) and the independence tolerance tau.
 * Outputs X, *iters, *status and optional histories of capacity hist_cap:
 * s_hist[k] = ||R^k||_F^2, e_hist[k] = ||X^k - Xref||/||Xref|| (k = 0..iters),
 * I_hist (hist_cap x s_max, -1 padded), J_hist (hist_cap x t_max),
 * nI_hist[k], nJ_hist[k] (k < iters). Stop tests run before every step. */
int mo_solve_2s(int64_t m, int64_t p, int64_t q, int64_t n, const double* A, const double* B,
                const double* C, const double* X0, double theta, int64_t s_max, int64_t t_max,
                double tau, int stop, double tol, const double* Xref, int64_t max_iters,
                double diverge, double* X, int64_t* iters, int* status, double* s_hist,
                double* e_hist, int64_t* I_hist, int64_t* J_hist, int64_t* nI_hist,
                int64_t* nJ_hist, int64_t hist_cap) {
    if (m <= 0 || p <= 0 || q <= 0 || n <= 0 || !A || !B || !C || !X || !iters || !status)
        return MO_EINVAL;
    if (s_max < 1 || t_max < 1 || !(theta >= 0.0 && theta <= 1.0) || !(tau >= 0.0))
        return MO_EINVAL;
    if (stop == MO_STOP_REL_ERR && !Xref) return MO_EINVAL;
    *iters = 0;
    const size_t mn = (size_t)(m * n), pq = (size_t)(p * q);
    double* a = (double*)calloc((size_t)m, sizeof(double));
    double* b = (double*)calloc((size_t)n, sizeof(double));
    double* R = (double*)malloc(sizeof(double) * mn);
    double* GA = (double*)malloc(sizeof(double) * (size_t)(m * m));
    double* GB = (double*)malloc(sizeof(double) * (size_t)(n * n));
    int64_t* I = (int64_t*)malloc(sizeof(int64_t) * (size_t)s_max);
    int64_t* J = (int64_t*)malloc(sizeof(int64_t) * (size_t)t_max);
    double* LI = (double*)calloc((size_t)(s_max * s_max), sizeof(double));
    double* LJ = (double*)calloc((size_t)(t_max * t_max), sizeof(double));
    double* Wm = (double*)malloc(sizeof(double) * (size_t)(s_max * t_max));
    double* Wt = (double*)malloc(sizeof(double) * (size_t)(s_max * t_max));
    double* U = (double*)malloc(sizeof(double) * (size_t)(s_max * q));
    double* V = (double*)malloc(sizeof(double) * (size_t)(s_max * n));
    int st = MO_MAXITER;
    if (!a || !b || !R || !GA || !GB || !I || !J || !LI || !LJ || !Wm || !Wt || !U || !V) {
        st = MO_ENOMEM;
        goto out;
    }
    double F_A = 0.0, F_B = 0.0;
    for (int64_t i = 0; i < m; ++i) {
        double s = 0.0;
        for (int64_t j = 0; j < p; ++j) s += A[i * p + j] * A[i * p + j];
        a[i] = s;
        F_A += s;
    }
    for (int64_t j = 0; j < n; ++j) {
        double s = 0.0;
        for (int64_t l = 0; l < q; ++l) s += B[l * n + j] * B[l * n + j];
        b[j] = s;
        F_B += s;
    }
    /* A A^T and B^T B. */
    for (int64_t i = 0; i < m; ++i)
        for (int64_t h2 = 0; h2 < m; ++h2) {
            double s = 0.0;
            for (int64_t j = 0; j < p; ++j) s += A[i * p + j] * A[h2 * p + j];
            GA[i * m + h2] = s;
        }
    for (int64_t j = 0; j < n; ++j)
        for (int64_t l = 0; l < n; ++l) {
            double s = 0.0;
            for (int64_t x = 0; x < q; ++x) s += B[x * n + j] * B[x * n + l];
            GB[j * n + l] = s;
        }
    /* X^0 and R^0 = C - A X^0 B. */
    if (X0) memcpy(X, X0, sizeof(double) * pq);
    else memset(X, 0, sizeof(double) * pq);
    for (int64_t i = 0; i < m; ++i)
        for (int64_t j = 0; j < n; ++j) {
            double s = 0.0;
            if (X0)
                for (int64_t l = 0; l < q; ++l) {
                    double ax = 0.0;
                    for (int64_t x = 0; x < p; ++x) ax += A[i * p + x] * X[x * q + l];
                    s += ax * B[l * n + j];
                }
            R[i * n + j] = C[i * n + j] - s;
        }
    double ref2 = 0.0, C2 = 0.0;
    if (Xref)
        for (size_t i = 0; i < pq; ++i) ref2 += Xref[i] * Xref[i];
    for (size_t i = 0; i < mn; ++i) C2 += C[i] * C[i];

    double S0 = -1.0;
    int64_t k = 0;
    for (;;) {
        double S = 0.0;
        for (size_t i = 0; i < mn; ++i) S += R[i] * R[i];
        if (S0 < 0.0) S0 = S;
        const double err =
            Xref ? sqrt(frob_diff2_2s((int64_t)pq, X, Xref) / (ref2 > 0.0 ? ref2 : 1.0)) : NAN;
        if (k < hist_cap) {
            if (s_hist) s_hist[k] = S;
            if (e_hist) e_hist[k] = err;
        }
        if (stop == MO_STOP_REL_ERR && err <= tol) { st = MO_OK; break; }
        if (stop == MO_STOP_REL_RESID && sqrt(S) <= tol * sqrt(C2)) { st = MO_OK; break; }
        if (S == 0.0) { st = MO_EXACT; break; }
        if (!isfinite(S) || (diverge > 0.0 && S > diverge * S0)) { st = MO_EDIVERGED; break; }
        if (k >= max_iters) { st = MO_MAXITER; break; }

        int64_t nI = 0, nJ = 0;
        if (mo_select_2s(m, n, R, a, b, F_A, F_B, theta, s_max, t_max, GA, GB, tau, I, &nI, J,
                         &nJ, NULL, NULL) != 0 || nI == 0 || nJ == 0) {
            st = MO_EINVAL;
            break;
        }
        if (k < hist_cap) {
            for (int64_t x = 0; x < s_max; ++x) if (I_hist) I_hist[k * s_max + x] = x < nI ? I[x] : -1;
            for (int64_t y = 0; y < t_max; ++y) if (J_hist) J_hist[k * t_max + y] = y < nJ ? J[y] : -1;
            if (nI_hist) nI_hist[k] = nI;
            if (nJ_hist) nJ_hist[k] = nJ;
        }
        /* W = (A_I A_I^T)^{-1} R_IJ (B_J^T B_J)^{-1}. */
        chol_sub(nI, I, GA, m, LI, s_max);
        chol_sub(nJ, J, GB, n, LJ, t_max);
        for (int64_t x = 0; x < nI; ++x)
            for (int64_t y = 0; y < nJ; ++y) Wm[x * t_max + y] = R[I[x] * n + J[y]];
        chol_solve_cols(nI, nJ, LI, s_max, Wm, t_max);            /* G_I^{-1} E */
        for (int64_t x = 0; x < nI; ++x)                           /* transpose */
            for (int64_t y = 0; y < nJ; ++y) Wt[y * s_max + x] = Wm[x * t_max + y];
        chol_solve_cols(nJ, nI, LJ, t_max, Wt, s_max);             /* G_J^{-1} (.)^T */
        for (int64_t x = 0; x < nI; ++x)
            for (int64_t y = 0; y < nJ; ++y) Wm[x * t_max + y] = Wt[y * s_max + x];
        /* X += A_I^T (W B_J^T). */
        for (int64_t x = 0; x < nI; ++x)
            for (int64_t l = 0; l < q; ++l) {
                double s = 0.0;
                for (int64_t y = 0; y < nJ; ++y) s += Wm[x * t_max + y] * B[l * n + J[y]];
                U[x * q + l] = s;
            }
        for (int64_t s_ = 0; s_ < p; ++s_)
            for (int64_t l = 0; l < q; ++l) {
                double s = 0.0;
                for (int64_t x = 0; x < nI; ++x) s += A[I[x] * p + s_] * U[x * q + l];
                X[s_ * q + l] += s;
            }
        /* R -= (A A^T)_{:,I} (W (B^T B)_{J,:}). */
        for (int64_t x = 0; x < nI; ++x)
            for (int64_t j = 0; j < n; ++j) {
                double s = 0.0;
                for (int64_t y = 0; y < nJ; ++y) s += Wm[x * t_max + y] * GB[J[y] * n + j];
                V[x * n + j] = s;
            }
        for (int64_t h2 = 0; h2 < m; ++h2)
            for (int64_t j = 0; j < n; ++j) {
                double s = 0.0;
                for (int64_t x = 0; x < nI; ++x) s += GA[h2 * m + I[x]] * V[x * n + j];
                R[h2 * n + j] -= s;
            }
        ++k;
    }
    *iters = k;
out:
    *status = st;
    free(a); free(b); free(R); free(GA); free(GB); free(I); free(J); free(LI); free(LJ);
    free(Wm); free(Wt); free(U); free(V);
    return st;
}
