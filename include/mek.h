/*
 * mek.h - C ABI of libmek.so: greedy randomized block Kaczmarz solvers for
 * the matrix equation A X B = C on AMD Instinct MI355X (gfx950).
 *
 * Problem (paper, Sec. 1, eq. 1.1): given A (m x p), B (q x n), C (m x n),
 * find X (p x q) with A X B = C; for a consistent system the greedy methods
 * converge to the least-norm solution X* = A^+ C B^+ (Sec. 2; Theorems 4.2,
 * 4.5, 4.7), ME-BK to A^+ C B^+ + X0 - A^+ A X0 B B^+ (Theorem 3.3).
 *
 * Iteration (Algs. 1-5): pick one row index i_k, then
 *     X^{k+1} = X^k + alpha/||A_i||^2 * A_i^T (R_i^k B^T),
 *     R^{k+1} = R^k - alpha/||A_i||^2 * (A A^T)_{:,i} (R_i^k B^T B),
 * where R = C - A X B. The variants differ in how i_k is chosen:
 *     MEK_BK     cyclic over the rows with nonzero norm      (Alg. 2)
 *     MEK_RBK    Pr(i) = ||A_i||^2/||A||_F^2                 (Alg. 1)
 *     MEK_GRBK   greedy threshold set + residual sampling    (Alg. 3)
 *     MEK_RGRBK  the same with relaxation theta in [0, 1]    (Alg. 4)
 *     MEK_MWRBK  argmax of ||R_i||^2/||A_i||^2, lowest index (Alg. 5)
 *   MEK_TWOSIDED extends the greedy criterion of Algs. 3/4 from rows to
 *   entries and projects exactly onto a block of equations A_I X B_J = C_IJ
 *   (an extension; the paper's iteration is the row form above). With
 *   omega_ij = R_ij^2 / (||A_i||^2 ||B_j||^2) (B_j a column of B), Omega =
 *   max omega and eps = min(Omega, theta Omega + (1 - theta) ||R||_F^2 /
 *   (||A||_F^2 ||B||_F^2)): rows with max_j omega_ij >= eps are ranked by
 *   that maximum (lower index first on ties); I = the first block_rows of
 *   them less those whose Cholesky pivot in A_I A_I^T (rank order) is at
 *   most tau times its diagonal; J likewise from the columns with B^T B, at
 *   most block_cols; then W = (A_I A_I^T)^{-1} R_IJ (B_J^T B_J)^{-1},
 *   X += A_I^T W B_J^T, R -= (A A^T)_{:,I} W (B^T B)_{J,:}. No step size.
 *
 * Conventions shared by every entry point:
 *   - Matrices are dense, row-major and contiguous (leading dimension equals
 *     the number of columns). Element type at the boundary is always double.
 *   - Pointers documented as "device" must point to memory of the current
 *     HIP device; the library never frees caller memory.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Blocking calls synchronise that stream before returning.
 *   - The return value is a status code (MEK_OK ... below). Negative values
 *     are errors; on an error, outputs are left untouched unless stated.
 *   - A plan is not thread-safe; use one plan per stream. Calls on one
 *     plan must not overlap.
 */
#ifndef MEK_H
#define MEK_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MEK_ABI_VERSION 4

/* Selection rules (Algs. 1-5), and the two-sided block projection. */
#define MEK_BK 0
#define MEK_RBK 1
#define MEK_GRBK 2
#define MEK_RGRBK 3
#define MEK_MWRBK 4
#define MEK_TWOSIDED 5

/* Stop rules, evaluated before every update (so 0 updates when X0 already
 * passes). REL_ERR: ||X^k - X_ref||_F <= tol ||X_ref||_F (Sec. 5's RRN is
 * the square of this ratio). REL_RESID: ||R^k||_F <= tol ||C||_F. */
#define MEK_STOP_NONE 0
#define MEK_STOP_REL_ERR 1
#define MEK_STOP_REL_RESID 2

/* Arithmetic of the iteration. FP64: everything in double. FP32: residual,
 * iterate and Gram matrices in float, norms / selection / stop test in
 * double. MIXED: FP64 outer refinement (true residual by FP64 GEMM), FP32
 * inner iterations on the correction equation A D B = R_true. */
#define MEK_FP64 0
#define MEK_FP32 1
#define MEK_MIXED 2

/* How an update is applied (mek_plan_opts.update). DENSE: every row of R
 * and X, the work of an update split over a team of work-groups. SPARSE:
 * only the rows of X where A_{i_k} is nonzero and the rows of R where
 * column i_k of A A^T is nonzero, with v = R_{i_k} B^T and w = v B summed
 * over the nonzeros of B; the terms left out are exactly zero, so the
 * iteration is the same (Alg. 3's update with its zero terms skipped). One
 * work-group runs each instance. For banded or otherwise sparse A and B
 * (a blur), where an update touches a few rows instead of all of them. */
#define MEK_UPDATE_DENSE 0
#define MEK_UPDATE_SPARSE 1

/* Status codes. */
#define MEK_OK 0            /* stop rule met */
#define MEK_MAXITER 1       /* max_iters updates made, rule not met */
#define MEK_EXACT 2         /* ||R^k||_F = 0 exactly */
#define MEK_EINVAL (-1)     /* bad argument (sizes, NULL, theta, alpha, ...) */
#define MEK_ENOMEM (-2)     /* device allocation failed */
#define MEK_EHIP (-3)       /* a HIP runtime call failed */
#define MEK_ENONFINITE (-4) /* NaN or Inf in an input */
#define MEK_EDIVERGED (-5)  /* ||R^k||_F^2 not finite or above diverge * ||R^0||_F^2 */
#define MEK_EUNSUPPORTED (-6) /* valid request this build cannot run */
#define MEK_ETIMEOUT (-7)   /* a cross-work-group wait exceeded its spin limit */

/* Opaque plan: device copies of A and B plus everything precomputed from
 * them (row norms ||A_i||^2, ||A||_F^2, A A^T, B^T B, alpha). */
typedef struct mek_plan_s* mek_plan;

typedef struct {
    int precision;   /* MEK_FP64 / MEK_FP32 / MEK_MIXED */
    double alpha;    /* > 0: the step alpha; <= 0: alpha = 1/||B||_2^2 (Sec. 5),
                        ||B||_2^2 from power iteration on B B^T */
    int team_wgs;    /* 0: automatic; > 0: number of work-groups that share one
                        solve (testing and tuning hook) */
    int r_in_lds;    /* -1: automatic; 0: keep R in device memory; 1: require R
                        resident in LDS (MEK_EUNSUPPORTED if it does not fit).
                        SPARSE plans: 0 keeps the row norms and row errors in
                        device memory (the form taken automatically when
                        8 (m + p) bytes of them do not fit in LDS or m is
                        above 8192), otherwise ignored */
    int update;      /* MEK_UPDATE_DENSE (0) or MEK_UPDATE_SPARSE. A SPARSE plan
                        takes FP64 or FP32 (MEK_MIXED: MEK_EUNSUPPORTED) and
                        finds the nonzeros of A, B and A A^T at creation;
                        MEK_EUNSUPPORTED when a row of A or A A^T, or a row or
                        column of B, holds more than 1024 nonzeros, or when
                        16 n + 8 q bytes plus 1 KiB exceed the LDS of one
                        work-group */
} mek_plan_opts;

typedef struct {
    int variant;          /* MEK_BK ... MEK_MWRBK */
    double theta;         /* relaxation of Alg. 4, in [0, 1]; GRBK uses 1/2 */
    double alpha;         /* > 0 overrides the plan's alpha; values outside
                             (0, 2/||B||_2^2), the range of the convergence
                             theorems, are rejected with MEK_EINVAL */
    int stop;             /* MEK_STOP_* */
    double tol;           /* tolerance of the stop rule */
    const double* X_ref;  /* device, p x q; needed for MEK_STOP_REL_ERR and for
                             err_hist, else may be NULL */
    int64_t max_iters;    /* cap on the number of updates (>= 0) */
    uint64_t seed;        /* Philox4x64-10 key word 0 */
    uint64_t instance;    /* Philox4x64-10 key word 1 */
    const int32_t* replay_idx; /* device, optional: forced row indices for
                             updates k < replay_len (test hook; in MEK_MIXED
                             k counts updates over all refinement passes) */
    int64_t replay_len;
    double diverge;       /* > 0: stop with MEK_EDIVERGED once ||R^k||^2 >
                             diverge * ||R^0||^2; <= 0: off */
    /* Histories, device, caller-owned, each of capacity hist_cap entries
     * (entries past the capacity are dropped; NULL = not recorded):
     *   resid_hist[k] = ||R^k||_F^2 for k = 0..iters,
     *   err_hist[k]   = ||X^k - X_ref||_F / ||X_ref||_F for k = 0..iters,
     *   idx_hist[k]   = i_k (0-based) for k = 0..iters-1,
     *   set_hist[k]   = size of the index set of update k (greedy variants). */
    double* resid_hist;
    double* err_hist;
    int32_t* idx_hist;
    int32_t* set_hist;
    int64_t hist_cap;
    /* MEK_MIXED only: FP32 updates per refinement pass (0: automatic). */
    int64_t inner_iters;
    /* MEK_TWOSIDED only (FP64 plans, one instance): the block caps s and t
     * (1 .. 32), the independence tolerance tau (<= 0: 1e-10), and optional
     * histories (device, caller-owned): rows_hist[k * block_rows + x] = the
     * x-th row of I at step k and cols_hist[k * block_cols + y] likewise
     * (-1 past the block's size), for k < hist_cap. replay_idx must be NULL. */
    int block_rows;
    int block_cols;
    double tau;
    int32_t* rows_hist;
    int32_t* cols_hist;
    /* MEK_FP32 and MEK_MIXED plans, DENSE update, mek_solve and
     * mek_solve_batched: every refresh_period updates the FP32 residual is
     * recomputed from the current iterate by the split-BF16 residual engine
     * (see mek_residual_split), so that the incrementally updated residual
     * does not drift: FP32 recomputes R = C - A X B with 3 bf16 terms per
     * operand (FP32 accuracy); MIXED recomputes the inner residual
     * R_true - A D B of its correction D with 2 terms (about 2^-17, far
     * below the inner stop). 0: automatic (every max(2048, 4 m) updates);
     * < 0: never. The stream-ordered and ragged calls run without refreshes
     * and return MEK_EUNSUPPORTED for refresh_period > 0. */
    int64_t refresh_period;
} mek_solve_opts;

typedef struct {
    int64_t iters;       /* updates made */
    int status;          /* MEK_OK / MEK_MAXITER / MEK_EXACT / MEK_EDIVERGED / MEK_ETIMEOUT */
    double resid2;       /* ||R||_F^2 of the returned iterate (as tracked) */
    double rel_err;      /* ||X - X_ref||_F/||X_ref||_F, NaN without X_ref */
    double alpha;        /* step used */
    int team_wgs;        /* work-groups per solve */
    int r_in_lds;        /* 1 if R stayed in LDS */
    int passes;          /* launches of the persistent solver: MEK_MIXED refinement
                            passes, MEK_FP32 residual refreshes + 1, else 1 */
    double kernel_ms;    /* time of the persistent solver launch(es), measured
                            with HIP events on `stream` around each launch */
} mek_report;

/* ABI version (MEK_ABI_VERSION). */
int mek_version(void);

/* Static string naming a status code. */
const char* mek_status_string(int status);

/* Build a plan for A (m x p) and B (q x n), both device pointers. The plan
 * copies A and B, so they may be freed after the call. Precomputes
 * ||A_i||^2, ||A||_F^2, the Gram matrices A A^T and B^T B (the remark after
 * Alg. 3) and alpha. Errors: MEK_EINVAL (sizes <= 0, NULL pointers, bad
 * options), MEK_ENONFINITE (NaN/Inf in A or B), MEK_EINVAL if A or B is
 * all zero, MEK_ENOMEM, MEK_EHIP. Blocking. `opts` may be NULL (defaults:
 * FP64, alpha = 1/||B||_2^2, automatic layout). */
int mek_plan_create(mek_plan* out, int64_t m, int64_t p, int64_t q, int64_t n,
                    const double* A, const double* B, const mek_plan_opts* opts, void* stream);

/* Release a plan and its device memory. NULL is accepted. */
int mek_plan_destroy(mek_plan plan);

/* Copy plan data to caller memory (device pointers, each may be NULL):
 * row_norms (m) = ||A_i||^2, gram_a (m x m) = A A^T, gram_b (n x n) =
 * B^T B; *alpha (host) = the plan's step. Blocking. */
int mek_plan_query(mek_plan plan, double* row_norms, double* gram_a, double* gram_b,
                   double* alpha, void* stream);

/* Nonzeros per line of a SPARSE plan's structure (host array of 4):
 * widths[0] = max over rows of A, [1] = over rows of B, [2] = over columns
 * of B, [3] = over columns of A A^T (an update touches widths[0] rows of X
 * and widths[3] rows of R at most). MEK_EUNSUPPORTED for a DENSE plan. */
int mek_plan_sparse_widths(mek_plan plan, int32_t* widths);

/* Solve A X B = C with the plan's A and B. C (m x n), X0 (p x q, NULL means
 * zero) and X (p x q, output) are device pointers; X may alias X0. Runs
 * the whole iteration on the GPU in one persistent launch (MIXED: one per
 * refinement pass) and synchronises `stream` before returning. The report
 * (host struct) may be NULL. Returns the final status (>= 0: X written). */
int mek_solve(mek_plan plan, const double* C, const double* X0, const mek_solve_opts* opts,
              double* X, mek_report* report, void* stream);

/* Uniform batch: solve A X_b B = C_b for b < batch with the plan's A and B
 * (for instance the channels of an image) in one persistent launch whose
 * work-groups are split evenly between the instances. All per-instance
 * arrays are stacked, instance b at b times the size of one: C (batch x m x
 * n), X0 (batch x p x q, NULL means zero), X (batch x p x q, may alias X0),
 * opts->X_ref (batch x p x q) and each history (batch x hist_cap entries).
 * Instance b draws its random numbers under Philox key (seed, instance + b),
 * so it follows the same trajectory as a mek_solve call with that key.
 * replay_idx, when given, forces the same rows in every instance. reports
 * (host, batch entries) may be NULL; kernel_ms is the time of the shared
 * launch(es). Returns a negative code if the call failed (nothing written)
 * or an instance failed; otherwise MEK_OK when every instance met the stop
 * rule, else the status of the first one that did not. Errors as mek_solve,
 * and MEK_EUNSUPPORTED when batch exceeds the device's compute units.
 * With a SPARSE plan each instance is one work-group of one launch, and the
 * batch is not bounded by the compute units (work-groups beyond them wait
 * for a free one); the two-sided variant returns MEK_EUNSUPPORTED. */
int mek_solve_batched(mek_plan plan, int64_t batch, const double* C, const double* X0,
                      const mek_solve_opts* opts, double* X, mek_report* reports, void* stream);

/* The report of a stream-ordered solve, in device memory. */
typedef struct mek_device_report {
    int64_t iters;    /* updates made */
    int32_t status;   /* MEK_OK, MEK_MAXITER, MEK_EXACT, MEK_EDIVERGED, ... */
    int32_t last_set; /* size of the last index set (GRBK/RGRBK) */
    double resid2;    /* ||R||_F^2 at exit */
    double rel_err;   /* ||X - X_ref||_F / ||X_ref||_F at exit, NaN without X_ref */
} mek_device_report;

/* Stream-ordered solve of Alg. 3 (and the other variants) for one instance:
 * the same iteration and result as mek_solve, but every step (residual,
 * norms, transposes, the persistent launch, X) is enqueued on `stream` and
 * the call returns without waiting; the report is written to dev_report
 * (device memory) when the stream reaches it. Nothing in the call reads
 * device data on the host or allocates (mek_plan_create makes the plan's
 * workspace for one instance), so it can be captured into a graph. FP64 and
 * FP32 plans, DENSE or SPARSE; MIXED plans, the two-sided variant and
 * replay_idx return MEK_EUNSUPPORTED. No finite check of the inputs is made (non-finite data
 * ends in MEK_EDIVERGED or a non-finite report). X, the histories and the
 * plan's workspace must not be touched until the stream has passed the
 * call; calls on one plan must be ordered on one stream. A later call that
 * grows the plan's workspace (a uniform batch larger than any before on the
 * plan) moves it, after which graphs captured on the plan must not be
 * replayed. */
int mek_solve_async(mek_plan plan, const double* C, const double* X0, const mek_solve_opts* opts,
                    double* X, mek_device_report* dev_report, void* stream);

/* Ragged batch: solve A_b X_b B_b = C_b for b < batch, each instance with
 * its own plan plans[b] (own sizes m_b, p_b, q_b, n_b; every plan distinct,
 * all of one precision, FP64 or FP32, on one device), in one persistent
 * launch. Each instance runs the iteration of Algs. 3-5 exactly as mek_solve
 * would (same selection, sampling, update and stop rule); instance b draws
 * under Philox key (seed, instance + b). The work-groups of the launch are
 * shared out in proportion to each instance's per-update work (m_b n_b +
 * p_b q_b), at most one per compute unit in all; residuals stay in device
 * memory. plans, C, X0, X_ref and X are host arrays of batch entries;
 * C[b] (m_b x n_b), X0[b] (p_b x q_b; X0 or an entry NULL means zero),
 * X_ref[b] (p_b x q_b; needed by MEK_STOP_REL_ERR) and X[b] (p_b x q_b,
 * output) are device pointers. opts is shared; opts->X_ref must be NULL
 * (references come through X_ref); each history holds batch x hist_cap
 * entries, instance b from b * hist_cap. Returns as mek_solve_batched.
 * SPARSE plans (all plans SPARSE, or none): every instance is one
 * work-group of one launch, the batch is not bounded by the compute units,
 * and instances may share a plan (the j-th instance on a plan uses the
 * j-th slice of its workspace, which grows to hold them).
 * Errors: MEK_EINVAL for bad arguments, a repeated DENSE plan, or mixed
 * precisions or update modes; MEK_EUNSUPPORTED for MEK_MIXED plans,
 * replay_idx, the two-sided variant or a DENSE batch above the compute
 * units. */
int mek_solve_multi(int64_t batch, const mek_plan* plans, const double* const* C,
                    const double* const* X0, const double* const* X_ref,
                    const mek_solve_opts* opts, double* const* X, mek_report* reports,
                    void* stream);

/* Stream-ordered ragged batch: the iteration and results of mek_solve_multi
 * (same arguments, same layout of work-groups), with every step enqueued on
 * `stream` and no host wait; instance b's report goes to dev_reports[b]
 * (device memory, batch entries) when the stream reaches it. The parameter
 * table of the launch reaches the device through kernel arguments, so once
 * every plan has a workspace and the first plan holds a table for this
 * batch size (one earlier mek_solve_multi or mek_solve_multi_async call on
 * the same plans), the call can be captured into a graph and replayed; a
 * captured call that would need either returns MEK_EUNSUPPORTED (outside
 * capture they are allocated). SPARSE plans as in mek_solve_multi (shared
 * plans, any batch size); their table holds at least 1024 instances and
 * moves only for a larger batch, after which graphs captured earlier on
 * that first plan must not be replayed. No finite check of the inputs is
 * made.
 * Other errors and refusals as mek_solve_multi. X, the histories and the
 * plans' workspaces must not be touched until the stream has passed the
 * call; calls sharing a plan must be ordered on one stream. A later call
 * that grows a plan's workspace (a uniform batch larger than any before on
 * that plan) moves it, after which graphs captured on that plan must not be
 * replayed; the parameter table never moves. */
int mek_solve_multi_async(int64_t batch, const mek_plan* plans, const double* const* C,
                          const double* const* X0, const double* const* X_ref,
                          const mek_solve_opts* opts, double* const* X,
                          mek_device_report* dev_reports, void* stream);

/* ---- Unit entry points: the hot path's stages run on their own. ---- */

/* out[j] = u_{k0+j} for j < count: the uniform draw of update k0+j,
 * (w0 >> 11) * 2^-53 with w0 the first word of Philox4x64-10 under key
 * (seed, instance) and counter (k+1, 0, 0, 0). `out` is device memory. */
int mek_philox_uniform(uint64_t seed, uint64_t instance, int64_t k0, int64_t count,
                       double* out, void* stream);

/* Run the selection step of update k (k0 <= k < k0+count) on fixed weights:
 * r (m, device) = ||R_i^k||^2, a (m, device) = ||A_i||^2, F_A = ||A||_F^2.
 * Writes idx[j] (device, count) = the row chosen for update k0+j. If
 * in_set (device, m bytes) is not NULL it receives the index set of
 * Algs. 3/4 (for MWRBK the chosen row), and if set_list (device, m int32)
 * is not NULL the set's rows compacted in ascending order; stats (device,
 * 4 doubles, optional) = {threshold t, set weight T, ||R||_F^2, set size}. */
int mek_select(int variant, int64_t m, const double* r, const double* a, double F_A,
               double theta, uint64_t seed, uint64_t instance, int64_t k0, int64_t count,
               int32_t* idx, uint8_t* in_set, int32_t* set_list, double* stats, void* stream);

/* Residual engine (the residual R^0 = C - A X^0 B with which Alg. 3 starts,
 * also used by the refinement passes): R = C - A X B for A (m x p),
 * X (p x q), B (q x n), C (m x n), all device double, computed as two FP64 MFMA GEMMs
 * (T = A X, then R = C - T B). R must not alias the inputs. Blocking. The
 * temporary T is kept in a per-device buffer between calls (the largest
 * m x q seen so far); calls from several threads are serialised. */
int mek_residual(int64_t m, int64_t p, int64_t q, int64_t n, const double* A, const double* X,
                 const double* B, const double* C, double* R, void* stream);

/* The residual engine of Alg. 3's start for a uniform batch that shares A
 * and B: for b < nb,
 * R_b = C_b - (A X_b) B with X_b = X + b p q, C_b = C + b m n and
 * R_b = R + b m n (all device double, row-major, instances contiguous).
 * Two strided-batched launches, one per product. R must not overlap any
 * input. Blocking; the temporaries share the per-device buffer of
 * mek_residual (nb x m x q doubles). Errors: MEK_EINVAL for sizes <= 0, null
 * or overlapping pointers; MEK_EHIP for host or unregistered pointers. */
int mek_residual_batched(int64_t nb, int64_t m, int64_t p, int64_t q, int64_t n, const double* A,
                         const double* X, const double* B, const double* C, double* R,
                         void* stream);

/* For callers that cannot allocate device memory (code under graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * residual engine of mek_residual, R = C - (A X) B (same arguments, same
 * kernels, same results), with the temporary T = A X (m x q doubles) in a
 * fixed per-device array of 2^21 doubles (16 MiB) that the library holds
 * until the process ends, so the call never allocates or frees. Stream
 * ordered: returns once both products are enqueued on `stream`, without
 * waiting. Every call on one device shares that device's array: calls that
 * overlap on one device (other streams, other threads) race and give
 * undefined results; order them on one stream. Errors: MEK_EINVAL for
 * m q > 2^21, sizes <= 0, null, host, short or overlapping pointers;
 * MEK_EHIP if a launch fails. */
int mek_residual_noalloc(int64_t m, int64_t p, int64_t q, int64_t n, const double* A,
                         const double* X, const double* B, const double* C, double* R,
                         void* stream);

/* Communication floor of the team solver (measurement): a cooperative
 * launch of W work-groups that repeats, `rounds` times, the exchanges and
 * block collectives of one update of Alg. 3 as the team kernel does them
 * (all-gather of m row-norm words and W error words, block reductions and
 * scan, broadcast of one row of n words, all-gather of the q words of
 * v = R_i B^T and of the n words of w = v B) with no arithmetic and no
 * operand traffic. *us_per_round (host) = kernel time per round, measured
 * with HIP events on `stream`: the floor those exchanges put under one
 * update at that team shape. Blocking. Errors: MEK_EINVAL for W < 1, m < W,
 * m > 8192, sizes < 1 or rounds < 1; MEK_EUNSUPPORTED for W above the
 * compute units; MEK_ETIMEOUT if a wait gave up. */
int mek_exchange_floor(int64_t W, int64_t m, int64_t n, int64_t q, int64_t rounds,
                       double* us_per_round, void* stream);

/* The FP32 residual engine of the FP32 and mixed iterations (the residual
 * R = C - A X B with which Alg. 3 starts, recomputed from the current
 * iterate so that the incrementally updated FP32 residual does not drift):
 * for b < nb, R_b = C_b - (A X_b) B with A (m x p), X_b = X + b p q
 * (p x q) and B (q x n) device float, C_b = C + b m n device double and
 * R_b = R + b m n device float (row-major, instances contiguous). Both
 * products run on the BF16 matrix cores with FP32 accumulation, every FP32
 * operand value split into `pieces` bf16 terms (1, 2 or 3) and the cross
 * terms of combined order below `pieces` summed: 1 term gives about bf16
 * accuracy (2^-9 relative per product), 2 about 2^-17, 3 about FP32
 * accuracy (2^-24). T = A X_b is rounded to FP32 between the products;
 * C_b - T B is formed in FP64 and rounded once. R must not overlap any
 * input. Blocking; the temporaries T (nb x m x q floats) use a per-device
 * buffer kept between calls. Errors: MEK_EINVAL for pieces outside 1..3,
 * sizes <= 0, null or overlapping pointers; MEK_EHIP for host or short
 * buffers. */
int mek_residual_split(int pieces, int64_t nb, int64_t m, int64_t p, int64_t q, int64_t n,
                       const float* A, const float* X, const float* B, const double* C, float* R,
                       void* stream);

/* Gram products by the FP64 MFMA GEMM: G = M M^T (transpose_first = 0,
 * G rows x rows) or G = M^T M (transpose_first = 1, G cols x cols) for M
 * (rows x cols), all device double. Blocking. */
int mek_gram(int64_t rows, int64_t cols, const double* M, int transpose_first, double* G,
             void* stream);

/* ---- Learned warm start X0 = C + f(C) (not in the paper: an extension of
 * its initial guess X^0). f is a network of 3 x 3 convolutions; these calls
 * are its layers, gradients and optimiser step. Tensors are device arrays:
 * with 3 channels in NCHW order (the image-shaped input C, the output, the
 * loss gradient), with 32 channels in NHWC order (channels innermost: the
 * hidden activations and their gradients, so that a pixel's 32 channels are
 * 64 contiguous bytes for the matrix cores); indices below are written
 * [n,c,h,w] in either case. BF16 tensors are uint16_t (the upper half of an
 * IEEE single, rounded to nearest even); weights are float arrays
 * (O, C, 3, 3) holding BF16-rounded values; sums are FP32 (the loss FP64).
 * Channel counts must be 3 or 32, N <= 65535, H, W <= 32768. The calls are
 * stream ordered (they return once their kernels are enqueued on `stream`)
 * except mek_cnn_mse_grad, which returns the loss and so synchronises.
 * grad_weight and mse_grad share a per-device scratch buffer, and the
 * convolutions a per-device buffer for their weights: order those calls on
 * one stream. Errors: MEK_EINVAL for bad sizes or pointers, MEK_EHIP for
 * host or short buffers and launch failures. */

/* y[n,o,h,w] = b[o] + sum_{c,i,j} w[o,c,i,j] x[n,c,h+i-1,w+j-1] (zero
 * padding 1), then max(., 0) when relu; written to exactly one of y_bf16
 * (BF16) or y_f64; an FP64 output adds add_f64 (same shape) when that is not
 * NULL (the warm start's X0 = C + f(C)). b may be NULL. */
int mek_cnn_conv3x3(int64_t N, int64_t Cin, int64_t H, int64_t W, int64_t Cout, const uint16_t* x,
                    const float* w, const float* b, int relu, uint16_t* y_bf16, double* y_f64,
                    const double* add_f64, void* stream);

/* Input gradient of that convolution for the upstream gradient g (N, Cout,
 * H, W; BF16): gx[n,c,h,w] = sum_{o,i,j} w[o,c,i,j] g'[n,o,h-i+1,w-j+1], with
 * g' = g where g_gate > 0 and 0 elsewhere (g_gate: the layer's ReLU output,
 * or NULL for no gate). gx (N, Cin, H, W) BF16. */
int mek_cnn_conv3x3_grad_input(int64_t N, int64_t Cout, int64_t H, int64_t W, int64_t Cin,
                               const uint16_t* g, const uint16_t* g_gate, const float* w,
                               uint16_t* gx, void* stream);

/* Weight and bias gradients: dw[o,c,i,j] = sum_{n,h,w} g'[n,o,h,w]
 * x[n,c,h+i-1,w+j-1], db[o] = sum g' (g' gated as above), FP32, summed over
 * 16 x 16 pixel tiles and then over the tiles in a fixed order. Uses a
 * per-device scratch buffer kept between calls. */
int mek_cnn_conv3x3_grad_weight(int64_t N, int64_t Cin, int64_t H, int64_t W, int64_t Cout,
                                const uint16_t* x, const uint16_t* g, const uint16_t* g_gate,
                                float* dw, float* db, void* stream);

/* *loss (host) = mean((y - label)^2) over len entries (device double), and,
 * when g is not NULL, g = BF16(2 (y - label) / len). */
int mek_cnn_mse_grad(int64_t len, const double* y, const double* label, uint16_t* g, double* loss,
                     void* stream);

/* One Adam step (t >= 1) on n FP32 master weights w with gradient g and
 * moments m, v; wq receives the BF16-rounded weights the layers use. */
int mek_cnn_adam(int64_t n, float* w, float* wq, const float* g, float* m, float* v, double lr,
                 double beta1, double beta2, double eps, int64_t t, void* stream);

/* y = BF16(scale x) for n doubles; y = BF16-rounded x for n floats. */
int mek_cnn_to_bf16(int64_t n, const double* x, double scale, uint16_t* y, void* stream);
int mek_cnn_round_bf16(int64_t n, const float* x, float* y, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* MEK_H */
