// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_common.h"

namespace mek {

// Status codes (mirror the public header's MEK_* values).
enum : int {
    kOK = 0,
    kMaxIter = 1,
    kExact = 2,
    kEInval = -1,
    kENoMem = -2,
    kEHip = -3,
    kENonFinite = -4,
    kEDiverged = -5,
    kEUnsupported = -6,
    kETimeout = -7,
};

enum : int { kBK = 0, kRBK = 1, kGRBK = 2, kRGRBK = 3, kMWRBK = 4 };
enum : int { kStopNone = 0, kStopRelErr = 1, kStopRelResid = 2 };

// Result of a solve as written by the kernel (device memory).
struct DevReport {
    long long iters;
    int status;
    int last_set;
    double S;       // ||R||_F^2 at exit
    double err;     // relative error at exit (NaN without a reference)
};

// Per-instance scalars of a batched launch (instances share A and B).
struct InstSlot {
    int id;                      // instance index: strides of its buffers
    int pad;
    double C2, ref2, S_target;
    long long max_iters, k_offset, hist_offset;
    unsigned long long inst;     // Philox key word 1
};

// Per-instance strides of the exchange and error buffers (words).
constexpr int kErrStride = 512;

// Everything the persistent solver kernel needs for one instance. T is the
// storage/update type of R, X and the Gram matrices (double or float);
// norms, selection and the stop test are always double.
template <typename T>
struct SolveParams {
    int m, p, q, n;
    // Plan data.
    const T* A;        // m x p
    const T* B;        // q x n
    const T* BT;       // n x q, B transposed
    const T* GA;       // m x m, A A^T
    const T* GB;       // n x n, B^T B
    const double* a;   // m, ||A_i||^2
    double F_A;        // ||A||_F^2
    const int* active; // rows with ||A_i|| > 0, ascending
    int n_active;
    // State.
    T* R;              // m x n residual (initial value in, storage if not in LDS)
    T* Xt;             // q x p, the iterate transposed
    const double* Xref_t;  // q x p or null
    double ref2;       // ||X_ref||_F^2
    double C2;         // ||C||_F^2 (REL_RESID denominator, squared)
    const double* norms;   // optional: {||C||_F^2, ||X_ref||_F^2} read from device memory at
                           // the start instead of C2 and ref2 (0 for ref2 means no reference)
    double* r;         // m row norms of R
    T* rowbuf;         // n, the published row R_{i_k}
    T* vbuf;           // q, v = R_{i_k} B^T
    T* wbuf;           // n, w = R_{i_k} B^T B
    double* errpart;   // 2 * W partial ||X - X_ref||^2
    TeamSync* sync;
    DevReport* report;
    // Options.
    int variant;
    double theta;
    double alpha;
    int stop;
    double tol;
    long long max_iters;
    unsigned long long seed, inst;
    long long k_offset;          // updates made before this launch (Philox counter and replay offset)
    const int32_t* replay;
    long long replay_len;
    double diverge;
    double* resid_hist;
    double* err_hist;
    int32_t* idx_hist;
    int32_t* set_hist;
    long long hist_cap;
    long long hist_offset;       // history index of this launch's k = 0
    double S_target;             // > 0: also stop (OK) once ||R||_F^2 <= S_target
    unsigned long long* phase;   // optional: per-phase wall-clock ticks (3 timed work-groups)
    int a_in_lds;                // keep ||A_i||^2 for all rows in LDS
    int x_in_lds;                // keep this work-group's rows of X^T in LDS
    int b_in_lds;                // keep B and B^T in LDS (one-work-group teams)
    int small;                   // one work-group, one row of R per thread (small instances)
    int poll_sleep;              // s_sleep length between polls of exchange words
    // Batch: with slots set, nb teams of W work-groups, team b on instance
    // slots[b].id, whose R, X^T, X_ref^T, r, rowbuf, vbuf, wbuf, errpart,
    // sync, report and histories sit at that index times their size from the
    // pointers above; its scalars come from the slot.
    int nb;
    const InstSlot* slots;
    // Ragged batch (the kernel's MULTI form): multi_n instances, each with
    // its own complete parameter block multi[b] (multi unset there), owning
    // work-groups [multi_start[b], multi_start[b + 1]) of a grid of
    // multi_wgs.
    const SolveParams* multi;
    const int* multi_start;
    int multi_n;
    int multi_wgs;
    // Team layout.
    int W;      // work-groups in the team
    int rpw;    // rows of R per work-group
    int xpw;    // columns of X (rows of X^T) per work-group
    int wpw;    // entries of w per work-group
};

// Sparse-aware update (sparse.hip): one work-group per instance; the
// nonzeros of A, B and A A^T in ELL form (index -1 pads a row).
template <typename T>
struct SparseParams {
    int m, p, q, n;
    const int* a_idx;  const T* a_val;  int ka;    // row i of A: m x ka, row-major
    const int* b_idx;  const T* b_val;  int kb;    // row j of B: kb x q, slot-major
    const int* bt_idx; const T* bt_val; int kbt;   // column l of B: kbt x n, slot-major
    const int* g_idx;  const T* g_val;  int kg;    // column i of A A^T: m x kg, row-major
    const double* a;   // m, ||A_i||^2
    double F_A;
    const int* active;
    int n_active;
    T* R;              // instance b at b * sR: m x n
    long long sR;
    T* X;              // instance b at b * sX: p x q, row-major
    long long sX;
    const double* Xref;   // p x q per instance (stride sX), or null
    DevReport* report;    // indexed by instance
    const InstSlot* slots;
    int nb;               // work-groups = instances of this launch
    int a_in_lds;         // ||A_i||^2 of all rows in LDS
    int b_in_lds;         // the ELL slots of B's rows and columns in LDS
    int g_in_lds;         // the ELL slots of A A^T and A in LDS
    int norms_in_lds;     // row norms and row errors in LDS (else in r_glob / e_glob)
    double* r_glob;       // {||R_i||^2, ||R_i||^2/||A_i||^2} pairs per instance (stride 2m),
                          // when not in LDS
    double* e_glob;       // p row errors per instance (stride sX), when not in LDS
    int variant;
    double theta, alpha;
    int stop;
    double tol;
    double diverge;
    unsigned long long seed;
    const int32_t* replay;
    long long replay_len;
    double* resid_hist;   // histories: instance b at b * hist_cap
    double* err_hist;
    int32_t* idx_hist;
    int32_t* set_hist;
    long long hist_cap;
    unsigned long long* phase;   // optional: per-phase wall-clock ticks of work-group 0
    // Ragged batch: nb instances, work-group b taking the complete
    // parameters multi[b] (whose slots hold one slot, of index 0).
    const SparseParams* multi;
    // Optional (stream-ordered solves, one instance): {||C||_F^2,
    // ||X_ref||_F^2} read from device memory instead of the slot's C2 and
    // ref2 (0 for the second means no reference).
    const double* norms;
};
hipError_t launch_sparse(const SparseParams<double>& P, size_t lds_bytes, hipStream_t s);
hipError_t launch_sparse(const SparseParams<float>& P, size_t lds_bytes, hipStream_t s);
// LDS of the sparse kernel; kb, kbt > 0 when B's ELL slots are cached, ka,
// kg > 0 when those of A and A A^T are.
size_t sparse_lds_bytes(int m, int p, int q, int n, size_t elem, bool norms_in_lds, bool a_in_lds,
                        int kb, int kbt, int ka, int kg);
// Largest count of nonzeros over the `rows` lines of M (line i: M[i*rs + j*cs],
// j < cols), combined into *width_dev with atomicMax (clear it first).
hipError_t ell_width(const double* M, int rows, int cols, long long rs, long long cs,
                     int* width_dev, hipStream_t s);
template <typename T>
hipError_t ell_fill(const double* M, int rows, int cols, long long rs, long long cs, int width,
                    bool slot_major, int* idx, T* val, hipStream_t s);

// Two-sided block projection (block2.hip): at most kBlkCap rows and columns
// per step.
constexpr int kBlkCap = 32;

struct Block2Params {
    int m, p, q, n;
    const double* A;       // m x p
    const double* B;       // q x n
    const double* GA;      // m x m, A A^T
    const double* GB;      // n x n, B^T B
    const double* a;       // m, ||A_i||^2
    const double* b;       // n, ||B_j||^2 (columns of B)
    double F_A, F_B;       // ||A||_F^2, ||B||_F^2
    double* R;             // m x n residual (initial value in, storage if not in LDS)
    double* Xt;            // q x p, the iterate transposed
    const double* Xref_t;  // q x p or null
    double ref2, C2;
    // Exchange words (64-bit, tagged).
    unsigned long long* hbuf;     // m: max_j omega_ij of row i
    unsigned long long* rbuf;     // m: ||R_i||^2
    unsigned long long* cpart;    // W x n: column maxima of omega over each work-group's rows
    unsigned long long* gcol;     // n: column maxima
    unsigned long long* ebuf;     // kBlkCap x kBlkCap: R_IJ
    unsigned long long* errpart;  // W: partial ||X - X_ref||^2
    TeamSync* sync;
    DevReport* report;
    double theta, tau;
    int s_cap, t_cap;
    int stop;
    double tol;
    long long max_iters;
    double diverge;
    double* resid_hist;
    double* err_hist;
    int32_t* rows_hist;    // hist_cap x s_cap
    int32_t* cols_hist;    // hist_cap x t_cap
    long long hist_cap;
    int W, rpw, xpw;
    int r_in_lds;
    int poll_sleep;
    unsigned long long* phase;   // optional: per-phase wall-clock ticks of work-group 0
};

// Bytes of the block kernel's LDS region shared by R_IJ / W (kBlkCap rows
// of kBlkCap + 1), the radix histograms and the column slice of exchange B.
__host__ __device__ inline size_t block2_ereg_bytes(int ncs) {
    size_t e = (size_t)kBlkCap * (kBlkCap + 1) * 8;
    e = e > 1024 * sizeof(int) ? e : 1024 * sizeof(int);
    e = e > (size_t)ncs * 8 ? e : (size_t)ncs * 8;
    return (e + 15) & ~(size_t)15;
}
// Doubles of the block kernel's factor region: L_I and L_J (s_cap and t_cap
// rows of kBlkCap), later the X update's two kXRows x kBlkCap arrays and the
// R update's kBlkCap x kChunk array (kXRows = kChunk = 8).
__host__ __device__ inline int block2_fac_doubles(int s_cap, int t_cap) {
    const int f = (s_cap + t_cap) * kBlkCap;
    return f > 2 * 8 * kBlkCap ? f : 2 * 8 * kBlkCap;
}
hipError_t launch_block2(const Block2Params& P, size_t lds_bytes, hipStream_t s);
size_t block2_lds_bytes(int rpw, int n, int W, int s_cap, int t_cap, bool r_in_lds);
size_t block2_lds_budget();

// Rows of a selection chunk per thread (1, 2, 4, 8 or 16) for m rows.
int sel_rows_for(int m);

// Launchers (solver.hip).
// Ragged batch: P carries multi, multi_start, multi_n and multi_wgs; R stays
// in device memory; max_m sizes the selection chunk; lds_bytes is the
// largest of the instances' LDS needs.
hipError_t launch_solve_multi(const SolveParams<double>& P, int max_m, size_t lds_bytes,
                              hipStream_t s);
hipError_t launch_solve_multi(const SolveParams<float>& P, int max_m, size_t lds_bytes,
                              hipStream_t s);
hipError_t launch_solve(const SolveParams<double>& P, bool r_in_lds, size_t lds_bytes,
                        hipStream_t s);
hipError_t launch_solve(const SolveParams<float>& P, bool r_in_lds, size_t lds_bytes,
                        hipStream_t s);
size_t solve_lds_bytes(int rpw, int n, int q, int xpw, int wpw, size_t elem, bool r_in_lds,
                       bool single);
size_t solve_lds_budget();
size_t solve_lds_bytes_a(int m);
size_t solve_small_lds_bytes(int m, int p, int q, int n, size_t elem);

hipError_t launch_select(int variant, int m, const double* r, const double* a, double F_A,
                         double theta, uint64_t seed, uint64_t inst, long long k0,
                         long long count, int32_t* idx, uint8_t* in_set, int32_t* set_list,
                         double* stats, const int* active, int n_active, hipStream_t s);
hipError_t launch_philox(uint64_t seed, uint64_t inst, long long k0, long long count,
                         double* out, hipStream_t s);

// Dense kernels (gemm.hip).
// D = beta * C + alpha * A B, A(i,k) = A[i*a_i + k*a_k], B(k,j) = B[k*b_k + j*b_j],
// C, D row-major with leading dimensions ldc, ldd (C may be null when beta == 0).
// The team solver's exchanges and block collectives without arithmetic,
// `rounds` times (probe.hip); words: 2n + m + q + W zeroed 64-bit words.
hipError_t exchange_probe(int W, int m, int n, int q, long long rounds, void* words,
                          TeamSync* sync, int* status, hipStream_t s);

// D_b = beta C_b + alpha A_b B_b (FP32 operands split into `pieces` bf16
// terms on the BF16 matrix cores, FP32 accumulation; C FP64, D FP32).
hipError_t gemm_bf16s_batched(int pieces, int nb, int M, int N, int K, double alpha,
                              const float* A, long long a_i, long long a_k, long long sA,
                              const float* B, long long b_k, long long b_j, long long sB,
                              double beta, const double* C, long long ldc, long long sC, float* D,
                              long long ldd, long long sD, hipStream_t s);
hipError_t gemm_f64(int M, int N, int K, double alpha, const double* A, long long a_i,
                    long long a_k, const double* B, long long b_k, long long b_j, double beta,
                    const double* C, long long ldc, double* D, long long ldd, hipStream_t s);
// The same for nb instances in one launch: instance b reads A + b sA, B + b sB,
// C + b sC and writes D + b sD (a stride of 0 shares the operand).
hipError_t gemm_f64_batched(int nb, int M, int N, int K, double alpha, const double* A,
                            long long a_i, long long a_k, long long sA, const double* B,
                            long long b_k, long long b_j, long long sB, double beta,
                            const double* C, long long ldc, long long sC, double* D,
                            long long ldd, long long sD, hipStream_t s);

// Warm-start network kernels (cnn.hip): BF16 tensors as uint16_t, NCHW;
// channel counts 3 or 32.
bool cnn_channels_ok(int64_t c);
size_t cnn_wgrad_partial_floats(int N, int Cin, int H, int W, int Cout);
// wb: device scratch of kCnnWeightScratch uint16 for the weights in MFMA
// order (used when the convolution's input has 32 channels).
constexpr int kCnnWeightScratch = 9 * 32 * 32;
hipError_t cnn_conv3x3(int N, int Cin, int H, int W, int Cout, const uint16_t* x,
                       const uint16_t* mask, const float* w, const float* b, int relu,
                       uint16_t* yb, double* yd, const double* add, uint16_t* wb, hipStream_t s);
hipError_t cnn_conv3x3_grad_input(int N, int Cout, int H, int W, int Cin, const uint16_t* g,
                                  const uint16_t* gmask, const float* w, uint16_t* gx,
                                  uint16_t* wb, hipStream_t s);
hipError_t cnn_conv3x3_grad_weight(int N, int Cin, int H, int W, int Cout, const uint16_t* x,
                                   const uint16_t* g, const uint16_t* gmask, float* partial,
                                   float* dw, float* db, hipStream_t s);
hipError_t cnn_mse_grad(long long len, const double* y, const double* label, double scale,
                        uint16_t* g, double* part, int nblocks, hipStream_t s);
hipError_t cnn_adam(long long n, float* w, float* wq, const float* g, float* m, float* v, float lr,
                    float b1, float b2, float eps, int t, hipStream_t s);
hipError_t cnn_to_bf16(long long n, const double* x, double scale, uint16_t* y, hipStream_t s);
hipError_t cnn_round_bf16(long long n, const float* x, float* y, hipStream_t s);

// Utility kernels (util.hip).
hipError_t row_sq_norms(const double* A, int m, int p, double* out, hipStream_t s);
// Fixed-order reductions; scratch holds 256 doubles of partial sums.
hipError_t sum_reduce(const double* x, long long len, double* out, double* scratch, hipStream_t s);
hipError_t sq_norm(const double* x, long long len, double* out, double* scratch, hipStream_t s);
hipError_t sq_diff_norm(const double* x, const double* y, long long len, double* out,
                        double* scratch, hipStream_t s);
hipError_t nonfinite_count(const double* x, long long len, int* out, hipStream_t s);
hipError_t active_rows(const double* a, int m, int* list, int* count, hipStream_t s);
template <typename T>
hipError_t transpose_to(const double* X, int rows, int cols, T* Xt, hipStream_t s);
template <typename T>
hipError_t transpose_from(const T* Xt, int rows, int cols, double* X, hipStream_t s);
hipError_t convert_f64_f32(const double* x, long long len, float* y, hipStream_t s);
hipError_t convert_f32_f64(const float* x, long long len, double* y, hipStream_t s);
hipError_t copy_f64(const double* x, long long len, double* y, hipStream_t s);
hipError_t fill_zero_bytes(void* x, long long bytes, hipStream_t s);
// Store `bytes` of host data at dst (device, 8-byte aligned, room for bytes
// rounded up to 8) through kernel arguments, kBlobWords words per launch.
constexpr int kBlobWords = 64;
hipError_t store_bytes(const void* src, size_t bytes, void* dst, hipStream_t s);
// out = a x + b y elementwise (out may alias x or y).
hipError_t lincomb_f64(double a, const double* x, double b, const double* y, long long len,
                       double* out, hipStream_t s);
hipError_t diag_argmax_col(const double* G, int q, double* v, hipStream_t s);

}  // namespace mek
