// C ABI of libmek.so (declared in include/mek.h): argument checking, plans,
// workspace, the team layout of the persistent solver and the precision
// drivers. Every numerical step runs in the library's own HIP kernels.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>

#include "../../include/mek.h"
#include "internal.h"

using namespace mek;

namespace {

struct Workspace {
    void* base = nullptr;
    size_t bytes = 0;
    double* R64 = nullptr;     // m x n
    float* R32 = nullptr;      // m x n (FP32 / MIXED)
    double* T64 = nullptr;     // m x q, GEMM temporary A X
    double* Xt64 = nullptr;    // q x p
    float* Xt32 = nullptr;     // q x p
    double* Xacc = nullptr;    // p x q, MIXED accumulated iterate
    double* Xtmp = nullptr;    // p x q
    double* Xref_t = nullptr;  // q x p
    double* r = nullptr;       // m
    void* rowbuf = nullptr;    // n * 8 bytes
    void* wbuf = nullptr;      // n * 8 bytes
    void* vbuf = nullptr;      // q * 8 bytes
    double* errpart = nullptr; // 2 * 256
    TeamSync* sync = nullptr;
    DevReport* report = nullptr;
    double* scal = nullptr;    // 8 scalars
    double* red = nullptr;     // 256 partial sums of the reductions
    int* iscal = nullptr;      // 8 ints
    unsigned long long* phase = nullptr;   // 16 phase-timing counters
};

}  // namespace

struct mek_plan_s {
    int64_t m = 0, p = 0, q = 0, n = 0;
    int precision = MEK_FP64;
    int team_wgs = 0;
    int r_in_lds = -1;
    double alpha = 0.0;
    double F_A = 0.0;
    double b2 = 0.0;          // ||B||_2^2
    int n_active = 0;
    int cus = 0;
    int device = 0;
    double *A = nullptr, *B = nullptr, *BT = nullptr, *GA = nullptr, *GB = nullptr, *a = nullptr;
    int* active = nullptr;
    float *A32 = nullptr, *B32 = nullptr, *BT32 = nullptr, *GA32 = nullptr, *GB32 = nullptr;
    Workspace ws;
};

namespace {

int hip_status(hipError_t e) {
    if (e == hipSuccess) return MEK_OK;
    if (e == hipErrorOutOfMemory) return MEK_ENOMEM;
    return MEK_EHIP;
}

#define MEK_TRY(expr)                                  \
    do {                                               \
        hipError_t _e = (expr);                        \
        if (_e != hipSuccess) return hip_status(_e);   \
    } while (0)

// The pointer must lie in one device allocation that holds `bytes` bytes
// from it on. Catches host pointers and short buffers before any kernel
// touches them.
int check_dev(const void* ptr, size_t bytes) {
    if (!ptr) return MEK_EINVAL;
    hipPointerAttribute_t attr;
    if (hipPointerGetAttributes(&attr, ptr) != hipSuccess) {
        (void)hipGetLastError();
        return MEK_EINVAL;
    }
    if (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged) return MEK_EINVAL;
    hipDeviceptr_t base = nullptr;
    size_t size = 0;
    if (hipMemGetAddressRange(&base, &size, (hipDeviceptr_t)ptr) != hipSuccess) {
        (void)hipGetLastError();
        return MEK_EINVAL;
    }
    const char* b = (const char*)base;
    const char* pc = (const char*)ptr;
    if (pc < b || (size_t)(pc - b) + bytes > size) return MEK_EINVAL;
    return MEK_OK;
}

int finite_check(const double* x, long long len, int* flag_dev, hipStream_t s) {
    MEK_TRY(nonfinite_count(x, len, flag_dev, s));
    int h = 0;
    MEK_TRY(hipMemcpyAsync(&h, flag_dev, sizeof(int), hipMemcpyDeviceToHost, s));
    MEK_TRY(hipStreamSynchronize(s));
    return h ? MEK_ENONFINITE : MEK_OK;
}

template <typename T>
T* carve(char*& cur, size_t count) {
    T* p = reinterpret_cast<T*>(cur);
    cur += (count * sizeof(T) + 255) & ~(size_t)255;
    return p;
}

int ensure_workspace(mek_plan_s* P) {
    if (P->ws.base) return MEK_OK;
    const size_t m = P->m, p = P->p, q = P->q, n = P->n;
    const bool f32 = P->precision != MEK_FP64;
    size_t need = 0;
    auto add = [&](size_t bytes) { need += (bytes + 255) & ~(size_t)255; };
    add(m * n * 8);
    add(f32 ? m * n * 4 : 0);
    add(m * q * 8);
    add(q * p * 8);
    add(f32 ? q * p * 4 : 0);
    add(p * q * 8);
    add(p * q * 8);
    add(q * p * 8);
    add(m * 8);
    add(n * 8);
    add(n * 8);
    add(q * 8);
    add(2 * 256 * 8);
    add(sizeof(TeamSync));
    add(sizeof(DevReport));
    add(8 * 8);
    add(8 * 4);
    add(32 * 8);
    add(256 * 8);
    void* base = nullptr;
    MEK_TRY(hipMalloc(&base, need));
    char* cur = (char*)base;
    Workspace& w = P->ws;
    w.base = base;
    w.bytes = need;
    w.R64 = carve<double>(cur, m * n);
    w.R32 = f32 ? carve<float>(cur, m * n) : nullptr;
    w.T64 = carve<double>(cur, m * q);
    w.Xt64 = carve<double>(cur, q * p);
    w.Xt32 = f32 ? carve<float>(cur, q * p) : nullptr;
    w.Xacc = carve<double>(cur, p * q);
    w.Xtmp = carve<double>(cur, p * q);
    w.Xref_t = carve<double>(cur, q * p);
    w.r = carve<double>(cur, m);
    w.rowbuf = carve<double>(cur, n);
    w.wbuf = carve<double>(cur, n);
    w.vbuf = carve<double>(cur, q);
    w.errpart = carve<double>(cur, 2 * 256);
    w.sync = carve<TeamSync>(cur, 1);
    w.report = carve<DevReport>(cur, 1);
    w.scal = carve<double>(cur, 8);
    w.iscal = carve<int>(cur, 8);
    w.phase = carve<unsigned long long>(cur, 32);
    w.red = carve<double>(cur, 256);
    return MEK_OK;
}

void free_plan(mek_plan_s* P) {
    if (!P) return;
    void* ptrs[] = {P->A, P->B, P->BT, P->GA, P->GB, P->a, P->active, P->A32, P->B32, P->BT32,
                    P->GA32, P->GB32, P->ws.base};
    for (void* x : ptrs)
        if (x) (void)hipFree(x);
    delete P;
}

struct Layout {
    int W, rpw, xpw, wpw;
    bool lds;
    bool a_lds;
    size_t lds_bytes;
};

int ceil_div(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

// Team layout: how many work-groups share the solve and whether their rows
// of R stay in LDS. Automatic choice: the fewest work-groups whose LDS can
// hold all of R, but at least one per 32K residual entries (so each
// work-group's pass stays short), capped by the number of CUs.
int choose_layout(const mek_plan_s* P, size_t elem, Layout* L) {
    const int64_t m = P->m, n = P->n, q = P->q;
    // The selection keeps at most kSelRows row norms per thread in registers,
    // and the n-vector staging buffer must fit in LDS.
    if (m > (int64_t)kSelRows * kThreads) return MEK_EUNSUPPORTED;
    if ((size_t)std::max(n, q) * elem + 4096 > solve_lds_budget()) return MEK_EUNSUPPORTED;
    const int cus = std::max(1, P->cus);
    const size_t budget = solve_lds_budget();
    int W;
    bool lds;
    auto fits = [&](int Wc) {
        const int rpw = ceil_div(m, Wc);
        const int Wr = ceil_div(m, rpw);
        return solve_lds_bytes(rpw, (int)n, (int)q, ceil_div(q, Wr), ceil_div(n, Wr), elem, true) <=
               budget;
    };
    if (P->team_wgs > 0) {
        W = (int)std::min<int64_t>({(int64_t)P->team_wgs, (int64_t)cus, m});
        lds = (P->r_in_lds != 0) && fits(W);
        if (P->r_in_lds == 1 && !lds) return MEK_EUNSUPPORTED;
    } else {
        const int64_t work = m * n;
        int Wt = (int)std::min<int64_t>(std::max<int64_t>(1, (work + 32767) / 32768), cus);
        Wt = (int)std::min<int64_t>(Wt, m);
        int Wl = -1;
        for (int Wc = 1; Wc <= std::min<int64_t>(cus, m); ++Wc)
            if (fits(Wc)) { Wl = Wc; break; }
        if (P->r_in_lds != 0 && Wl > 0) {
            // With R in LDS, spread the rows over as many CUs as there are
            // (fewer rows per work-group, even load): the LDS fits any W >= Wl.
            W = std::max(Wt, Wl);
            if (work >= (int64_t)cus * 4096) W = std::max(W, (int)std::min<int64_t>(cus, m));
            lds = true;
        } else {
            if (P->r_in_lds == 1) return MEK_EUNSUPPORTED;
            W = Wt;
            lds = false;
        }
    }
    const int rpw = ceil_div(m, W);
    W = ceil_div(m, rpw);   // no work-group without rows
    L->W = W;
    L->rpw = rpw;
    L->xpw = ceil_div(q, W);
    L->wpw = ceil_div(n, W);
    L->lds = lds && fits(W);
    L->lds_bytes = solve_lds_bytes(L->rpw, (int)n, (int)q, L->xpw, L->wpw, elem, L->lds);
    if (L->lds_bytes > budget || W > kMaxTeam) return MEK_EUNSUPPORTED;
    // ||A_i||^2 of all rows goes to LDS too when there is room.
    L->a_lds = L->lds_bytes + solve_lds_bytes_a((int)m) <= budget;
    if (L->a_lds) L->lds_bytes += solve_lds_bytes_a((int)m);
    return MEK_OK;
}

int validate_opts(const mek_plan_s* P, const mek_solve_opts* o) {
    if (!o) return MEK_EINVAL;
    if (o->variant < MEK_BK || o->variant > MEK_MWRBK) return MEK_EINVAL;
    if (!(o->theta >= 0.0 && o->theta <= 1.0)) return MEK_EINVAL;
    if (o->stop < MEK_STOP_NONE || o->stop > MEK_STOP_REL_RESID) return MEK_EINVAL;
    if (o->stop != MEK_STOP_NONE && !(o->tol >= 0.0)) return MEK_EINVAL;
    if (o->stop == MEK_STOP_REL_ERR && !o->X_ref) return MEK_EINVAL;
    if (o->max_iters < 0) return MEK_EINVAL;
    if (o->replay_len < 0 || (o->replay_len > 0 && !o->replay_idx)) return MEK_EINVAL;
    if (o->hist_cap < 0) return MEK_EINVAL;
    if (!(o->alpha <= 0.0 || isfinite(o->alpha))) return MEK_EINVAL;
    if (o->alpha > 0.0 && P && P->b2 > 0.0 && !(o->alpha < 2.0 / P->b2 * (1.0 + 1e-9)))
        return MEK_EINVAL;
    return MEK_OK;
}

// Fill the scalar part of the kernel parameters.
template <typename T>
void fill_common(SolveParams<T>& K, const mek_plan_s* P, const mek_solve_opts* o,
                 const Layout& L, double alpha) {
    K.m = (int)P->m;
    K.p = (int)P->p;
    K.q = (int)P->q;
    K.n = (int)P->n;
    K.a = P->a;
    K.F_A = P->F_A;
    K.active = P->active;
    K.n_active = P->n_active;
    K.r = P->ws.r;
    K.rowbuf = (T*)P->ws.rowbuf;
    K.vbuf = (T*)P->ws.vbuf;
    K.wbuf = (T*)P->ws.wbuf;
    K.errpart = P->ws.errpart;
    K.sync = P->ws.sync;
    K.report = P->ws.report;
    K.variant = o->variant;
    K.theta = o->theta;
    K.alpha = alpha;
    K.stop = o->stop;
    K.tol = o->tol;
    K.max_iters = o->max_iters;
    K.seed = o->seed;
    K.inst = o->instance;
    K.k_offset = 0;
    K.replay = o->replay_idx;
    K.replay_len = o->replay_len;
    K.diverge = o->diverge;
    K.resid_hist = o->resid_hist;
    K.err_hist = o->err_hist;
    K.idx_hist = o->idx_hist;
    K.set_hist = o->set_hist;
    K.hist_cap = o->hist_cap;
    K.hist_offset = 0;
    K.W = L.W;
    K.rpw = L.rpw;
    K.xpw = L.xpw;
    K.wpw = L.wpw;
}

int read_report(mek_plan_s* P, DevReport* h, hipStream_t s) {
    MEK_TRY(hipMemcpyAsync(h, P->ws.report, sizeof(DevReport), hipMemcpyDeviceToHost, s));
    MEK_TRY(hipStreamSynchronize(s));
    return MEK_OK;
}

// One persistent launch on the residual already stored in ws.R64 / ws.R32.
template <typename T>
int run_kernel(mek_plan_s* P, const mek_solve_opts* o, const Layout& L, double alpha,
               double C2, double ref2, const double* Xref_t, long long max_iters,
               long long k_offset, long long hist_offset, double S_target, T* R, T* Xt,
               hipStream_t s, DevReport* out, double* kernel_ms) {
    SolveParams<T> K;
    fill_common(K, P, o, L, alpha);
    if (sizeof(T) == 8) {
        K.A = (const T*)P->A;
        K.B = (const T*)P->B;
        K.BT = (const T*)P->BT;
        K.GA = (const T*)P->GA;
        K.GB = (const T*)P->GB;
    } else {
        K.A = (const T*)P->A32;
        K.B = (const T*)P->B32;
        K.BT = (const T*)P->BT32;
        K.GA = (const T*)P->GA32;
        K.GB = (const T*)P->GB32;
    }
    K.R = R;
    K.Xt = Xt;
    K.Xref_t = Xref_t;
    K.ref2 = ref2;
    K.C2 = C2;
    K.max_iters = max_iters;
    K.k_offset = k_offset;
    K.hist_offset = hist_offset;
    K.S_target = S_target;
    // MEK_PHASES=1 in the environment: time the phases of each update on
    // work-group 0 and print the averages to stderr (profiling aid).
    static const bool phases = getenv("MEK_PHASES") && getenv("MEK_PHASES")[0] == '1';
    K.phase = phases ? P->ws.phase : nullptr;
    K.a_in_lds = L.a_lds ? 1 : 0;
    // Pause between polls of exchange words (tuning knob MEK_POLL_SLEEP).
    static const int poll_sleep = getenv("MEK_POLL_SLEEP") ? atoi(getenv("MEK_POLL_SLEEP")) : 1;
    K.poll_sleep = poll_sleep;
    if (phases) MEK_TRY(fill_zero_bytes(P->ws.phase, 32 * 8, s));
    // Exchange words start with tag 0, which no update waits for.
    MEK_TRY(fill_zero_bytes(P->ws.sync, sizeof(TeamSync), s));
    MEK_TRY(fill_zero_bytes(P->ws.errpart, 2 * 256 * 8, s));
    MEK_TRY(fill_zero_bytes(P->ws.r, (long long)P->m * 8, s));
    MEK_TRY(fill_zero_bytes(P->ws.rowbuf, (long long)P->n * 8, s));
    MEK_TRY(fill_zero_bytes(P->ws.wbuf, (long long)P->n * 8, s));
    MEK_TRY(fill_zero_bytes(P->ws.vbuf, (long long)P->q * 8, s));
    hipEvent_t ev[2];
    MEK_TRY(hipEventCreate(&ev[0]));
    if (hipEventCreate(&ev[1]) != hipSuccess) {
        (void)hipEventDestroy(ev[0]);
        return MEK_EHIP;
    }
    hipError_t e = hipEventRecord(ev[0], s);
    if (e == hipSuccess) e = launch_solve(K, L.lds, L.lds_bytes, s);
    if (e == hipSuccess) e = hipEventRecord(ev[1], s);
    int st = (e == hipSuccess) ? read_report(P, out, s) : hip_status(e);
    float ms = 0.0f;
    if (st == MEK_OK && hipEventElapsedTime(&ms, ev[0], ev[1]) == hipSuccess && kernel_ms)
        *kernel_ms += (double)ms;
    if (st == MEK_OK && phases && out->iters > 0) {
        unsigned long long h[24];
        int rate_khz = 100000;
        (void)hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, P->device);
        if (hipMemcpy(h, P->ws.phase, sizeof(h), hipMemcpyDeviceToHost) == hipSuccess) {
            const char* names[8] = {"reduce", "select", "row", "dots", "waitw", "xupd", "update", "end"};
            const int wg[3] = {0, L.W / 2, L.W - 1};
            for (int t = 0; t < (L.W > 1 ? 3 : 1); ++t) {
                fprintf(stderr, "[mek phases] W=%d lds=%d a_lds=%d wg=%d iters=%lld us/update:", L.W,
                        (int)L.lds, (int)L.a_lds, wg[t], (long long)out->iters);
                for (int i = 0; i < 8; ++i)
                    fprintf(stderr, " %s=%.2f", names[i],
                            (double)h[t * 8 + i] / (rate_khz * 1e-3) / out->iters);
                fprintf(stderr, " total_kernel=%.2f\n", ms * 1e3 / out->iters);
            }
        }
    }
    (void)hipEventDestroy(ev[0]);
    (void)hipEventDestroy(ev[1]);
    return st;
}

int read_scalar(const double* dev, double* host, hipStream_t s) {
    MEK_TRY(hipMemcpyAsync(host, dev, sizeof(double), hipMemcpyDeviceToHost, s));
    MEK_TRY(hipStreamSynchronize(s));
    return MEK_OK;
}

}  // namespace

extern "C" {

int mek_version(void) { return MEK_ABI_VERSION; }

const char* mek_status_string(int st) {
    switch (st) {
        case MEK_OK: return "ok: stop rule met";
        case MEK_MAXITER: return "max_iters reached";
        case MEK_EXACT: return "exact: residual is zero";
        case MEK_EINVAL: return "invalid argument";
        case MEK_ENOMEM: return "device out of memory";
        case MEK_EHIP: return "HIP runtime error";
        case MEK_ENONFINITE: return "NaN or Inf in an input";
        case MEK_EDIVERGED: return "iteration diverged";
        case MEK_EUNSUPPORTED: return "unsupported configuration";
        case MEK_ETIMEOUT: return "cross-work-group wait timed out";
        default: return "unknown status";
    }
}

int mek_plan_create(mek_plan* out, int64_t m, int64_t p, int64_t q, int64_t n, const double* A,
                    const double* B, const mek_plan_opts* opts, void* stream) {
    if (!out) return MEK_EINVAL;
    *out = nullptr;
    if (m <= 0 || p <= 0 || q <= 0 || n <= 0) return MEK_EINVAL;
    if (m > INT32_MAX / 2 || p > INT32_MAX / 2 || q > INT32_MAX / 2 || n > INT32_MAX / 2)
        return MEK_EINVAL;
    if (!A || !B) return MEK_EINVAL;
    mek_plan_opts o = {MEK_FP64, 0.0, 0, -1};
    if (opts) o = *opts;
    if (o.precision < MEK_FP64 || o.precision > MEK_MIXED) return MEK_EINVAL;
    if (o.team_wgs < 0 || o.r_in_lds < -1 || o.r_in_lds > 1) return MEK_EINVAL;
    if (!(o.alpha <= 0.0 || isfinite(o.alpha))) return MEK_EINVAL;
    int st = check_dev(A, (size_t)(m * p) * 8);
    if (st) return st;
    st = check_dev(B, (size_t)(q * n) * 8);
    if (st) return st;
    hipStream_t s = (hipStream_t)stream;

    mek_plan_s* P = new mek_plan_s();
    P->m = m; P->p = p; P->q = q; P->n = n;
    P->precision = o.precision;
    P->team_wgs = o.team_wgs;
    P->r_in_lds = o.r_in_lds;
    int dev = 0;
    (void)hipGetDevice(&dev);
    P->device = dev;
    (void)hipDeviceGetAttribute(&P->cus, hipDeviceAttributeMultiprocessorCount, dev);

    auto fail = [&](int code) { free_plan(P); return code; };
    auto alloc = [&](void** ptr, size_t bytes) { return hipMalloc(ptr, bytes); };
    if (alloc((void**)&P->A, (size_t)(m * p) * 8) || alloc((void**)&P->B, (size_t)(q * n) * 8) ||
        alloc((void**)&P->BT, (size_t)(q * n) * 8) ||
        alloc((void**)&P->GA, (size_t)(m * m) * 8) || alloc((void**)&P->GB, (size_t)(n * n) * 8) ||
        alloc((void**)&P->a, (size_t)m * 8) || alloc((void**)&P->active, (size_t)m * 4) ||
        ensure_workspace(P))
        return fail(MEK_ENOMEM);
    Workspace& w = P->ws;
    if (copy_f64(A, m * p, P->A, s) || copy_f64(B, q * n, P->B, s) ||
        transpose_to<double>(P->B, (int)q, (int)n, P->BT, s))
        return fail(MEK_EHIP);
    if ((st = finite_check(P->A, m * p, w.iscal, s))) return fail(st);
    if ((st = finite_check(P->B, q * n, w.iscal, s))) return fail(st);
    // ||A_i||^2, ||A||_F^2 and the rows that can be selected.
    if (row_sq_norms(P->A, (int)m, (int)p, P->a, s) || sum_reduce(P->a, m, w.scal, w.red, s) ||
        active_rows(P->a, (int)m, P->active, w.iscal + 1, s))
        return fail(MEK_EHIP);
    if ((st = read_scalar(w.scal, &P->F_A, s))) return fail(st);
    if (hipMemcpyAsync(&P->n_active, w.iscal + 1, sizeof(int), hipMemcpyDeviceToHost, s) ||
        hipStreamSynchronize(s))
        return fail(MEK_EHIP);
    if (P->n_active == 0 || !(P->F_A > 0.0)) return fail(MEK_EINVAL);
    // Gram matrices A A^T (m x m) and B^T B (n x n) on the matrix cores.
    if (gemm_f64((int)m, (int)m, (int)p, 1.0, P->A, p, 1, P->A, 1, p, 0.0, nullptr, 0, P->GA, m, s) ||
        gemm_f64((int)n, (int)n, (int)q, 1.0, P->B, 1, n, P->B, n, 1, 0.0, nullptr, 0, P->GB, n, s))
        return fail(MEK_EHIP);
    // ||B||_2^2: largest eigenvalue of the smaller Gram matrix.
    if (q <= n) {
        double* BBt = nullptr;
        if (alloc((void**)&BBt, (size_t)(q * q) * 8)) return fail(MEK_ENOMEM);
        hipError_t e = gemm_f64((int)q, (int)q, (int)n, 1.0, P->B, n, 1, P->B, 1, n, 0.0, nullptr, 0, BBt, q, s);
        if (e == hipSuccess) e = power_iteration_max_eig(BBt, (int)q, w.scal + 1, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        (void)hipFree(BBt);
        if (e != hipSuccess) return fail(MEK_EHIP);
    } else {
        if (power_iteration_max_eig(P->GB, (int)n, w.scal + 1, s)) return fail(MEK_EHIP);
    }
    if ((st = read_scalar(w.scal + 1, &P->b2, s))) return fail(st);
    if (!(P->b2 > 0.0)) return fail(MEK_EINVAL);   // B is all zero
    P->alpha = (o.alpha > 0.0) ? o.alpha : 1.0 / P->b2;
    if (!(P->alpha < 2.0 / P->b2 * (1.0 + 1e-9))) return fail(MEK_EINVAL);
    if (P->precision != MEK_FP64) {
        if (alloc((void**)&P->A32, (size_t)(m * p) * 4) || alloc((void**)&P->B32, (size_t)(q * n) * 4) ||
            alloc((void**)&P->BT32, (size_t)(q * n) * 4) ||
            alloc((void**)&P->GA32, (size_t)(m * m) * 4) || alloc((void**)&P->GB32, (size_t)(n * n) * 4))
            return fail(MEK_ENOMEM);
        if (convert_f64_f32(P->A, m * p, P->A32, s) || convert_f64_f32(P->B, q * n, P->B32, s) ||
            convert_f64_f32(P->BT, q * n, P->BT32, s) ||
            convert_f64_f32(P->GA, m * m, P->GA32, s) || convert_f64_f32(P->GB, n * n, P->GB32, s))
            return fail(MEK_EHIP);
    }
    if (hipStreamSynchronize(s)) return fail(MEK_EHIP);
    *out = P;
    return MEK_OK;
}

int mek_plan_destroy(mek_plan plan) {
    if (plan) {
        (void)hipDeviceSynchronize();
        free_plan(plan);
    }
    return MEK_OK;
}

int mek_plan_query(mek_plan P, double* row_norms, double* gram_a, double* gram_b, double* alpha,
                   void* stream) {
    if (!P) return MEK_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    int st;
    if (row_norms) {
        if ((st = check_dev(row_norms, (size_t)P->m * 8))) return st;
        MEK_TRY(copy_f64(P->a, P->m, row_norms, s));
    }
    if (gram_a) {
        if ((st = check_dev(gram_a, (size_t)(P->m * P->m) * 8))) return st;
        MEK_TRY(copy_f64(P->GA, P->m * P->m, gram_a, s));
    }
    if (gram_b) {
        if ((st = check_dev(gram_b, (size_t)(P->n * P->n) * 8))) return st;
        MEK_TRY(copy_f64(P->GB, P->n * P->n, gram_b, s));
    }
    if (alpha) *alpha = P->alpha;
    MEK_TRY(hipStreamSynchronize(s));
    return MEK_OK;
}

int mek_solve(mek_plan P, const double* C, const double* X0, const mek_solve_opts* o, double* X,
              mek_report* report, void* stream) {
    if (!P || !C || !X) return MEK_EINVAL;
    int st = validate_opts(P, o);
    if (st) return st;
    const int64_t m = P->m, p = P->p, q = P->q, n = P->n;
    hipStream_t s = (hipStream_t)stream;
    if ((st = check_dev(C, (size_t)(m * n) * 8))) return st;
    if (X0 && (st = check_dev(X0, (size_t)(p * q) * 8))) return st;
    if ((st = check_dev(X, (size_t)(p * q) * 8))) return st;
    if (o->X_ref && (st = check_dev(o->X_ref, (size_t)(p * q) * 8))) return st;
    if (o->replay_len > 0 && (st = check_dev(o->replay_idx, (size_t)o->replay_len * 4))) return st;
    if (o->hist_cap > 0) {
        if (o->resid_hist && (st = check_dev(o->resid_hist, (size_t)o->hist_cap * 8))) return st;
        if (o->err_hist && (st = check_dev(o->err_hist, (size_t)o->hist_cap * 8))) return st;
        if (o->idx_hist && (st = check_dev(o->idx_hist, (size_t)o->hist_cap * 4))) return st;
        if (o->set_hist && (st = check_dev(o->set_hist, (size_t)o->hist_cap * 4))) return st;
    }
    Workspace& w = P->ws;
    if ((st = finite_check(C, m * n, w.iscal, s))) return st;
    if (X0 && (st = finite_check(X0, p * q, w.iscal, s))) return st;
    if (o->X_ref && (st = finite_check(o->X_ref, p * q, w.iscal, s))) return st;
    if (o->replay_len > 0) {
        // Forced indices must name rows that can be projected on.
        int32_t* hidx = (int32_t*)malloc((size_t)o->replay_len * 4);
        int* hact = (int*)malloc((size_t)P->n_active * 4);
        if (!hidx || !hact) { free(hidx); free(hact); return MEK_ENOMEM; }
        hipError_t e1 = hipMemcpy(hidx, o->replay_idx, (size_t)o->replay_len * 4, hipMemcpyDeviceToHost);
        hipError_t e2 = hipMemcpy(hact, P->active, (size_t)P->n_active * 4, hipMemcpyDeviceToHost);
        int bad = (e1 != hipSuccess || e2 != hipSuccess);
        for (int64_t j = 0; !bad && j < o->replay_len; ++j)
            bad = (hidx[j] < 0 || hidx[j] >= m || !std::binary_search(hact, hact + P->n_active, hidx[j]));
        free(hidx);
        free(hact);
        if (bad) return MEK_EINVAL;
    }
    const double alpha = (o->alpha > 0.0) ? o->alpha : P->alpha;

    // ||C||_F^2 and ||X_ref||_F^2.
    double C2 = 0.0, ref2 = 0.0;
    MEK_TRY(sq_norm(C, m * n, w.scal + 2, w.red, s));
    if ((st = read_scalar(w.scal + 2, &C2, s))) return st;
    if (o->X_ref) {
        MEK_TRY(sq_norm(o->X_ref, p * q, w.scal + 3, w.red, s));
        if ((st = read_scalar(w.scal + 3, &ref2, s))) return st;
        if (!(ref2 > 0.0)) ref2 = 1.0;
    }

    const int prec = P->precision;
    Layout L;
    if ((st = choose_layout(P, prec == MEK_FP64 ? 8 : 4, &L))) return st;

    // R^0 = C - A X^0 B (residual engine), or C when X^0 = 0.
    auto residual_into_R64 = [&](const double* Xcur) -> int {
        if (Xcur) {
            MEK_TRY(gemm_f64((int)m, (int)q, (int)p, 1.0, P->A, p, 1, Xcur, q, 1, 0.0, nullptr, 0,
                             w.T64, q, s));
            MEK_TRY(gemm_f64((int)m, (int)n, (int)q, -1.0, w.T64, q, 1, P->B, n, 1, 1.0, C, n,
                             w.R64, n, s));
        } else {
            MEK_TRY(copy_f64(C, m * n, w.R64, s));
        }
        return MEK_OK;
    };

    DevReport rep;
    memset(&rep, 0, sizeof(rep));
    int passes = 1;
    double kms = 0.0;
    if (prec == MEK_FP64 || prec == MEK_FP32) {
        if ((st = residual_into_R64(X0))) return st;
        if (o->X_ref) MEK_TRY(transpose_to<double>(o->X_ref, (int)p, (int)q, w.Xref_t, s));
        if (prec == MEK_FP64) {
            if (X0) MEK_TRY(transpose_to<double>(X0, (int)p, (int)q, w.Xt64, s));
            else MEK_TRY(fill_zero_bytes(w.Xt64, (long long)(p * q) * 8, s));
            st = run_kernel<double>(P, o, L, alpha, C2, ref2, o->X_ref ? w.Xref_t : nullptr,
                                    o->max_iters, 0, 0, 0.0, w.R64, w.Xt64, s, &rep, &kms);
            if (st) return st;
            MEK_TRY(transpose_from<double>(w.Xt64, (int)p, (int)q, X, s));
        } else {
            MEK_TRY(convert_f64_f32(w.R64, m * n, w.R32, s));
            if (X0) MEK_TRY(transpose_to<float>(X0, (int)p, (int)q, w.Xt32, s));
            else MEK_TRY(fill_zero_bytes(w.Xt32, (long long)(p * q) * 4, s));
            st = run_kernel<float>(P, o, L, alpha, C2, ref2, o->X_ref ? w.Xref_t : nullptr,
                                   o->max_iters, 0, 0, 0.0, w.R32, w.Xt32, s, &rep, &kms);
            if (st) return st;
            MEK_TRY(transpose_from<float>(w.Xt32, (int)p, (int)q, X, s));
        }
    } else {
        // MIXED: FP64 refinement around FP32 inner solves of A D B = R_true.
        if (X0) MEK_TRY(copy_f64(X0, p * q, w.Xacc, s));
        else MEK_TRY(fill_zero_bytes(w.Xacc, (long long)(p * q) * 8, s));
        // The inner stop is a 1e-3 drop of the residual norm, which FP32 reaches
        // well above its drift floor; the cap only bounds a pass.
        const long long inner_cap = o->inner_iters > 0 ? o->inner_iters
                                                       : std::max<long long>(20000, 200 * m);
        long long done = 0;
        passes = 0;
        double S0 = -1.0;
        for (;;) {
            if ((st = residual_into_R64(w.Xacc))) return st;
            double S = 0.0, err2 = NAN;
            MEK_TRY(sq_norm(w.R64, m * n, w.scal + 4, w.red, s));
            if ((st = read_scalar(w.scal + 4, &S, s))) return st;
            if (S0 < 0.0) S0 = S;
            double err = NAN;
            if (o->X_ref) {
                MEK_TRY(sq_diff_norm(w.Xacc, o->X_ref, p * q, w.scal + 5, w.red, s));
                if ((st = read_scalar(w.scal + 5, &err2, s))) return st;
                err = sqrt(err2 / ref2);
            }
            rep.S = S;
            rep.err = err;
            rep.iters = done;
            if (o->hist_cap > done) {
                if (o->resid_hist)
                    MEK_TRY(hipMemcpyAsync(o->resid_hist + done, &S, 8, hipMemcpyHostToDevice, s));
                if (o->err_hist)
                    MEK_TRY(hipMemcpyAsync(o->err_hist + done, &err, 8, hipMemcpyHostToDevice, s));
                MEK_TRY(hipStreamSynchronize(s));
            }
            if (o->stop == MEK_STOP_REL_ERR && err <= o->tol) { rep.status = MEK_OK; break; }
            if (o->stop == MEK_STOP_REL_RESID && sqrt(S) <= o->tol * sqrt(C2)) { rep.status = MEK_OK; break; }
            if (S == 0.0) { rep.status = MEK_EXACT; break; }
            if (!isfinite(S) || (o->diverge > 0.0 && S > o->diverge * S0)) { rep.status = MEK_EDIVERGED; break; }
            if (done >= o->max_iters) { rep.status = MEK_MAXITER; break; }
            // Inner problem: A D B = R_true from D = 0, error against X_ref - X_acc.
            MEK_TRY(convert_f64_f32(w.R64, m * n, w.R32, s));
            MEK_TRY(fill_zero_bytes(w.Xt32, (long long)(p * q) * 4, s));
            mek_solve_opts io = *o;
            io.replay_idx = nullptr;
            io.replay_len = 0;
            io.diverge = 0.0;
            const double* xref_t = nullptr;
            if (o->X_ref) {
                // The inner iterate D is judged against X_ref - X_acc, so its
                // error is the error of X_acc + D.
                MEK_TRY(lincomb_f64(1.0, o->X_ref, -1.0, w.Xacc, p * q, w.Xtmp, s));
                MEK_TRY(transpose_to<double>(w.Xtmp, (int)p, (int)q, w.Xref_t, s));
                xref_t = w.Xref_t;
            }
            // Inner stop: the outer rule on the true error when it is REL_ERR,
            // and in every case a drop of the inner residual by 1e-3 (the range
            // in which the FP32 incremental residual is still accurate).
            io.stop = (o->stop == MEK_STOP_REL_ERR) ? MEK_STOP_REL_ERR : MEK_STOP_NONE;
            io.tol = o->tol;
            const double S_target = 1e-6 * S;
            const long long cap = std::min<long long>(inner_cap, o->max_iters - done);
            DevReport ir;
            st = run_kernel<float>(P, &io, L, alpha, S, ref2, xref_t, cap, done, done, S_target,
                                   w.R32, w.Xt32, s, &ir, &kms);
            if (st) return st;
            // X_acc += D, accumulated in FP64.
            MEK_TRY(transpose_from<float>(w.Xt32, (int)p, (int)q, w.Xtmp, s));
            MEK_TRY(lincomb_f64(1.0, w.Xacc, 1.0, w.Xtmp, p * q, w.Xacc, s));
            done += ir.iters;
            ++passes;
            if (ir.status == MEK_ETIMEOUT || ir.status == MEK_EDIVERGED) { rep.status = ir.status; break; }
            if (ir.iters == 0 && ir.status != MEK_OK) { rep.status = MEK_MAXITER; break; }
        }
        MEK_TRY(copy_f64(w.Xacc, p * q, X, s));
    }
    MEK_TRY(hipStreamSynchronize(s));
    if (report) {
        report->iters = rep.iters;
        report->status = rep.status;
        report->resid2 = rep.S;
        report->rel_err = o->X_ref ? rep.err : NAN;
        report->alpha = alpha;
        report->team_wgs = L.W;
        report->r_in_lds = L.lds ? 1 : 0;
        report->passes = passes;
        report->kernel_ms = kms;
    }
    return rep.status;
}

int mek_philox_uniform(uint64_t seed, uint64_t instance, int64_t k0, int64_t count, double* out,
                       void* stream) {
    if (count < 0 || k0 < 0) return MEK_EINVAL;
    if (count == 0) return MEK_OK;
    int st = check_dev(out, (size_t)count * 8);
    if (st) return st;
    hipStream_t s = (hipStream_t)stream;
    MEK_TRY(launch_philox(seed, instance, k0, count, out, s));
    MEK_TRY(hipStreamSynchronize(s));
    return MEK_OK;
}

int mek_select(int variant, int64_t m, const double* r, const double* a, double F_A, double theta,
               uint64_t seed, uint64_t instance, int64_t k0, int64_t count, int32_t* idx,
               uint8_t* in_set, int32_t* set_list, double* stats, void* stream) {
    if (variant < MEK_BK || variant > MEK_MWRBK) return MEK_EINVAL;
    if (m <= 0 || m > INT32_MAX / 2 || count < 0 || k0 < 0) return MEK_EINVAL;
    if (m > (int64_t)kSelRows * kThreads) return MEK_EUNSUPPORTED;
    if (!(theta >= 0.0 && theta <= 1.0) || !(F_A > 0.0) || !isfinite(F_A)) return MEK_EINVAL;
    if (!r || !a || (count > 0 && !idx)) return MEK_EINVAL;
    int st;
    if ((st = check_dev(r, (size_t)m * 8)) || (st = check_dev(a, (size_t)m * 8))) return st;
    if (count > 0 && (st = check_dev(idx, (size_t)count * 4))) return st;
    if (in_set && (st = check_dev(in_set, (size_t)m))) return st;
    if (set_list && (st = check_dev(set_list, (size_t)m * 4))) return st;
    if (stats && (st = check_dev(stats, 4 * 8))) return st;
    hipStream_t s = (hipStream_t)stream;
    int* tmp = nullptr;
    MEK_TRY(hipMalloc((void**)&tmp, (size_t)(m + 1) * 4));
    int n_active = 0;
    hipError_t e = active_rows(a, (int)m, tmp, tmp + m, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&n_active, tmp + m, 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess && n_active == 0) {
        (void)hipFree(tmp);
        return MEK_EINVAL;
    }
    if (e == hipSuccess && in_set) e = fill_zero_bytes(in_set, m, s);
    if (e == hipSuccess && count > 0)
        e = launch_select(variant, (int)m, r, a, F_A, theta, seed, instance, k0, count, idx,
                          in_set, set_list, stats, tmp, n_active, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(tmp);
    return hip_status(e);
}

int mek_residual(int64_t m, int64_t p, int64_t q, int64_t n, const double* A, const double* X,
                 const double* B, const double* C, double* R, void* stream) {
    if (m <= 0 || p <= 0 || q <= 0 || n <= 0) return MEK_EINVAL;
    if (m > INT32_MAX / 2 || p > INT32_MAX / 2 || q > INT32_MAX / 2 || n > INT32_MAX / 2) return MEK_EINVAL;
    if (!A || !X || !B || !C || !R) return MEK_EINVAL;
    if ((const double*)R == A || (const double*)R == X || (const double*)R == B || (const double*)R == C)
        return MEK_EINVAL;
    int st;
    if ((st = check_dev(A, (size_t)(m * p) * 8)) || (st = check_dev(X, (size_t)(p * q) * 8)) ||
        (st = check_dev(B, (size_t)(q * n) * 8)) || (st = check_dev(C, (size_t)(m * n) * 8)) ||
        (st = check_dev(R, (size_t)(m * n) * 8)))
        return st;
    hipStream_t s = (hipStream_t)stream;
    double* T = nullptr;
    MEK_TRY(hipMalloc((void**)&T, (size_t)(m * q) * 8));
    hipError_t e = gemm_f64((int)m, (int)q, (int)p, 1.0, A, p, 1, X, q, 1, 0.0, nullptr, 0, T, q, s);
    if (e == hipSuccess)
        e = gemm_f64((int)m, (int)n, (int)q, -1.0, T, q, 1, B, n, 1, 1.0, C, n, R, n, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(T);
    return hip_status(e);
}

int mek_gram(int64_t rows, int64_t cols, const double* M, int transpose_first, double* G,
             void* stream) {
    if (rows <= 0 || cols <= 0 || rows > INT32_MAX / 2 || cols > INT32_MAX / 2) return MEK_EINVAL;
    if (!M || !G || (const double*)G == M) return MEK_EINVAL;
    if (transpose_first != 0 && transpose_first != 1) return MEK_EINVAL;
    const int64_t g = transpose_first ? cols : rows;
    int st;
    if ((st = check_dev(M, (size_t)(rows * cols) * 8)) || (st = check_dev(G, (size_t)(g * g) * 8)))
        return st;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e;
    if (!transpose_first)   // M M^T: A(i,k) = M[i,k], B(k,j) = M[j,k]
        e = gemm_f64((int)rows, (int)rows, (int)cols, 1.0, M, cols, 1, M, 1, cols, 0.0, nullptr, 0, G, rows, s);
    else                    // M^T M: A(i,k) = M[k,i], B(k,j) = M[k,j]
        e = gemm_f64((int)cols, (int)cols, (int)rows, 1.0, M, 1, cols, M, cols, 1, 0.0, nullptr, 0, G, cols, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return hip_status(e);
}

}  // extern "C"
