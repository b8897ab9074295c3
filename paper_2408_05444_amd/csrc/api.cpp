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
#include <cstddef>
#include <mutex>
#include <vector>

#include "../../include/mek.h"
#include "internal.h"

using namespace mek;

namespace {

struct Workspace {
    void* base = nullptr;
    size_t bytes = 0;
    int64_t cap = 0;           // instances the per-instance buffers hold
    // Per-instance buffers: instance b at b times the size given.
    double* R64 = nullptr;     // m x n
    float* R32 = nullptr;      // m x n (FP32 / MIXED)
    double* Xt64 = nullptr;    // q x p
    float* Xt32 = nullptr;     // q x p
    double* Xacc = nullptr;    // p x q, MIXED accumulated iterate
    double* Xtmp = nullptr;    // p x q
    double* Xref_t = nullptr;  // q x p
    double* r = nullptr;       // m
    double* r2 = nullptr;      // 2m: {||R_i||^2, ratio} pairs of the sparse form in device memory
    void* rowbuf = nullptr;    // n * 8 bytes
    void* wbuf = nullptr;      // n * 8 bytes
    void* vbuf = nullptr;      // q * 8 bytes
    double* errpart = nullptr; // kErrStride
    TeamSync* sync = nullptr;
    DevReport* report = nullptr;
    InstSlot* slots = nullptr;
    // Shared scratch.
    double* T64 = nullptr;     // per instance m x q, GEMM temporary A X
    double* scal = nullptr;    // 8 scalars
    double* red = nullptr;     // 256 partial sums of the reductions
    int* iscal = nullptr;      // 8 ints
    unsigned long long* phase = nullptr;   // 32 phase-timing counters
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
    double* bcol = nullptr;   // n, ||B_j||^2 (columns of B), for the two-sided variant
    double F_B = 0.0;         // ||B||_F^2
    int* active = nullptr;
    // Exchange buffers of the two-sided block kernel (allocated on first use).
    void* blk = nullptr;
    unsigned long long *hbuf = nullptr, *rbuf = nullptr, *cpart = nullptr, *gcol = nullptr,
                       *ebuf = nullptr, *epart = nullptr;
    float *A32 = nullptr, *B32 = nullptr, *BT32 = nullptr, *GA32 = nullptr, *GB32 = nullptr;
    // SPARSE plans: the nonzeros of the rows of A, the rows and columns of B
    // and the columns of A A^T in ELL form (values in the plan's precision),
    // in one allocation.
    int update = MEK_UPDATE_DENSE;
    int ell_w[4] = {0, 0, 0, 0};    // ka, kb, kbt, kg
    void* ell = nullptr;
    int *a_idx = nullptr, *b_idx = nullptr, *bt_idx = nullptr, *g_idx = nullptr;
    void *a_val = nullptr, *b_val = nullptr, *bt_val = nullptr, *g_val = nullptr;
    // Parameter table of a ragged launch whose first instance is this plan
    // (kept across calls, so that stream-ordered calls allocate nothing).
    void* mtab = nullptr;
    size_t mtab_bytes = 0;
    // Parameter table of a ragged launch of sparse plans (grown as needed).
    void* stab = nullptr;
    size_t stab_bytes = 0;
    Workspace ws;
};

static_assert(sizeof(mek_device_report) == sizeof(DevReport), "device report layout");
static_assert(offsetof(mek_device_report, iters) == offsetof(DevReport, iters) &&
                  offsetof(mek_device_report, status) == offsetof(DevReport, status) &&
                  offsetof(mek_device_report, resid2) == offsetof(DevReport, S) &&
                  offsetof(mek_device_report, rel_err) == offsetof(DevReport, err),
              "device report layout");

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

// Workspace for nb instances; grows (and never shrinks) with the batch size.
int ensure_workspace(mek_plan_s* P, int64_t nb) {
    if (P->ws.base && P->ws.cap >= nb) return MEK_OK;
    if (P->ws.base) {
        MEK_TRY(hipDeviceSynchronize());
        (void)hipFree(P->ws.base);
        P->ws = Workspace();
    }
    const size_t m = P->m, p = P->p, q = P->q, n = P->n, B = (size_t)nb;
    const bool f32 = P->precision != MEK_FP64;
    size_t need = 0;
    auto add = [&](size_t bytes) { need += (bytes + 255) & ~(size_t)255; };
    add(B * m * n * 8);
    add(f32 ? B * m * n * 4 : 0);
    add(B * q * p * 8);
    add(f32 ? B * q * p * 4 : 0);
    add(B * p * q * 8);
    add(B * p * q * 8);
    add(B * q * p * 8);
    add(B * m * 8);
    add(B * m * 16);
    add(B * n * 8);
    add(B * n * 8);
    add(B * q * 8);
    add(B * kErrStride * 8);
    add(B * sizeof(TeamSync));
    add(B * sizeof(DevReport));
    add(B * sizeof(InstSlot));
    add(B * m * q * 8);
    add(8 * 8);
    add(256 * 8);
    add(8 * 4);
    add(32 * 8);
    void* base = nullptr;
    MEK_TRY(hipMalloc(&base, need));
    char* cur = (char*)base;
    Workspace& w = P->ws;
    w.base = base;
    w.bytes = need;
    w.cap = nb;
    w.R64 = carve<double>(cur, B * m * n);
    w.R32 = f32 ? carve<float>(cur, B * m * n) : nullptr;
    w.Xt64 = carve<double>(cur, B * q * p);
    w.Xt32 = f32 ? carve<float>(cur, B * q * p) : nullptr;
    w.Xacc = carve<double>(cur, B * p * q);
    w.Xtmp = carve<double>(cur, B * p * q);
    w.Xref_t = carve<double>(cur, B * q * p);
    w.r = carve<double>(cur, B * m);
    w.r2 = carve<double>(cur, B * m * 2);
    w.rowbuf = carve<double>(cur, B * n);
    w.wbuf = carve<double>(cur, B * n);
    w.vbuf = carve<double>(cur, B * q);
    w.errpart = carve<double>(cur, B * kErrStride);
    w.sync = carve<TeamSync>(cur, B);
    w.report = carve<DevReport>(cur, B);
    w.slots = carve<InstSlot>(cur, B);
    w.T64 = carve<double>(cur, B * m * q);
    w.scal = carve<double>(cur, 8);
    w.red = carve<double>(cur, 256);
    w.iscal = carve<int>(cur, 8);
    w.phase = carve<unsigned long long>(cur, 32);
    return MEK_OK;
}

void free_plan(mek_plan_s* P) {
    if (!P) return;
    void* ptrs[] = {P->A, P->B, P->BT, P->GA, P->GB, P->a, P->bcol, P->active, P->A32, P->B32,
                    P->BT32, P->GA32, P->GB32, P->ws.base, P->blk, P->ell, P->mtab, P->stab};
    for (void* x : ptrs)
        if (x) (void)hipFree(x);
    delete P;
}

struct Layout {
    int W, rpw, xpw, wpw;
    bool lds;
    bool a_lds;
    bool x_lds;
    bool b_lds;
    bool small;   // the one-row-per-thread kernel (W = 1, R, B, X^T in LDS)
    size_t lds_bytes;
};

int ceil_div(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

constexpr int kRowsPerWG = 8;   // target rows of R per work-group (automatic layout)

// Team layout: how many work-groups share the solve and whether their rows
// of R stay in LDS. Automatic choice: one work-group per kRowsPerWG rows of
// R (at least as many as it takes for R to fit in LDS), capped by the CUs
// available to the instance.
// Team layout of one instance with at most cap work-groups; R may live in
// LDS only when allow_lds (and the plan's r_in_lds option permits it).
int choose_layout_cap(const mek_plan_s* P, size_t elem, int cap, bool allow_lds, Layout* L) {
    const int64_t m = P->m, n = P->n, q = P->q;
    // The selection keeps at most kSelRows row norms per thread in registers,
    // and the n-vector staging buffer must fit in LDS.
    if (m > (int64_t)kSelRows * kThreads) return MEK_EUNSUPPORTED;
    if ((size_t)std::max(n, q) * elem + 4096 > solve_lds_budget()) return MEK_EUNSUPPORTED;
    if (!allow_lds && P->r_in_lds == 1) return MEK_EUNSUPPORTED;
    const int cus = std::max(1, cap);
    const size_t budget = solve_lds_budget();
    L->small = false;
    L->b_lds = false;
    // Small instances under the automatic layout: one work-group, one row of
    // R per thread, R, B and X^T in LDS, no exchanges.
    if (allow_lds && P->team_wgs <= 0 && P->r_in_lds != 0 && m <= kThreads && n <= kThreads &&
        q <= kThreads && P->p <= kThreads &&
        solve_small_lds_bytes((int)m, (int)P->p, (int)q, (int)n, elem) <= budget) {
        L->W = 1;
        L->rpw = (int)m;
        L->xpw = (int)q;
        L->wpw = (int)n;
        L->lds = true;
        L->a_lds = L->x_lds = false;
        L->small = true;
        L->lds_bytes = solve_small_lds_bytes((int)m, (int)P->p, (int)q, (int)n, elem);
        return MEK_OK;
    }
    int W;
    bool lds;
    auto fits = [&](int Wc) {
        const int rpw = ceil_div(m, Wc);
        const int Wr = ceil_div(m, rpw);
        return solve_lds_bytes(rpw, (int)n, (int)q, ceil_div(q, Wr), ceil_div(n, Wr), elem, true,
                               Wr == 1) <= budget;
    };
    if (P->team_wgs > 0) {
        W = (int)std::min<int64_t>({(int64_t)P->team_wgs, (int64_t)cus, m});
        lds = allow_lds && (P->r_in_lds != 0) && fits(W);
        if (P->r_in_lds == 1 && !lds) return MEK_EUNSUPPORTED;
    } else {
        // About kRowsPerWG rows of R per work-group: measured on MI355X, the
        // time per update falls as rows per work-group drop to about 8 and
        // is flat below (the exchanges cost the same for any team size).
        int Wt = (int)std::min<int64_t>(std::max<int64_t>(1, (m + kRowsPerWG - 1) / kRowsPerWG), cus);
        int Wl = -1;
        for (int Wc = 1; Wc <= std::min<int64_t>(cus, m); ++Wc)
            if (fits(Wc)) { Wl = Wc; break; }
        if (allow_lds && P->r_in_lds != 0 && Wl > 0) {
            // With R in LDS the LDS fits any W >= Wl.
            W = std::max(Wt, Wl);
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
    L->lds_bytes = solve_lds_bytes(L->rpw, (int)n, (int)q, L->xpw, L->wpw, elem, L->lds, W == 1);
    if (L->lds_bytes > budget || W > kMaxTeam) return MEK_EUNSUPPORTED;
    // With room left: this work-group's rows of X^T (updated every step),
    // then ||A_i||^2 of all rows.
    // One work-group with R in LDS: B and B^T first (the dot products then
    // read no device memory).
    const size_t bb = 2 * (size_t)q * n * elem;
    L->b_lds = L->W == 1 && L->lds && L->lds_bytes + bb <= budget;
    if (L->b_lds) L->lds_bytes += bb;
    const size_t xb = (size_t)L->xpw * P->p * elem;
    L->x_lds = L->lds_bytes + xb <= budget;
    if (L->x_lds) L->lds_bytes += xb;
    L->a_lds = L->lds_bytes + solve_lds_bytes_a((int)m) <= budget;
    if (L->a_lds) L->lds_bytes += solve_lds_bytes_a((int)m);
    return MEK_OK;
}

// A uniform batch splits the CUs evenly between its instances' teams.
int choose_layout(const mek_plan_s* P, size_t elem, int64_t nb, Layout* L) {
    if (nb > std::max(1, P->cus)) return MEK_EUNSUPPORTED;
    return choose_layout_cap(P, elem, std::max(1, P->cus / (int)nb), true, L);
}

int validate_opts(const mek_plan_s* P, const mek_solve_opts* o) {
    if (!o) return MEK_EINVAL;
    if (o->variant < MEK_BK || o->variant > MEK_TWOSIDED) return MEK_EINVAL;
    if (o->variant == MEK_TWOSIDED) {
        if (o->block_rows < 1 || o->block_rows > kBlkCap) return MEK_EINVAL;
        if (o->block_cols < 1 || o->block_cols > kBlkCap) return MEK_EINVAL;
        if (!(o->tau <= 0.0 || (o->tau < 1.0 && isfinite(o->tau)))) return MEK_EINVAL;
        if (o->replay_len > 0) return MEK_EINVAL;
    }
    if (o->hist_cap > 0 && (o->rows_hist || o->cols_hist) && o->variant != MEK_TWOSIDED)
        return MEK_EINVAL;
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
    memset(&K, 0, sizeof(K));
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
    K.nb = 1;
    K.slots = nullptr;
    K.norms = nullptr;
    K.multi = nullptr;
    K.multi_start = nullptr;
    K.multi_n = 0;
    K.multi_wgs = 0;
    K.W = L.W;
    K.rpw = L.rpw;
    K.xpw = L.xpw;
    K.wpw = L.wpw;
}

// One persistent launch on the residuals already stored in ws.R64 / ws.R32.
// nb = 1 without slots: one instance, its scalars in `one`. With slots (host
// array of nb entries): a team per slot, instance slots[j].id's buffers.
// Each launched instance's report goes to out[id].
template <typename T>
int run_kernel(mek_plan_s* P, const mek_solve_opts* o, const Layout& L, double alpha,
               const InstSlot& one, const InstSlot* slots, int nb, const double* Xref_t, T* R,
               T* Xt, hipStream_t s, DevReport* out, double* kernel_ms) {
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
    K.ref2 = one.ref2;
    K.C2 = one.C2;
    K.max_iters = one.max_iters;
    K.k_offset = one.k_offset;
    K.hist_offset = one.hist_offset;
    K.S_target = one.S_target;
    K.inst = one.inst;
    Workspace& w = P->ws;
    // Instances touched by this launch: their exchange words start at tag 0,
    // which no update waits for.
    int lo = 0, hi = 1;
    if (slots) {
        MEK_TRY(hipMemcpyAsync(w.slots, slots, sizeof(InstSlot) * nb, hipMemcpyHostToDevice, s));
        MEK_TRY(hipStreamSynchronize(s));
        K.nb = nb;
        K.slots = w.slots;
        lo = slots[0].id;
        hi = slots[0].id + 1;
        for (int j = 0; j < nb; ++j) {
            lo = std::min(lo, slots[j].id);
            hi = std::max(hi, slots[j].id + 1);
        }
    }
    const long long span = hi - lo;
    // MEK_PHASES=1 in the environment: time the phases of each update on
    // three work-groups and print the averages to stderr (profiling aid).
    static const bool phases = getenv("MEK_PHASES") && getenv("MEK_PHASES")[0] == '1';
    K.phase = phases ? w.phase : nullptr;
    K.a_in_lds = L.a_lds ? 1 : 0;
    K.x_in_lds = L.x_lds ? 1 : 0;
    K.b_in_lds = L.b_lds ? 1 : 0;
    K.small = L.small ? 1 : 0;
    // Pause between polls of exchange words (tuning knob MEK_POLL_SLEEP).
    static const int poll_sleep = getenv("MEK_POLL_SLEEP") ? atoi(getenv("MEK_POLL_SLEEP")) : 1;
    K.poll_sleep = poll_sleep;
    if (phases) MEK_TRY(fill_zero_bytes(w.phase, 32 * 8, s));
    MEK_TRY(fill_zero_bytes(w.sync + lo, span * (long long)sizeof(TeamSync), s));
    MEK_TRY(fill_zero_bytes(w.errpart + lo * kErrStride, span * kErrStride * 8, s));
    MEK_TRY(fill_zero_bytes(w.r + lo * P->m, span * P->m * 8, s));
    MEK_TRY(fill_zero_bytes((char*)w.rowbuf + lo * P->n * 8, span * P->n * 8, s));
    MEK_TRY(fill_zero_bytes((char*)w.wbuf + lo * P->n * 8, span * P->n * 8, s));
    MEK_TRY(fill_zero_bytes((char*)w.vbuf + lo * P->q * 8, span * P->q * 8, s));
    hipEvent_t ev[2];
    MEK_TRY(hipEventCreate(&ev[0]));
    if (hipEventCreate(&ev[1]) != hipSuccess) {
        (void)hipEventDestroy(ev[0]);
        return MEK_EHIP;
    }
    hipError_t e = hipEventRecord(ev[0], s);
    if (e == hipSuccess) e = launch_solve(K, L.lds, L.lds_bytes, s);
    if (e == hipSuccess) e = hipEventRecord(ev[1], s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(out + lo, w.report + lo, sizeof(DevReport) * span,
                           hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    int st = hip_status(e);
    float ms = 0.0f;
    if (st == MEK_OK && hipEventElapsedTime(&ms, ev[0], ev[1]) == hipSuccess && kernel_ms)
        *kernel_ms += (double)ms;
    const long long iters0 = out[lo].iters;
    if (st == MEK_OK && phases && iters0 > 0) {
        unsigned long long h[24];
        int rate_khz = 100000;
        (void)hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, P->device);
        if (hipMemcpy(h, w.phase, sizeof(h), hipMemcpyDeviceToHost) == hipSuccess) {
            const char* names[8] = {"reduce", "select", "row", "dots", "waitw", "xupd", "update", "end"};
            const int wg[3] = {0, L.W / 2, L.W - 1};
            for (int t = 0; t < (L.W > 1 ? 3 : 1); ++t) {
                fprintf(stderr, "[mek phases] W=%d lds=%d a_lds=%d x_lds=%d wg=%d iters=%lld us/update:",
                        L.W, (int)L.lds, (int)L.a_lds, (int)L.x_lds, wg[t], iters0);
                for (int i = 0; i < 8; ++i)
                    fprintf(stderr, " %s=%.2f", names[i],
                            (double)h[t * 8 + i] / (rate_khz * 1e-3) / iters0);
                fprintf(stderr, " total_kernel=%.2f\n", ms * 1e3 / iters0);
            }
        }
    }
    (void)hipEventDestroy(ev[0]);
    (void)hipEventDestroy(ev[1]);
    return st;
}

// Most nonzeros per line that a SPARSE plan accepts.
constexpr int kSparseMaxWidth = 1024;

// The ELL structure of a SPARSE plan, from the plan's dense A, B and A A^T
// (entries of A A^T between rows of A with no common nonzero column are
// sums of exact zeros, so its pattern is exact).
int build_sparse(mek_plan_s* P, hipStream_t s) {
    const int m = (int)P->m, p = (int)P->p, q = (int)P->q, n = (int)P->n;
    const size_t elem = P->precision == MEK_FP64 ? 8 : 4;
    if (sparse_lds_bytes(m, p, q, n, elem, false, false, 0, 0, 0, 0) > solve_lds_budget())
        return MEK_EUNSUPPORTED;
    int* wd_dev = P->ws.iscal + 2;
    MEK_TRY(fill_zero_bytes(wd_dev, 4 * sizeof(int), s));
    MEK_TRY(ell_width(P->A, m, p, p, 1, wd_dev + 0, s));
    MEK_TRY(ell_width(P->B, q, n, n, 1, wd_dev + 1, s));
    MEK_TRY(ell_width(P->B, n, q, 1, n, wd_dev + 2, s));
    MEK_TRY(ell_width(P->GA, m, m, m, 1, wd_dev + 3, s));
    MEK_TRY(hipMemcpyAsync(P->ell_w, wd_dev, sizeof(P->ell_w), hipMemcpyDeviceToHost, s));
    MEK_TRY(hipStreamSynchronize(s));
    for (int& x : P->ell_w) {
        if (x > kSparseMaxWidth) return MEK_EUNSUPPORTED;
        x = std::max(x, 1);
    }
    const int ka = P->ell_w[0], kb = P->ell_w[1], kbt = P->ell_w[2], kg = P->ell_w[3];
    const size_t cnt[4] = {(size_t)m * ka, (size_t)q * kb, (size_t)n * kbt, (size_t)m * kg};
    size_t need = 0;
    for (size_t c : cnt) need += ((c * 4 + 255) & ~(size_t)255) + ((c * elem + 255) & ~(size_t)255);
    MEK_TRY(hipMalloc(&P->ell, need));
    char* cur = (char*)P->ell;
    int** idx[4] = {&P->a_idx, &P->b_idx, &P->bt_idx, &P->g_idx};
    void** val[4] = {&P->a_val, &P->b_val, &P->bt_val, &P->g_val};
    for (int t = 0; t < 4; ++t) {
        *idx[t] = carve<int>(cur, cnt[t]);
        *val[t] = elem == 8 ? (void*)carve<double>(cur, cnt[t]) : (void*)carve<float>(cur, cnt[t]);
    }
    auto fill = [&](const double* M, int rows, int cols, long long rs, long long cs, int width,
                    bool slot_major, int* ix, void* v) -> hipError_t {
        return elem == 8 ? ell_fill<double>(M, rows, cols, rs, cs, width, slot_major, ix, (double*)v, s)
                         : ell_fill<float>(M, rows, cols, rs, cs, width, slot_major, ix, (float*)v, s);
    };
    MEK_TRY(fill(P->A, m, p, p, 1, ka, false, P->a_idx, P->a_val));
    MEK_TRY(fill(P->B, q, n, n, 1, kb, true, P->b_idx, P->b_val));
    MEK_TRY(fill(P->B, n, q, 1, n, kbt, true, P->bt_idx, P->bt_val));
    MEK_TRY(fill(P->GA, m, m, m, 1, kg, false, P->g_idx, P->g_val));
    MEK_TRY(hipStreamSynchronize(s));
    return MEK_OK;
}

// One launch of the sparse-update kernel for the instances in `slots` (their
// residuals already in ws.R64), X0 (stacked, or NULL) as the start and X
// (stacked) as the output.
// The kernel parameters of a sparse plan's solve (R, X and X_ref pointers,
// reports, slots and batch size are the caller's); returns the LDS bytes.
template <typename T>
size_t fill_sparse(const mek_plan_s* P, const mek_solve_opts* o, double alpha, SparseParams<T>& K,
                   bool norms_mem = false) {
    const int64_t m = P->m, p = P->p, q = P->q, n = P->n;
    memset(&K, 0, sizeof(K));
    K.m = (int)m; K.p = (int)p; K.q = (int)q; K.n = (int)n;
    K.a_idx = P->a_idx;   K.a_val = (const T*)P->a_val;   K.ka = P->ell_w[0];
    K.b_idx = P->b_idx;   K.b_val = (const T*)P->b_val;   K.kb = P->ell_w[1];
    K.bt_idx = P->bt_idx; K.bt_val = (const T*)P->bt_val; K.kbt = P->ell_w[2];
    K.g_idx = P->g_idx;   K.g_val = (const T*)P->g_val;   K.kg = P->ell_w[3];
    K.a = P->a;
    K.F_A = P->F_A;
    K.active = P->active;
    K.n_active = P->n_active;
    K.sR = m * n;
    K.sX = p * q;
    // The row norms and row errors stay in LDS when they fit and the
    // selection's register chunks cover m (the plan's r_in_lds = 0 keeps them
    // in device memory: the form for instances too large for LDS). The LDS
    // left is taken in this order while it fits: ||A_i||^2 (read by every
    // selection), B's ELL slots (every v and w), then those of A A^T and A
    // (every update's row lists).
    const size_t elem = sizeof(T);
    const size_t budget = solve_lds_budget();
    K.norms_in_lds = 1;
    auto lds_for = [&](bool a_lds, bool b_lds, bool g_lds) {
        return sparse_lds_bytes((int)m, (int)p, (int)q, (int)n, elem, K.norms_in_lds != 0, a_lds,
                                b_lds ? K.kb : 0, b_lds ? K.kbt : 0, g_lds ? K.ka : 0,
                                g_lds ? K.kg : 0);
    };
    K.norms_in_lds = (!norms_mem && P->r_in_lds != 0 && m <= (int64_t)kSelRows * kThreads &&
                      lds_for(false, false, false) <= budget) ? 1 : 0;
    K.r_glob = P->ws.r2;
    K.e_glob = P->ws.Xtmp;
    K.a_in_lds = lds_for(true, false, false) <= budget ? 1 : 0;
    K.b_in_lds = lds_for(K.a_in_lds, true, false) <= budget ? 1 : 0;
    K.g_in_lds = lds_for(K.a_in_lds, K.b_in_lds, true) <= budget ? 1 : 0;
    K.variant = o->variant;
    K.theta = o->theta;
    K.alpha = alpha;
    K.stop = o->stop;
    K.tol = o->tol;
    K.diverge = o->diverge;
    K.seed = o->seed;
    K.replay = o->replay_idx;
    K.replay_len = o->replay_len;
    K.resid_hist = o->resid_hist;
    K.err_hist = o->err_hist;
    K.idx_hist = o->idx_hist;
    K.set_hist = o->set_hist;
    K.hist_cap = o->hist_cap;
    return lds_for(K.a_in_lds, K.b_in_lds, K.g_in_lds);
}

// R^0 already in ws.R64 (nb instances): the start X^0 into the kernel's X
// buffer (row-major p x q per instance), R in the kernel's precision.
template <typename T>
int sparse_state(mek_plan_s* P, int nb, const double* X0, T** R, T** Xs, hipStream_t s) {
    Workspace& w = P->ws;
    const long long mn = P->m * P->n, pq = P->p * P->q;
    const bool f64 = sizeof(T) == 8;
    *R = f64 ? (T*)w.R64 : (T*)w.R32;
    *Xs = f64 ? (T*)w.Xacc : (T*)w.Xt32;
    if (!f64) MEK_TRY(convert_f64_f32(w.R64, nb * mn, w.R32, s));
    if (X0) {
        if (f64) MEK_TRY(copy_f64(X0, nb * pq, w.Xacc, s));
        else MEK_TRY(convert_f64_f32(X0, nb * pq, w.Xt32, s));
    } else {
        MEK_TRY(fill_zero_bytes(*Xs, nb * pq * (long long)sizeof(T), s));
    }
    return MEK_OK;
}

template <typename T>
int run_sparse(mek_plan_s* P, const mek_solve_opts* o, double alpha,
               const std::vector<InstSlot>& slots, const double* X0, double* X, hipStream_t s,
               DevReport* out, double* kernel_ms) {
    Workspace& w = P->ws;
    const int nb = (int)slots.size();
    const int64_t m = P->m, n = P->n;
    const long long pq = P->p * P->q;
    const bool f64 = sizeof(T) == 8;
    T *R = nullptr, *Xs = nullptr;
    int st0 = sparse_state<T>(P, nb, X0, &R, &Xs, s);
    if (st0) return st0;
    SparseParams<T> K;
    const size_t lds = fill_sparse<T>(P, o, alpha, K);
    K.R = R;
    K.X = Xs;
    K.Xref = o->X_ref;
    K.report = w.report;
    K.slots = w.slots;
    K.nb = nb;
    MEK_TRY(hipMemcpyAsync(w.slots, slots.data(), sizeof(InstSlot) * nb, hipMemcpyHostToDevice, s));
    // MEK_PHASES=1: time the phases of each update on work-group 0 and print
    // the averages to stderr (profiling aid).
    static const bool phases = getenv("MEK_PHASES") && getenv("MEK_PHASES")[0] == '1';
    K.phase = phases ? w.phase : nullptr;
    if (phases) MEK_TRY(fill_zero_bytes(w.phase, 32 * 8, s));
    hipEvent_t ev[2];
    MEK_TRY(hipEventCreate(&ev[0]));
    if (hipEventCreate(&ev[1]) != hipSuccess) {
        (void)hipEventDestroy(ev[0]);
        return MEK_EHIP;
    }
    hipError_t e = hipEventRecord(ev[0], s);
    if (e == hipSuccess) e = launch_sparse(K, lds, s);
    if (e == hipSuccess) e = hipEventRecord(ev[1], s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(out, w.report, sizeof(DevReport) * nb, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    int st = hip_status(e);
    float ms = 0.0f;
    if (st == MEK_OK && hipEventElapsedTime(&ms, ev[0], ev[1]) == hipSuccess && kernel_ms)
        *kernel_ms += (double)ms;
    (void)hipEventDestroy(ev[0]);
    (void)hipEventDestroy(ev[1]);
    if (st) return st;
    if (phases && out[0].iters > 0) {
        unsigned long long h[6];
        int rate_khz = 100000;
        (void)hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, P->device);
        if (hipMemcpy(h, w.phase, sizeof(h), hipMemcpyDeviceToHost) == hipSuccess) {
            const char* names[6] = {"reduce", "select", "load", "v", "w_x", "r"};
            fprintf(stderr, "[mek sparse phases] m=%lld n=%lld widths=%d,%d,%d,%d a_lds=%d b_lds=%d "
                    "g_lds=%d iters=%lld us/update:", (long long)m, (long long)n, K.ka, K.kb, K.kbt,
                    K.kg, K.a_in_lds, K.b_in_lds, K.g_in_lds, out[0].iters);
            for (int i = 0; i < 6; ++i)
                fprintf(stderr, " %s=%.2f", names[i], (double)h[i] / (rate_khz * 1e-3) / out[0].iters);
            fprintf(stderr, " total_kernel=%.2f\n", ms * 1e3 / out[0].iters);
        }
    }
    if (f64) MEK_TRY(copy_f64(w.Xacc, nb * pq, X, s));
    else MEK_TRY(convert_f32_f64(w.Xt32, nb * pq, X, s));
    return MEK_OK;
}

int read_scalar(const double* dev, double* host, hipStream_t s) {
    MEK_TRY(hipMemcpyAsync(host, dev, sizeof(double), hipMemcpyDeviceToHost, s));
    MEK_TRY(hipStreamSynchronize(s));
    return MEK_OK;
}

// Largest eigenvalue of the symmetric positive semidefinite q x q matrix G
// (device) by repeated squaring: G_0 = G, G_{j+1} = G_j^2 / ||G_j||_F^2 on
// the FP64 matrix cores, until G_j is numerically rank one (||G_j||_F^2
// within 1e-13 of 1, at most 24 squarings: G^(2^24)); its column with the
// largest diagonal entry is then the top eigenvector v, and the eigenvalue
// is ||G v|| / ||v||. The error of that estimate is second order in the
// part of v outside the top eigenspace. Returns the value on the host.
int max_eig_by_squaring(const double* G, int q, double* lam, double* scal, double* red,
                        hipStream_t s) {
    double *buf = nullptr;
    const size_t qq = (size_t)q * q;
    MEK_TRY(hipMalloc((void**)&buf, (2 * qq + 2 * (size_t)q) * 8));
    double* P0 = buf;
    double* P1 = buf + qq;
    double* v = buf + 2 * qq;
    double* w = v + q;
    int st = MEK_OK;
    const double* cur = G;
    for (int it = 0; it < 24 && st == MEK_OK; ++it) {
        double f = 0.0;
        if (sq_norm(cur, (long long)qq, scal, red, s) != hipSuccess) { st = MEK_EHIP; break; }
        if ((st = read_scalar(scal, &f, s))) break;
        if (!(f > 0.0) || !isfinite(f)) break;
        if (it > 0 && fabs(f - 1.0) <= 1e-13) break;   // rank one: G_j^2 = G_j
        double* nxt = (cur == P0) ? P1 : P0;
        if (gemm_f64(q, q, q, 1.0 / f, cur, q, 1, cur, q, 1, 0.0, nullptr, 0, nxt, q, s) !=
            hipSuccess) { st = MEK_EHIP; break; }
        cur = nxt;
    }
    double vv = 0.0, ww = 0.0;
    if (st == MEK_OK && diag_argmax_col(cur, q, v, s) != hipSuccess) st = MEK_EHIP;
    if (st == MEK_OK &&
        gemm_f64(q, 1, q, 1.0, G, q, 1, v, 1, 1, 0.0, nullptr, 0, w, 1, s) != hipSuccess)
        st = MEK_EHIP;
    if (st == MEK_OK && sq_norm(v, q, scal, red, s) != hipSuccess) st = MEK_EHIP;
    if (st == MEK_OK) st = read_scalar(scal, &vv, s);
    if (st == MEK_OK && sq_norm(w, q, scal, red, s) != hipSuccess) st = MEK_EHIP;
    if (st == MEK_OK) st = read_scalar(scal, &ww, s);
    (void)hipStreamSynchronize(s);
    (void)hipFree(buf);
    if (st) return st;
    *lam = (vv > 0.0) ? sqrt(ww / vv) : 0.0;
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
    mek_plan_opts o = {MEK_FP64, 0.0, 0, -1, MEK_UPDATE_DENSE};
    if (opts) o = *opts;
    if (o.precision < MEK_FP64 || o.precision > MEK_MIXED) return MEK_EINVAL;
    if (o.update != MEK_UPDATE_DENSE && o.update != MEK_UPDATE_SPARSE) return MEK_EINVAL;
    if (o.update == MEK_UPDATE_SPARSE && o.precision == MEK_MIXED) return MEK_EUNSUPPORTED;
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
    P->update = o.update;
    int dev = 0;
    (void)hipGetDevice(&dev);
    P->device = dev;
    (void)hipDeviceGetAttribute(&P->cus, hipDeviceAttributeMultiprocessorCount, dev);

    auto fail = [&](int code) { free_plan(P); return code; };
    auto alloc = [&](void** ptr, size_t bytes) { return hipMalloc(ptr, bytes); };
    if (alloc((void**)&P->A, (size_t)(m * p) * 8) || alloc((void**)&P->B, (size_t)(q * n) * 8) ||
        alloc((void**)&P->BT, (size_t)(q * n) * 8) ||
        alloc((void**)&P->GA, (size_t)(m * m) * 8) || alloc((void**)&P->GB, (size_t)(n * n) * 8) ||
        alloc((void**)&P->a, (size_t)m * 8) || alloc((void**)&P->bcol, (size_t)n * 8) ||
        alloc((void**)&P->active, (size_t)m * 4) || ensure_workspace(P, 1))
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
    // ||B_j||^2 (rows of B^T) and ||B||_F^2.
    if (row_sq_norms(P->BT, (int)n, (int)q, P->bcol, s) || sum_reduce(P->bcol, n, w.scal + 6, w.red, s))
        return fail(MEK_EHIP);
    if ((st = read_scalar(w.scal + 6, &P->F_B, s))) return fail(st);
    // Gram matrices A A^T (m x m) and B^T B (n x n) on the matrix cores.
    if (gemm_f64((int)m, (int)m, (int)p, 1.0, P->A, p, 1, P->A, 1, p, 0.0, nullptr, 0, P->GA, m, s) ||
        gemm_f64((int)n, (int)n, (int)q, 1.0, P->B, 1, n, P->B, n, 1, 0.0, nullptr, 0, P->GB, n, s))
        return fail(MEK_EHIP);
    // ||B||_2^2: largest eigenvalue of the smaller Gram matrix.
    if (q <= n) {
        double* BBt = nullptr;
        if (alloc((void**)&BBt, (size_t)(q * q) * 8)) return fail(MEK_ENOMEM);
        hipError_t e = gemm_f64((int)q, (int)q, (int)n, 1.0, P->B, n, 1, P->B, 1, n, 0.0, nullptr, 0, BBt, q, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        st = (e == hipSuccess) ? max_eig_by_squaring(BBt, (int)q, &P->b2, w.scal + 1, w.red, s)
                               : MEK_EHIP;
        (void)hipFree(BBt);
        if (st) return fail(st);
    } else {
        if ((st = max_eig_by_squaring(P->GB, (int)n, &P->b2, w.scal + 1, w.red, s))) return fail(st);
    }
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
    if (P->update == MEK_UPDATE_SPARSE && (st = build_sparse(P, s))) return fail(st);
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

int mek_plan_sparse_widths(mek_plan P, int32_t* widths) {
    if (!P || !widths) return MEK_EINVAL;
    if (P->update != MEK_UPDATE_SPARSE) return MEK_EUNSUPPORTED;
    for (int t = 0; t < 4; ++t) widths[t] = P->ell_w[t];
    return MEK_OK;
}

}  // extern "C"

namespace {

// Team layout of the two-sided block kernel: the same policy as the row
// solver (all CUs when the residual is large, R in LDS when it fits).
int choose_layout_block2(const mek_plan_s* P, int s_cap, int t_cap, Layout* L) {
    const int64_t m = P->m, n = P->n, q = P->q;
    if (m > (int64_t)kSelRows * kThreads || n > (int64_t)kSelRows * kThreads) return MEK_EUNSUPPORTED;
    const int cus = std::max(1, P->cus);
    const size_t budget = block2_lds_budget();
    auto bytes = [&](int Wc, bool lds) {
        const int rpw = ceil_div(m, Wc);
        const int Wr = ceil_div(m, rpw);
        return block2_lds_bytes(rpw, (int)n, Wr, s_cap, t_cap, lds);
    };
    int W;
    bool lds;
    if (P->team_wgs > 0) {
        W = (int)std::min<int64_t>({(int64_t)P->team_wgs, (int64_t)cus, m});
        lds = (P->r_in_lds != 0) && bytes(W, true) <= budget;
        if (P->r_in_lds == 1 && !lds) return MEK_EUNSUPPORTED;
    } else {
        int Wt = (int)std::min<int64_t>(std::max<int64_t>(1, (m + kRowsPerWG - 1) / kRowsPerWG), cus);
        int Wl = -1;
        for (int Wc = 1; Wc <= std::min<int64_t>(cus, m); ++Wc)
            if (bytes(Wc, true) <= budget) { Wl = Wc; break; }
        if (P->r_in_lds != 0 && Wl > 0) {
            W = std::max(Wt, Wl);
            lds = true;
        } else {
            if (P->r_in_lds == 1) return MEK_EUNSUPPORTED;
            W = Wt;
            lds = false;
        }
    }
    const int rpw = ceil_div(m, W);
    W = ceil_div(m, rpw);
    L->W = W;
    L->rpw = rpw;
    L->xpw = ceil_div(q, W);
    L->wpw = 0;
    L->lds = lds && bytes(W, true) <= budget;
    L->a_lds = false;
    L->x_lds = false;
    L->lds_bytes = bytes(W, L->lds);
    if (L->lds_bytes > budget || W > kMaxTeam) return MEK_EUNSUPPORTED;
    return MEK_OK;
}

int ensure_block_ws(mek_plan_s* P) {
    if (P->blk) return MEK_OK;
    const size_t m = P->m, n = P->n, cus = std::max(1, P->cus);
    const size_t words = 2 * m + cus * n + n + (size_t)kBlkCap * kBlkCap + kMaxTeam;
    MEK_TRY(hipMalloc(&P->blk, words * 8));
    unsigned long long* w = (unsigned long long*)P->blk;
    P->hbuf = w;
    P->rbuf = P->hbuf + m;
    P->cpart = P->rbuf + m;
    P->gcol = P->cpart + cus * n;
    P->ebuf = P->gcol + n;
    P->epart = P->ebuf + kBlkCap * kBlkCap;
    return MEK_OK;
}

// One launch of the two-sided block kernel on the residual in ws.R64.
int run_block2(mek_plan_s* P, const mek_solve_opts* o, const Layout& L, double C2, double ref2,
               const double* Xref_t, hipStream_t s, DevReport* out, double* kernel_ms) {
    Workspace& w = P->ws;
    int st = ensure_block_ws(P);
    if (st) return st;
    Block2Params K;
    memset(&K, 0, sizeof(K));
    K.m = (int)P->m;
    K.p = (int)P->p;
    K.q = (int)P->q;
    K.n = (int)P->n;
    K.A = P->A;
    K.B = P->B;
    K.GA = P->GA;
    K.GB = P->GB;
    K.a = P->a;
    K.b = P->bcol;
    K.F_A = P->F_A;
    K.F_B = P->F_B;
    K.R = w.R64;
    K.Xt = w.Xt64;
    K.Xref_t = Xref_t;
    K.ref2 = ref2;
    K.C2 = C2;
    K.hbuf = P->hbuf;
    K.rbuf = P->rbuf;
    K.cpart = P->cpart;
    K.gcol = P->gcol;
    K.ebuf = P->ebuf;
    K.errpart = P->epart;
    K.sync = w.sync;
    K.report = w.report;
    K.theta = o->theta;
    K.tau = o->tau > 0.0 ? o->tau : 1e-10;
    K.s_cap = o->block_rows;
    K.t_cap = o->block_cols;
    K.stop = o->stop;
    K.tol = o->tol;
    K.max_iters = o->max_iters;
    K.diverge = o->diverge;
    K.resid_hist = o->resid_hist;
    K.err_hist = o->err_hist;
    K.rows_hist = o->rows_hist;
    K.cols_hist = o->cols_hist;
    K.hist_cap = o->hist_cap;
    K.W = L.W;
    K.rpw = L.rpw;
    K.xpw = L.xpw;
    K.r_in_lds = L.lds ? 1 : 0;
    static const int poll_sleep = getenv("MEK_POLL_SLEEP") ? atoi(getenv("MEK_POLL_SLEEP")) : 1;
    K.poll_sleep = poll_sleep;
    // MEK_PHASES=1: time the phases of each step on work-group 0 and print
    // the averages to stderr (profiling aid).
    static const bool phases = getenv("MEK_PHASES") && getenv("MEK_PHASES")[0] == '1';
    K.phase = phases ? w.phase : nullptr;
    if (phases) MEK_TRY(fill_zero_bytes(w.phase, 32 * 8, s));
    // Exchange words start with tag 0, which no step waits for.
    const size_t words = 2 * P->m + (size_t)std::max(1, P->cus) * P->n + P->n +
                         (size_t)kBlkCap * kBlkCap + kMaxTeam;
    MEK_TRY(fill_zero_bytes(P->blk, (long long)(words * 8), s));
    MEK_TRY(fill_zero_bytes(w.sync, sizeof(TeamSync), s));
    hipEvent_t ev[2];
    MEK_TRY(hipEventCreate(&ev[0]));
    if (hipEventCreate(&ev[1]) != hipSuccess) {
        (void)hipEventDestroy(ev[0]);
        return MEK_EHIP;
    }
    hipError_t e = hipEventRecord(ev[0], s);
    if (e == hipSuccess) e = launch_block2(K, L.lds_bytes, s);
    if (e == hipSuccess) e = hipEventRecord(ev[1], s);
    if (e == hipSuccess) e = hipMemcpyAsync(out, w.report, sizeof(DevReport), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    st = hip_status(e);
    float ms = 0.0f;
    if (st == MEK_OK && hipEventElapsedTime(&ms, ev[0], ev[1]) == hipSuccess && kernel_ms)
        *kernel_ms += (double)ms;
    if (st == MEK_OK && phases && out->iters > 0) {
        unsigned long long h[11];
        int rate_khz = 100000;
        (void)hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, P->device);
        if (hipMemcpy(h, w.phase, sizeof(h), hipMemcpyDeviceToHost) == hipSuccess) {
            const char* names[11] = {"rows", "cols", "select", "gram", "chol", "factor", "E",
                                     "W",    "X",    "R_upd",  "R_score"};
            fprintf(stderr, "[mek block phases] W=%d lds=%d steps=%lld us/step:", L.W, (int)L.lds,
                    (long long)out->iters);
            for (int i = 0; i < 11; ++i)
                fprintf(stderr, " %s=%.2f", names[i], (double)h[i] / (rate_khz * 1e-3) / out->iters);
            fprintf(stderr, " total_kernel=%.2f\n", ms * 1e3 / out->iters);
        }
    }
    (void)hipEventDestroy(ev[0]);
    (void)hipEventDestroy(ev[1]);
    return st;
}

// The solve of nb instances that share the plan's A and B (nb = 1: mek_solve).
// C, X0, X, X_ref and the histories are stacked per instance.
int solve_impl(mek_plan P, int64_t nb, const double* C, const double* X0,
               const mek_solve_opts* o, double* X, mek_report* reports, hipStream_t s) {
    if (!P || !C || !X || nb < 1) return MEK_EINVAL;
    int st = validate_opts(P, o);
    if (st) return st;
    const int64_t m = P->m, p = P->p, q = P->q, n = P->n;
    const size_t mn = (size_t)(m * n), pq = (size_t)(p * q);
    if ((st = check_dev(C, nb * mn * 8))) return st;
    if (X0 && (st = check_dev(X0, nb * pq * 8))) return st;
    if ((st = check_dev(X, nb * pq * 8))) return st;
    if (o->X_ref && (st = check_dev(o->X_ref, nb * pq * 8))) return st;
    if (o->replay_len > 0 && (st = check_dev(o->replay_idx, (size_t)o->replay_len * 4))) return st;
    if (o->hist_cap > 0) {
        const size_t hc = (size_t)(nb * o->hist_cap);
        if (o->resid_hist && (st = check_dev(o->resid_hist, hc * 8))) return st;
        if (o->err_hist && (st = check_dev(o->err_hist, hc * 8))) return st;
        if (o->idx_hist && (st = check_dev(o->idx_hist, hc * 4))) return st;
        if (o->set_hist && (st = check_dev(o->set_hist, hc * 4))) return st;
        if (o->rows_hist && (st = check_dev(o->rows_hist, hc * (size_t)o->block_rows * 4))) return st;
        if (o->cols_hist && (st = check_dev(o->cols_hist, hc * (size_t)o->block_cols * 4))) return st;
    }
    const int prec = P->precision;
    const bool twosided = o->variant == MEK_TWOSIDED;
    const bool sparse = P->update == MEK_UPDATE_SPARSE;
    if (twosided && (prec != MEK_FP64 || nb != 1 || sparse)) return MEK_EUNSUPPORTED;
    Layout L;
    memset(&L, 0, sizeof(L));
    L.W = 1;
    if (twosided) st = choose_layout_block2(P, o->block_rows, o->block_cols, &L);
    else if (!sparse) st = choose_layout(P, prec == MEK_FP64 ? 8 : 4, nb, &L);
    if (st) return st;
    if ((st = ensure_workspace(P, nb))) return st;
    Workspace& w = P->ws;
    if ((st = finite_check(C, nb * m * n, w.iscal, s))) return st;
    if (X0 && (st = finite_check(X0, nb * p * q, w.iscal, s))) return st;
    if (o->X_ref && (st = finite_check(o->X_ref, nb * p * q, w.iscal, s))) return st;
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

    // Per instance: ||C_b||_F^2 and ||X_ref,b||_F^2.
    std::vector<double> C2(nb, 0.0), ref2(nb, 1.0);
    for (int64_t b = 0; b < nb; ++b) {
        MEK_TRY(sq_norm(C + b * mn, m * n, w.scal + 2, w.red, s));
        if ((st = read_scalar(w.scal + 2, &C2[b], s))) return st;
        if (o->X_ref) {
            MEK_TRY(sq_norm(o->X_ref + b * pq, p * q, w.scal + 3, w.red, s));
            if ((st = read_scalar(w.scal + 3, &ref2[b], s))) return st;
            if (!(ref2[b] > 0.0)) ref2[b] = 1.0;
        }
    }

    // R^0_b = C_b - A X^0_b B (residual engine), or C_b when X^0 = 0.
    auto residual_into_R64 = [&](int64_t b, const double* Xcur) -> int {
        double* Rb = w.R64 + b * mn;
        if (Xcur) {
            MEK_TRY(gemm_f64((int)m, (int)q, (int)p, 1.0, P->A, p, 1, Xcur, q, 1, 0.0, nullptr, 0,
                             w.T64, q, s));
            MEK_TRY(gemm_f64((int)m, (int)n, (int)q, -1.0, w.T64, q, 1, P->B, n, 1, 1.0,
                             C + b * mn, n, Rb, n, s));
        } else {
            MEK_TRY(copy_f64(C + b * mn, m * n, Rb, s));
        }
        return MEK_OK;
    };
    // All instances at once (uniform batches share A and B): one launch per
    // product for the whole batch.
    auto residual_all_into_R64 = [&](const double* Xall) -> int {
        if (nb == 1) return residual_into_R64(0, Xall);
        if (!Xall) return copy_f64(C, nb * mn, w.R64, s) == hipSuccess ? MEK_OK : MEK_EHIP;
        MEK_TRY(gemm_f64_batched((int)nb, (int)m, (int)q, (int)p, 1.0, P->A, p, 1, 0, Xall, q, 1,
                                 pq, 0.0, nullptr, 0, 0, w.T64, q, m * q, s));
        MEK_TRY(gemm_f64_batched((int)nb, (int)m, (int)n, (int)q, -1.0, w.T64, q, 1, m * q, P->B,
                                 n, 1, 0, 1.0, C, n, mn, w.R64, n, mn, s));
        return MEK_OK;
    };
    auto slot_for = [&](int64_t b) {
        InstSlot sl;
        memset(&sl, 0, sizeof(sl));
        sl.id = (int)b;
        sl.C2 = C2[b];
        sl.ref2 = ref2[b];
        sl.max_iters = o->max_iters;
        sl.inst = o->instance + (uint64_t)b;
        return sl;
    };

    // FP32 residual refresh from the current FP32 iterate on the split-BF16
    // residual engine: R32_b = base_b - A32 (Xt32_b)^T B32 for the listed
    // instances (one batched launch per product when the list is the whole
    // batch). base is C (FP32 plans) or the FP64 true residual (MIXED).
    auto refresh_r32 = [&](const double* base, const std::vector<int64_t>& ids,
                           int pieces) -> int {
        float* T = reinterpret_cast<float*>(w.T64);
        const bool all = nb > 1 && (int64_t)ids.size() == nb;
        for (size_t j = 0; j < (all ? 1 : ids.size()); ++j) {
            const int64_t b = all ? 0 : ids[j];
            const int cnt = all ? (int)nb : 1;
            MEK_TRY(gemm_bf16s_batched(pieces, cnt, (int)m, (int)q, (int)p, 1.0, P->A32, p, 1, 0,
                                       w.Xt32 + b * pq, 1, p, pq, 0.0, nullptr, 0, 0, T, q,
                                       m * q, s));
            MEK_TRY(gemm_bf16s_batched(pieces, cnt, (int)m, (int)n, (int)q, -1.0, T, q, 1, m * q,
                                       P->B32, n, 1, 0, 1.0, base + b * mn, n, mn,
                                       w.R32 + b * mn, n, mn, s));
        }
        return MEK_OK;
    };
    const long long refresh = o->refresh_period > 0 ? o->refresh_period
                              : o->refresh_period == 0 ? std::max<long long>(2048, 4 * m)
                                                       : 0;

    std::vector<DevReport> rep(nb);
    std::vector<int> passes(nb, 1);
    memset(rep.data(), 0, sizeof(DevReport) * nb);
    double kms = 0.0;
    if (sparse) {
        // One work-group per instance; R^0 from the residual engine.
        std::vector<InstSlot> slots(nb);
        for (int64_t b = 0; b < nb; ++b) slots[b] = slot_for(b);
        if ((st = residual_all_into_R64(X0))) return st;
        st = prec == MEK_FP64 ? run_sparse<double>(P, o, alpha, slots, X0, X, s, rep.data(), &kms)
                              : run_sparse<float>(P, o, alpha, slots, X0, X, s, rep.data(), &kms);
        if (st) return st;
    } else if (prec == MEK_FP64 || prec == MEK_FP32) {
        std::vector<InstSlot> slots(nb);
        if ((st = residual_all_into_R64(X0))) return st;
        for (int64_t b = 0; b < nb; ++b) {
            if (o->X_ref)
                MEK_TRY(transpose_to<double>(o->X_ref + b * pq, (int)p, (int)q, w.Xref_t + b * pq, s));
            slots[b] = slot_for(b);
        }
        const double* xr = o->X_ref ? w.Xref_t : nullptr;
        const InstSlot* sp = nb > 1 ? slots.data() : nullptr;
        if (prec == MEK_FP64) {
            for (int64_t b = 0; b < nb; ++b) {
                if (X0) MEK_TRY(transpose_to<double>(X0 + b * pq, (int)p, (int)q, w.Xt64 + b * pq, s));
                else MEK_TRY(fill_zero_bytes(w.Xt64 + b * pq, (long long)pq * 8, s));
            }
            if (twosided)
                st = run_block2(P, o, L, C2[0], ref2[0], xr, s, rep.data(), &kms);
            else
                st = run_kernel<double>(P, o, L, alpha, slots[0], sp, (int)nb, xr, w.R64, w.Xt64, s,
                                        rep.data(), &kms);
            if (st) return st;
            for (int64_t b = 0; b < nb; ++b)
                MEK_TRY(transpose_from<double>(w.Xt64 + b * pq, (int)p, (int)q, X + b * pq, s));
        } else {
            MEK_TRY(convert_f64_f32(w.R64, nb * m * n, w.R32, s));
            for (int64_t b = 0; b < nb; ++b) {
                if (X0) MEK_TRY(transpose_to<float>(X0 + b * pq, (int)p, (int)q, w.Xt32 + b * pq, s));
                else MEK_TRY(fill_zero_bytes(w.Xt32 + b * pq, (long long)pq * 4, s));
            }
            // Passes of `refresh` updates, the residual recomputed (3 bf16
            // terms, FP32 accuracy) between them; the Philox counter, replay
            // position and histories continue across passes.
            std::vector<long long> done(nb, 0);
            std::vector<int64_t> ids;
            for (int64_t b = 0; b < nb; ++b) ids.push_back(b);
            std::vector<DevReport> ir(nb);
            for (;;) {
                std::vector<InstSlot> ps;
                for (int64_t b : ids) {
                    InstSlot sl = slots[b];
                    const long long left = o->max_iters - done[b];
                    sl.max_iters = refresh > 0 ? std::min<long long>(refresh, left) : left;
                    sl.k_offset = done[b];
                    sl.hist_offset = done[b];
                    ps.push_back(sl);
                }
                st = run_kernel<float>(P, o, L, alpha, ps[0], nb > 1 ? ps.data() : nullptr,
                                       (int)ps.size(), xr, w.R32, w.Xt32, s, ir.data(), &kms);
                if (st) return st;
                std::vector<int64_t> again;
                for (const InstSlot& sl : ps) {
                    const int64_t b = sl.id;
                    done[b] += ir[b].iters;
                    rep[b] = ir[b];
                    rep[b].iters = done[b];
                    if (ir[b].status == MEK_MAXITER && done[b] < o->max_iters) again.push_back(b);
                }
                if (again.empty()) break;
                for (int64_t b : again) ++passes[b];
                if ((st = refresh_r32(C, again, 3))) return st;
                ids = again;
            }
            for (int64_t b = 0; b < nb; ++b)
                MEK_TRY(transpose_from<float>(w.Xt32 + b * pq, (int)p, (int)q, X + b * pq, s));
        }
    } else {
        // MIXED: FP64 refinement around FP32 inner solves of A D B = R_true,
        // for every instance that has not met its stop rule yet.
        for (int64_t b = 0; b < nb; ++b) {
            if (X0) MEK_TRY(copy_f64(X0 + b * pq, p * q, w.Xacc + b * pq, s));
            else MEK_TRY(fill_zero_bytes(w.Xacc + b * pq, (long long)pq * 8, s));
        }
        // The inner stop is a 1e-3 drop of the residual norm, which FP32 reaches
        // well above its drift floor; the cap only bounds a pass.
        const long long inner_cap = o->inner_iters > 0 ? o->inner_iters
                                                       : std::max<long long>(20000, 200 * m);
        std::vector<long long> done(nb, 0);
        std::vector<double> S0(nb, -1.0);
        std::vector<char> running(nb, 1);
        for (int64_t b = 0; b < nb; ++b) passes[b] = 0;
        // Replayed indices continue across passes: the kernel reads entry
        // k_offset + k, with k_offset the updates already made.
        mek_solve_opts io = *o;
        io.diverge = 0.0;
        // Inner stop: the outer rule on the true error when it is REL_ERR, and
        // in every case a drop of the inner residual by 1e-3 (the range in
        // which the FP32 incremental residual is still accurate).
        io.stop = (o->stop == MEK_STOP_REL_ERR) ? MEK_STOP_REL_ERR : MEK_STOP_NONE;
        io.tol = o->tol;
        std::vector<DevReport> ir(nb);
        for (;;) {
            std::vector<InstSlot> slots;
            const bool all_running = nb > 1 && std::all_of(running.begin(), running.end(),
                                                           [](char c) { return c != 0; });
            if (all_running && (st = residual_all_into_R64(w.Xacc))) return st;
            for (int64_t b = 0; b < nb; ++b) {
                if (!running[b]) continue;
                double* Xacc = w.Xacc + b * pq;
                if (!all_running && (st = residual_into_R64(b, Xacc))) return st;
                double S = 0.0, err2 = NAN, err = NAN;
                MEK_TRY(sq_norm(w.R64 + b * mn, m * n, w.scal + 4, w.red, s));
                if ((st = read_scalar(w.scal + 4, &S, s))) return st;
                if (S0[b] < 0.0) S0[b] = S;
                if (o->X_ref) {
                    MEK_TRY(sq_diff_norm(Xacc, o->X_ref + b * pq, p * q, w.scal + 5, w.red, s));
                    if ((st = read_scalar(w.scal + 5, &err2, s))) return st;
                    err = sqrt(err2 / ref2[b]);
                }
                DevReport& r = rep[b];
                r.S = S;
                r.err = err;
                r.iters = done[b];
                const long long hk = done[b];
                if (o->hist_cap > hk) {
                    const size_t ho = (size_t)(b * o->hist_cap + hk);
                    if (o->resid_hist)
                        MEK_TRY(hipMemcpyAsync(o->resid_hist + ho, &S, 8, hipMemcpyHostToDevice, s));
                    if (o->err_hist)
                        MEK_TRY(hipMemcpyAsync(o->err_hist + ho, &err, 8, hipMemcpyHostToDevice, s));
                    MEK_TRY(hipStreamSynchronize(s));
                }
                int fin = 1;
                if (o->stop == MEK_STOP_REL_ERR && err <= o->tol) r.status = MEK_OK;
                else if (o->stop == MEK_STOP_REL_RESID && sqrt(S) <= o->tol * sqrt(C2[b])) r.status = MEK_OK;
                else if (S == 0.0) r.status = MEK_EXACT;
                else if (!isfinite(S) || (o->diverge > 0.0 && S > o->diverge * S0[b])) r.status = MEK_EDIVERGED;
                else if (done[b] >= o->max_iters) r.status = MEK_MAXITER;
                else fin = 0;
                if (fin) { running[b] = 0; continue; }
                // Inner problem: A D B = R_true from D = 0, error against
                // X_ref - X_acc, so that its error is the error of X_acc + D.
                MEK_TRY(convert_f64_f32(w.R64 + b * mn, m * n, w.R32 + b * mn, s));
                MEK_TRY(fill_zero_bytes(w.Xt32 + b * pq, (long long)pq * 4, s));
                if (o->X_ref) {
                    MEK_TRY(lincomb_f64(1.0, o->X_ref + b * pq, -1.0, Xacc, p * q, w.Xtmp + b * pq, s));
                    MEK_TRY(transpose_to<double>(w.Xtmp + b * pq, (int)p, (int)q, w.Xref_t + b * pq, s));
                }
                InstSlot sl = slot_for(b);
                sl.C2 = S;
                // The inner residual tracks the true residual of X_acc + D,
                // so under REL_RESID the inner pass also ends where the
                // outer rule would (the next pass checks it in FP64).
                sl.S_target = std::max(1e-6 * S, o->stop == MEK_STOP_REL_RESID
                                                     ? o->tol * o->tol * C2[b] : 0.0);
                sl.max_iters = std::min<long long>(inner_cap, o->max_iters - done[b]);
                sl.k_offset = done[b];
                sl.hist_offset = done[b];
                slots.push_back(sl);
            }
            if (slots.empty()) break;
            const bool batched = nb > 1;
            // The inner pass in sub-passes of `refresh` updates; between them
            // the inner residual R_true - A D B is recomputed from D (2 bf16
            // terms: about 2^-17 relative, far below the inner stop).
            std::vector<long long> idone(nb, 0), icap(nb, 0);
            for (const InstSlot& sl : slots) icap[sl.id] = sl.max_iters;
            std::vector<InstSlot> cur = slots;
            for (;;) {
                for (InstSlot& sl : cur) {
                    const long long left = icap[sl.id] - idone[sl.id];
                    sl.max_iters = refresh > 0 ? std::min<long long>(refresh, left) : left;
                    sl.k_offset = done[sl.id] + idone[sl.id];
                    sl.hist_offset = sl.k_offset;
                }
                st = run_kernel<float>(P, &io, L, alpha, cur[0], batched ? cur.data() : nullptr,
                                       (int)cur.size(), o->X_ref ? w.Xref_t : nullptr, w.R32,
                                       w.Xt32, s, ir.data(), &kms);
                if (st) return st;
                std::vector<InstSlot> next;
                std::vector<int64_t> again;
                for (const InstSlot& sl : cur) {
                    idone[sl.id] += ir[sl.id].iters;
                    if (ir[sl.id].status == MEK_MAXITER && idone[sl.id] < icap[sl.id]) {
                        next.push_back(sl);
                        again.push_back(sl.id);
                    }
                }
                if (again.empty()) break;
                if ((st = refresh_r32(w.R64, again, 2))) return st;
                cur = next;
            }
            for (const InstSlot& sl : slots) ir[sl.id].iters = idone[sl.id];
            for (const InstSlot& sl : slots) {
                const int64_t b = sl.id;
                // X_acc += D, accumulated in FP64.
                MEK_TRY(transpose_from<float>(w.Xt32 + b * pq, (int)p, (int)q, w.Xtmp + b * pq, s));
                MEK_TRY(lincomb_f64(1.0, w.Xacc + b * pq, 1.0, w.Xtmp + b * pq, p * q, w.Xacc + b * pq, s));
                done[b] += ir[b].iters;
                ++passes[b];
                if (ir[b].status == MEK_ETIMEOUT || ir[b].status == MEK_EDIVERGED) {
                    rep[b].status = ir[b].status;
                    rep[b].iters = done[b];
                    running[b] = 0;
                } else if (ir[b].iters == 0 && ir[b].status != MEK_OK) {
                    rep[b].status = MEK_MAXITER;
                    rep[b].iters = done[b];
                    running[b] = 0;
                }
            }
        }
        for (int64_t b = 0; b < nb; ++b)
            MEK_TRY(copy_f64(w.Xacc + b * pq, p * q, X + b * pq, s));
    }
    MEK_TRY(hipStreamSynchronize(s));
    int ret = MEK_OK;
    for (int64_t b = 0; b < nb; ++b) {
        if (reports) {
            mek_report& r = reports[b];
            r.iters = rep[b].iters;
            r.status = rep[b].status;
            r.resid2 = rep[b].S;
            r.rel_err = o->X_ref ? rep[b].err : NAN;
            r.alpha = alpha;
            r.team_wgs = L.W;
            r.r_in_lds = L.lds ? 1 : 0;
            r.passes = passes[b];
            r.kernel_ms = kms;
        }
        const int sb = rep[b].status;
        if (ret == MEK_OK && sb != MEK_OK) ret = sb;
        else if (ret >= 0 && sb < 0) ret = sb;
    }
    return ret;
}

// Ragged batch: instance b of plan plans[b] (sizes of its own), one
// persistent launch of the MULTI kernel form. Teams get work-groups in
// proportion to their per-update work (R and X touched), within one
// work-group per CU for the whole grid; R stays in device memory.
// True while `s` is being captured into a graph (which must not allocate).
bool capturing(hipStream_t s) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return cs != hipStreamCaptureStatusNone;
}

// The ragged launch's parameter table in the first plan, allocated once at
// the size of the largest batch (one instance per compute unit), so that it
// never moves under a captured graph; never allocated during capture.
int ensure_multi_table(mek_plan_s* P, size_t bytes, hipStream_t s) {
    if (P->mtab && P->mtab_bytes >= bytes) return MEK_OK;
    if (P->mtab) return MEK_EINVAL;   // larger than any batch the launch takes
    if (capturing(s)) return MEK_EUNSUPPORTED;
    const size_t nmax = (size_t)std::max(1, P->cus);
    const size_t want = std::max<size_t>(
        bytes, nmax * sizeof(SolveParams<double>) + (((nmax + 1) * sizeof(int) + 7) & ~(size_t)7));
    MEK_TRY(hipMalloc(&P->mtab, want));
    P->mtab_bytes = want;
    return MEK_OK;
}

template <typename T>
int run_multi(int64_t nb, mek_plan_s* const* plans, const std::vector<Layout>& Ls,
              const mek_solve_opts* o, const std::vector<double>& C2,
              const std::vector<double>& ref2, const double* const* Xref, hipStream_t s,
              std::vector<DevReport>& rep, double* kernel_ms, DevReport* dev_reports = nullptr) {
    std::vector<SolveParams<T>> K(nb);
    std::vector<int> start(nb + 1, 0);
    size_t lds = 0;
    int max_m = 1;
    static const int poll_sleep = getenv("MEK_POLL_SLEEP") ? atoi(getenv("MEK_POLL_SLEEP")) : 1;
    for (int64_t b = 0; b < nb; ++b) {
        mek_plan_s* P = plans[b];
        const Layout& L = Ls[b];
        Workspace& w = P->ws;
        SolveParams<T>& k = K[b];
        fill_common(k, P, o, L, o->alpha > 0.0 ? o->alpha : P->alpha);
        if (sizeof(T) == 8) {
            k.A = (const T*)P->A;
            k.B = (const T*)P->B;
            k.BT = (const T*)P->BT;
            k.GA = (const T*)P->GA;
            k.GB = (const T*)P->GB;
            k.R = (T*)w.R64;
            k.Xt = (T*)w.Xt64;
        } else {
            k.A = (const T*)P->A32;
            k.B = (const T*)P->B32;
            k.BT = (const T*)P->BT32;
            k.GA = (const T*)P->GA32;
            k.GB = (const T*)P->GB32;
            k.R = (T*)w.R32;
            k.Xt = (T*)w.Xt32;
        }
        k.Xref_t = (Xref && Xref[b]) ? w.Xref_t : nullptr;
        k.C2 = C2[b];
        k.ref2 = ref2[b];
        k.S_target = 0.0;
        k.inst = o->instance + (uint64_t)b;
        if (dev_reports) {
            k.norms = w.scal + 2;   // {||C_b||^2, ||X_ref,b||^2} computed on the device
            k.report = dev_reports + b;
        }
        const size_t hc = (size_t)b * (size_t)std::max<int64_t>(o->hist_cap, 0);
        k.resid_hist = o->resid_hist ? o->resid_hist + hc : nullptr;
        k.err_hist = o->err_hist ? o->err_hist + hc : nullptr;
        k.idx_hist = o->idx_hist ? o->idx_hist + hc : nullptr;
        k.set_hist = o->set_hist ? o->set_hist + hc : nullptr;
        k.phase = nullptr;
        k.a_in_lds = L.a_lds ? 1 : 0;
        k.x_in_lds = L.x_lds ? 1 : 0;
        k.b_in_lds = L.b_lds ? 1 : 0;
        k.poll_sleep = poll_sleep;
        start[b + 1] = start[b] + L.W;
        lds = std::max(lds, L.lds_bytes);
        max_m = std::max(max_m, (int)P->m);
        MEK_TRY(fill_zero_bytes(w.sync, (long long)sizeof(TeamSync), s));
        MEK_TRY(fill_zero_bytes(w.errpart, kErrStride * 8, s));
        MEK_TRY(fill_zero_bytes(w.r, P->m * 8, s));
        MEK_TRY(fill_zero_bytes((char*)w.rowbuf, P->n * 8, s));
        MEK_TRY(fill_zero_bytes((char*)w.wbuf, P->n * 8, s));
        MEK_TRY(fill_zero_bytes((char*)w.vbuf, P->q * 8, s));
    }
    const size_t pbytes = sizeof(SolveParams<T>) * (size_t)nb;
    const size_t tbytes = pbytes + ((sizeof(int) * (size_t)(nb + 1) + 7) & ~(size_t)7);
    int st = ensure_multi_table(plans[0], tbytes, s);
    if (st) return st;
    char* dbuf = (char*)plans[0]->mtab;
    SolveParams<T> head = K[0];
    head.multi = reinterpret_cast<const SolveParams<T>*>(dbuf);
    head.multi_start = reinterpret_cast<const int*>(dbuf + pbytes);
    head.multi_n = (int)nb;
    head.multi_wgs = start[nb];
    if (dev_reports) {
        // Stream-ordered: the table goes in through kernel arguments, the
        // kernel reads the norms from device memory and writes the reports
        // to the caller's structs; nothing waits.
        MEK_TRY(store_bytes(K.data(), pbytes, dbuf, s));
        MEK_TRY(store_bytes(start.data(), sizeof(int) * (size_t)(nb + 1), dbuf + pbytes, s));
        MEK_TRY(launch_solve_multi(head, max_m, lds, s));
        return MEK_OK;
    }
    hipEvent_t ev[2] = {nullptr, nullptr};
    hipError_t e = hipMemcpyAsync(dbuf, K.data(), pbytes, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(dbuf + pbytes, start.data(), sizeof(int) * (size_t)(nb + 1),
                           hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipEventCreate(&ev[0]);
    if (e == hipSuccess) e = hipEventCreate(&ev[1]);
    if (e == hipSuccess) e = hipEventRecord(ev[0], s);
    if (e == hipSuccess) e = launch_solve_multi(head, max_m, lds, s);
    if (e == hipSuccess) e = hipEventRecord(ev[1], s);
    for (int64_t b = 0; b < nb && e == hipSuccess; ++b)
        e = hipMemcpyAsync(&rep[b], plans[b]->ws.report, sizeof(DevReport), hipMemcpyDeviceToHost,
                           s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    st = hip_status(e);
    float ms = 0.0f;
    if (st == MEK_OK && hipEventElapsedTime(&ms, ev[0], ev[1]) == hipSuccess && kernel_ms)
        *kernel_ms += (double)ms;
    for (hipEvent_t x : ev)
        if (x) (void)hipEventDestroy(x);
    return st;
}

// Ragged batch of sparse plans: every instance one work-group of one plain
// launch, its complete parameters in a table in the first plan. Instances
// may share a plan: the j-th instance on a plan uses the j-th per-instance
// slice of that plan's workspace (R, X, slot, report).
template <typename T>
int run_sparse_multi(int64_t nb, mek_plan_s* const* Ps, const mek_solve_opts* o,
                     const double* const* C, const double* const* X0, const double* const* Xref,
                     double* const* X, hipStream_t s, std::vector<DevReport>& rep,
                     double* kernel_ms, DevReport* dev_reports = nullptr) {
    // Stream-ordered (dev_reports set): no host reads or waits; the norms go
    // to the kernel through device memory, slots and table through kernel
    // arguments, and nothing is allocated while the stream is captured.
    const bool async = dev_reports != nullptr;
    const bool cap = async && capturing(s);
    // Occurrence of each instance on its plan, and the workspaces.
    std::vector<int> occ(nb, 0);
    {
        std::vector<std::pair<mek_plan_s*, int>> seen;
        for (int64_t b = 0; b < nb; ++b) {
            int j = 0;
            for (auto& pr : seen)
                if (pr.first == Ps[b]) j = ++pr.second;
            if (j == 0) seen.push_back({Ps[b], 0});
            occ[b] = j;
        }
        for (auto& pr : seen) {
            if (cap && (!pr.first->ws.base || pr.first->ws.cap < pr.second + 1))
                return MEK_EUNSUPPORTED;   // a captured call must not allocate
            int st = ensure_workspace(pr.first, pr.second + 1);
            if (st) return st;
        }
    }
    std::vector<SparseParams<T>> K(nb);
    std::vector<InstSlot> slots(nb);
    size_t lds = 0;
    int max_m = 1;
    const bool f64 = sizeof(T) == 8;
    // One launch has one selection form: if any instance needs its norms in
    // device memory, every instance keeps them there.
    bool norms_mem = false;
    for (int64_t b = 0; b < nb; ++b) {
        SparseParams<T> probe;
        fill_sparse<T>(Ps[b], o, 1.0, probe);
        norms_mem = norms_mem || !probe.norms_in_lds;
    }
    for (int64_t b = 0; b < nb; ++b) {
        mek_plan_s* P = Ps[b];
        Workspace& w = P->ws;
        const int j = occ[b];
        const int64_t m = P->m, p = P->p, q = P->q, n = P->n;
        const long long mn = m * n, pq = p * q;
        const double* x0 = X0 ? X0[b] : nullptr;
        const double* xr = Xref ? Xref[b] : nullptr;
        int st;
        InstSlot& sl = slots[b];
        memset(&sl, 0, sizeof(sl));
        sl.ref2 = 1.0;
        double* norms = w.errpart + (size_t)j * kErrStride;   // unused by this kernel otherwise
        if (async) {
            sl.C2 = 1.0;
            MEK_TRY(sq_norm(C[b], mn, norms, w.red, s));
            if (xr) MEK_TRY(sq_norm(xr, pq, norms + 1, w.red, s));
            else MEK_TRY(fill_zero_bytes(norms + 1, 8, s));
        } else {
            if ((st = finite_check(C[b], mn, w.iscal, s))) return st;
            if (x0 && (st = finite_check(x0, pq, w.iscal, s))) return st;
            if (xr && (st = finite_check(xr, pq, w.iscal, s))) return st;
            MEK_TRY(sq_norm(C[b], mn, w.scal + 2, w.red, s));
            if ((st = read_scalar(w.scal + 2, &sl.C2, s))) return st;
            if (xr) {
                MEK_TRY(sq_norm(xr, pq, w.scal + 3, w.red, s));
                if ((st = read_scalar(w.scal + 3, &sl.ref2, s))) return st;
                if (!(sl.ref2 > 0.0)) sl.ref2 = 1.0;
            }
        }
        sl.id = 0;
        sl.max_iters = o->max_iters;
        sl.inst = o->instance + (uint64_t)b;
        // R^0 = C - A X^0 B (or C) into slice j, then the kernel's state.
        double* R64 = w.R64 + (size_t)j * mn;
        if (x0) {
            MEK_TRY(gemm_f64((int)m, (int)q, (int)p, 1.0, P->A, p, 1, x0, q, 1, 0.0, nullptr, 0,
                             w.T64, q, s));
            MEK_TRY(gemm_f64((int)m, (int)n, (int)q, -1.0, w.T64, q, 1, P->B, n, 1, 1.0, C[b], n,
                             R64, n, s));
        } else {
            MEK_TRY(copy_f64(C[b], mn, R64, s));
        }
        T* R = f64 ? (T*)R64 : (T*)(w.R32 + (size_t)j * mn);
        T* Xs = f64 ? (T*)(w.Xacc + (size_t)j * pq) : (T*)(w.Xt32 + (size_t)j * pq);
        if (!f64) MEK_TRY(convert_f64_f32(R64, mn, (float*)R, s));
        if (x0) {
            if (f64) MEK_TRY(copy_f64(x0, pq, (double*)Xs, s));
            else MEK_TRY(convert_f64_f32(x0, pq, (float*)Xs, s));
        } else {
            MEK_TRY(fill_zero_bytes(Xs, pq * (long long)sizeof(T), s));
        }
        lds = std::max(lds, fill_sparse<T>(P, o, o->alpha > 0.0 ? o->alpha : P->alpha, K[b],
                                           norms_mem));
        SparseParams<T>& k = K[b];
        k.R = R;
        k.X = Xs;
        k.Xref = xr;
        k.r_glob = w.r2 + (size_t)j * 2 * m;
        k.e_glob = w.Xtmp + (size_t)j * pq;
        k.report = async ? dev_reports + b : w.report + j;
        k.slots = w.slots + j;
        k.nb = 1;
        if (async) k.norms = norms;
        const size_t hc = (size_t)b * (size_t)std::max<int64_t>(o->hist_cap, 0);
        k.resid_hist = o->resid_hist ? o->resid_hist + hc : nullptr;
        k.err_hist = o->err_hist ? o->err_hist + hc : nullptr;
        k.idx_hist = o->idx_hist ? o->idx_hist + hc : nullptr;
        k.set_hist = o->set_hist ? o->set_hist + hc : nullptr;
        if (async) MEK_TRY(store_bytes(&sl, sizeof(sl), w.slots + j, s));
        else MEK_TRY(hipMemcpyAsync(w.slots + j, &sl, sizeof(sl), hipMemcpyHostToDevice, s));
        max_m = std::max(max_m, (int)m);
    }
    // The table, in the first plan: at least 1024 entries, so that batches
    // up to that size never move it under a captured graph.
    mek_plan_s* P0 = Ps[0];
    const size_t tbytes = sizeof(SparseParams<T>) * (size_t)nb;
    if (!P0->stab || P0->stab_bytes < tbytes) {
        if (cap) return MEK_EUNSUPPORTED;
        if (P0->stab) {
            MEK_TRY(hipDeviceSynchronize());
            (void)hipFree(P0->stab);
            P0->stab = nullptr;
            P0->stab_bytes = 0;
        }
        const size_t want = std::max(tbytes, sizeof(SparseParams<double>) * (size_t)1024);
        MEK_TRY(hipMalloc(&P0->stab, want));
        P0->stab_bytes = want;
    }
    SparseParams<T> head = K[0];
    head.m = max_m;   // sizes the selection chunk of every instance
    head.nb = (int)nb;
    head.multi = (const SparseParams<T>*)P0->stab;
    if (async) {
        MEK_TRY(store_bytes(K.data(), tbytes, P0->stab, s));
        MEK_TRY(launch_sparse(head, lds, s));
        for (int64_t b = 0; b < nb; ++b) {
            const mek_plan_s* P = Ps[b];
            const long long pq = P->p * P->q;
            if (f64) MEK_TRY(copy_f64(P->ws.Xacc + (size_t)occ[b] * pq, pq, X[b], s));
            else MEK_TRY(convert_f32_f64(P->ws.Xt32 + (size_t)occ[b] * pq, pq, X[b], s));
        }
        return MEK_OK;
    }
    MEK_TRY(hipMemcpyAsync(P0->stab, K.data(), tbytes, hipMemcpyHostToDevice, s));
    hipEvent_t ev[2];
    MEK_TRY(hipEventCreate(&ev[0]));
    if (hipEventCreate(&ev[1]) != hipSuccess) {
        (void)hipEventDestroy(ev[0]);
        return MEK_EHIP;
    }
    hipError_t e = hipEventRecord(ev[0], s);
    if (e == hipSuccess) e = launch_sparse(head, lds, s);
    if (e == hipSuccess) e = hipEventRecord(ev[1], s);
    for (int64_t b = 0; b < nb && e == hipSuccess; ++b)
        e = hipMemcpyAsync(&rep[b], Ps[b]->ws.report + occ[b], sizeof(DevReport),
                           hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    int st = hip_status(e);
    float ms = 0.0f;
    if (st == MEK_OK && hipEventElapsedTime(&ms, ev[0], ev[1]) == hipSuccess && kernel_ms)
        *kernel_ms += (double)ms;
    (void)hipEventDestroy(ev[0]);
    (void)hipEventDestroy(ev[1]);
    if (st) return st;
    for (int64_t b = 0; b < nb; ++b) {
        const mek_plan_s* P = Ps[b];
        const long long pq = P->p * P->q;
        if (f64) MEK_TRY(copy_f64(P->ws.Xacc + (size_t)occ[b] * pq, pq, X[b], s));
        else MEK_TRY(convert_f32_f64(P->ws.Xt32 + (size_t)occ[b] * pq, pq, X[b], s));
    }
    return MEK_OK;
}

// Host reports of a ragged batch and its combined status: MEK_OK when every
// instance met the stop rule, else the first failing status (errors first).
int finish_reports(int64_t nb, mek_plan_s* const* Ps, const std::vector<Layout>& Ls,
                   const mek_solve_opts* o, const double* const* Xref,
                   const std::vector<DevReport>& rep, double kms, mek_report* reports,
                   bool sparse) {
    int ret = MEK_OK;
    for (int64_t b = 0; b < nb; ++b) {
        if (reports) {
            mek_report& r = reports[b];
            r.iters = rep[b].iters;
            r.status = rep[b].status;
            r.resid2 = rep[b].S;
            r.rel_err = (Xref && Xref[b]) ? rep[b].err : NAN;
            r.alpha = o->alpha > 0.0 ? o->alpha : Ps[b]->alpha;
            r.team_wgs = sparse ? 1 : Ls[b].W;
            r.r_in_lds = 0;
            r.passes = 1;
            r.kernel_ms = kms;
        }
        const int sb = rep[b].status;
        if (ret == MEK_OK && sb != MEK_OK) ret = sb;
        else if (ret >= 0 && sb < 0) ret = sb;
    }
    return ret;
}

// Checks and team layouts of a ragged batch (host only, nothing enqueued).
int multi_setup(int64_t nb, const mek_plan* plans, const double* const* C,
                const double* const* X0, const double* const* Xref, const mek_solve_opts* o,
                double* const* X, std::vector<mek_plan_s*>& Ps, std::vector<Layout>& Ls) {
    if (nb < 1 || !plans || !C || !X || !o) return MEK_EINVAL;
    // References come per instance through Xref; forced indices and the
    // two-sided projection are single-instance features.
    if (o->X_ref) return MEK_EINVAL;
    if (o->replay_len > 0 || o->variant == MEK_TWOSIDED) return MEK_EUNSUPPORTED;
    Ps.assign(nb, nullptr);
    for (int64_t b = 0; b < nb; ++b) {
        Ps[b] = plans[b];
        if (!Ps[b] || !C[b] || !X[b]) return MEK_EINVAL;
        if (Ps[b]->update != MEK_UPDATE_SPARSE)
            for (int64_t c = 0; c < b; ++c)
                if (Ps[c] == Ps[b]) return MEK_EINVAL;   // a team needs its plan's workspace
        if (Ps[b]->precision != Ps[0]->precision || Ps[b]->device != Ps[0]->device)
            return MEK_EINVAL;
        if (Ps[b]->update != Ps[0]->update) return MEK_EINVAL;
        mek_solve_opts ob = *o;
        ob.X_ref = Xref ? Xref[b] : nullptr;
        int st = validate_opts(Ps[b], &ob);
        if (st) return st;
    }
    const int prec = Ps[0]->precision;
    if (prec == MEK_MIXED) return MEK_EUNSUPPORTED;
    const bool sparse = Ps[0]->update == MEK_UPDATE_SPARSE;
    const int cus = std::max(1, Ps[0]->cus);
    if (!sparse && nb > cus) return MEK_EUNSUPPORTED;
    if (nb > INT32_MAX / 2) return MEK_EINVAL;
    int st;
    for (int64_t b = 0; b < nb; ++b) {
        const mek_plan_s* P = Ps[b];
        const size_t mn = (size_t)(P->m * P->n), pq = (size_t)(P->p * P->q);
        if ((st = check_dev(C[b], mn * 8)) || (st = check_dev(X[b], pq * 8))) return st;
        if (X0 && X0[b] && (st = check_dev(X0[b], pq * 8))) return st;
        if (Xref && Xref[b] && (st = check_dev(Xref[b], pq * 8))) return st;
    }
    if (o->hist_cap > 0) {
        const size_t hc = (size_t)(nb * o->hist_cap);
        if (o->resid_hist && (st = check_dev(o->resid_hist, hc * 8))) return st;
        if (o->err_hist && (st = check_dev(o->err_hist, hc * 8))) return st;
        if (o->idx_hist && (st = check_dev(o->idx_hist, hc * 4))) return st;
        if (o->set_hist && (st = check_dev(o->set_hist, hc * 4))) return st;
    }
    Ls.assign(nb, Layout());
    if (sparse) return MEK_OK;   // one work-group per instance, no team layout
    // Work-group caps: starting from one each, every further work-group goes
    // to the instance with the most elements per work-group that one update
    // touches (R, B twice for v and w, X), so the slowest team is as fast as
    // the budget allows; no team beyond about kRowsPerWG rows per work-group.
    std::vector<double> cost(nb);
    std::vector<int> cap(nb, 1), wmax(nb);
    for (int64_t b = 0; b < nb; ++b) {
        const mek_plan_s* P = Ps[b];
        cost[b] = (double)P->m * P->n + 2.0 * P->q * P->n + 2.0 * P->p * P->q;
        wmax[b] = (int)std::max<int64_t>(1, (P->m + kRowsPerWG - 1) / kRowsPerWG);
    }
    // Team sizes given on every plan (an autotuned allocation) and fitting the
    // device are taken as they are.
    int64_t given = 0;
    bool all_given = true;
    for (int64_t b = 0; b < nb; ++b) {
        all_given = all_given && Ps[b]->team_wgs > 0;
        given += std::max(0, Ps[b]->team_wgs);
    }
    if (all_given && given <= cus)
        for (int64_t b = 0; b < nb; ++b) cap[b] = wmax[b] = Ps[b]->team_wgs;
    for (int spare = cus - (int)nb; !(all_given && given <= cus) && spare > 0; --spare) {
        int64_t best = -1;
        for (int64_t b = 0; b < nb; ++b)
            if (cap[b] < wmax[b] && (best < 0 || cost[b] / cap[b] > cost[best] / cap[best]))
                best = b;
        if (best < 0) break;
        ++cap[best];
    }
    const size_t elem = prec == MEK_FP64 ? 8 : 4;
    Ls.assign(nb, Layout());
    for (int64_t b = 0; b < nb; ++b)
        if ((st = choose_layout_cap(Ps[b], elem, cap[b], false, &Ls[b]))) return st;
    return MEK_OK;
}

int solve_multi_impl(int64_t nb, const mek_plan* plans, const double* const* C,
                     const double* const* X0, const double* const* Xref,
                     const mek_solve_opts* o, double* const* X, mek_report* reports,
                     hipStream_t s) {
    if (o && o->refresh_period > 0) return MEK_EUNSUPPORTED;
    std::vector<mek_plan_s*> Ps;
    std::vector<Layout> Ls;
    int st = multi_setup(nb, plans, C, X0, Xref, o, X, Ps, Ls);
    if (st) return st;
    const int prec = Ps[0]->precision;
    const bool sparse = Ps[0]->update == MEK_UPDATE_SPARSE;
    if (sparse) {
        std::vector<DevReport> rep(nb);
        memset(rep.data(), 0, sizeof(DevReport) * nb);
        double kms = 0.0;
        st = prec == MEK_FP64
                 ? run_sparse_multi<double>(nb, Ps.data(), o, C, X0, Xref, X, s, rep, &kms)
                 : run_sparse_multi<float>(nb, Ps.data(), o, C, X0, Xref, X, s, rep, &kms);
        if (st) return st;
        MEK_TRY(hipStreamSynchronize(s));
        return finish_reports(nb, Ps.data(), Ls, o, Xref, rep, kms, reports, true);
    }
    // Per instance: workspace, the finite checks, ||C||^2, ||X_ref||^2, the
    // starting residual, X^0 and X_ref transposed.
    std::vector<double> C2(nb, 0.0), ref2(nb, 1.0);
    for (int64_t b = 0; b < nb; ++b) {
        mek_plan_s* P = Ps[b];
        const int64_t m = P->m, p = P->p, q = P->q, n = P->n;
        const double* x0 = X0 ? X0[b] : nullptr;
        const double* xr = Xref ? Xref[b] : nullptr;
        if ((st = ensure_workspace(P, 1))) return st;
        Workspace& w = P->ws;
        if ((st = finite_check(C[b], m * n, w.iscal, s))) return st;
        if (x0 && (st = finite_check(x0, p * q, w.iscal, s))) return st;
        if (xr && (st = finite_check(xr, p * q, w.iscal, s))) return st;
        MEK_TRY(sq_norm(C[b], m * n, w.scal + 2, w.red, s));
        if ((st = read_scalar(w.scal + 2, &C2[b], s))) return st;
        if (xr) {
            MEK_TRY(sq_norm(xr, p * q, w.scal + 3, w.red, s));
            if ((st = read_scalar(w.scal + 3, &ref2[b], s))) return st;
            if (!(ref2[b] > 0.0)) ref2[b] = 1.0;
            MEK_TRY(transpose_to<double>(xr, (int)p, (int)q, w.Xref_t, s));
        }
        if (x0) {
            MEK_TRY(gemm_f64((int)m, (int)q, (int)p, 1.0, P->A, p, 1, x0, q, 1, 0.0, nullptr, 0,
                             w.T64, q, s));
            MEK_TRY(gemm_f64((int)m, (int)n, (int)q, -1.0, w.T64, q, 1, P->B, n, 1, 1.0, C[b], n,
                             w.R64, n, s));
        } else {
            MEK_TRY(copy_f64(C[b], m * n, w.R64, s));
        }
        if (prec == MEK_FP64) {
            if (x0) MEK_TRY(transpose_to<double>(x0, (int)p, (int)q, w.Xt64, s));
            else MEK_TRY(fill_zero_bytes(w.Xt64, (long long)(p * q) * 8, s));
        } else {
            MEK_TRY(convert_f64_f32(w.R64, m * n, w.R32, s));
            if (x0) MEK_TRY(transpose_to<float>(x0, (int)p, (int)q, w.Xt32, s));
            else MEK_TRY(fill_zero_bytes(w.Xt32, (long long)(p * q) * 4, s));
        }
    }
    std::vector<DevReport> rep(nb);
    memset(rep.data(), 0, sizeof(DevReport) * nb);
    double kms = 0.0;
    st = prec == MEK_FP64 ? run_multi<double>(nb, Ps.data(), Ls, o, C2, ref2, Xref, s, rep, &kms)
                          : run_multi<float>(nb, Ps.data(), Ls, o, C2, ref2, Xref, s, rep, &kms);
    if (st) return st;
    for (int64_t b = 0; b < nb; ++b) {
        mek_plan_s* P = Ps[b];
        if (prec == MEK_FP64)
            MEK_TRY(transpose_from<double>(P->ws.Xt64, (int)P->p, (int)P->q, X[b], s));
        else
            MEK_TRY(transpose_from<float>(P->ws.Xt32, (int)P->p, (int)P->q, X[b], s));
    }
    MEK_TRY(hipStreamSynchronize(s));
    return finish_reports(nb, Ps.data(), Ls, o, Xref, rep, kms, reports, false);
}

// Stream-ordered ragged batch: the steps of solve_multi_impl without a host
// wait (norms on the device, table through kernel arguments, reports to the
// caller's device structs). Every plan's workspace and the first plan's
// table must exist (one earlier call on the same plans).
int solve_multi_async_impl(int64_t nb, const mek_plan* plans, const double* const* C,
                           const double* const* X0, const double* const* Xref,
                           const mek_solve_opts* o, double* const* X, void* dev_reports,
                           hipStream_t s) {
    if (!dev_reports) return MEK_EINVAL;
    if (o && o->refresh_period > 0) return MEK_EUNSUPPORTED;
    std::vector<mek_plan_s*> Ps;
    std::vector<Layout> Ls;
    int st = multi_setup(nb, plans, C, X0, Xref, o, X, Ps, Ls);
    if (st) return st;
    if ((st = check_dev(dev_reports, sizeof(DevReport) * (size_t)nb))) return st;
    const int prec = Ps[0]->precision;
    if (Ps[0]->update == MEK_UPDATE_SPARSE) {
        std::vector<DevReport> unused(nb);
        DevReport* dr = (DevReport*)dev_reports;
        return prec == MEK_FP64
                   ? run_sparse_multi<double>(nb, Ps.data(), o, C, X0, Xref, X, s, unused, nullptr, dr)
                   : run_sparse_multi<float>(nb, Ps.data(), o, C, X0, Xref, X, s, unused, nullptr, dr);
    }
    const bool cap = capturing(s);
    for (int64_t b = 0; b < nb; ++b) {
        if (Ps[b]->ws.base) continue;
        if (cap) return MEK_EUNSUPPORTED;   // a captured call must not allocate
        if ((st = ensure_workspace(Ps[b], 1))) return st;
    }
    for (int64_t b = 0; b < nb; ++b) {
        mek_plan_s* P = Ps[b];
        const int64_t m = P->m, p = P->p, q = P->q, n = P->n;
        const double* x0 = X0 ? X0[b] : nullptr;
        const double* xr = Xref ? Xref[b] : nullptr;
        Workspace& w = P->ws;
        MEK_TRY(sq_norm(C[b], m * n, w.scal + 2, w.red, s));
        if (xr) {
            MEK_TRY(sq_norm(xr, p * q, w.scal + 3, w.red, s));
            MEK_TRY(transpose_to<double>(xr, (int)p, (int)q, w.Xref_t, s));
        } else {
            MEK_TRY(fill_zero_bytes(w.scal + 3, 8, s));
        }
        if (x0) {
            MEK_TRY(gemm_f64((int)m, (int)q, (int)p, 1.0, P->A, p, 1, x0, q, 1, 0.0, nullptr, 0,
                             w.T64, q, s));
            MEK_TRY(gemm_f64((int)m, (int)n, (int)q, -1.0, w.T64, q, 1, P->B, n, 1, 1.0, C[b], n,
                             w.R64, n, s));
        } else {
            MEK_TRY(copy_f64(C[b], m * n, w.R64, s));
        }
        if (prec == MEK_FP64) {
            if (x0) MEK_TRY(transpose_to<double>(x0, (int)p, (int)q, w.Xt64, s));
            else MEK_TRY(fill_zero_bytes(w.Xt64, (long long)(p * q) * 8, s));
        } else {
            MEK_TRY(convert_f64_f32(w.R64, m * n, w.R32, s));
            if (x0) MEK_TRY(transpose_to<float>(x0, (int)p, (int)q, w.Xt32, s));
            else MEK_TRY(fill_zero_bytes(w.Xt32, (long long)(p * q) * 4, s));
        }
    }
    std::vector<double> C2(nb, 1.0), ref2(nb, 1.0);
    std::vector<DevReport> rep(nb);
    DevReport* dr = (DevReport*)dev_reports;
    st = prec == MEK_FP64
             ? run_multi<double>(nb, Ps.data(), Ls, o, C2, ref2, Xref, s, rep, nullptr, dr)
             : run_multi<float>(nb, Ps.data(), Ls, o, C2, ref2, Xref, s, rep, nullptr, dr);
    if (st) return st;
    for (int64_t b = 0; b < nb; ++b) {
        mek_plan_s* P = Ps[b];
        if (prec == MEK_FP64)
            MEK_TRY(transpose_from<double>(P->ws.Xt64, (int)P->p, (int)P->q, X[b], s));
        else
            MEK_TRY(transpose_from<float>(P->ws.Xt32, (int)P->p, (int)P->q, X[b], s));
    }
    return MEK_OK;
}

// Stream-ordered solve (FP64 / FP32, one instance): every step is a kernel
// or a device copy on the stream, nothing waits on the host, and the kernel
// writes its report to the caller's device struct, so the call can be
// captured into a graph once the plan's workspace exists.
template <typename T>
int enqueue_solve(mek_plan_s* P, const mek_solve_opts* o, const Layout& L, const double* C,
                  const double* X0, double* X, DevReport* dev_report, hipStream_t s) {
    Workspace& w = P->ws;
    const int64_t m = P->m, p = P->p, q = P->q, n = P->n;
    // ||C||^2 and ||X_ref||^2 (0 without a reference) into the scalar slots
    // the kernel reads at its start.
    MEK_TRY(sq_norm(C, m * n, w.scal + 2, w.red, s));
    if (o->X_ref) {
        MEK_TRY(sq_norm(o->X_ref, p * q, w.scal + 3, w.red, s));
        MEK_TRY(transpose_to<double>(o->X_ref, (int)p, (int)q, w.Xref_t, s));
    } else {
        MEK_TRY(fill_zero_bytes(w.scal + 3, 8, s));
    }
    if (X0) {
        MEK_TRY(gemm_f64((int)m, (int)q, (int)p, 1.0, P->A, p, 1, X0, q, 1, 0.0, nullptr, 0, w.T64,
                         q, s));
        MEK_TRY(gemm_f64((int)m, (int)n, (int)q, -1.0, w.T64, q, 1, P->B, n, 1, 1.0, C, n, w.R64, n,
                         s));
    } else {
        MEK_TRY(copy_f64(C, m * n, w.R64, s));
    }
    T* R = (T*)w.R64;
    T* Xt = (T*)w.Xt64;
    if (sizeof(T) == 4) {
        MEK_TRY(convert_f64_f32(w.R64, m * n, w.R32, s));
        R = (T*)w.R32;
        Xt = (T*)w.Xt32;
    }
    if (X0) MEK_TRY(transpose_to<T>(X0, (int)p, (int)q, Xt, s));
    else MEK_TRY(fill_zero_bytes(Xt, (long long)(p * q) * (long long)sizeof(T), s));
    SolveParams<T> K;
    fill_common(K, P, o, L, o->alpha > 0.0 ? o->alpha : P->alpha);
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
    K.Xref_t = o->X_ref ? w.Xref_t : nullptr;
    K.norms = w.scal + 2;
    K.C2 = 1.0;
    K.ref2 = 1.0;
    K.S_target = 0.0;
    K.report = dev_report;
    K.phase = nullptr;
    K.a_in_lds = L.a_lds ? 1 : 0;
    K.x_in_lds = L.x_lds ? 1 : 0;
    K.b_in_lds = L.b_lds ? 1 : 0;
    K.small = L.small ? 1 : 0;
    static const int poll_sleep = getenv("MEK_POLL_SLEEP") ? atoi(getenv("MEK_POLL_SLEEP")) : 1;
    K.poll_sleep = poll_sleep;
    MEK_TRY(fill_zero_bytes(w.sync, (long long)sizeof(TeamSync), s));
    MEK_TRY(fill_zero_bytes(w.errpart, kErrStride * 8, s));
    MEK_TRY(fill_zero_bytes(w.r, m * 8, s));
    MEK_TRY(fill_zero_bytes((char*)w.rowbuf, n * 8, s));
    MEK_TRY(fill_zero_bytes((char*)w.wbuf, n * 8, s));
    MEK_TRY(fill_zero_bytes((char*)w.vbuf, q * 8, s));
    MEK_TRY(launch_solve(K, L.lds, L.lds_bytes, s));
    MEK_TRY(transpose_from<T>(Xt, (int)p, (int)q, X, s));
    return MEK_OK;
}

// Stream-ordered solve of a SPARSE plan: the steps of run_sparse with the
// norms computed on the device and the instance slot stored through kernel
// arguments, the report written to the caller's device struct.
template <typename T>
int enqueue_sparse(mek_plan_s* P, const mek_solve_opts* o, const double* C, const double* X0,
                   double* X, DevReport* dev_report, hipStream_t s) {
    Workspace& w = P->ws;
    const int64_t m = P->m, p = P->p, q = P->q, n = P->n;
    MEK_TRY(sq_norm(C, m * n, w.scal + 2, w.red, s));
    if (o->X_ref) MEK_TRY(sq_norm(o->X_ref, p * q, w.scal + 3, w.red, s));
    else MEK_TRY(fill_zero_bytes(w.scal + 3, 8, s));
    if (X0) {
        MEK_TRY(gemm_f64((int)m, (int)q, (int)p, 1.0, P->A, p, 1, X0, q, 1, 0.0, nullptr, 0, w.T64,
                         q, s));
        MEK_TRY(gemm_f64((int)m, (int)n, (int)q, -1.0, w.T64, q, 1, P->B, n, 1, 1.0, C, n, w.R64, n,
                         s));
    } else {
        MEK_TRY(copy_f64(C, m * n, w.R64, s));
    }
    T *R = nullptr, *Xs = nullptr;
    int st = sparse_state<T>(P, 1, X0, &R, &Xs, s);
    if (st) return st;
    SparseParams<T> K;
    const size_t lds = fill_sparse<T>(P, o, o->alpha > 0.0 ? o->alpha : P->alpha, K);
    K.R = R;
    K.X = Xs;
    K.Xref = o->X_ref;
    K.report = dev_report;
    K.slots = w.slots;
    K.nb = 1;
    K.norms = w.scal + 2;
    InstSlot sl;
    memset(&sl, 0, sizeof(sl));
    sl.id = 0;
    sl.C2 = 1.0;
    sl.ref2 = 1.0;
    sl.max_iters = o->max_iters;
    sl.inst = o->instance;
    MEK_TRY(store_bytes(&sl, sizeof(sl), w.slots, s));
    MEK_TRY(launch_sparse(K, lds, s));
    const long long pq = p * q;
    if (sizeof(T) == 8) MEK_TRY(copy_f64(w.Xacc, pq, X, s));
    else MEK_TRY(convert_f32_f64(w.Xt32, pq, X, s));
    return MEK_OK;
}

int solve_async_impl(mek_plan P, const double* C, const double* X0, const mek_solve_opts* o,
                     double* X, void* dev_report, hipStream_t s) {
    if (!P || !C || !X || !dev_report || !o) return MEK_EINVAL;
    if (P->precision == MEK_MIXED || o->variant == MEK_TWOSIDED || o->replay_len > 0 ||
        o->refresh_period > 0)
        return MEK_EUNSUPPORTED;
    int st = validate_opts(P, o);
    if (st) return st;
    const int64_t m = P->m, p = P->p, q = P->q, n = P->n;
    const size_t mn = (size_t)(m * n), pq = (size_t)(p * q);
    if ((st = check_dev(C, mn * 8)) || (X0 && (st = check_dev(X0, pq * 8))) ||
        (st = check_dev(X, pq * 8)) || (o->X_ref && (st = check_dev(o->X_ref, pq * 8))) ||
        (st = check_dev(dev_report, sizeof(DevReport))))
        return st;
    if (o->hist_cap > 0) {
        const size_t hc = (size_t)o->hist_cap;
        if (o->resid_hist && (st = check_dev(o->resid_hist, hc * 8))) return st;
        if (o->err_hist && (st = check_dev(o->err_hist, hc * 8))) return st;
        if (o->idx_hist && (st = check_dev(o->idx_hist, hc * 4))) return st;
        if (o->set_hist && (st = check_dev(o->set_hist, hc * 4))) return st;
    }
    const bool f64 = P->precision == MEK_FP64;
    if (P->update == MEK_UPDATE_SPARSE) {
        if ((st = ensure_workspace(P, 1))) return st;
        return f64 ? enqueue_sparse<double>(P, o, C, X0, X, (DevReport*)dev_report, s)
                   : enqueue_sparse<float>(P, o, C, X0, X, (DevReport*)dev_report, s);
    }
    Layout L;
    if ((st = choose_layout(P, f64 ? 8 : 4, 1, &L))) return st;
    if ((st = ensure_workspace(P, 1))) return st;
    return f64 ? enqueue_solve<double>(P, o, L, C, X0, X, (DevReport*)dev_report, s)
               : enqueue_solve<float>(P, o, L, C, X0, X, (DevReport*)dev_report, s);
}

}  // namespace

extern "C" {

int mek_solve_async(mek_plan P, const double* C, const double* X0, const mek_solve_opts* o,
                    double* X, mek_device_report* dev_report, void* stream) {
    return solve_async_impl(P, C, X0, o, X, dev_report, (hipStream_t)stream);
}

int mek_solve_multi_async(int64_t nb, const mek_plan* plans, const double* const* C,
                          const double* const* X0, const double* const* X_ref,
                          const mek_solve_opts* o, double* const* X, mek_device_report* dev_reports,
                          void* stream) {
    return solve_multi_async_impl(nb, plans, C, X0, X_ref, o, X, dev_reports, (hipStream_t)stream);
}

int mek_solve_multi(int64_t nb, const mek_plan* plans, const double* const* C,
                    const double* const* X0, const double* const* X_ref,
                    const mek_solve_opts* opts, double* const* X, mek_report* reports,
                    void* stream) {
    return solve_multi_impl(nb, plans, C, X0, X_ref, opts, X, reports, (hipStream_t)stream);
}

int mek_solve(mek_plan P, const double* C, const double* X0, const mek_solve_opts* o, double* X,
              mek_report* report, void* stream) {
    return solve_impl(P, 1, C, X0, o, X, report, (hipStream_t)stream);
}

int mek_solve_batched(mek_plan P, int64_t batch, const double* C, const double* X0,
                      const mek_solve_opts* o, double* X, mek_report* reports, void* stream) {
    if (batch < 1) return MEK_EINVAL;
    return solve_impl(P, batch, C, X0, o, X, reports, (hipStream_t)stream);
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

int mek_residual_batched(int64_t nb, int64_t m, int64_t p, int64_t q, int64_t n, const double* A,
                         const double* X, const double* B, const double* C, double* R,
                         void* stream) {
    if (nb <= 0 || m <= 0 || p <= 0 || q <= 0 || n <= 0) return MEK_EINVAL;
    if (m > INT32_MAX / 2 || p > INT32_MAX / 2 || q > INT32_MAX / 2 || n > INT32_MAX / 2 ||
        nb > INT32_MAX / 2)
        return MEK_EINVAL;
    if (!A || !X || !B || !C || !R) return MEK_EINVAL;
    const size_t rb = (size_t)(nb * m * n) * 8;
    auto overlaps = [&](const double* x, size_t bytes) {
        const char *r0 = (const char*)R, *x0 = (const char*)x;
        return r0 < x0 + bytes && x0 < r0 + rb;
    };
    if (overlaps(A, (size_t)(m * p) * 8) || overlaps(X, (size_t)(nb * p * q) * 8) ||
        overlaps(B, (size_t)(q * n) * 8) || overlaps(C, rb))
        return MEK_EINVAL;
    int st;
    if ((st = check_dev(A, (size_t)(m * p) * 8)) || (st = check_dev(X, (size_t)(nb * p * q) * 8)) ||
        (st = check_dev(B, (size_t)(q * n) * 8)) || (st = check_dev(C, rb)) ||
        (st = check_dev(R, rb)))
        return st;
    hipStream_t s = (hipStream_t)stream;
    // The temporaries A X_b (nb x m x q) live in a per-device buffer kept
    // between calls (grown when a call needs more); calls are serialised on it.
    static std::mutex mtx;
    static double* tbuf[64] = {nullptr};
    static size_t tbytes[64] = {0};
    std::lock_guard<std::mutex> lock(mtx);
    int dev = 0;
    MEK_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return MEK_EUNSUPPORTED;
    const size_t need = (size_t)(nb * m * q) * 8;
    if (tbytes[dev] < need) {
        if (tbuf[dev]) {
            MEK_TRY(hipDeviceSynchronize());
            (void)hipFree(tbuf[dev]);
            tbuf[dev] = nullptr;
            tbytes[dev] = 0;
        }
        MEK_TRY(hipMalloc((void**)&tbuf[dev], need));
        tbytes[dev] = need;
    }
    double* T = tbuf[dev];
    const int b = (int)nb;
    hipError_t e = gemm_f64_batched(b, (int)m, (int)q, (int)p, 1.0, A, p, 1, 0, X, q, 1, p * q,
                                    0.0, nullptr, 0, 0, T, q, m * q, s);
    if (e == hipSuccess)
        e = gemm_f64_batched(b, (int)m, (int)n, (int)q, -1.0, T, q, 1, m * q, B, n, 1, 0, 1.0, C, n,
                             m * n, R, n, m * n, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return hip_status(e);
}

int mek_residual(int64_t m, int64_t p, int64_t q, int64_t n, const double* A, const double* X,
                 const double* B, const double* C, double* R, void* stream) {
    return mek_residual_batched(1, m, p, q, n, A, X, B, C, R, stream);
}

}  // extern "C"

// ---- Residual engine without allocation: the temporary T = A X lives in a
// fixed device array of kNoAllocScratch doubles (16 MiB), one per device,
// held until the process ends. Host code never passes the array's name to
// a kernel (on the host it only stands in for the symbol): its device
// address is looked up once per device with hipGetSymbolAddress and kept.
namespace {
constexpr size_t kNoAllocScratch = (size_t)1 << 21;
__device__ __align__(256) double scratch[kNoAllocScratch];
std::mutex g_scratch_mtx;
double* g_scratch_ptr[64] = {nullptr};

int noalloc_scratch(double** out) {
    int dev = 0;
    MEK_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return MEK_EUNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mtx);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return MEK_EHIP;
        }
        g_scratch_ptr[dev] = (double*)ptr;
    }
    *out = g_scratch_ptr[dev];
    return MEK_OK;
}
}  // namespace

extern "C" {

int mek_residual_noalloc(int64_t m, int64_t p, int64_t q, int64_t n, const double* A,
                         const double* X, const double* B, const double* C, double* R,
                         void* stream) {
    if (m <= 0 || p <= 0 || q <= 0 || n <= 0) return MEK_EINVAL;
    if (m > INT32_MAX / 2 || p > INT32_MAX / 2 || q > INT32_MAX / 2 || n > INT32_MAX / 2)
        return MEK_EINVAL;
    if ((uint64_t)m * (uint64_t)q > kNoAllocScratch) return MEK_EINVAL;   // T does not fit
    if (!A || !X || !B || !C || !R) return MEK_EINVAL;
    const size_t rb = (size_t)(m * n) * 8;
    auto overlaps = [&](const double* x, size_t bytes) {
        const char *r0 = (const char*)R, *x0 = (const char*)x;
        return r0 < x0 + bytes && x0 < r0 + rb;
    };
    if (overlaps(A, (size_t)(m * p) * 8) || overlaps(X, (size_t)(p * q) * 8) ||
        overlaps(B, (size_t)(q * n) * 8) || overlaps(C, rb))
        return MEK_EINVAL;
    int st;
    if ((st = check_dev(A, (size_t)(m * p) * 8)) || (st = check_dev(X, (size_t)(p * q) * 8)) ||
        (st = check_dev(B, (size_t)(q * n) * 8)) || (st = check_dev(C, rb)) ||
        (st = check_dev(R, rb)))
        return st;
    double* T = nullptr;
    if ((st = noalloc_scratch(&T))) return st;
    hipStream_t s = (hipStream_t)stream;
    // T = A X fills the first m q doubles completely (beta = 0), so nothing
    // has to be cleared between calls.
    MEK_TRY(gemm_f64((int)m, (int)q, (int)p, 1.0, A, p, 1, X, q, 1, 0.0, nullptr, 0, T, q, s));
    MEK_TRY(gemm_f64((int)m, (int)n, (int)q, -1.0, T, q, 1, B, n, 1, 1.0, C, n, R, n, s));
    return MEK_OK;
}

int mek_exchange_floor(int64_t W, int64_t m, int64_t n, int64_t q, int64_t rounds,
                       double* us_per_round, void* stream) {
    if (!us_per_round || W < 1 || m < W || n < 1 || q < 1 || rounds < 1) return MEK_EINVAL;
    if (m > (int64_t)kSelRows * kThreads || n > INT32_MAX / 2 || q > INT32_MAX / 2)
        return MEK_EINVAL;
    int dev = 0, cus = 0;
    MEK_TRY(hipGetDevice(&dev));
    MEK_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    if (W > cus) return MEK_EUNSUPPORTED;
    hipStream_t s = (hipStream_t)stream;
    const size_t words = (size_t)(2 * n + m + q + W) * 8;
    const size_t need = ((words + 255) & ~(size_t)255) + sizeof(TeamSync) + 256;
    char* buf = nullptr;
    MEK_TRY(hipMalloc((void**)&buf, need));
    TeamSync* ts = reinterpret_cast<TeamSync*>(buf + ((words + 255) & ~(size_t)255));
    int* status = reinterpret_cast<int*>(reinterpret_cast<char*>(ts) + sizeof(TeamSync));
    hipEvent_t ev[2] = {nullptr, nullptr};
    hipError_t e = fill_zero_bytes(buf, (long long)need, s);
    if (e == hipSuccess) e = hipEventCreate(&ev[0]);
    if (e == hipSuccess) e = hipEventCreate(&ev[1]);
    if (e == hipSuccess) e = hipEventRecord(ev[0], s);
    if (e == hipSuccess)
        e = exchange_probe((int)W, (int)m, (int)n, (int)q, rounds, buf, ts, status, s);
    if (e == hipSuccess) e = hipEventRecord(ev[1], s);
    int hst = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&hst, status, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev[0], ev[1]);
    for (hipEvent_t x : ev)
        if (x) (void)hipEventDestroy(x);
    (void)hipFree(buf);
    if (e != hipSuccess) return hip_status(e);
    if (hst != MEK_OK) return hst;
    *us_per_round = (double)ms * 1e3 / (double)rounds;
    return MEK_OK;
}

int mek_residual_split(int pieces, int64_t nb, int64_t m, int64_t p, int64_t q, int64_t n,
                       const float* A, const float* X, const float* B, const double* C, float* R,
                       void* stream) {
    if (pieces < 1 || pieces > 3) return MEK_EINVAL;
    if (nb <= 0 || m <= 0 || p <= 0 || q <= 0 || n <= 0) return MEK_EINVAL;
    if (m > INT32_MAX / 2 || p > INT32_MAX / 2 || q > INT32_MAX / 2 || n > INT32_MAX / 2 ||
        nb > INT32_MAX / 2)
        return MEK_EINVAL;
    if (!A || !X || !B || !C || !R) return MEK_EINVAL;
    const size_t rb = (size_t)(nb * m * n) * 4;
    auto overlaps = [&](const void* x, size_t bytes) {
        const char *r0 = (const char*)R, *x0 = (const char*)x;
        return r0 < x0 + bytes && x0 < r0 + rb;
    };
    if (overlaps(A, (size_t)(m * p) * 4) || overlaps(X, (size_t)(nb * p * q) * 4) ||
        overlaps(B, (size_t)(q * n) * 4) || overlaps(C, (size_t)(nb * m * n) * 8))
        return MEK_EINVAL;
    int st;
    if ((st = check_dev(A, (size_t)(m * p) * 4)) || (st = check_dev(X, (size_t)(nb * p * q) * 4)) ||
        (st = check_dev(B, (size_t)(q * n) * 4)) || (st = check_dev(C, (size_t)(nb * m * n) * 8)) ||
        (st = check_dev(R, rb)))
        return st;
    hipStream_t s = (hipStream_t)stream;
    // The temporaries A X_b (nb x m x q floats) live in a per-device buffer
    // kept between calls (grown when a call needs more); calls are
    // serialised on it.
    static std::mutex mtx;
    static float* tbuf[64] = {nullptr};
    static size_t tbytes[64] = {0};
    std::lock_guard<std::mutex> lock(mtx);
    int dev = 0;
    MEK_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return MEK_EUNSUPPORTED;
    const size_t need = (size_t)(nb * m * q) * 4;
    if (tbytes[dev] < need) {
        if (tbuf[dev]) {
            MEK_TRY(hipDeviceSynchronize());
            (void)hipFree(tbuf[dev]);
            tbuf[dev] = nullptr;
            tbytes[dev] = 0;
        }
        MEK_TRY(hipMalloc((void**)&tbuf[dev], need));
        tbytes[dev] = need;
    }
    float* T = tbuf[dev];
    const int b = (int)nb;
    hipError_t e = gemm_bf16s_batched(pieces, b, (int)m, (int)q, (int)p, 1.0, A, p, 1, 0, X, q, 1,
                                      p * q, 0.0, nullptr, 0, 0, T, q, m * q, s);
    if (e == hipSuccess)
        e = gemm_bf16s_batched(pieces, b, (int)m, (int)n, (int)q, -1.0, T, q, 1, m * q, B, n, 1, 0,
                               1.0, C, n, m * n, R, n, m * n, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return hip_status(e);
}

}  // extern "C"

// ---- Warm-start network (cnn.hip). Scratch for the weight-gradient
// partials and the loss partials: a per-device buffer kept between calls
// (grown when needed); calls are serialised on it.
namespace {
std::mutex g_cnn_mtx;
void* g_cnn_buf[64] = {nullptr};
size_t g_cnn_bytes[64] = {0};

int cnn_scratch(size_t need, void** out) {
    int dev = 0;
    MEK_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return MEK_EUNSUPPORTED;
    if (g_cnn_bytes[dev] < need) {
        if (g_cnn_buf[dev]) {
            MEK_TRY(hipDeviceSynchronize());
            (void)hipFree(g_cnn_buf[dev]);
            g_cnn_buf[dev] = nullptr;
            g_cnn_bytes[dev] = 0;
        }
        MEK_TRY(hipMalloc(&g_cnn_buf[dev], need));
        g_cnn_bytes[dev] = need;
    }
    *out = g_cnn_buf[dev];
    return MEK_OK;
}

// The weights of a matrix-core convolution in MFMA order: a per-device
// buffer made on first use (calls are ordered on their stream, so one
// buffer serves every call).
uint16_t* g_cnn_wb[64] = {nullptr};

int cnn_weight_buf(uint16_t** out) {
    int dev = 0;
    MEK_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return MEK_EUNSUPPORTED;
    if (!g_cnn_wb[dev]) MEK_TRY(hipMalloc((void**)&g_cnn_wb[dev], kCnnWeightScratch * 2));
    *out = g_cnn_wb[dev];
    return MEK_OK;
}

bool cnn_dims_ok(int64_t N, int64_t H, int64_t W) {
    return N > 0 && H > 0 && W > 0 && N <= 65535 && H <= (1 << 15) && W <= (1 << 15);
}
}  // namespace

extern "C" {

int mek_cnn_conv3x3(int64_t N, int64_t Cin, int64_t H, int64_t W, int64_t Cout, const uint16_t* x,
                    const float* w, const float* b, int relu, uint16_t* y_bf16, double* y_f64,
                    const double* add_f64, void* stream) {
    if (!cnn_dims_ok(N, H, W) || !cnn_channels_ok(Cin) || !cnn_channels_ok(Cout)) return MEK_EINVAL;
    if (!x || !w || (!y_bf16) == (!y_f64) || (add_f64 && !y_f64)) return MEK_EINVAL;
    const size_t in = (size_t)(N * Cin * H * W), outn = (size_t)(N * Cout * H * W);
    int st;
    if ((st = check_dev(x, in * 2)) || (st = check_dev(w, (size_t)(Cout * Cin * 9) * 4)) ||
        (b && (st = check_dev(b, (size_t)Cout * 4))) ||
        (y_bf16 && (st = check_dev(y_bf16, outn * 2))) || (y_f64 && (st = check_dev(y_f64, outn * 8))) ||
        (add_f64 && (st = check_dev(add_f64, outn * 8))))
        return st;
    hipStream_t s = (hipStream_t)stream;
    std::lock_guard<std::mutex> lock(g_cnn_mtx);
    uint16_t* wb = nullptr;
    if ((st = cnn_weight_buf(&wb))) return st;
    return hip_status(cnn_conv3x3((int)N, (int)Cin, (int)H, (int)W, (int)Cout, x, nullptr, w, b,
                                  relu ? 1 : 0, y_bf16, y_f64, add_f64, wb, s));
}

int mek_cnn_conv3x3_grad_input(int64_t N, int64_t Cout, int64_t H, int64_t W, int64_t Cin,
                               const uint16_t* g, const uint16_t* g_gate, const float* w,
                               uint16_t* gx, void* stream) {
    if (!cnn_dims_ok(N, H, W) || !cnn_channels_ok(Cin) || !cnn_channels_ok(Cout)) return MEK_EINVAL;
    if (!g || !w || !gx) return MEK_EINVAL;
    const size_t gn = (size_t)(N * Cout * H * W), xn = (size_t)(N * Cin * H * W);
    int st;
    if ((st = check_dev(g, gn * 2)) || (g_gate && (st = check_dev(g_gate, gn * 2))) ||
        (st = check_dev(w, (size_t)(Cout * Cin * 9) * 4)) || (st = check_dev(gx, xn * 2)))
        return st;
    hipStream_t s = (hipStream_t)stream;
    std::lock_guard<std::mutex> lock(g_cnn_mtx);
    uint16_t* wb = nullptr;
    if ((st = cnn_weight_buf(&wb))) return st;
    return hip_status(cnn_conv3x3_grad_input((int)N, (int)Cout, (int)H, (int)W, (int)Cin, g, g_gate,
                                             w, gx, wb, s));
}

int mek_cnn_conv3x3_grad_weight(int64_t N, int64_t Cin, int64_t H, int64_t W, int64_t Cout,
                                const uint16_t* x, const uint16_t* g, const uint16_t* g_gate,
                                float* dw, float* db, void* stream) {
    if (!cnn_dims_ok(N, H, W) || !cnn_channels_ok(Cin) || !cnn_channels_ok(Cout)) return MEK_EINVAL;
    if (!x || !g || !dw || !db) return MEK_EINVAL;
    const size_t gn = (size_t)(N * Cout * H * W), xn = (size_t)(N * Cin * H * W);
    int st;
    if ((st = check_dev(x, xn * 2)) || (st = check_dev(g, gn * 2)) ||
        (g_gate && (st = check_dev(g_gate, gn * 2))) ||
        (st = check_dev(dw, (size_t)(Cout * Cin * 9) * 4)) || (st = check_dev(db, (size_t)Cout * 4)))
        return st;
    hipStream_t s = (hipStream_t)stream;
    std::lock_guard<std::mutex> lock(g_cnn_mtx);
    void* part = nullptr;
    if ((st = cnn_scratch(cnn_wgrad_partial_floats((int)N, (int)Cin, (int)H, (int)W, (int)Cout) * 4,
                          &part)))
        return st;
    return hip_status(cnn_conv3x3_grad_weight((int)N, (int)Cin, (int)H, (int)W, (int)Cout, x, g,
                                              g_gate, (float*)part, dw, db, s));
}

int mek_cnn_mse_grad(int64_t len, const double* y, const double* label, uint16_t* g, double* loss,
                     void* stream) {
    if (len <= 0 || !y || !label || !loss) return MEK_EINVAL;
    int st;
    if ((st = check_dev(y, (size_t)len * 8)) || (st = check_dev(label, (size_t)len * 8)) ||
        (g && (st = check_dev(g, (size_t)len * 2))))
        return st;
    hipStream_t s = (hipStream_t)stream;
    std::lock_guard<std::mutex> lock(g_cnn_mtx);
    constexpr int kBlocks = 256;
    void* buf = nullptr;
    if ((st = cnn_scratch((kBlocks + 256 + 8) * 8, &buf))) return st;
    double* part = (double*)buf;
    double* scratch = part + kBlocks;
    double* out = scratch + 256;
    hipError_t e = cnn_mse_grad(len, y, label, 2.0 / (double)len, g, part, kBlocks, s);
    if (e == hipSuccess) e = sum_reduce(part, kBlocks, out, scratch, s);
    double h = 0.0;
    if (e == hipSuccess) e = hipMemcpyAsync(&h, out, 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess) *loss = h / (double)len;
    return hip_status(e);
}

int mek_cnn_adam(int64_t n, float* w, float* wq, const float* g, float* m, float* v, double lr,
                 double beta1, double beta2, double eps, int64_t t, void* stream) {
    if (n <= 0 || !w || !wq || !g || !m || !v || t < 1) return MEK_EINVAL;
    if (!(lr > 0.0) || !(beta1 >= 0.0 && beta1 < 1.0) || !(beta2 >= 0.0 && beta2 < 1.0) || !(eps > 0.0))
        return MEK_EINVAL;
    int st;
    const size_t b = (size_t)n * 4;
    if ((st = check_dev(w, b)) || (st = check_dev(wq, b)) || (st = check_dev(g, b)) ||
        (st = check_dev(m, b)) || (st = check_dev(v, b)))
        return st;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = cnn_adam(n, w, wq, g, m, v, (float)lr, (float)beta1, (float)beta2, (float)eps,
                            (int)std::min<int64_t>(t, INT32_MAX), s);
    return hip_status(e);
}

int mek_cnn_to_bf16(int64_t n, const double* x, double scale, uint16_t* y, void* stream) {
    if (n <= 0 || !x || !y) return MEK_EINVAL;
    int st;
    if ((st = check_dev(x, (size_t)n * 8)) || (st = check_dev(y, (size_t)n * 2))) return st;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = cnn_to_bf16(n, x, scale, y, s);
    return hip_status(e);
}

int mek_cnn_round_bf16(int64_t n, const float* x, float* y, void* stream) {
    if (n <= 0 || !x || !y) return MEK_EINVAL;
    int st;
    if ((st = check_dev(x, (size_t)n * 4)) || (st = check_dev(y, (size_t)n * 4))) return st;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = cnn_round_bf16(n, x, y, s);
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
