// Device-side building blocks shared by the gfx950 kernels: wave/block
// reductions and scans, the cross-work-group team barrier, and the
// Philox4x64-10 counter-based generator.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mek {

// Blocks of a tiled product are dealt to the 8 XCDs round-robin by linear
// id. Give each XCD a contiguous range of a grouped tile order (G tile rows,
// column by column) so that the tiles sharing one L2 touch few distinct
// panels of the two operands. Block b of a tm x tn tile grid -> (ti, tj).
__device__ __forceinline__ void tile_coords(int b, int tm, int tn, int& ti, int& tj) {
    constexpr int G = 4;
    const int nt = tm * tn;
    const int xcd = b & 7, local = b >> 3, base = nt >> 3, rem = nt & 7;
    const int lin = xcd < rem ? xcd * (base + 1) + local
                              : rem * (base + 1) + (xcd - rem) * base + local;
    const int group = lin / (G * tn), first = group * G;
    const int rows = min(G, tm - first), within = lin - group * G * tn;
    ti = first + within % rows;
    tj = within / rows;
}

constexpr int kWave = 64;         // CDNA wavefront width
constexpr int kThreads = 512;     // threads per work-group of the solver
constexpr int kWaves = kThreads / kWave;
constexpr int kSelRows = 16;      // rows of the selection chunk per thread (m <= 8192)
constexpr int kDotUnroll = 16;    // loads in flight per lane in a dot-product task
constexpr int kDotSeg = kDotUnroll * kWave;   // entries per dot-product task
constexpr int kVecRegs = 8;       // n-vector entries per thread held in registers
constexpr int kUTable = 128;      // Philox draws computed ahead, per refill

// LDS doubles for dot-product partial sums: the larger of the two dot
// batches of an update (xpw dots over n entries, wpw dots over q entries),
// plus n more for w when the team is a single work-group (`single`).
__host__ __device__ inline int dot_parts(int xpw, int n, int wpw, int q, bool single) {
    const int seg = kDotUnroll * kWave;
    const int a = xpw * ((n + seg - 1) / seg), b = wpw * ((q + seg - 1) / seg);
    return (a > b ? a : b) + (single ? n : 0);
}

constexpr int kAPre = 8;          // entries of A_{i_k} per lane loaded ahead of the X update
constexpr int kRowBatch = 8;      // loads in flight per lane when rows of R sit in device memory

// ---------------------------------------------------------------------------
// Wave-level reductions and scans on DPP row permutations (register-level
// lane exchange, no LDS round trip). A 64-lane wave is four rows of 16
// lanes: four DPP steps (swap neighbours, swap pairs, mirror within 8,
// mirror within 16) leave every lane of a row holding the row's total, and
// the four row totals are then combined in a fixed order. Every lane gets
// the same bits, and the order of the additions is fixed, so equal inputs
// give equal results in every wave and work-group.
// ---------------------------------------------------------------------------
constexpr int kDppSwap1 = 0xB1;        // quad_perm [1,0,3,2]
constexpr int kDppSwap2 = 0x4E;        // quad_perm [2,3,0,1]
constexpr int kDppHalfMirror = 0x141;  // row_half_mirror
constexpr int kDppMirror = 0x140;      // row_mirror
constexpr int kDppShr = 0x110;         // row_shr:n is kDppShr + n

template <int CTRL>
__device__ __forceinline__ int dpp_i(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, true);
}
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
    const int lo = dpp_i<CTRL>(__double2loint(v));
    const int hi = dpp_i<CTRL>(__double2hiint(v));
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double readlane_d(double v, int lane) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double wave_sum(double v) {
    v += dpp_d<kDppSwap1>(v);
    v += dpp_d<kDppSwap2>(v);
    v += dpp_d<kDppHalfMirror>(v);
    v += dpp_d<kDppMirror>(v);
    return ((readlane_d(v, 0) + readlane_d(v, 16)) + readlane_d(v, 32)) + readlane_d(v, 48);
}
__device__ __forceinline__ double wave_max(double v) {
    v = fmax(v, dpp_d<kDppSwap1>(v));
    v = fmax(v, dpp_d<kDppSwap2>(v));
    v = fmax(v, dpp_d<kDppHalfMirror>(v));
    v = fmax(v, dpp_d<kDppMirror>(v));
    return fmax(fmax(readlane_d(v, 0), readlane_d(v, 16)), fmax(readlane_d(v, 32), readlane_d(v, 48)));
}
__device__ __forceinline__ int wave_min_int(int v) {
    v = min(v, dpp_i<kDppSwap1>(v));
    v = min(v, dpp_i<kDppSwap2>(v));
    v = min(v, dpp_i<kDppHalfMirror>(v));
    v = min(v, dpp_i<kDppMirror>(v));
    return min(min(__builtin_amdgcn_readlane(v, 0), __builtin_amdgcn_readlane(v, 16)),
               min(__builtin_amdgcn_readlane(v, 32), __builtin_amdgcn_readlane(v, 48)));
}
__device__ __forceinline__ int wave_max_int(int v) {
    v = max(v, dpp_i<kDppSwap1>(v));
    v = max(v, dpp_i<kDppSwap2>(v));
    v = max(v, dpp_i<kDppHalfMirror>(v));
    v = max(v, dpp_i<kDppMirror>(v));
    return max(max(__builtin_amdgcn_readlane(v, 0), __builtin_amdgcn_readlane(v, 16)),
               max(__builtin_amdgcn_readlane(v, 32), __builtin_amdgcn_readlane(v, 48)));
}

// Inclusive scan over the 64 lanes: Hillis-Steele within each row of 16
// (row_shr 1, 2, 4, 8; lanes with no source add zero), then each row adds
// the totals of the rows before it.
__device__ __forceinline__ double wave_incl_scan(double v) {
    v += dpp_d<kDppShr + 1>(v);
    v += dpp_d<kDppShr + 2>(v);
    v += dpp_d<kDppShr + 4>(v);
    v += dpp_d<kDppShr + 8>(v);
    const double t0 = readlane_d(v, 15), t1 = readlane_d(v, 31), t2 = readlane_d(v, 47);
    const int row = (threadIdx.x & (kWave - 1)) >> 4;
    const double t01 = t0 + t1;
    const double off = row == 0 ? 0.0 : row == 1 ? t0 : row == 2 ? t01 : t01 + t2;
    return row == 0 ? v : v + off;
}
__device__ __forceinline__ int wave_incl_scan_int(int v) {
    v += dpp_i<kDppShr + 1>(v);
    v += dpp_i<kDppShr + 2>(v);
    v += dpp_i<kDppShr + 4>(v);
    v += dpp_i<kDppShr + 8>(v);
    const int t0 = __builtin_amdgcn_readlane(v, 15), t1 = __builtin_amdgcn_readlane(v, 31),
              t2 = __builtin_amdgcn_readlane(v, 47);
    const int row = (threadIdx.x & (kWave - 1)) >> 4;
    return v + (row == 0 ? 0 : row == 1 ? t0 : row == 2 ? t0 + t1 : t0 + t1 + t2);
}

// Shared scratch used by the block-level collectives below. One instance per
// work-group (declared __shared__ by each kernel that uses the helpers).
struct BlockScratch {
    double d[kWaves][8];
    int i[kWaves][4];
    double out_d[8];
    int out_i[4];
};

// Sum of NV values per thread over the block; every thread receives the
// totals. Waves reduce on DPP, then every thread adds the wave totals in
// wave order from LDS, so identical inputs give bit-identical results in
// every work-group.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], BlockScratch& s) {
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
#pragma unroll
    for (int j = 0; j < NV; ++j) v[j] = wave_sum(v[j]);
    if (lane == 0) {
#pragma unroll
        for (int j = 0; j < NV; ++j) s.d[wv][j] = v[j];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < NV; ++j) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) t += s.d[w][j];
        v[j] = t;
    }
    __syncthreads();
}

// Sum (a, b) and max (mx) in one pass.
__device__ __forceinline__ void block_sum_max_sum(double& a, double& mx, double& b,
                                                  BlockScratch& s) {
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    a = wave_sum(a);
    mx = wave_max(mx);
    b = wave_sum(b);
    if (lane == 0) {
        s.d[wv][0] = a;
        s.d[wv][1] = mx;
        s.d[wv][2] = b;
    }
    __syncthreads();
    double ta = 0.0, tm = s.d[0][1], tb = 0.0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
        ta += s.d[w][0];
        tm = fmax(tm, s.d[w][1]);
        tb += s.d[w][2];
    }
    a = ta;
    mx = tm;
    b = tb;
    __syncthreads();
}

__device__ __forceinline__ void block_min_max_int(int& mn, int& mx, BlockScratch& s) {
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    mn = wave_min_int(mn);
    mx = wave_max_int(mx);
    if (lane == 0) {
        s.i[wv][0] = mn;
        s.i[wv][1] = mx;
    }
    __syncthreads();
    int a = s.i[0][0], b = s.i[0][1];
#pragma unroll
    for (int w = 1; w < kWaves; ++w) {
        a = min(a, s.i[w][0]);
        b = max(b, s.i[w][1]);
    }
    mn = a;
    mx = b;
    __syncthreads();
}

// Exclusive scan of one double and one int per thread (thread order).
// Returns the exclusive prefixes and the block totals. Each thread adds the
// totals of the waves before its own in wave order.
__device__ __forceinline__ void block_excl_scan(double v, int c, double& pre_v, int& pre_c,
                                                double& tot_v, int& tot_c, BlockScratch& s) {
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    const double iv = wave_incl_scan(v);
    const int ic = wave_incl_scan_int(c);
    if (lane == kWave - 1) {
        s.d[wv][3] = iv;
        s.i[wv][2] = ic;
    }
    __syncthreads();
    double off = 0.0, tot = 0.0;
    int offc = 0, totc = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
        const double t = s.d[w][3];
        const int tc = s.i[w][2];
        if (w < wv) {
            off += t;
            offc += tc;
        }
        tot += t;
        totc += tc;
    }
    pre_v = off + (iv - v);
    pre_c = offc + (ic - c);
    tot_v = tot;
    tot_c = totc;
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon et al., SC'11): four 64-bit counter words, two key
// words, ten rounds of the multiply/xor S-box with a Weyl key schedule.
// ---------------------------------------------------------------------------
struct U64x4 {
    uint64_t w[4];
};

__device__ __forceinline__ U64x4 philox4x64_10(U64x4 c, uint64_t k0, uint64_t k1) {
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0_hi = __umul64hi(M0, c.w[0]), p0_lo = M0 * c.w[0];
        const uint64_t p1_hi = __umul64hi(M1, c.w[2]), p1_lo = M1 * c.w[2];
        U64x4 o;
        o.w[0] = p1_hi ^ c.w[1] ^ k0;
        o.w[1] = p1_lo;
        o.w[2] = p0_hi ^ c.w[3] ^ k1;
        o.w[3] = p0_lo;
        c = o;
        k0 += W0;
        k1 += W1;
    }
    return c;
}

// The uniform in [0, 1) drawn for update k (counter (k+1, 0, 0, 0)).
__device__ __forceinline__ double philox_uniform(uint64_t seed, uint64_t inst, int64_t k) {
    U64x4 c;
    c.w[0] = (uint64_t)k + 1ull;
    c.w[1] = 0;
    c.w[2] = 0;
    c.w[3] = 0;
    U64x4 o = philox4x64_10(c, seed, inst);
    return (double)(o.w[0] >> 11) * 0x1.0p-53;
}

// ---------------------------------------------------------------------------
// Team synchronisation. A team is a set of W co-resident work-groups (one
// cooperative launch) that solve one instance together. All counters only
// grow; targets are compared with wrap-safe signed differences.
// ---------------------------------------------------------------------------
constexpr int kMaxTeam = 512;     // work-groups per team (one arrival slot each)

struct alignas(256) TeamSync {
    unsigned int arrive[kMaxTeam];   // arrive[g] = barriers work-group g has reached
    unsigned int flag;               // "row of update k published" = k + 1
    unsigned int pad1[63];
    int abort;                       // set when any wait times out
    unsigned int pad2[63];
};

constexpr long long kSpinLimit = 1ll << 24;   // polls before a wait gives up

__device__ __forceinline__ unsigned int sync_load(const unsigned int* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wait until *p reaches `target` (wrap-safe), polling with short sleeps; the
// abort flag and the spin limit are checked every 64 polls. Thread 0 only.
__device__ __forceinline__ int spin_until(TeamSync* ts, const unsigned int* p,
                                          unsigned int target) {
    long long spins = 0;
    while ((int)(sync_load(p) - target) < 0) {
        if ((++spins & 63) == 0 &&
            (spins > kSpinLimit ||
             __hip_atomic_load(&ts->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) {
            __hip_atomic_store(&ts->abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return 0;
        }
        __builtin_amdgcn_s_sleep(1);
    }
    return 1;
}

// Barrier over the W work-groups of a team. Every thread first waits for
// its own outstanding memory operations (so exchange stores are complete);
// work-group g then records its arrival in its own slot, and thread t < W
// of every work-group waits for slot t, so no two work-groups contend for
// one address. `epoch` counts the barriers passed (identical in all
// work-groups). *s_fail is set (never cleared) if a wait gives up.
__device__ __forceinline__ bool team_barrier(TeamSync* ts, unsigned int& epoch, unsigned int W,
                                             int* s_fail) {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    ++epoch;
    if (threadIdx.x == 0)
        __hip_atomic_store(&ts->arrive[blockIdx.x], epoch, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    if (threadIdx.x < W && !spin_until(ts, &ts->arrive[threadIdx.x], epoch)) *s_fail = 1;
    __syncthreads();
    return *s_fail == 0;
}

// One work-group publishes (flag = value) after its exchange stores; the
// others wait for it.
__device__ __forceinline__ void team_flag_set(TeamSync* ts, unsigned int value) {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0)
        __hip_atomic_store(&ts->flag, value, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ bool team_flag_wait(TeamSync* ts, unsigned int value, int* s_fail) {
    if (threadIdx.x == 0 && !spin_until(ts, &ts->flag, value)) *s_fail = 1;
    __syncthreads();
    return *s_fail == 0;
}

}  // namespace mek
