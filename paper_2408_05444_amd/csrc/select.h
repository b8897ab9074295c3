// The selection step of Algs. 1-5 for one work-group that holds every row
// norm of its instance (shared by the persistent solver kernels).
#pragma once

#include <limits.h>

#include "device_common.h"
#include "internal.h"

namespace mek {

struct SelectOut {
    int idx;
    int setsize;
    double t;
    double T;
};

// Inverse-CDF draw over a row set held in registers (thread t owns the rows
// [b, b + cnt)). GREEDY: the set is {i : a_i > 0, r_i / a_i >= t} with
// weights r_i (Algs. 3/4); otherwise every row with a_i > 0, weight a_i
// (Alg. 1). A block-wide exclusive scan of the chunk sums and counts gives
// each chunk its starting prefix and each member its position in the
// compacted set. The chosen row is the first whose running sum exceeds
// u * T (T the set's total weight), else the set's last row.
template <bool GREEDY, int SR>
__device__ __forceinline__ SelectOut sample_set(int b, int cnt, const double (&rr)[SR],
                                                const double (&aa)[SR], const double (&rho)[SR],
                                                double t, double u, BlockScratch& sc,
                                                int32_t* set_list, uint8_t* in_set) {
    unsigned int mask = 0;
    double ws = 0.0;
    int c = 0, lastm = -1;
#pragma unroll
    for (int j = 0; j < SR; ++j) {
        const bool mem = j < cnt && aa[j] > 0.0 && (!GREEDY || rho[j] >= t);
        if (mem) {
            mask |= 1u << j;
            ws += rr[j];
            ++c;
            lastm = b + j;
        }
    }
    if (threadIdx.x == 0) {
        sc.out_i[2] = INT_MAX;   // first crossing row
        sc.out_i[3] = -1;        // last row of the set
    }
    double pre_w, T;
    int pre_c, tot_c;
    block_excl_scan(ws, c, pre_w, pre_c, T, tot_c, sc);
    const double target = u * T;
    int cand = INT_MAX;
    double run = pre_w;
    int pos = pre_c;
#pragma unroll
    for (int j = 0; j < SR; ++j) {
        if ((mask >> j) & 1u) {
            if (set_list) set_list[pos] = b + j;
            if (in_set) in_set[b + j] = 1;
            ++pos;
            run += rr[j];
            if (cand == INT_MAX && run > target) cand = b + j;
        }
    }
    // First crossing and last member: wave min / max on DPP, then one LDS
    // atomic per wave (integer min / max do not depend on arrival order).
    cand = wave_min_int(cand);
    lastm = wave_max_int(lastm);
    if ((threadIdx.x & (kWave - 1)) == 0) {
        if (cand != INT_MAX) atomicMin(&sc.out_i[2], cand);
        if (lastm >= 0) atomicMax(&sc.out_i[3], lastm);
    }
    __syncthreads();
    SelectOut o;
    o.idx = (sc.out_i[2] != INT_MAX) ? sc.out_i[2] : sc.out_i[3];
    o.setsize = tot_c;
    o.t = t;
    o.T = T;
    __syncthreads();
    return o;
}

// The selection step of update k for Algs. 1-5, run by one whole work-group.
// Thread t holds rows [b, b + cnt) (cnt <= SR, contiguous chunks in
// thread order) with rr[j] = ||R_i||^2 and aa[j] = ||A_i||^2 in registers.
// S = sum of all r, M = max over rows with a_i > 0 of r_i / a_i; the greedy
// threshold is t = min(M, theta M + (1 - theta) S / F_A).
template <int SR>
__device__ __forceinline__ SelectOut select_rows(int variant, int b, int cnt,
                                                 const double (&rr)[SR], const double (&aa)[SR],
                                                 const double (&rho)[SR], double S, double M,
                                                 double F_A, double theta, double u, long long k,
                                                 const int* __restrict__ active, int n_active,
                                                 BlockScratch& sc, int32_t* set_list,
                                                 uint8_t* in_set) {
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
#pragma unroll
        for (int j = 0; j < SR; ++j)
            if (j < cnt && aa[j] > 0.0 && rho[j] == M) cand = min(cand, b + j);
        if (threadIdx.x == 0) sc.out_i[2] = INT_MAX;
        cand = wave_min_int(cand);
        __syncthreads();
        if ((threadIdx.x & (kWave - 1)) == 0 && cand != INT_MAX) atomicMin(&sc.out_i[2], cand);
        __syncthreads();
        o.idx = sc.out_i[2];
        __syncthreads();
        o.setsize = 1;
        o.t = M;
        if (threadIdx.x == 0) {
            if (in_set) in_set[o.idx] = 1;
            if (set_list) set_list[0] = o.idx;
        }
        return o;
    }
    if (variant == kGRBK || variant == kRGRBK) {
        // Evaluated as written (no fused multiply-add): each operation is
        // rounded in turn, as in a plain evaluation of the formula.
#pragma clang fp contract(off)
        const double th = (variant == kGRBK) ? 0.5 : theta;
        double t = th * M + (1.0 - th) * (S / F_A);
        if (t > M) t = M;
        return sample_set<true, SR>(b, cnt, rr, aa, rho, t, u, sc, set_list, in_set);
    }
    return sample_set<false, SR>(b, cnt, aa, aa, rho, 0.0, u, sc, set_list, in_set);
}

}  // namespace mek
