// Communication floor of the team solver: the exchanges and block
// collectives of one update with none of its arithmetic, repeated for a
// number of rounds. Per round, as in an update of the team kernel:
//   1. every thread polls its chunk of the m row-norm words and threads
//      t < W poll the W error words; a block sum/max and an exclusive scan
//      stand for the reduction and the selection's collectives;
//   2. the owner of the round's row (work-group k mod W) publishes n words,
//      every work-group polls them;
//   3. every work-group publishes its ceil(q / W) words of v, polls all q;
//   4. every work-group publishes its ceil(n / W) words of w, polls all n;
//   5. every wave publishes its rows' norm words, thread 0 the error word,
//      with the next round's tag.
// Words carry the same 2-bit sequence tags and use the same relaxed
// agent-scope loads and stores as the solver. The time per round is the
// floor that the exchanges alone put under an update at that team shape.
#include "exchange.h"
#include "internal.h"

namespace mek {

namespace {

constexpr int kProbeSR = 16;

struct ProbeParams {
    int W, m, n, q, rpw, xpw, wpw;
    long long rounds;
    xword *r, *e, *row, *v, *w;
    TeamSync* sync;
    int* status;
};

__global__ void __launch_bounds__(kThreads, 1) exchange_probe_kernel(ProbeParams P) {
    __shared__ BlockScratch sc;
    __shared__ int s_fail;
    if (threadIdx.x == 0) s_fail = 0;
    const int g = blockIdx.x, tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
    const int m = P.m, n = P.n, q = P.q, W = P.W;
    const int row0 = g * P.rpw, nrow = max(0, min(P.rpw, m - row0));
    const int nx = max(0, min(P.xpw, q - g * P.xpw)), nw = max(0, min(P.wpw, n - g * P.wpw));
    const int cs = (m + kThreads - 1) / kThreads;
    const int sb = min(m, tid * cs), scnt = min(m, sb + cs) - sb;
    // Round 0's norm and error words.
    for (int ii = wv; ii < nrow; ii += kWaves)
        if (lane == 0) xstore(&P.r[row0 + ii], pack_word(0.0, seq_tag(0)));
    if (tid == 0) xstore(&P.e[g], pack_word(0.0, seq_tag(0)));
    __syncthreads();
    for (long long k = 0; k < P.rounds; ++k) {
        const unsigned int tag = seq_tag(k), ntag = seq_tag(k + 1);
        double rr[kProbeSR];
        if (!poll_words<double, kProbeSR>(P.r + sb, scnt, tag, rr, P.sync, 1)) s_fail = 1;
        double e1[1] = {0.0};
        if (tid < W && !poll_words<double, 1>(P.e + tid, 1, tag, e1, P.sync, 1)) s_fail = 1;
        double a = 0.0, mx = -1.0, b = e1[0];
        for (int j = 0; j < kProbeSR; ++j)
            if (j < scnt) a += rr[j];
        block_sum_max_sum(a, mx, b, sc);
        double pre_v, tot_v;
        int pre_c, tot_c;
        block_excl_scan(a, scnt, pre_v, pre_c, tot_v, tot_c, sc);
        __syncthreads();
        if (s_fail) break;
        // 2. The row.
        if ((int)(k % W) == g)
            for (int j = tid; j < n; j += kThreads) xstore(&P.row[j], pack_word(0.0, tag));
        for (int j0 = 0; j0 < n; j0 += kThreads * kVecRegs) {
            double t[kVecRegs];
            const int cnt = max(0, min(kVecRegs, (n - j0 - tid + kThreads - 1) / kThreads));
            if (!poll_strided<double, kVecRegs>(P.row + j0 + tid, kThreads, cnt, tag, t, P.sync, 1))
                s_fail = 1;
        }
        __syncthreads();
        // 3. v.
        if (tid < nx) xstore(&P.v[g * P.xpw + tid], pack_word(0.0, tag));
        for (int l0 = 0; l0 < q; l0 += kThreads * kVecRegs) {
            double t[kVecRegs];
            const int cnt = max(0, min(kVecRegs, (q - l0 - tid + kThreads - 1) / kThreads));
            if (!poll_strided<double, kVecRegs>(P.v + l0 + tid, kThreads, cnt, tag, t, P.sync, 1))
                s_fail = 1;
        }
        __syncthreads();
        // 4. w.
        if (tid < nw) xstore(&P.w[g * P.wpw + tid], pack_word(0.0, tag));
        for (int j0 = 0; j0 < n; j0 += kThreads * kVecRegs) {
            double t[kVecRegs];
            const int cnt = max(0, min(kVecRegs, (n - j0 - tid + kThreads - 1) / kThreads));
            if (!poll_strided<double, kVecRegs>(P.w + j0 + tid, kThreads, cnt, tag, t, P.sync, 1))
                s_fail = 1;
        }
        __syncthreads();
        if (s_fail) break;
        // 5. Next round's norms and error word.
        for (int ii = wv; ii < nrow; ii += kWaves)
            if (lane == 0) xstore(&P.r[row0 + ii], pack_word(0.0, ntag));
        if (tid == 0) xstore(&P.e[g], pack_word(0.0, ntag));
        __syncthreads();
    }
    if (g == 0 && tid == 0) *P.status = s_fail ? kETimeout : kOK;
}

}  // namespace

hipError_t exchange_probe(int W, int m, int n, int q, long long rounds, void* words,
                          TeamSync* sync, int* status, hipStream_t s) {
    ProbeParams P;
    P.W = W;
    P.m = m;
    P.n = n;
    P.q = q;
    P.rpw = (m + W - 1) / W;
    P.xpw = (q + W - 1) / W;
    P.wpw = (n + W - 1) / W;
    P.rounds = rounds;
    xword* x = reinterpret_cast<xword*>(words);
    P.r = x;
    P.e = P.r + m;
    P.row = P.e + W;
    P.v = P.row + n;
    P.w = P.v + q;
    P.sync = sync;
    P.status = status;
    void* args[] = {&P};
    return hipLaunchCooperativeKernel((const void*)exchange_probe_kernel, dim3(W), dim3(kThreads),
                                      args, 0, s);
}

}  // namespace mek
