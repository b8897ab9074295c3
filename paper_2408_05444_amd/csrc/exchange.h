// Cross-work-group exchange of the persistent solvers: tagged 64-bit words
// written and polled with agent-scope relaxed atomics.
#pragma once

#include "device_common.h"

namespace mek {

// ---------------------------------------------------------------------------
// Cross-work-group exchange. The few values that work-groups hand to each
// other every update are written and read with relaxed agent-scope atomics,
// which the compiler turns into plain stores/loads that go to the
// device-wide coherence point (cache policy sc1). No L2 write-back or
// invalidate is needed, so read-only operands (A, B, A A^T, B^T B, the row
// and column norms) stay cached in L2.
// ---------------------------------------------------------------------------
template <typename U>
__device__ __forceinline__ U xload(const U* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename U>
__device__ __forceinline__ void xstore(U* p, U v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------------------
// Tagged exchange words. Work-groups of a team hand each other a few kinds of
// values every update (in the row solver: row norms r_i, error partials, the
// selected row R_{i_k} and the slices of w). Each value travels in one 64-bit
// word that
// also carries a 2-bit sequence tag, so a reader polls the data itself
// until the tags show the current update: the signal and the data arrive
// together, and no team-wide barrier is needed. A double keeps the tag in its
// two lowest mantissa bits (a change of at most 3 units in the last place,
// the size of one rounding; an exact zero stays zero); a float keeps its 32
// bits and the tag sits in the upper half of the word. Words are written
// and read with agent-scope relaxed atomics (aligned 64-bit, so a reader
// never sees half of a word).
//
// One buffer per kind suffices when every rewrite of a word is causally after
// every work-group has read its previous contents (row solver: the next r
// needs every slice of w, a work-group publishes its slice of w only after
// its own selection has read every r and it has the published row, and the
// next row needs every r), so a reader waiting for tag t can only see tag t
// or the tag of the update before.
// ---------------------------------------------------------------------------
typedef unsigned long long xword;

__device__ __forceinline__ unsigned int seq_tag(long long k) { return (unsigned int)((k + 1) & 3); }

__device__ __forceinline__ xword pack_word(double v, unsigned int tag) {
    return ((xword)__double_as_longlong(v) & ~3ull) | tag;
}
__device__ __forceinline__ xword pack_word(float v, unsigned int tag) {
    return ((xword)tag << 32) | (xword)__float_as_uint(v);
}
template <typename T> __device__ __forceinline__ T word_value(xword w);
template <> __device__ __forceinline__ double word_value<double>(xword w) {
    return ((w & 0x7FFFFFFFFFFFFFFCull) == 0) ? 0.0 : __longlong_as_double((long long)w);
}
template <> __device__ __forceinline__ float word_value<float>(xword w) {
    return __uint_as_float((unsigned int)w);
}
template <typename T> __device__ __forceinline__ unsigned int word_tag(xword w);
template <> __device__ __forceinline__ unsigned int word_tag<double>(xword w) {
    return (unsigned int)(w & 3);
}
template <> __device__ __forceinline__ unsigned int word_tag<float>(xword w) {
    return (unsigned int)(w >> 32) & 3;
}

// Pause between two polls: s_sleep takes an immediate, so the few allowed
// lengths are dispatched on a (wave-uniform) runtime value.
__device__ __forceinline__ void poll_pause(int sleep) {
    switch (sleep) {
        case 0: break;
        case 2: __builtin_amdgcn_s_sleep(2); break;
        case 4: __builtin_amdgcn_s_sleep(4); break;
        case 8: __builtin_amdgcn_s_sleep(8); break;
        case 16: __builtin_amdgcn_s_sleep(16); break;
        default: __builtin_amdgcn_s_sleep(1); break;
    }
}

// Read cnt (<= N) words p[0..cnt) until every one carries `tag`. Returns
// false if the wait gives up (spin limit, or another work-group aborted).
template <typename T, int N>
__device__ __forceinline__ bool poll_words(const xword* p, int cnt, unsigned int tag, T (&out)[N],
                                           TeamSync* ts, int sleep) {
    long long spins = 0;
    for (;;) {
        xword w[N];
#pragma unroll
        for (int j = 0; j < N; ++j) w[j] = (j < cnt) ? xload(p + j) : 0ull;
        bool ready = true;
#pragma unroll
        for (int j = 0; j < N; ++j) {
            if (j < cnt) {
                ready = ready && (word_tag<T>(w[j]) == tag);
                out[j] = word_value<T>(w[j]);
            }
        }
        if (ready) return true;
        if ((++spins & 63) == 0 &&
            (spins > kSpinLimit ||
             __hip_atomic_load(&ts->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) {
            __hip_atomic_store(&ts->abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
        poll_pause(sleep);
    }
}

// Strided variant: words p[j * stride] for j < cnt.
template <typename T, int N>
__device__ __forceinline__ bool poll_strided(const xword* p, int stride, int cnt, unsigned int tag,
                                             T (&out)[N], TeamSync* ts, int sleep) {
    long long spins = 0;
    for (;;) {
        xword w[N];
#pragma unroll
        for (int j = 0; j < N; ++j) w[j] = (j < cnt) ? xload(p + (size_t)j * stride) : 0ull;
        bool ready = true;
#pragma unroll
        for (int j = 0; j < N; ++j) {
            if (j < cnt) {
                ready = ready && (word_tag<T>(w[j]) == tag);
                out[j] = word_value<T>(w[j]);
            }
        }
        if (ready) return true;
        if ((++spins & 63) == 0 &&
            (spins > kSpinLimit ||
             __hip_atomic_load(&ts->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) {
            __hip_atomic_store(&ts->abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
        poll_pause(sleep);
    }
}

// Gather variant: words *ptr[j] for j < cnt.
template <typename T, int N>
__device__ __forceinline__ bool poll_gather(const xword* const (&ptr)[N], int cnt,
                                            unsigned int tag, T (&out)[N], TeamSync* ts,
                                            int sleep) {
    long long spins = 0;
    for (;;) {
        xword w[N];
#pragma unroll
        for (int j = 0; j < N; ++j) w[j] = (j < cnt) ? xload(ptr[j]) : 0ull;
        bool ready = true;
#pragma unroll
        for (int j = 0; j < N; ++j) {
            if (j < cnt) {
                ready = ready && (word_tag<T>(w[j]) == tag);
                out[j] = word_value<T>(w[j]);
            }
        }
        if (ready) return true;
        if ((++spins & 63) == 0 &&
            (spins > kSpinLimit ||
             __hip_atomic_load(&ts->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) {
            __hip_atomic_store(&ts->abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
        poll_pause(sleep);
    }
}

}  // namespace mek
