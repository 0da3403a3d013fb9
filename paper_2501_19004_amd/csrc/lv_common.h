// lv_common.h -- shared device helpers and data structures of the gfx950
// Louvain library (local-moving and aggregation phases).
//
// Integer conventions: vertex and community ids are int32; weighted degrees
// K, community totals Sigma and super-graph weights are int64; modularity
// gains (Eq. (2) of the paper, multiplied by W^2/2) are int64 when
// W * max(K) < 2^62 and __int128 otherwise; per-iteration gain sums are
// 128-bit.  Floating point appears only in the optional learned pruner
// (lv_learn.hip), whose FP32 keep decisions follow a fixed operation order.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace lv {

constexpr int WAVE = 64;
constexpr int32_t EMPTY_KEY = 0x7fffffff;  // hash-table empty slot; sorts after every id
constexpr int MAX_BUCKETS = 8;

typedef unsigned long long u64;
typedef long long i64;
typedef __int128 i128;

// Device control block: counters written by kernels and read back by the host.
// Hot counters are striped over STRIPES slots (a block uses slot
// blockIdx % STRIPES) so that thousands of blocks do not serialise on one
// address; the host adds the stripes.
constexpr int STRIPES = 32;
struct Ctl {
    // ---- zeroed before every local-moving iteration
    int32_t qcount[MAX_BUCKETS];  // next-iteration queue sizes, per move bucket
    int32_t pad0[2];
    // sums of applied gains, split so that every part is added without a
    // returning atomic: gain = hi * 2^64 + mid * 2^32 + lo with lo, mid in
    // [0, 2^32); the host adds the parts modulo 2^128
    u64 s_lo[STRIPES];
    u64 s_mid[STRIPES];
    u64 s_hi[STRIPES];
    u64 moves[STRIPES];           // moves applied
    u64 positive[STRIPES];        // evaluated vertices whose best gain was positive (before Pick-Less)
    u64 pruned;                   // flagged vertices the learned pruner skipped (for the next iteration)
    // ---- other state
    int32_t err;                  // validation error bits
    int32_t unsorted;             // validation: some row is not strictly ascending by neighbour id
    u64 kmax;                     // largest weighted degree of the level
    u64 wsum;                     // total weight (validation pass)
    int32_t bcount[MAX_BUCKETS];  // bucket sizes (classification)
    int32_t bcursor[MAX_BUCKETS]; // fill cursors
    u64 q_lo;                     // modularity numerator accumulator (128-bit)
    u64 q_hi;
    u64 nsamples;                 // training samples claimed during the run
    // ---- run totals per move bucket (last = hub): evaluations, arcs,
    // distinct communities, moves, arcs of movers
    u64 bstat[5][MAX_BUCKETS][STRIPES];
};
constexpr size_t CTL_ITER_BYTES = offsetof(Ctl, err);

// CSR view of one level.  WK: 0 = unit weights, 1 = int32, 2 = int64.
template <typename OffT, int WK>
struct Graph {
    const OffT* __restrict__ off;
    const int32_t* __restrict__ idx;
    const void* __restrict__ w;
    __device__ __forceinline__ i64 weight(i64 e) const {
        if constexpr (WK == 0) return 1;
        else if constexpr (WK == 1) return (i64)((const int32_t*)w)[e];
        else return ((const i64*)w)[e];
    }
};

// ---------------------------------------------------------------- hashing
// Multiplicative (Fibonacci) hash into a power-of-two table, then triangular
// probing s, s+1, s+3, s+6, ... which visits every slot of such a table.
template <int LOG2CAP>
__device__ __forceinline__ uint32_t hash_slot(int32_t key) {
    return ((uint32_t)key * 0x9E3779B1u) >> (32 - LOG2CAP);
}
__device__ __forceinline__ uint32_t hash_slot_rt(int32_t key, int log2cap) {
    return log2cap == 0 ? 0u : (((uint32_t)key * 0x9E3779B1u) >> (32 - log2cap));
}

// Accumulate (key, v) into an open-addressing table with atomics; the caller
// guarantees a free slot exists (capacity >= 2 * distinct keys).
template <typename AccT>
__device__ __forceinline__ void table_add(int32_t* keys, AccT* vals, uint32_t mask, uint32_t s, int32_t key,
                                          AccT v) {
    for (uint32_t step = 1;; ++step) {
        int32_t k = *(volatile int32_t*)&keys[s];
        if (k == key) { atomicAdd(&vals[s], v); return; }
        if (k == EMPTY_KEY) {
            int32_t old = atomicCAS(&keys[s], EMPTY_KEY, key);
            if (old == EMPTY_KEY || old == key) { atomicAdd(&vals[s], v); return; }
        }
        s = (s + step) & mask;
    }
}

// As table_add; returns the slot if this call claimed a previously empty
// slot for key, else -1 (so that callers can list the occupied slots).
template <typename AccT>
__device__ __forceinline__ int64_t table_add_claim(int32_t* keys, AccT* vals, uint32_t mask, uint32_t s,
                                                   int32_t key, AccT v) {
    for (uint32_t step = 1;; ++step) {
        int32_t k = *(volatile int32_t*)&keys[s];
        if (k == key) { atomicAdd(&vals[s], v); return -1; }
        if (k == EMPTY_KEY) {
            int32_t old = atomicCAS(&keys[s], EMPTY_KEY, key);
            if (old == EMPTY_KEY || old == key) {
                atomicAdd(&vals[s], v);
                return old == EMPTY_KEY ? (int64_t)s : -1;
            }
        }
        s = (s + step) & mask;
    }
}

// ------------------------------------------------------------ reductions
__device__ __forceinline__ i64 shfl_xor64(i64 v, int m, int width) { return __shfl_xor(v, m, width); }
__device__ __forceinline__ i128 shfl_xor128(i128 v, int m, int width) {
    i64 lo = (i64)(u64)v, hi = (i64)(v >> 64);
    lo = __shfl_xor(lo, m, width);
    hi = __shfl_xor(hi, m, width);
    return ((i128)hi << 64) | (i128)(u64)lo;
}

// Best candidate: larger key wins, ties go to the smaller community id.
template <typename KeyT>
struct Best {
    KeyT key;
    int32_t d;
};
template <typename KeyT>
__device__ __forceinline__ bool better(KeyT k1, int32_t d1, KeyT k2, int32_t d2) {
    return k1 > k2 || (k1 == k2 && d1 < d2);
}

// Butterfly reduction inside an aligned group of G <= 64 lanes; the winner's
// payload v (its K_{i->d}) travels with it.
template <int G>
__device__ __forceinline__ void group_best64(i64& key, int32_t& d, i64& v) {
#pragma unroll
    for (int m = G / 2; m >= 1; m >>= 1) {
        i64 k2 = shfl_xor64(key, m, G);
        int32_t d2 = __shfl_xor(d, m, G);
        i64 v2 = shfl_xor64(v, m, G);
        if (better(k2, d2, key, d)) { key = k2; d = d2; v = v2; }
    }
}
template <int G>
__device__ __forceinline__ void group_best128(i128& key, int32_t& d, i64& v) {
#pragma unroll
    for (int m = G / 2; m >= 1; m >>= 1) {
        i128 k2 = shfl_xor128(key, m, G);
        int32_t d2 = __shfl_xor(d, m, G);
        i64 v2 = shfl_xor64(v, m, G);
        if (better(k2, d2, key, d)) { key = k2; d = d2; v = v2; }
    }
}
template <int G>
__device__ __forceinline__ i64 group_max64(i64 v) {
#pragma unroll
    for (int m = G / 2; m >= 1; m >>= 1) {
        i64 o = shfl_xor64(v, m, G);
        v = o > v ? o : v;
    }
    return v;
}
template <int G>
__device__ __forceinline__ i64 group_sum64(i64 v) {
#pragma unroll
    for (int m = G / 2; m >= 1; m >>= 1) v += shfl_xor64(v, m, G);
    return v;
}

// Exact 128-bit accumulation into (lo, hi) with two 64-bit atomics.
__device__ __forceinline__ void atomic_add_i128(u64* lo, u64* hi, i128 v) {
    u64 vlo = (u64)v, vhi = (u64)(v >> 64);
    u64 old = atomicAdd(lo, vlo);
    vhi += (old + vlo < old) ? 1ull : 0ull;
    if (vhi) atomicAdd(hi, vhi);
}

// Parts of a 128-bit value for split accumulation (lo and mid < 2^32, so
// sums of up to 2^32 parts cannot overflow; hi wraps modulo 2^64, which is
// exact modulo 2^128 once recombined).
struct Split128 {
    u64 lo, mid, hi;
};
__device__ __forceinline__ Split128 split128(i128 v) {
    return Split128{(u64)v & 0xffffffffull, (u64)(v >> 32) & 0xffffffffull, (u64)(v >> 64)};
}

// Barrier for a group of G threads (G <= 64: inside one wave).
template <int G>
__device__ __forceinline__ void group_sync() {
    if constexpr (G > WAVE) {
        __syncthreads();
    } else {
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        __builtin_amdgcn_wave_barrier();
    }
}

}  // namespace lv
