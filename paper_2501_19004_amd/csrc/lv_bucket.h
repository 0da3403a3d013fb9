// lv_bucket.h -- ordered, atomic-free partition of items into buckets.
//
// Used for the per-pass degree buckets, the per-iteration queues of flagged
// vertices and the aggregation buckets.  Two passes over the items with a
// scan in between: (1) every block counts its items per bucket; (2) an
// exclusive scan over the bucket-major count matrix gives every (bucket,
// block) its output offset; (3) every block writes its items, in item order,
// to its slots.  The output lists are therefore sorted by item id within each
// bucket, which keeps neighbouring rows of the CSR together in memory.
#pragma once

#include "lv_common.h"

namespace lv {

constexpr int BK_TPB = 256;   // threads per block
constexpr int BK_IPT = 16;    // consecutive items per thread
constexpr int BK_ITEMS = BK_TPB * BK_IPT;

inline int64_t bucket_blocks(int64_t n) { return (n + BK_ITEMS - 1) / BK_ITEMS; }

// Exclusive scan across the block of NB per-thread counters at once.
template <int NB>
__device__ __forceinline__ void block_excl_scan_nb(int32_t (&v)[NB], int32_t (&tot)[NB]) {
    __shared__ int32_t s_w[NB][BK_TPB / WAVE];
    const int lane = threadIdx.x % WAVE, wid = threadIdx.x / WAVE;
#pragma unroll
    for (int b = 0; b < NB; b++) {
        int32_t x = v[b];
#pragma unroll
        for (int d = 1; d < WAVE; d <<= 1) {
            const int32_t y = __shfl_up(x, d, WAVE);
            if (lane >= d) x += y;
        }
        if (lane == WAVE - 1) s_w[b][wid] = x;
        v[b] = x - v[b];  // exclusive within the wave
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < NB; b++) {
        int32_t before = 0, all = 0;
#pragma unroll
        for (int k = 0; k < BK_TPB / WAVE; k++) {
            const int32_t ws = s_w[b][k];
            before += k < wid ? ws : 0;
            all += ws;
        }
        v[b] += before;
        tot[b] = all;
    }
    __syncthreads();
}

// bucket functor: __device__ int operator()(int64_t item) const, returns a
// bucket in [0, NB) or a value >= NB for "no bucket".  halt (may be NULL):
// the launch does nothing when *halt != 0.
template <int NB, typename BF>
__global__ void __launch_bounds__(BK_TPB) k_bucket_count(BF bf, int64_t n, int32_t* __restrict__ blkcnt,
                                                         int64_t nblocks, const int32_t* __restrict__ halt) {
    if (halt && *halt) return;
    int32_t cnt[NB];
#pragma unroll
    for (int b = 0; b < NB; b++) cnt[b] = 0;
    const int64_t base = (int64_t)blockIdx.x * BK_ITEMS + (int64_t)threadIdx.x * BK_IPT;
#pragma unroll 4
    for (int k = 0; k < BK_IPT; k++) {
        const int64_t it = base + k;
        if (it < n) {
            const int b = bf(it);
#pragma unroll
            for (int q = 0; q < NB; q++) cnt[q] += (b == q);
        }
    }
    int32_t tot[NB];
    block_excl_scan_nb<NB>(cnt, tot);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int b = 0; b < NB; b++) blkcnt[(int64_t)b * nblocks + blockIdx.x] = tot[b];
    }
}

template <int NB, typename BF>
__global__ void __launch_bounds__(BK_TPB) k_bucket_fill(BF bf, int64_t n, const int32_t* __restrict__ blkoff,
                                                        int64_t nblocks, int32_t* __restrict__ out,
                                                        const int32_t* __restrict__ halt) {
    if (halt && *halt) return;
    int32_t cnt[NB];
#pragma unroll
    for (int b = 0; b < NB; b++) cnt[b] = 0;
    const int64_t base = (int64_t)blockIdx.x * BK_ITEMS + (int64_t)threadIdx.x * BK_IPT;
#pragma unroll 4
    for (int k = 0; k < BK_IPT; k++) {
        const int64_t it = base + k;
        if (it < n) {
            const int b = bf(it);
#pragma unroll
            for (int q = 0; q < NB; q++) cnt[q] += (b == q);
        }
    }
    int32_t tot[NB];
    block_excl_scan_nb<NB>(cnt, tot);
    int32_t pos[NB];
#pragma unroll
    for (int b = 0; b < NB; b++) pos[b] = blkoff[(int64_t)b * nblocks + blockIdx.x] + cnt[b];
#pragma unroll 4
    for (int k = 0; k < BK_IPT; k++) {
        const int64_t it = base + k;
        if (it < n) {
            const int b = bf(it);
#pragma unroll
            for (int q = 0; q < NB; q++)
                if (b == q) out[pos[q]++] = (int32_t)it;
        }
    }
}

// Bucket totals: tot[b] = blkoff[(b+1)*nblocks] - blkoff[b*nblocks].
static __global__ void k_bucket_totals(const int32_t* __restrict__ blkoff, int64_t nblocks, int nb,
                                int32_t* __restrict__ tot) {
    const int b = threadIdx.x;
    if (b < nb) tot[b] = blkoff[(int64_t)(b + 1) * nblocks] - blkoff[(int64_t)b * nblocks];
}

}  // namespace lv
