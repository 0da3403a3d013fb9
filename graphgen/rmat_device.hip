/*
 * R-MAT tuple generation on the GPU, for graphs too large to build on the
 * host (scale 27 and up).  Each tuple k draws exactly the numbers the host
 * generator in graphgen.c draws (the same counter-based SplitMix64 stream,
 * the same doubles and comparisons, the same relabelling permutation passed
 * in from the host), so both produce the same edge multiset; deduplication
 * and CSR layout are done by the caller.  Like graphgen.c this file holds
 * no community-detection arithmetic.
 *
 * Two entry points, both asynchronous on the given stream:
 *   gg_dev_rmat_hist    counts the canonical keys (u < v, self-loops
 *                       dropped) per bin of u >> shift;
 *   gg_dev_rmat_select  appends the keys u * n + v whose bin lies in
 *                       [blo, bhi) to out (at most cap of them; *count
 *                       receives the number found, which may exceed cap).
 * Return 0, or -1 on a bad argument or a launch error.
 */
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

struct Rmat {
    int scale;
    int64_t ntuples;
    double a, ab, abc;
    uint64_t base;        // SplitMix64 of (seed ^ SplitMix64(stream)): the per-stream start
    const int32_t* perm;  // may be null
    int shift;
};

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z += 0x9e3779b97f4a7c15ULL;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

// Canonical key of tuple k, or UINT64_MAX for a self-loop.
__device__ __forceinline__ uint64_t tuple_key(const Rmat& p, int64_t k, int64_t* umin) {
    int64_t u = 0, v = 0;
    const uint64_t c0 = (uint64_t)k * (uint64_t)p.scale;
    for (int l = 0; l < p.scale; l++) {
        const double r = (double)(mix64(p.base + c0 + (uint64_t)l) >> 11) * (1.0 / 9007199254740992.0);
        int bu = 0, bv = 0;
        if (r < p.a) {
        } else if (r < p.ab) {
            bv = 1;
        } else if (r < p.abc) {
            bu = 1;
        } else {
            bu = 1;
            bv = 1;
        }
        u = (u << 1) | bu;
        v = (v << 1) | bv;
    }
    if (p.perm) {
        u = p.perm[u];
        v = p.perm[v];
    }
    if (u == v) return UINT64_MAX;
    if (u > v) {
        const int64_t t = u;
        u = v;
        v = t;
    }
    *umin = u;
    return ((uint64_t)u << p.scale) | (uint64_t)v;
}

constexpr int HB = 4096;  // histogram bins held in LDS

__global__ void __launch_bounds__(256) k_hist(Rmat p, unsigned long long* hist, int nbins) {
    __shared__ uint32_t s_h[HB];
    for (int b = threadIdx.x; b < HB; b += 256) s_h[b] = 0;
    __syncthreads();
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < p.ntuples; k += stride) {
        int64_t u = 0;
        if (tuple_key(p, k, &u) != UINT64_MAX) atomicAdd(&s_h[u >> p.shift], 1u);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < nbins; b += 256)
        if (s_h[b]) atomicAdd(&hist[b], (unsigned long long)s_h[b]);
}

__global__ void __launch_bounds__(256) k_select(Rmat p, int64_t blo, int64_t bhi, uint64_t* out, int64_t cap,
                                                unsigned long long* count) {
    const int64_t stride = (int64_t)gridDim.x * 256;
    const int lane = threadIdx.x % 64;
    // every lane of a wave runs the same number of rounds (the wave-wide ballot needs all of them)
    const int64_t k0 = (int64_t)blockIdx.x * 256 + (threadIdx.x - lane);
    for (int64_t kw = k0; kw < p.ntuples; kw += stride) {
        const int64_t k = kw + lane;
        uint64_t key = UINT64_MAX;
        int64_t u = 0;
        bool keep = false;
        if (k < p.ntuples) {
            key = tuple_key(p, k, &u);
            if (key != UINT64_MAX) {
                const int64_t b = u >> p.shift;
                keep = b >= blo && b < bhi;
            }
        }
        const uint64_t mask = __ballot(keep);
        if (!mask) continue;
        unsigned long long at = 0;
        const int leader = __ffsll((long long)mask) - 1;
        if (lane == leader) at = atomicAdd(count, (unsigned long long)__popcll(mask));
        at = __shfl(at, leader, 64);
        if (keep) {
            const uint64_t below = lane ? (mask & ((~0ull) >> (64 - lane))) : 0ull;
            const int64_t pos = (int64_t)at + __popcll(below);
            if (pos < cap) out[pos] = key;
        }
    }
}

bool fill(Rmat* p, int scale, int64_t ntuples, double a, double ab, double abc, uint64_t base,
          const int32_t* perm, int shift) {
    if (scale < 1 || scale > 31 || ntuples < 0 || shift < 0 || shift > scale || scale - shift > 12) return false;
    p->scale = scale;
    p->ntuples = ntuples;
    p->a = a;
    p->ab = ab;
    p->abc = abc;
    p->base = base;
    p->perm = perm;
    p->shift = shift;
    return true;
}

unsigned grid_for(int64_t ntuples) {
    const int64_t want = (ntuples + 255) / 256;
    return (unsigned)(want < 8192 ? (want > 0 ? want : 1) : 8192);
}

}  // namespace

extern "C" int gg_dev_rmat_hist(int scale, int64_t ntuples, double a, double ab, double abc, uint64_t base,
                                const int32_t* perm, int shift, unsigned long long* hist, void* stream) {
    Rmat p;
    if (!fill(&p, scale, ntuples, a, ab, abc, base, perm, shift) || !hist) return -1;
    const int nbins = 1 << (scale - shift);
    hipLaunchKernelGGL(k_hist, dim3(grid_for(ntuples)), dim3(256), 0, (hipStream_t)stream, p, hist, nbins);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

extern "C" int gg_dev_rmat_select(int scale, int64_t ntuples, double a, double ab, double abc, uint64_t base,
                                  const int32_t* perm, int shift, int64_t blo, int64_t bhi, uint64_t* out,
                                  int64_t cap, unsigned long long* count, void* stream) {
    Rmat p;
    if (!fill(&p, scale, ntuples, a, ab, abc, base, perm, shift) || !out || !count || cap < 0) return -1;
    hipLaunchKernelGGL(k_select, dim3(grid_for(ntuples)), dim3(256), 0, (hipStream_t)stream, p, blo, bhi, out, cap,
                       count);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}
