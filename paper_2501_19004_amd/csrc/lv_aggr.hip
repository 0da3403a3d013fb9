// lv_aggr.hip -- aggregation phase, dendrogram lookup, modularity, validation.
//
// Aggregation (the paper's Algorithm 3 / Algorithm 6) merges each community
// into one super-vertex: the super-arc (c, d) carries the summed weight of all
// arcs (i, j) with C'[i] = c and C'[j] = d, self-loops included
// (scanCommunities with self = true).  Steps here:
//   used flags -> exclusive scan -> dense ids (renumber, ascending old id);
//   community-vertex CSR by counting + scan + scatter;
//   community total degree + scan -> "holey" row bounds;
//   per community: hash (d, w) in an LDS table, bitonic-sort the table in
//   LDS, write the sorted distinct entries into the holey row;
//   big communities: many workgroups per community, LDS pre-aggregation
//   into a global table, sorted extraction through a key bitmap;
//   scan of distinct counts -> compacted, row-sorted super-graph CSR.
#include <algorithm>

#include "lv_bucket.h"
#include "lv_internal.h"

namespace lv {
namespace {

template <int N>
struct Log2 { static constexpr int v = 1 + Log2<N / 2>::v; };
template <>
struct Log2<1> { static constexpr int v = 0; };
template <typename T>
struct TypeTag { using type = T; };
template <int V>
struct IntTag { static constexpr int value = V; };

template <typename Fn>
void dispatch_types(const LevelTypes& t, Fn&& fn) {
    auto acc = [&](auto o, auto w) {
        if (t.acc64) fn(o, w, TypeTag<u64>{});
        else fn(o, w, TypeTag<uint32_t>{});
    };
    auto wk = [&](auto o) {
        if (t.wk == 0) acc(o, IntTag<0>{});
        else if (t.wk == 1) acc(o, IntTag<1>{});
        else acc(o, IntTag<2>{});
    };
    if (t.off64) wk(TypeTag<int64_t>{});
    else wk(TypeTag<int32_t>{});
}

inline unsigned blocks_for(int64_t items, int per_block) { return (unsigned)((items + per_block - 1) / per_block); }

// Inclusive scan over a group of G lanes (G > 64: whole workgroup via LDS).
template <int G>
__device__ __forceinline__ i64 group_incl_scan(i64 v, i64* s_t) {
    constexpr int GW = G < WAVE ? G : WAVE;
    const int l = threadIdx.x % GW;
#pragma unroll
    for (int d = 1; d < GW; d <<= 1) {
        i64 y = __shfl_up(v, d, GW);
        if (l >= d) v += y;
    }
    if constexpr (G > WAVE) {
        const int w = threadIdx.x / WAVE;
        if (threadIdx.x % WAVE == WAVE - 1) s_t[w] = v;
        __syncthreads();
        i64 before = 0;
        for (int k = 0; k < w; k++) before += s_t[k];
        __syncthreads();
        v += before;
    }
    return v;
}
template <int G>
__device__ __forceinline__ i64 group_sum(i64 v, i64* s_t) {
    constexpr int GW = G < WAVE ? G : WAVE;
    v = group_sum64<GW>(v);
    if constexpr (G > WAVE) {
        const int w = threadIdx.x / WAVE;
        if (threadIdx.x % WAVE == 0) s_t[w] = v;
        __syncthreads();
        v = 0;
        for (int k = 0; k < G / WAVE; k++) v += s_t[k];
        __syncthreads();
    }
    return v;
}
// Broadcast lane 0's value to the group.
template <int G>
__device__ __forceinline__ i64 group_bcast(i64 v, i64* s_t) {
    if constexpr (G <= WAVE) {
        return __shfl(v, 0, G);
    } else {
        if (threadIdx.x == 0) s_t[0] = v;
        __syncthreads();
        v = s_t[0];
        __syncthreads();
        return v;
    }
}

// Feed every arc (j, w) of every member of community c into the table:
// members are taken G at a time; their arc ranges are laid end to end and
// the group strides over the concatenation (a lane finds its member by
// binary search over the group's prefix of degrees).
template <typename OffT, int WK, typename AccT, int G, typename InsertFn>
__device__ __forceinline__ void feed_members(const Graph<OffT, WK>& g, const int32_t* __restrict__ Cp,
                                             const int32_t* __restrict__ members, i64 m0, i64 m1, int lane,
                                             i64* s_start, i64* s_pre, i64* s_t, InsertFn&& ins) {
    for (i64 mb = m0; mb < m1; mb += G) {
        i64 start = 0, deg = 0;
        if (mb + lane < m1) {
            const int32_t m = members[mb + lane];
            start = (i64)g.off[m];
            deg = (i64)g.off[m + 1] - start;
        }
        const i64 pre = group_incl_scan<G>(deg, s_t);
        s_start[lane] = start;
        s_pre[lane] = pre;
        group_sync<G>();
        const i64 total = s_pre[G - 1];
        for (i64 f = lane; f < total; f += G) {
            int lo = 0, hi = G - 1;  // first k with pre[k] > f
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (s_pre[mid] > f) hi = mid; else lo = mid + 1;
            }
            const i64 e = s_start[lo] + (f - (lo ? s_pre[lo - 1] : 0));
            ins(Cp[g.idx[e]], (AccT)g.weight(e));
        }
        group_sync<G>();
    }
}

// In-place bitonic sort of CAP (key, value) pairs held by one group; keys
// ascending, EMPTY_KEY last.
template <int G, typename AccT>
__device__ __forceinline__ void bitonic_sort_group(int32_t* keys, AccT* vals, int64_t cap, int lane) {
    for (int64_t k = 2; k <= cap; k <<= 1) {
        for (int64_t j = k >> 1; j > 0; j >>= 1) {
            for (int64_t x = lane; x < cap; x += G) {
                const int64_t y = x ^ j;
                if (y > x) {
                    const bool up = (x & k) == 0;
                    const int32_t kx = keys[x], ky = keys[y];
                    if ((kx > ky) == up) {
                        keys[x] = ky; keys[y] = kx;
                        const AccT t = vals[x]; vals[x] = vals[y]; vals[y] = t;
                    }
                }
            }
            group_sync<G>();
        }
    }
}

template <typename OffT, int WK, typename AccT, int G, int CAP>
__global__ void __launch_bounds__(G > 256 ? G : 256) k_aggregate_lds(Graph<OffT, WK> g, AggArgs a,
                                                                     const int32_t* __restrict__ list,
                                                                     int32_t count) {
    constexpr int BLOCK = G > 256 ? G : 256;
    constexpr int NG = BLOCK / G;
    constexpr int L2C = Log2<CAP>::v;
    __shared__ int32_t s_keys[NG * CAP];
    __shared__ AccT s_vals[NG * CAP];
    __shared__ i64 s_start[NG * G], s_pre[NG * G];
    __shared__ i64 s_t[BLOCK / WAVE];
    const int grp = threadIdx.x / G, lane = threadIdx.x % G;
    const int64_t slot = (int64_t)blockIdx.x * NG + grp;
    const bool active = slot < count;
    const int32_t c = active ? list[slot] : 0;
    int32_t* keys = s_keys + grp * CAP;
    AccT* vals = s_vals + grp * CAP;
    for (int s = lane; s < CAP; s += G) { keys[s] = EMPTY_KEY; vals[s] = 0; }
    group_sync<G>();
    const i64 m0 = active ? a.coff[c] : 0, m1 = active ? a.coff[c + 1] : 0;
    feed_members<OffT, WK, AccT, G>(g, a.Cp, a.members, m0, m1, lane, s_start + grp * G, s_pre + grp * G, s_t,
                                    [&](int32_t d, AccT w) {
                                        table_add<AccT>(keys, vals, CAP - 1, hash_slot<L2C>(d), d, w);
                                    });
    // Move the occupied slots to the front, then sort only the next power of
    // two above their count (the rest of the table stays empty).
    constexpr int PER = CAP / G;
    int32_t rk[PER];
    AccT rv[PER];
    i64 mine = 0;
#pragma unroll
    for (int q = 0; q < PER; q++) {
        rk[q] = keys[lane + q * G];
        rv[q] = vals[lane + q * G];
        mine += rk[q] != EMPTY_KEY;
    }
    const i64 incl = group_incl_scan<G>(mine, s_t);
    const i64 L = group_sum<G>(mine, s_t);
    group_sync<G>();
    i64 at = incl - mine;
#pragma unroll
    for (int q = 0; q < PER; q++)
        if (rk[q] != EMPTY_KEY) { keys[at] = rk[q]; vals[at] = rv[q]; at++; }
    if (a.sorted) {
        int64_t P = 1;
        while (P < L) P <<= 1;
        for (i64 x = L + lane; x < P; x += G) { keys[x] = EMPTY_KEY; vals[x] = 0; }
        group_sync<G>();
        bitonic_sort_group<G, AccT>(keys, vals, P, lane);
    } else {
        group_sync<G>();
    }
    if (active) {
        const i64 h = a.hoff[c];
        for (i64 x = lane; x < L; x += G) {
            a.hidx[h + x] = keys[x];
            if (a.out_w64) ((i64*)a.hw)[h + x] = (i64)vals[x];
            else ((int32_t*)a.hw)[h + x] = (int32_t)vals[x];
        }
        if (lane == 0) a.rowlen[c] = (int32_t)L;
    }
}

// ------------------------------------------------------------ big communities
// A community whose distinct-neighbour bound exceeds the largest LDS bucket,
// or whose arcs exceed BIG_ARCS, is spread over many workgroups.  Its arcs
// are laid end to end in community-vertex order ("virtual arcs": virtual arc
// f belongs to the member k with mpos[k] <= f < mpos[k+1], where mpos is the
// exclusive prefix of member degrees; community c's virtual range starts at
// hoff[c]).  Each chunk of BIG_CH virtual arcs is hashed into an LDS table,
// then the table's distinct entries are added into the community's global
// table.  Extraction marks the keys in a bitmap over [0, ncom) and walks it
// in order, which yields the row sorted by neighbour id.

// Exclusive-prefix input: degree of each member in community-vertex order.
template <typename OffT>
__global__ void k_member_deg(const OffT* __restrict__ off, const int32_t* __restrict__ members, int64_t n,
                             int64_t* __restrict__ md) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int32_t m = members[k];
    md[k] = (int64_t)off[m + 1] - (int64_t)off[m];
}

__global__ void k_big_info(const int32_t* __restrict__ list, int32_t nbig, const int64_t* __restrict__ hoff,
                           int64_t ncom, int64_t* __restrict__ nch, int64_t* __restrict__ cap) {
    const int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= nbig) return;
    const int32_t c = list[h];
    const int64_t cdeg = hoff[c + 1] - hoff[c];
    nch[h] = (cdeg + BIG_CH - 1) / BIG_CH;
    const int64_t bound = cdeg < ncom ? cdeg : ncom;
    uint64_t t = 1;
    while (t < 2 * (uint64_t)bound) t <<= 1;
    cap[h] = (int64_t)t;
}

__global__ void k_big_clear(int32_t* __restrict__ keys, u64* __restrict__ vals, int64_t count) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < count; s += stride) {
        keys[s] = EMPTY_KEY;
        vals[s] = 0;
    }
}

// largest h in [0, n) with pre[h] - base <= x (pre non-decreasing, pre[0] - base <= x)
__device__ __forceinline__ int32_t find_owner(const int64_t* pre, int32_t n, int64_t base, int64_t x) {
    int32_t lo = 0, hi = n - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (pre[mid] - base <= x) lo = mid; else hi = mid - 1;
    }
    return lo;
}

template <typename OffT, int WK, typename AccT>
__global__ void __launch_bounds__(1024) k_big_insert(Graph<OffT, WK> g, BigArgs a) {
    constexpr int G = 1024;
    constexpr int L2C = Log2<BIG_LCAP>::v;
    __shared__ int32_t s_keys[BIG_LCAP];
    __shared__ AccT s_vals[BIG_LCAP];
    __shared__ i64 s_start[G], s_pre[G];
    __shared__ i64 s_t[G / WAVE];
    __shared__ int64_t s_info[4];
    const int tid = threadIdx.x;
    const int64_t chunk = blockIdx.x;
    for (int s = tid; s < BIG_LCAP; s += G) { s_keys[s] = EMPTY_KEY; s_vals[s] = 0; }
    if (tid == 0) {
        const int32_t h = find_owner(a.chunk_pre, a.nbig, a.chunk_base, chunk);
        const int32_t c = a.list[h];
        const int64_t f0 = a.hoff[c] + (chunk - (a.chunk_pre[h] - a.chunk_base)) * BIG_CH;
        const int64_t f1 = min(f0 + (int64_t)BIG_CH, a.hoff[c + 1]);
        // first member whose virtual range contains f0; first member starting at or after f1
        int64_t lo = a.coff[c], hi = a.coff[c + 1] - 1;
        while (lo < hi) {
            const int64_t mid = (lo + hi + 1) >> 1;
            if (a.mpos[mid] <= f0) lo = mid; else hi = mid - 1;
        }
        int64_t k1lo = lo, k1hi = a.coff[c + 1];
        while (k1lo < k1hi) {
            const int64_t mid = (k1lo + k1hi) >> 1;
            if (a.mpos[mid] < f1) k1lo = mid + 1; else k1hi = mid;
        }
        s_info[0] = h;
        s_info[1] = lo;
        s_info[2] = k1lo;
        s_info[3] = f0;
        s_t[0] = f1;
    }
    __syncthreads();
    const int32_t h = (int32_t)s_info[0];
    const int64_t k0 = s_info[1], k1 = s_info[2], f0 = s_info[3];
    const int64_t f1 = s_t[0];
    __syncthreads();
    for (int64_t kb = k0; kb < k1; kb += G) {
        i64 start = 0, deg = 0;
        if (kb + tid < k1) {
            const int64_t k = kb + tid;
            const int32_t m = a.members[k];
            const int64_t v0 = max(a.mpos[k], f0), v1 = min(a.mpos[k + 1], f1);
            start = (i64)g.off[m] + (v0 - a.mpos[k]);
            deg = v1 > v0 ? v1 - v0 : 0;
        }
        const i64 pre = group_incl_scan<G>(deg, s_t);
        s_start[tid] = start;
        s_pre[tid] = pre;
        __syncthreads();
        const i64 total = s_pre[G - 1];
        // U virtual arcs per round: their index loads, then their C' gathers, are issued together
        constexpr int U = 4;
        for (i64 fb = tid; fb < total; fb += U * G) {
            i64 ee[U];
            int32_t jj[U], dd[U];
#pragma unroll
            for (int u = 0; u < U; u++) {
                const i64 f = fb + (i64)u * G;
                ee[u] = -1;
                if (f < total) {
                    int lo = 0, hi = G - 1;
                    while (lo < hi) {
                        const int mid = (lo + hi) >> 1;
                        if (s_pre[mid] > f) hi = mid; else lo = mid + 1;
                    }
                    ee[u] = s_start[lo] + (f - (lo ? s_pre[lo - 1] : 0));
                }
            }
#pragma unroll
            for (int u = 0; u < U; u++) jj[u] = ee[u] >= 0 ? g.idx[ee[u]] : 0;
#pragma unroll
            for (int u = 0; u < U; u++) dd[u] = ee[u] >= 0 ? a.Cp[jj[u]] : EMPTY_KEY;
#pragma unroll
            for (int u = 0; u < U; u++)
                if (ee[u] >= 0)
                    table_add<AccT>(s_keys, s_vals, BIG_LCAP - 1, hash_slot<L2C>(dd[u]), dd[u], (AccT)g.weight(ee[u]));
        }
        __syncthreads();
    }
    // merge the chunk's distinct entries into the community's global table
    const int64_t toff = a.tab_pre[h] - a.tab_base;
    const int64_t cap = a.tab_pre[h + 1] - a.tab_pre[h];
    const int log2cap = __ffsll((long long)cap) - 1;
    int32_t* keys = a.keys + toff;
    AccT* vals = (AccT*)a.vals + toff;
    int32_t* slots = a.slots + toff / 2;  // cap >= 2 * distinct keys
    // the first probes of all of this thread's keys are issued together; a
    // key whose home slot holds another key continues along its probe sequence
    constexpr int PER = BIG_LCAP / G;
    const uint32_t mask = (uint32_t)(cap - 1);
    int32_t kk[PER], old[PER];
    uint32_t home[PER];
    int64_t got[PER];
#pragma unroll
    for (int u = 0; u < PER; u++) kk[u] = s_keys[tid + u * G];
#pragma unroll
    for (int u = 0; u < PER; u++) {
        home[u] = kk[u] != EMPTY_KEY ? hash_slot_rt(kk[u], log2cap) : 0u;
        old[u] = kk[u] != EMPTY_KEY ? atomicCAS(&keys[home[u]], EMPTY_KEY, kk[u]) : EMPTY_KEY;
    }
    int nclaim = 0;
#pragma unroll
    for (int u = 0; u < PER; u++) {
        got[u] = -1;
        if (kk[u] == EMPTY_KEY) continue;
        const AccT val = s_vals[tid + u * G];
        if (old[u] == EMPTY_KEY || old[u] == kk[u]) {
            atomicAdd(&vals[home[u]], val);
            if (old[u] == EMPTY_KEY) got[u] = home[u];
        } else {
            got[u] = table_add_claim<AccT>(keys, vals, mask, home[u], kk[u], val);
        }
        nclaim += got[u] >= 0;
    }
    // list the newly occupied slots: one global counter update per block
    __shared__ int32_t s_claim[2];
    if (tid == 0) s_claim[0] = 0;
    __syncthreads();
    const int mine = nclaim ? atomicAdd(&s_claim[0], nclaim) : 0;
    __syncthreads();
    if (tid == 0) s_claim[1] = s_claim[0] ? atomicAdd(&a.cnt[h], s_claim[0]) : 0;
    __syncthreads();
    if (nclaim) {
        int32_t p = s_claim[1] + mine;
#pragma unroll
        for (int u = 0; u < PER; u++)
            if (got[u] >= 0) slots[p++] = (int32_t)got[u];
    }
}

template <typename AccT>
__device__ __forceinline__ AccT table_get(const int32_t* keys, const AccT* vals, uint32_t mask, uint32_t s,
                                          int32_t key) {
    for (uint32_t step = 1;; ++step) {
        if (keys[s] == key) return vals[s];
        s = (s + step) & mask;
    }
}

template <typename AccT>
__global__ void __launch_bounds__(1024) k_big_extract(BigArgs a) {
    constexpr int G = 1024;
    __shared__ i64 s_t[G / WAVE];
    __shared__ int32_t s_k[BIG_SORT_MAX];
    __shared__ AccT s_v[BIG_SORT_MAX];
    const int tid = threadIdx.x;
    uint32_t* bm = a.bitmaps + (int64_t)blockIdx.x * a.words;
    for (int32_t h = blockIdx.x; h < a.nbig; h += gridDim.x) {
        const int32_t c = a.list[h];
        const int64_t toff = a.tab_pre[h] - a.tab_base;
        const int64_t cap = a.tab_pre[h + 1] - a.tab_pre[h];
        const int log2cap = __ffsll((long long)cap) - 1;
        const int32_t* keys = a.keys + toff;
        const AccT* vals = (const AccT*)a.vals + toff;
        const int32_t* slots = a.slots + toff / 2;
        const int64_t L = a.cnt[h];
        const int64_t base = a.hoff[c];
        if (!a.sorted) {
            // table order: the listed occupied slots as they are
            for (int64_t x = tid; x < L; x += G) {
                const int32_t sl = slots[x];
                a.hidx[base + x] = keys[sl];
                if (a.out_w64) ((i64*)a.hw)[base + x] = (i64)vals[sl];
                else ((int32_t*)a.hw)[base + x] = (int32_t)vals[sl];
            }
            if (tid == 0) a.rowlen[c] = (int32_t)L;
            continue;
        }
        if (L <= BIG_SORT_MAX) {
            // the listed entries, padded to a power of two, sorted in LDS
            int64_t P = 1;
            while (P < L) P <<= 1;
            for (int64_t k = tid; k < P; k += G) {
                if (k < L) {
                    const int32_t sl = slots[k];
                    s_k[k] = keys[sl];
                    s_v[k] = vals[sl];
                } else {
                    s_k[k] = EMPTY_KEY;
                    s_v[k] = 0;
                }
            }
            __syncthreads();
            bitonic_sort_group<G, AccT>(s_k, s_v, P, tid);
            for (int64_t x = tid; x < L; x += G) {
                a.hidx[base + x] = s_k[x];
                if (a.out_w64) ((i64*)a.hw)[base + x] = (i64)s_v[x];
                else ((int32_t*)a.hw)[base + x] = (int32_t)s_v[x];
            }
            if (tid == 0) a.rowlen[c] = (int32_t)L;
            __syncthreads();
            continue;
        }
        // long rows: mark the keys in a bitmap over [0, ncom) and walk it in order
        for (int64_t w = tid; w < a.words; w += G) bm[w] = 0;
        __syncthreads();
        for (int64_t k = tid; k < L; k += G) {
            const int32_t d = keys[slots[k]];
            atomicOr(&bm[d >> 5], 1u << (d & 31));
        }
        __syncthreads();
        const int64_t per = (a.words + G - 1) / G;
        const int64_t w0 = min((int64_t)tid * per, a.words), w1 = min(w0 + per, a.words);
        i64 cnt = 0;
        for (int64_t w = w0; w < w1; w++) cnt += __popc(bm[w]);
        const i64 incl = group_incl_scan<G>(cnt, s_t);
        i64 rank = incl - cnt;
        for (int64_t w = w0; w < w1; w++) {
            uint32_t bits = bm[w];
            while (bits) {
                const int b = __ffs(bits) - 1;
                bits &= bits - 1;
                const int32_t d = (int32_t)(w * 32 + b);
                const AccT v = table_get<AccT>(keys, vals, (uint32_t)(cap - 1), hash_slot_rt(d, log2cap), d);
                a.hidx[base + rank] = d;
                if (a.out_w64) ((i64*)a.hw)[base + rank] = (i64)v;
                else ((int32_t*)a.hw)[base + rank] = (int32_t)v;
                rank++;
            }
        }
        if (tid == G - 1) a.rowlen[c] = (int32_t)incl;
        __syncthreads();
    }
}

// ------------------------------------------------------------ small kernels
__global__ void k_mark_used(const int32_t* __restrict__ Cp, int64_t n, int32_t* __restrict__ used) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n) used[Cp[v]] = 1;
}
__global__ void k_relabel(int32_t* __restrict__ Cp, int64_t n, const int32_t* __restrict__ newid) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n) Cp[v] = newid[Cp[v]];
}
__global__ void k_dendrogram(int32_t* __restrict__ C, int64_t n0, const int32_t* __restrict__ Cp) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n0) C[v] = Cp[C[v]];
}
__global__ void k_final_lookup(int32_t* __restrict__ C, int64_t n0, const int32_t* __restrict__ Cp,
                               const int32_t* __restrict__ newid) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n0) C[v] = newid[Cp[C[v]]];
}
// Community sizes, total degrees and member lists.  Large communities hold
// many vertices, so a global atomic per vertex would serialise on their
// counters; instead every block first combines its tile of CT_TILE vertices
// in an LDS table keyed by community and issues one global atomic per
// (block, community).
constexpr int CT_TPB = 256;
constexpr int CT_PER = 4;
constexpr int CT_TILE = CT_TPB * CT_PER;
constexpr int CT_CAP = 2 * CT_TILE;  // >= 2 * distinct communities of a tile
constexpr int CT_L2C = 11;
static_assert((1 << CT_L2C) == CT_CAP, "table size");

// Slot of key c in the tile table (inserting it if absent).
__device__ __forceinline__ uint32_t ct_slot(int32_t* keys, int32_t c) {
    uint32_t s = hash_slot<CT_L2C>(c);
    for (uint32_t step = 1;; ++step) {
        const int32_t k = *(volatile int32_t*)&keys[s];
        if (k == c) return s;
        if (k == EMPTY_KEY) {
            const int32_t old = atomicCAS(&keys[s], EMPTY_KEY, c);
            if (old == EMPTY_KEY || old == c) return s;
        }
        s = (s + step) & (CT_CAP - 1);
    }
}

template <typename OffT>
__global__ void __launch_bounds__(CT_TPB) k_comm_count(const OffT* __restrict__ off, int64_t n,
                                                       const int32_t* __restrict__ Cp, int32_t* __restrict__ cnt,
                                                       int64_t* __restrict__ cdeg) {
    __shared__ int32_t s_keys[CT_CAP];
    __shared__ int32_t s_cnt[CT_CAP];
    __shared__ u64 s_deg[CT_CAP];
    for (int k = threadIdx.x; k < CT_CAP; k += CT_TPB) { s_keys[k] = EMPTY_KEY; s_cnt[k] = 0; s_deg[k] = 0; }
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * CT_TILE;
    for (int q = 0; q < CT_PER; q++) {
        const int64_t v = base + q * CT_TPB + threadIdx.x;
        if (v >= n) break;
        const uint32_t sl = ct_slot(s_keys, Cp[v]);
        atomicAdd(&s_cnt[sl], 1);
        const u64 deg = (u64)((int64_t)off[v + 1] - (int64_t)off[v]);
        if (deg) atomicAdd(&s_deg[sl], deg);
    }
    __syncthreads();
    for (int k = threadIdx.x; k < CT_CAP; k += CT_TPB) {
        const int32_t c = s_keys[k];
        if (c == EMPTY_KEY) continue;
        atomicAdd(&cnt[c], s_cnt[k]);
        if (s_deg[k]) atomicAdd((u64*)&cdeg[c], s_deg[k]);
    }
}

__global__ void __launch_bounds__(CT_TPB) k_comm_fill(int64_t n, const int32_t* __restrict__ Cp,
                                                      const int32_t* __restrict__ coff, int32_t* __restrict__ cursor,
                                                      int32_t* __restrict__ members) {
    __shared__ int32_t s_keys[CT_CAP];
    __shared__ int32_t s_cnt[CT_CAP];
    __shared__ int32_t s_pos[CT_CAP];
    for (int k = threadIdx.x; k < CT_CAP; k += CT_TPB) { s_keys[k] = EMPTY_KEY; s_cnt[k] = 0; }
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * CT_TILE;
    uint32_t slot[CT_PER];
    for (int q = 0; q < CT_PER; q++) {
        const int64_t v = base + q * CT_TPB + threadIdx.x;
        slot[q] = 0xffffffffu;
        if (v >= n) continue;
        slot[q] = ct_slot(s_keys, Cp[v]);
        atomicAdd(&s_cnt[slot[q]], 1);
    }
    __syncthreads();
    // one global reservation per (block, community)
    for (int k = threadIdx.x; k < CT_CAP; k += CT_TPB) {
        const int32_t c = s_keys[k];
        if (c != EMPTY_KEY) s_pos[k] = coff[c] + atomicAdd(&cursor[c], s_cnt[k]);
    }
    __syncthreads();
    for (int q = 0; q < CT_PER; q++) {
        if (slot[q] == 0xffffffffu) continue;
        const int64_t v = base + q * CT_TPB + threadIdx.x;
        members[atomicAdd(&s_pos[slot[q]], 1)] = (int32_t)v;
    }
}
// Aggregation bucket of community c: by the bound min(total degree, ncom)
// on its distinct neighbours; communities with more than BIG_ARCS arcs, or
// a bound above every LDS bucket, take the big path (bucket nb); empty rows
// (isolated members only) need no work.
struct AggBucket {
    const int64_t* hoff;
    int64_t bound_cap;
    Buckets B;
    __device__ __forceinline__ int operator()(int64_t c) const {
        const int64_t cdeg = hoff[c + 1] - hoff[c];
        const int64_t bound = cdeg < bound_cap ? cdeg : bound_cap;
        if (bound <= 0) return 255;
        if (cdeg <= BIG_ARCS)
            for (int k = 0; k < B.nb; k++)
                if (bound <= B.maxdeg[k]) return k;
        return B.nb;
    }
};

// Copy each holey row to its compacted position; 32 lanes per row.
template <typename GOffT>
__global__ void __launch_bounds__(256) k_compact(int64_t ncom, const int64_t* __restrict__ hoff,
                                                 const int32_t* __restrict__ hidx, const void* __restrict__ hw,
                                                 const GOffT* __restrict__ goff, int32_t* __restrict__ gidx,
                                                 void* __restrict__ gw, int w64) {
    const int64_t c = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 32;
    const int lane = threadIdx.x % 32;
    if (c >= ncom) return;
    const int64_t src = hoff[c], dst = (int64_t)goff[c], len = (int64_t)goff[c + 1] - dst;
    for (int64_t x = lane; x < len; x += 32) {
        gidx[dst + x] = hidx[src + x];
        if (w64) ((i64*)gw)[dst + x] = ((const i64*)hw)[src + x];
        else ((int32_t*)gw)[dst + x] = ((const int32_t*)hw)[src + x];
    }
}

// Modularity pieces on the input graph: sigma_c (arcs inside c) and Sigma_c.
template <typename OffT, int WK>
__global__ void __launch_bounds__(256) k_mod_arcs(Graph<OffT, WK> g, int64_t n, const int32_t* __restrict__ C,
                                                  i64* __restrict__ sigin, i64* __restrict__ sigtot) {
    const int lane = threadIdx.x % WAVE;
    const int64_t nw = (int64_t)gridDim.x * (256 / WAVE);
    for (int64_t v = (int64_t)blockIdx.x * (256 / WAVE) + threadIdx.x / WAVE; v < n; v += nw) {
        const int32_t cv = C[v];
        i64 in = 0, tot = 0;
        for (i64 e = (i64)g.off[v] + lane; e < (i64)g.off[v + 1]; e += WAVE) {
            const i64 w = g.weight(e);
            tot += w;
            if (C[g.idx[e]] == cv) in += w;
        }
        in = group_sum64<WAVE>(in);
        tot = group_sum64<WAVE>(tot);
        if (lane == 0 && tot) {
            atomicAdd((u64*)&sigtot[cv], (u64)tot);
            if (in) atomicAdd((u64*)&sigin[cv], (u64)in);
        }
    }
}
__global__ void __launch_bounds__(256) k_mod_terms(int64_t ncom, i64 W, const i64* __restrict__ sigin,
                                                   const i64* __restrict__ sigtot, Ctl* ctl) {
    __shared__ i128 s_part[256 / WAVE];
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    i128 t = 0;
    if (c < ncom) t = (i128)W * sigin[c] - (i128)sigtot[c] * sigtot[c];
    // wave reduction of 128-bit values
    for (int m = WAVE / 2; m >= 1; m >>= 1) t += shfl_xor128(t, m, WAVE);
    if (threadIdx.x % WAVE == 0) s_part[threadIdx.x / WAVE] = t;
    __syncthreads();
    if (threadIdx.x == 0) {
        i128 s = 0;
        for (int k = 0; k < 256 / WAVE; k++) s += s_part[k];
        if (s != 0) atomic_add_i128(&ctl->q_lo, &ctl->q_hi, s);
    }
}

// Validation: offsets monotone, indices in range, weights positive; sums W.
template <typename OffT, int WK>
__global__ void __launch_bounds__(256) k_validate(Graph<OffT, WK> g, int64_t n, int64_t nnz, int check, Ctl* ctl) {
    const int lane = threadIdx.x % WAVE;
    const int64_t nw = (int64_t)gridDim.x * (256 / WAVE);
    u64 wsum = 0;
    int err = 0, uns = 0;
    for (int64_t v = (int64_t)blockIdx.x * (256 / WAVE) + threadIdx.x / WAVE; v < n; v += nw) {
        const i64 o0 = (i64)g.off[v], o1 = (i64)g.off[v + 1];
        if (check && (o1 < o0 || o0 < 0 || o1 > nnz)) { err |= 1; continue; }
        for (i64 e = o0 + lane; e < o1; e += WAVE) {
            const i64 w = g.weight(e);
            if (check) {
                const int32_t j = g.idx[e];
                if (j < 0 || j >= n) err |= 2;
                if (w <= 0) err |= 4;
            }
            if (e > o0 && g.idx[e - 1] >= g.idx[e]) uns = 1;  // a repeated or out-of-order neighbour
            wsum += (u64)w;
        }
    }
    wsum = (u64)group_sum64<WAVE>((i64)wsum);
    const bool any_uns = __any(uns);
    if (lane == 0 && wsum) atomicAdd(&ctl->wsum, wsum);
    if (lane == 0 && any_uns) atomicOr(&ctl->unsorted, 1);
    if (err) atomicOr(&ctl->err, err);
}

}  // namespace

void launch_mark_used(const int32_t* Cp, int64_t n, int32_t* used, hipStream_t s) {
    if (n > 0) k_mark_used<<<blocks_for(n, 256), 256, 0, s>>>(Cp, n, used);
}
void launch_relabel(int32_t* Cp, int64_t n, const int32_t* newid, hipStream_t s) {
    if (n > 0) k_relabel<<<blocks_for(n, 256), 256, 0, s>>>(Cp, n, newid);
}
void launch_dendrogram(int32_t* C, int64_t n0, const int32_t* Cp, hipStream_t s) {
    if (n0 > 0) k_dendrogram<<<blocks_for(n0, 256), 256, 0, s>>>(C, n0, Cp);
}
void launch_final_lookup(int32_t* C, int64_t n0, const int32_t* Cp, const int32_t* newid, hipStream_t s) {
    if (n0 > 0) k_final_lookup<<<blocks_for(n0, 256), 256, 0, s>>>(C, n0, Cp, newid);
}
void launch_comm_count(const LevelView& L, const int32_t* Cp, int32_t* cnt, int64_t* cdeg, hipStream_t s) {
    if (L.n <= 0) return;
    if (L.t.off64)
        k_comm_count<int64_t><<<blocks_for(L.n, CT_TILE), CT_TPB, 0, s>>>((const int64_t*)L.off, L.n, Cp, cnt, cdeg);
    else
        k_comm_count<int32_t><<<blocks_for(L.n, CT_TILE), CT_TPB, 0, s>>>((const int32_t*)L.off, L.n, Cp, cnt, cdeg);
}
void launch_comm_fill(int64_t n, const int32_t* Cp, const int32_t* coff, int32_t* cursor, int32_t* members,
                      hipStream_t s) {
    if (n > 0) k_comm_fill<<<blocks_for(n, CT_TILE), CT_TPB, 0, s>>>(n, Cp, coff, cursor, members);
}
void bucketize_communities(int64_t ncom, const int64_t* hoff, int64_t bound_cap, const Buckets& B, int32_t* rowlen,
                           int32_t* blkcnt, int32_t* blkoff, int32_t* out, int32_t* totals, void* scratch,
                           hipStream_t s) {
    constexpr int NB = NB_AGG + 1;
    if (ncom <= 0) {
        hipMemsetAsync(totals, 0, NB * sizeof(int32_t), s);
        return;
    }
    hipMemsetAsync(rowlen, 0, (size_t)(ncom + 1) * sizeof(int32_t), s);
    const int64_t nb = bucket_blocks(ncom);
    AggBucket bf{hoff, bound_cap, B};
    k_bucket_count<NB><<<(unsigned)nb, BK_TPB, 0, s>>>(bf, ncom, blkcnt, nb, nullptr);
    scan_i32_to_i32(blkcnt, blkoff, NB * nb, scratch, s);
    k_bucket_fill<NB><<<(unsigned)nb, BK_TPB, 0, s>>>(bf, ncom, blkoff, nb, out, nullptr);
    k_bucket_totals<<<1, 32, 0, s>>>(blkoff, nb, NB, totals);
}

void launch_aggregate(const LevelView& L, int bucket, const AggArgs& a, const int32_t* list, int32_t count,
                      hipStream_t s) {
    if (count <= 0) return;
    dispatch_types(L.t, [&](auto o, auto w, auto ac) {
        using OffT = typename decltype(o)::type;
        constexpr int WK = decltype(w)::value;
        using AccT = typename decltype(ac)::type;
        Graph<OffT, WK> g{(const OffT*)L.off, L.idx, L.w};
        auto go = [&](auto btag) {
            constexpr int b = decltype(btag)::value;
            constexpr int G = AGG_G[b], CAP = AGG_CAP[b];
            constexpr int BLOCK = G > 256 ? G : 256;
            k_aggregate_lds<OffT, WK, AccT, G, CAP><<<blocks_for(count, BLOCK / G), BLOCK, 0, s>>>(g, a, list, count);
        };
        switch (bucket) {
            case 0: go(IntTag<0>{}); break;
            case 1: go(IntTag<1>{}); break;
            case 2: go(IntTag<2>{}); break;
            default: go(IntTag<3>{}); break;
        }
    });
}

void launch_member_deg(const LevelView& L, const int32_t* members, int64_t n, int64_t* md, hipStream_t s) {
    if (n <= 0) return;
    if (L.t.off64) k_member_deg<int64_t><<<blocks_for(n, 256), 256, 0, s>>>((const int64_t*)L.off, members, n, md);
    else k_member_deg<int32_t><<<blocks_for(n, 256), 256, 0, s>>>((const int32_t*)L.off, members, n, md);
}
void launch_big_info(const int32_t* list, int32_t nbig, const int64_t* hoff, int64_t ncom, int64_t* nch,
                     int64_t* cap, hipStream_t s) {
    if (nbig > 0) k_big_info<<<blocks_for(nbig, 256), 256, 0, s>>>(list, nbig, hoff, ncom, nch, cap);
}
void launch_big_clear(int32_t* keys, void* vals, int64_t count, hipStream_t s) {
    if (count <= 0) return;
    const unsigned grid = (unsigned)std::min<int64_t>(8192, (count + 255) / 256);
    k_big_clear<<<grid, 256, 0, s>>>(keys, (u64*)vals, count);
}
void launch_big_insert(const LevelView& L, const BigArgs& a, int64_t nchunks, hipStream_t s) {
    if (nchunks <= 0) return;
    dispatch_types(L.t, [&](auto o, auto w, auto ac) {
        using OffT = typename decltype(o)::type;
        constexpr int WK = decltype(w)::value;
        using AccT = typename decltype(ac)::type;
        Graph<OffT, WK> g{(const OffT*)L.off, L.idx, L.w};
        k_big_insert<OffT, WK, AccT><<<(unsigned)nchunks, 1024, 0, s>>>(g, a);
    });
}
void launch_big_extract(const LevelView& L, const BigArgs& a, hipStream_t s) {
    if (a.nbig <= 0) return;
    const unsigned grid = (unsigned)std::min<int64_t>(BIG_EXTRACT_BLOCKS, a.nbig);
    if (L.t.acc64) k_big_extract<u64><<<grid, 1024, 0, s>>>(a);
    else k_big_extract<uint32_t><<<grid, 1024, 0, s>>>(a);
}

void launch_compact(int64_t ncom, const int64_t* hoff, const int32_t* hidx, const void* hw, const void* goff,
                    int goff64, int32_t* gidx, void* gw, int w64, hipStream_t s) {
    if (ncom <= 0) return;
    const unsigned grid = blocks_for(ncom * 32, 256);
    if (goff64)
        k_compact<int64_t><<<grid, 256, 0, s>>>(ncom, hoff, hidx, hw, (const int64_t*)goff, gidx, gw, w64);
    else
        k_compact<int32_t><<<grid, 256, 0, s>>>(ncom, hoff, hidx, hw, (const int32_t*)goff, gidx, gw, w64);
}

void launch_rowlen_to_offsets(const int32_t* rowlen, int64_t ncom, void* goff, int goff64, void* scratch,
                              hipStream_t s) {
    if (goff64) scan_i32_to_i64(rowlen, (int64_t*)goff, ncom, scratch, s);
    else scan_i32_to_i32(rowlen, (int32_t*)goff, ncom, scratch, s);
}

void launch_modularity_arcs(const LevelView& L0, const int32_t* C, i64* sigin, i64* sigtot, hipStream_t s) {
    if (L0.n <= 0) return;
    LevelTypes t = L0.t;
    t.acc64 = 0;
    dispatch_types(t, [&](auto o, auto w, auto) {
        using OffT = typename decltype(o)::type;
        constexpr int WK = decltype(w)::value;
        Graph<OffT, WK> g{(const OffT*)L0.off, L0.idx, L0.w};
        const unsigned grid = (unsigned)std::min<int64_t>(16384, (L0.n + 3) / 4);
        k_mod_arcs<OffT, WK><<<grid, 256, 0, s>>>(g, L0.n, C, sigin, sigtot);
    });
}

void launch_modularity(const LevelView& L0, const int32_t* C, int64_t ncom, i64 W, i64* sigin, i64* sigtot,
                       Ctl* ctl, hipStream_t s) {
    if (L0.n <= 0) return;
    LevelTypes t = L0.t;
    t.acc64 = 0;
    dispatch_types(t, [&](auto o, auto w, auto) {
        using OffT = typename decltype(o)::type;
        constexpr int WK = decltype(w)::value;
        Graph<OffT, WK> g{(const OffT*)L0.off, L0.idx, L0.w};
        const unsigned grid = (unsigned)std::min<int64_t>(16384, (L0.n + 3) / 4);
        k_mod_arcs<OffT, WK><<<grid, 256, 0, s>>>(g, L0.n, C, sigin, sigtot);
    });
    if (ncom > 0) k_mod_terms<<<blocks_for(ncom, 256), 256, 0, s>>>(ncom, W, sigin, sigtot, ctl);
}

void launch_validate(const LevelView& L, int check, Ctl* ctl, hipStream_t s) {
    if (L.n <= 0) return;
    LevelTypes t = L.t;
    t.acc64 = 0;
    dispatch_types(t, [&](auto o, auto w, auto) {
        using OffT = typename decltype(o)::type;
        constexpr int WK = decltype(w)::value;
        Graph<OffT, WK> g{(const OffT*)L.off, L.idx, L.w};
        const unsigned grid = (unsigned)std::min<int64_t>(16384, (L.n + 3) / 4);
        k_validate<OffT, WK><<<grid, 256, 0, s>>>(g, L.n, L.nnz, check, ctl);
    });
}

}  // namespace lv
