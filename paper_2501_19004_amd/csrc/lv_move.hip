// lv_move.hip -- pass initialisation and the local-moving phase.
//
// Local moving (the paper's Algorithm 2 / Algorithm 5) evaluates each queued
// vertex i: it accumulates K_{i->d}, the weight from i to every neighbouring
// community d (self-loop excluded, as scanCommunities with self = false),
// then picks the community of largest integer gain
//     gain(d) = W*(K_{i->d} - K_{i->c}) - K_i*(Sigma_d - Sigma_c + K_i)
// (Eq. (2) times W^2/2; c = current community, Sigma_c includes K_i),
// ties to the smaller id, and moves when the gain is positive and Pick-Less
// allows it.  Because the term -W*K_{i->c} + K_i*Sigma_c - K_i^2 is common to
// all candidates, the argmax runs over key(d) = W*K_{i->d} - K_i*Sigma_d and
// the gain is key(best) - (W*K_{i->c} - K_i*(Sigma_c - K_i)).
//
// Work layout on gfx950: vertices are split into degree buckets; a bucket is
// processed by groups of G lanes per vertex (G = 8 .. 1024) with a private
// open-addressing table of CAP slots in LDS, or -- above the largest LDS
// bucket -- by one 1024-thread workgroup per vertex with a table in a global
// memory pool.  Pruning flags are per-vertex bytes in two buffers (this
// iteration's queue, the next one's): a mover sets its neighbours' next flags
// with plain byte stores, and the next queue is built by an ordered
// compaction of the flagged vertices (lv_bucket.h).
#include <algorithm>
#include <type_traits>

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

// ---------------------------------------------------------- group reductions
// Reductions over a group of G lanes; for G > 64 the group is the whole
// workgroup and the cross-wave step goes through LDS.
template <int G, typename KeyT>
__device__ __forceinline__ void reduce_best(KeyT& key, int32_t& d, i64& v, KeyT* s_k, int32_t* s_d, i64* s_v) {
    constexpr int GW = G < WAVE ? G : WAVE;
    if constexpr (sizeof(KeyT) == 8) group_best64<GW>(*(i64*)&key, d, v);
    else group_best128<GW>(*(i128*)&key, d, v);
    if constexpr (G > WAVE) {
        const int w = threadIdx.x / WAVE;
        if (threadIdx.x % WAVE == 0) { s_k[w] = key; s_d[w] = d; s_v[w] = v; }
        __syncthreads();
        key = s_k[0];
        d = s_d[0];
        v = s_v[0];
#pragma unroll
        for (int k = 1; k < G / WAVE; k++)
            if (better(s_k[k], s_d[k], key, d)) { key = s_k[k]; d = s_d[k]; v = s_v[k]; }
        __syncthreads();
    }
}
template <int G>
__device__ __forceinline__ i64 reduce_sum(i64 v, i64* s_t) {
    constexpr int GW = G < WAVE ? G : WAVE;
    v = group_sum64<GW>(v);
    if constexpr (G > WAVE) {
        const int w = threadIdx.x / WAVE;
        if (threadIdx.x % WAVE == 0) s_t[w] = v;
        __syncthreads();
        v = 0;
#pragma unroll
        for (int k = 0; k < G / WAVE; k++) v += s_t[k];
        __syncthreads();
    }
    return v;
}
template <int G>
__device__ __forceinline__ i64 reduce_max(i64 v, i64* s_t) {
    constexpr int GW = G < WAVE ? G : WAVE;
    v = group_max64<GW>(v);
    if constexpr (G > WAVE) {
        const int w = threadIdx.x / WAVE;
        if (threadIdx.x % WAVE == 0) s_t[w] = v;
        __syncthreads();
        v = s_t[0];
#pragma unroll
        for (int k = 1; k < G / WAVE; k++) v = s_t[k] > v ? s_t[k] : v;
        __syncthreads();
    }
    return v;
}
// Broadcast lane 0's value to the group.
template <int G>
__device__ __forceinline__ int32_t group_bcast(int32_t v, int32_t* s_x) {
    if constexpr (G <= WAVE) {
        return __shfl(v, 0, G);
    } else {
        if (threadIdx.x == 0) s_x[0] = v;
        __syncthreads();
        v = s_x[0];
        __syncthreads();
        return v;
    }
}

// ------------------------------------------------------------ pass init
// The level's largest weighted degree: one atomic per block whose maximum
// exceeds the value already there (read first), so that millions of blocks do
// not serialise on the one address.
__device__ __forceinline__ void raise_kmax(Ctl* ctl, u64 m) {
    if (m > __hip_atomic_load(&ctl->kmax, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(&ctl->kmax, m);
}

// Degree bucket of every vertex; C' = identity.  K' = Sigma' = 0, to be
// filled by the row sums -- except for unit weights (UNIT), where the row
// sum is the degree and is written here together with its maximum.
template <typename OffT, bool UNIT>
__global__ void __launch_bounds__(256) k_classify(const OffT* __restrict__ off, int64_t n, Buckets B,
                                                  uint8_t* __restrict__ vbucket, int32_t* __restrict__ Cp,
                                                  i64* __restrict__ K, i64* __restrict__ Sig, Ctl* ctl) {
    __shared__ u64 s_max;
    if (UNIT && threadIdx.x == 0) s_max = 0;
    if (UNIT) __syncthreads();
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n) {
        int b = 255;
        const int64_t deg = (int64_t)off[v + 1] - (int64_t)off[v];
        if (deg > 0) {
            b = B.nb;
            for (int k = 0; k < B.nb; k++)
                if (deg <= B.maxdeg[k]) { b = k; break; }
        }
        vbucket[v] = (uint8_t)b;
        Cp[v] = (int32_t)v;
        K[v] = UNIT ? deg : 0;
        Sig[v] = UNIT ? deg : 0;
        if (UNIT && deg > 0) atomicMax(&s_max, (u64)deg);
    }
    if (UNIT) {
        __syncthreads();
        if (threadIdx.x == 0 && s_max) raise_kmax(ctl, s_max);
    }
}

struct VBucket {
    const uint8_t* vb;
    __device__ __forceinline__ int operator()(int64_t v) const { return vb[v]; }
};
struct MarkBucket {
    const uint8_t* vb;
    const uint8_t* flags;
    const int32_t* gid;   // batched runs: only vertices of graphs still moving
    const uint8_t* gact;
    __device__ __forceinline__ int operator()(int64_t v) const {
        return (flags[v] && (!gid || gact[gid[v]])) ? (int)vb[v] : 255;
    }
};

// K'[i] = sum of i's arc weights (self-loop once); Sigma'[i] = K'[i].
template <typename OffT, int WK, int G>
__global__ void __launch_bounds__(G > 256 ? G : 256) k_rowsum(Graph<OffT, WK> g, const int32_t* __restrict__ list,
                                                              int32_t count, i64* __restrict__ K,
                                                              i64* __restrict__ Sig, Ctl* ctl) {
    constexpr int BLOCK = G > 256 ? G : 256;
    constexpr int NG = BLOCK / G;
    static_assert(G <= WAVE || G == BLOCK, "a group is at most one wave or the whole workgroup");
    __shared__ i64 s_t[BLOCK / WAVE];
    __shared__ u64 s_max;
    const int grp = threadIdx.x / G, lane = threadIdx.x % G;
    const int64_t slot = (int64_t)blockIdx.x * NG + grp;
    const bool active = slot < count;
    const int32_t i = active ? list[slot] : 0;
    if (threadIdx.x == 0) s_max = 0;
    __syncthreads();
    i64 s = 0;
    if constexpr (WK == 0) {
        if (active && lane == 0) s = (i64)g.off[i + 1] - (i64)g.off[i];
    } else if (active) {
        for (i64 e = (i64)g.off[i] + lane; e < (i64)g.off[i + 1]; e += G) s += g.weight(e);
    }
    s = reduce_sum<G>(s, s_t);
    if (active && lane == 0) {
        K[i] = s;
        Sig[i] = s;
        atomicMax(&s_max, (u64)s);
    }
    __syncthreads();
    if (threadIdx.x == 0 && s_max) raise_kmax(ctl, s_max);
}

// Static position of each hub and its table capacity: next power of two >=
// 2 * (bound on distinct neighbour communities) = 2 * min(degree, n).
template <typename OffT>
__global__ void k_hub_caps(const OffT* __restrict__ off, int64_t n, const int32_t* __restrict__ list, int32_t count,
                           int64_t* __restrict__ caps, int64_t* __restrict__ nch) {
    const int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= count) return;
    const int32_t v = list[h];
    const int64_t deg = (int64_t)off[v + 1] - (int64_t)off[v];
    const uint64_t want = 2 * (uint64_t)(deg < n ? deg : n);
    uint64_t cap = 1;
    while (cap < want) cap <<= 1;
    caps[h] = (int64_t)cap;
    nch[h] = (deg + HUB_CH - 1) / HUB_CH;
}

// ------------------------------------------------------------ local moving
// Modes: SYNC decides against the iteration's snapshot and records moves;
// ASYNC_CACHED applies moves in place with ordinary (XCD-L2 cached) loads;
// ASYNC_COHERENT does the same with device-scope loads and stores of C' and
// Sigma', so moves made on other chiplets are seen within the launch.
enum { M_SYNC = 0, M_ASYNC_CACHED = 1, M_ASYNC_COHERENT = 2 };

template <int MODE>
__device__ __forceinline__ int32_t ld_c(const int32_t* p) {
    if constexpr (MODE == M_ASYNC_COHERENT) return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else return *p;
}
template <int MODE>
__device__ __forceinline__ i64 ld_s(const i64* p) {
    if constexpr (MODE == M_ASYNC_COHERENT) return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else return *p;
}
template <int MODE>
__device__ __forceinline__ void st_c(int32_t* p, int32_t v) {
    if constexpr (MODE == M_ASYNC_COHERENT) __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else *p = v;
}

struct Decision {
    int32_t target;  // -1: stay
    i64 kid;         // K_{i->target}
    i64 kic;         // K_{i->c}
    i128 gain;       // gain against the state read
    i64 nd;          // distinct neighbour communities
    i64 bestk;       // K_{i->d*} of the best candidate d* (0 without one)
    int32_t positive;  // the best candidate's gain was positive (before Pick-Less)
};

// Best candidate of a group's table: the largest key W*K_{i->d} - K_i*Sigma_d
// over the communities d != c (ties to the smaller d), with K_{i->c} and the
// number of distinct communities.  bd = EMPTY_KEY when there is no candidate.
template <typename KeyT>
struct Best {
    KeyT bk;
    int32_t bd;
    i64 bv, kic, nd;
};

// Scans the table slots owned by this lane (all cap slots, or the nlist slots
// listed in `list`) and reduces over the group; every lane returns the same.
template <int G, int MODE, typename KeyT, typename AccT, typename ListT = int32_t>
__device__ __forceinline__ Best<KeyT> scan_table(const MoveArgs& a, i64 W, const int32_t* keys, const AccT* vals,
                                                 int64_t cap, int lane, int32_t c, i64 Ki, KeyT* s_k, int32_t* s_d,
                                                 i64* s_v, i64* s_t, const ListT* list, int64_t nlist) {
    KeyT bk = 0;
    int32_t bd = EMPTY_KEY;
    i64 bv = 0, kic = 0, nd = 0;
    const int64_t span = list ? nlist : cap;
    // U slots per round: their Sigma gathers are issued together.
    constexpr int U = 4;
    for (int64_t k0 = lane; k0 < span; k0 += U * G) {
        int32_t dd[U];
        i64 vv[U], ss[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int64_t k = k0 + (int64_t)u * G;
            dd[u] = EMPTY_KEY;
            vv[u] = 0;
            if (k < span) {
                const int64_t s = list ? (int64_t)list[k] : k;
                dd[u] = keys[s];
                vv[u] = (i64)vals[s];
            }
        }
#pragma unroll
        for (int u = 0; u < U; u++) ss[u] = (dd[u] != EMPTY_KEY && dd[u] != c) ? ld_s<MODE>(&a.Sig[dd[u]]) : 0;
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int32_t d = dd[u];
            if (d == EMPTY_KEY) continue;
            ++nd;
            if (d == c) { kic = vv[u]; continue; }
            const KeyT key = (KeyT)W * vv[u] - (KeyT)Ki * ss[u];
            if (bd == EMPTY_KEY || better(key, d, bk, bd)) { bk = key; bd = d; bv = vv[u]; }
        }
    }
    // Lanes without a candidate must not win: give them the smallest key.
    if (bd == EMPTY_KEY) bk = (sizeof(KeyT) == 8) ? (KeyT)INT64_MIN : (KeyT)(((i128)1) << 127);
    reduce_best<G, KeyT>(bk, bd, bv, s_k, s_d, s_v);
    kic = reduce_max<G>(kic, s_t);
    nd = reduce_sum<G>(nd, s_t);
    return Best<KeyT>{bk, bd, bd != EMPTY_KEY ? bv : 0, kic, nd};
}

// The move of vertex i (community c) from its best candidate: the gain
// against staying, Pick-Less, and (concurrent modes) the minimum-label rule.
template <int MODE, typename KeyT>
__device__ __forceinline__ Decision finish_decision(const MoveArgs& a, i64 W, bool active, int32_t i, int32_t c,
                                                    i64 Ki, const Best<KeyT>& b, i64 Sc) {
    Decision r{-1, 0, b.kic, 0, b.nd, b.bd != EMPTY_KEY ? b.bv : 0, 0};
    if (active && b.bd != EMPTY_KEY) {
        const KeyT stay = (KeyT)W * b.kic - (KeyT)Ki * (Sc - Ki);
        const KeyT gk = b.bk - stay;
        r.positive = gk > 0;
        bool ok = gk > 0 && (!a.pl || b.bd < c);
        if constexpr (MODE != M_SYNC) {
            // a positive move refused by Pick-Less is still pending: i stays
            // queued for the next iteration, as a mover's neighbours are
            if (gk > 0 && !ok && a.prune) a.fnext[i] = 1;
            // i alone in c, d a single-vertex community of larger id: let d's vertex come to c instead
            if (ok && a.min_label && b.bd > c && Sc == Ki && ld_c<MODE>(&a.Cp[b.bd]) == b.bd &&
                ld_s<MODE>(&a.Sig[b.bd]) == a.K[b.bd])
                ok = false;
        }
        if (ok) { r.target = b.bd; r.kid = b.bv; r.gain = (i128)gk; }
    }
    return r;
}

// Per-group decision after the table is filled (Sc: Sigma of c as read);
// list/nlist: the table's occupied slots.
template <int G, int MODE, typename KeyT, typename AccT>
__device__ __forceinline__ Decision decide(const MoveArgs& a, i64 W, const int32_t* keys, const AccT* vals, int64_t cap,
                                           int lane, bool active, int32_t c, i64 Ki, i64 Sc, KeyT* s_k, int32_t* s_d,
                                           i64* s_v, i64* s_t, const uint16_t* list, int64_t nlist, int32_t i) {
    const Best<KeyT> b = scan_table<G, MODE, KeyT, AccT, uint16_t>(a, W, keys, vals, cap, lane, c, Ki, s_k, s_d, s_v,
                                                                   s_t, list, nlist);
    return finish_decision<MODE, KeyT>(a, W, active, i, c, Ki, b, Sc);
}

// ASYNC move with validation: Sigma of the target is updated by an atomic
// add whose return value is the exact total before this vertex joins; the
// gain is recomputed from that value and the current Sigma_c, and the move is
// undone if it is no longer positive.  Concurrent joins of one community are
// therefore each checked against the community as it really is.
template <int MODE>
__device__ __forceinline__ bool apply_async(const MoveArgs& a, i64 W, int32_t i, int32_t c, i64 Ki, Decision& dcs) {
    const i64 old_d = (i64)atomicAdd((u64*)&a.Sig[dcs.target], (u64)Ki);
    const i64 Sc = ld_s<MODE>(&a.Sig[c]);
    const i128 g = (i128)W * (dcs.kid - dcs.kic) - (i128)Ki * ((i128)old_d - Sc + Ki);
    if (g > 0) {
        atomicAdd((u64*)&a.Sig[c], (u64)(-Ki));
        st_c<MODE>(&a.Cp[i], dcs.target);
        if (a.learn) a.f_moved[i] = a.itag;
        dcs.gain = g;
        return true;
    }
    atomicAdd((u64*)&a.Sig[dcs.target], (u64)(-Ki));
    dcs.target = -1;
    dcs.gain = 0;
    return false;
}

// Stamp the neighbours of mover i for the next iteration's queue (pruning)
// and count i among their moved neighbours (learned-pruner features).
__device__ __forceinline__ void mark_one(const MoveArgs& a, int32_t i, int32_t j) {
    if (j == i) return;
    if (a.prune) a.fnext[j] = 1;
    if (a.learn) atomicAdd(&a.f_nm[j], 1);
}
template <int G, typename OffT, int WK>
__device__ __forceinline__ void mark_neighbours(const MoveArgs& a, const Graph<OffT, WK>& g, int32_t i, i64 o0,
                                                i64 o1, int lane) {
    for (i64 e = o0 + lane; e < o1; e += G) mark_one(a, i, g.idx[e]);
}

// Feature state of an evaluated vertex: its own-community weight and the
// best candidate's advantage over it.
__device__ __forceinline__ void note_evaluation(const MoveArgs& a, int32_t i, const Decision& d) {
    a.f_own[i] = d.kic;
    a.f_adv[i] = d.bestk - d.kic;
}

// Block totals into the striped counters; no atomic here waits for its
// result, so the block retires as soon as they are issued.
__device__ __forceinline__ void add_block_totals_split(Ctl* ctl, int bucket, u64 ne, u64 na, u64 nd, u64 nm, u64 nma,
                                                       const Split128& gain, u64 npos) {
    const int st = blockIdx.x & (STRIPES - 1);
    if (!ne) return;
    if (npos) atomicAdd(&ctl->positive[st], npos);
    atomicAdd(&ctl->bstat[0][bucket][st], ne);
    atomicAdd(&ctl->bstat[1][bucket][st], na);
    atomicAdd(&ctl->bstat[2][bucket][st], nd);
    if (nm) {
        if (gain.lo) atomicAdd(&ctl->s_lo[st], gain.lo);
        if (gain.mid) atomicAdd(&ctl->s_mid[st], gain.mid);
        if (gain.hi) atomicAdd(&ctl->s_hi[st], gain.hi);
        atomicAdd(&ctl->moves[st], nm);
        atomicAdd(&ctl->bstat[3][bucket][st], nm);
        atomicAdd(&ctl->bstat[4][bucket][st], nma);
    }
}
__device__ __forceinline__ void add_block_totals(Ctl* ctl, int bucket, u64 ne, u64 na, u64 nd, u64 nm, u64 nma,
                                                 i128 gain, u64 npos) {
    add_block_totals_split(ctl, bucket, ne, na, nd, nm, nma, split128(gain), npos);
}

// Block-level scratch shared by every local-moving path (sized for the
// largest block, 1024 threads, and the most groups per block, 32).
struct MoveShm {
    i128 k128[16];
    i64 k64[16];
    int32_t d[16];
    i64 v[16];
    i64 t[16];
    int32_t x[1];
    i128 gain[32];
    int32_t dec[32];
    int32_t pos[32];
    int32_t gi[32];
    int32_t ncl[32];  // occupied slots listed per group
    i64 arcs[32], nd[32];
    u64 wsum[256 / WAVE][9];  // lane path: per-wave partial block totals
};

// Queue entry of work slot `slot` of a launch: the slot-th entry of the
// launch's list (strided for interleaved slices), or, for batched ASYNC
// slices, the entry of the slot's graph segment.
__device__ __forceinline__ int64_t queue_entry(const MoveArgs& a, int64_t slot) {
    int64_t e = slot * a.lstride + a.lphase;
    if (a.seg_pre) {
        int32_t lo = 0, hi = a.seg_n - 1;  // graph of this slot: largest g with seg_pre[g] <= slot
        while (lo < hi) {
            const int32_t mid = (lo + hi + 1) >> 1;
            if (a.seg_pre[mid] <= slot) lo = mid; else hi = mid - 1;
        }
        const int64_t len = a.seg_cnt[lo];
        e = a.seg_start[lo] + len * a.seg_k / a.seg_ns + (slot - a.seg_pre[lo]);
    }
    return e;
}

// Device-driven iterations: this launch's share of bucket b's queue (list is
// the queue's base on entry); false once the pass has ended.
__device__ __forceinline__ bool dev_share(const MoveArgs& a, const int32_t* seg_pre, int b, const int32_t*& list,
                                          int32_t& count) {
    if (a.dit->halt) return false;
    if (seg_pre) {  // batched slices: the slice's slots over all graphs
        list += a.dit->seg[b];
        count = seg_pre[a.seg_n];
        return true;
    }
    const int32_t* e = a.dshare + 2 * (a.slice * NB_MOVE + b);
    list += e[0];
    count = e[1];
    return true;
}

// One block of a degree bucket: NG = BLOCK/G vertices, each evaluated by G
// lanes with a CAP-slot table in LDS (keys/vals point at this block's LDS).
template <typename OffT, int WK, typename AccT, int G, int CAP, int MODE, bool WIDE>
__device__ __forceinline__ void move_block(const MoveArgs& a, const int32_t* __restrict__ list, int32_t count,
                                           int64_t blk, int bucket, int32_t* s_keys, AccT* s_vals, uint16_t* s_list,
                                           MoveShm& sh) {
    constexpr int BLOCK = G > 256 ? G : 256;
    constexpr int NG = BLOCK / G;
    constexpr int L2C = Log2<CAP>::v;
    // group reductions work inside one wave or over the whole workgroup, and
    // the per-group slots of MoveShm hold 32 groups
    static_assert(G <= WAVE || G == BLOCK, "a group is at most one wave or the whole workgroup");
    static_assert(NG <= 32, "MoveShm holds 32 groups per block");
    static_assert(CAP <= 65536, "slot lists hold 16-bit slot numbers");
    const Graph<OffT, WK> g{(const OffT*)a.off, a.idx, a.w};
    const int grp = threadIdx.x / G, lane = threadIdx.x % G;
    const int64_t slot = blk * NG + grp;
    const bool listed = slot < count;
    const int32_t i = listed ? list[queue_entry(a, slot)] : -1;
    const int32_t gi = (listed && a.gid) ? a.gid[i] : -1;  // batched runs: graph of i
    const bool active = listed && (gi < 0 || a.gact[gi]);
    const i64 Wi = gi >= 0 ? (i64)a.Wg[gi] : a.W;
    int32_t* keys = s_keys + grp * CAP;
    AccT* vals = s_vals + grp * CAP;
    uint16_t* occ = s_list + grp * (CAP / 2);  // distinct keys <= degree <= CAP / 2
    for (int s = lane; s < CAP; s += G) { keys[s] = EMPTY_KEY; vals[s] = 0; }
    if (lane == 0) sh.ncl[grp] = 0;
    group_sync<G>();

    int32_t c = 0;
    i64 Ki = 0, o0 = 0, o1 = 0, Sc = 0;
    if (active) {
        c = ld_c<MODE>(&a.Cp[i]);
        Ki = a.K[i];
        o0 = (i64)g.off[i];
        o1 = (i64)g.off[i + 1];
        Sc = ld_s<MODE>(&a.Sig[c]);  // in flight while the row is read
    }
    // U arcs per round: their index loads, then their C' gathers, are issued
    // together.  The first round's neighbours stay in registers: when the row
    // fits in one round they are flagged from there if the vertex moves.
    constexpr int U = 4;
    int32_t j0[U];
#pragma unroll
    for (int u = 0; u < U; u++) j0[u] = i;
    for (i64 e0 = o0 + lane; e0 < o1; e0 += U * G) {
        int32_t jj[U], dd[U];
        AccT ww[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
            const i64 e = e0 + (i64)u * G;
            jj[u] = e < o1 ? g.idx[e] : i;
            ww[u] = e < o1 ? (AccT)g.weight(e) : (AccT)0;
        }
        if (e0 == o0 + lane) {
#pragma unroll
            for (int u = 0; u < U; u++) j0[u] = jj[u];
        }
#pragma unroll
        for (int u = 0; u < U; u++) dd[u] = jj[u] != i ? ld_c<MODE>(&a.Cp[jj[u]]) : EMPTY_KEY;
#pragma unroll
        for (int u = 0; u < U; u++) {
            if (dd[u] == EMPTY_KEY) continue;
            const int64_t got = table_add_claim<AccT>(keys, vals, CAP - 1, hash_slot<L2C>(dd[u]), dd[u], ww[u]);
            if (got >= 0) occ[atomicAdd(&sh.ncl[grp], 1)] = (uint16_t)got;
        }
    }
    group_sync<G>();
    const int32_t nocc = sh.ncl[grp];

    Decision dcs;
    if constexpr (!WIDE)
        dcs = decide<G, MODE, i64, AccT>(a, Wi, keys, vals, CAP, lane, active, c, Ki, Sc, sh.k64, sh.d, sh.v, sh.t,
                                         occ, nocc, i);
    else
        dcs = decide<G, MODE, i128, AccT>(a, Wi, keys, vals, CAP, lane, active, c, Ki, Sc, sh.k128, sh.d, sh.v, sh.t,
                                          occ, nocc, i);

    if (a.learn && active && lane == 0) note_evaluation(a, i, dcs);
    if constexpr (MODE == M_SYNC) {
        if (lane == 0 && listed) a.sdec[i] = dcs.target;  // -1 for a vertex of a graph that has converged
    } else {
        int32_t t = -1;
        if (lane == 0 && dcs.target >= 0 && apply_async<MODE>(a, Wi, i, c, Ki, dcs)) t = dcs.target;
        t = group_bcast<G>(t, sh.x);
        if ((a.prune || a.learn) && t >= 0) {
            if (o1 - o0 <= (i64)U * G) {
#pragma unroll
                for (int u = 0; u < U; u++) mark_one(a, i, j0[u]);
            } else {
                mark_neighbours<G>(a, g, i, o0, o1, lane);
            }
        }
    }
    if (lane == 0) {
        sh.gain[grp] = dcs.gain;
        sh.dec[grp] = dcs.target;
        sh.pos[grp] = active ? dcs.positive : 0;
        sh.gi[grp] = gi;
        sh.arcs[grp] = active ? (o1 - o0) : -1;
        sh.nd[grp] = dcs.nd;
    }
    __syncthreads();
    if (!a.Sg) {
        // block totals: wave 0 reduces the NG group results in parallel
        if (threadIdx.x < WAVE) {
            const int k = threadIdx.x;
            i64 ne = 0, na = 0, ndt = 0, nm = 0, nma = 0, np = 0;
            Split128 sp{0, 0, 0};
            if (k < NG && sh.arcs[k] >= 0) {
                ne = 1;
                na = sh.arcs[k];
                ndt = sh.nd[k];
                np = sh.pos[k];
                if (sh.dec[k] >= 0) {
                    nm = 1;
                    nma = sh.arcs[k];
                    sp = split128(sh.gain[k]);
                }
            }
            if constexpr (NG > 1) {
                ne = group_sum64<WAVE>(ne);
                na = group_sum64<WAVE>(na);
                ndt = group_sum64<WAVE>(ndt);
                nm = group_sum64<WAVE>(nm);
                nma = group_sum64<WAVE>(nma);
                np = group_sum64<WAVE>(np);
                sp.lo = (u64)group_sum64<WAVE>((i64)sp.lo);
                sp.mid = (u64)group_sum64<WAVE>((i64)sp.mid);
                sp.hi = (u64)group_sum64<WAVE>((i64)sp.hi);
            }
            if (k == 0)
                add_block_totals_split(a.ctl, bucket, (u64)ne, (u64)na, (u64)ndt, (u64)nm, (u64)nma, sp, (u64)np);
        }
    } else if (threadIdx.x == 0) {
        i128 sg = 0;
        u64 nm = 0, ne = 0, na = 0, ndt = 0, nma = 0, np = 0;
        for (int k = 0; k < NG; k++) {
            if (sh.arcs[k] < 0) continue;
            ne++;
            na += (u64)sh.arcs[k];
            ndt += (u64)sh.nd[k];
            np += (u64)sh.pos[k];
            if (sh.dec[k] >= 0) { sg += sh.gain[k]; nm++; nma += (u64)sh.arcs[k]; }
        }
        add_block_totals(a.ctl, bucket, ne, na, ndt, nm, nma, sg, np);
        // per-graph gain sums, one 128-bit atomic per run of equal graph id
        int32_t cur = -1;
        i128 acc = 0;
        for (int k = 0; k < NG; k++) {
            if (sh.arcs[k] < 0 || sh.dec[k] < 0) continue;
            if (sh.gi[k] != cur) {
                if (cur >= 0 && acc != 0) atomic_add_i128(&a.Sg[2 * cur], &a.Sg[2 * cur + 1], acc);
                cur = sh.gi[k];
                acc = 0;
            }
            acc += sh.gain[k];
        }
        if (cur >= 0 && acc != 0) atomic_add_i128(&a.Sg[2 * cur], &a.Sg[2 * cur + 1], acc);
        if (a.Pg) {
            // per-graph positive-gain evaluations, one atomic per run of equal graph id
            int32_t gcur = -1;
            u64 pos = 0;
            for (int k = 0; k < NG; k++) {
                if (sh.arcs[k] < 0 || !sh.pos[k]) continue;
                if (sh.gi[k] != gcur) {
                    if (gcur >= 0 && pos) atomicAdd(&a.Pg[gcur], pos);
                    gcur = sh.gi[k];
                    pos = 0;
                }
                pos++;
            }
            if (gcur >= 0 && pos) atomicAdd(&a.Pg[gcur], pos);
        }
    }
}

// Bucket 0: one vertex per lane, 256 per block.  A row of at most D = LANE_DEG
// arcs stays in registers: K_{i->d} of each distinct neighbour community is
// the sum over the row's entries of that community, found by comparing the
// entries pairwise (D^2 register compares, no table, no barrier), and the
// Sigma of each distinct candidate is gathered once.  The decision rule is the
// groups' (finish_decision), so both paths pick the same community.
constexpr int LANE_DEG = MOVE_CAP[0] / 2;

template <typename OffT, int WK, int MODE, typename KeyT>
__device__ __forceinline__ void move_lanes(const MoveArgs& a, const int32_t* __restrict__ list, int32_t count,
                                           int64_t blk, int bucket, MoveShm& sh) {
    constexpr int D = LANE_DEG;
    const Graph<OffT, WK> g{(const OffT*)a.off, a.idx, a.w};
    const int64_t slot = blk * 256 + threadIdx.x;
    const bool listed = slot < count;
    const int32_t i = listed ? list[queue_entry(a, slot)] : -1;
    const int32_t gi = (listed && a.gid) ? a.gid[i] : -1;  // batched runs: graph of i
    const bool active = listed && (gi < 0 || a.gact[gi]);
    const i64 Wi = gi >= 0 ? (i64)a.Wg[gi] : a.W;
    int32_t c = 0;
    i64 Ki = 0, o0 = 0, Sc = 0;
    int deg = 0;
    if (active) {
        c = ld_c<MODE>(&a.Cp[i]);
        Ki = a.K[i];
        o0 = (i64)g.off[i];
        deg = (int)((i64)g.off[i + 1] - o0);
        Sc = ld_s<MODE>(&a.Sig[c]);  // in flight while the row is read
    }
    int32_t jj[D], dd[D];
    i64 ww[D];
#pragma unroll
    for (int u = 0; u < D; u++) {
        jj[u] = u < deg ? g.idx[o0 + u] : i;
        ww[u] = u < deg ? g.weight(o0 + u) : 0;
    }
#pragma unroll
    for (int u = 0; u < D; u++) dd[u] = jj[u] != i ? ld_c<MODE>(&a.Cp[jj[u]]) : EMPTY_KEY;
    // kd[u]: weight from i to community dd[u]; first[u]: u is that community's first entry
    i64 kd[D];
    bool first[D];
#pragma unroll
    for (int u = 0; u < D; u++) {
        i64 sum = 0;
        bool f = dd[u] != EMPTY_KEY;
#pragma unroll
        for (int v = 0; v < D; v++) {
            const bool same = dd[v] == dd[u];
            sum += same ? ww[v] : 0;
            if (v < u && same) f = false;
        }
        kd[u] = sum;
        first[u] = f;
    }
    i64 kic = 0, nd = 0;
#pragma unroll
    for (int u = 0; u < D; u++) {
        nd += first[u] ? 1 : 0;
        if (first[u] && dd[u] == c) kic = kd[u];
    }
    i64 sd[D];
#pragma unroll
    for (int u = 0; u < D; u++) sd[u] = (first[u] && dd[u] != c) ? ld_s<MODE>(&a.Sig[dd[u]]) : 0;
    KeyT bk = 0;
    int32_t bd = EMPTY_KEY;
    i64 bv = 0;
#pragma unroll
    for (int u = 0; u < D; u++) {
        if (!first[u] || dd[u] == c) continue;
        const KeyT key = (KeyT)Wi * kd[u] - (KeyT)Ki * sd[u];
        if (bd == EMPTY_KEY || better(key, dd[u], bk, bd)) { bk = key; bd = dd[u]; bv = kd[u]; }
    }
    Decision dcs = finish_decision<MODE, KeyT>(a, Wi, active, i, c, Ki, Best<KeyT>{bk, bd, bv, kic, nd}, Sc);

    if (a.learn && active) note_evaluation(a, i, dcs);
    if constexpr (MODE == M_SYNC) {
        if (listed) a.sdec[i] = dcs.target;  // -1 for a vertex of a graph that has converged
    } else if (dcs.target >= 0 && apply_async<MODE>(a, Wi, i, c, Ki, dcs) && (a.prune || a.learn)) {
#pragma unroll
        for (int u = 0; u < D; u++)
            if (u < deg) mark_one(a, i, jj[u]);
    }
    // batched runs: per-graph gain sums and positive-gain counts, per lane
    if (a.Sg && active && dcs.target >= 0 && dcs.gain != 0)
        atomic_add_i128(&a.Sg[2 * gi], &a.Sg[2 * gi + 1], dcs.gain);
    if (a.Pg && active && dcs.positive) atomicAdd(&a.Pg[gi], 1ull);
    // block totals: wave sums, then one lane adds the block's
    const bool moved = active && dcs.target >= 0;
    const Split128 sp = moved ? split128(dcs.gain) : Split128{0, 0, 0};
    u64 v9[9] = {active ? 1ull : 0ull, active ? (u64)deg : 0ull, active ? (u64)nd : 0ull, moved ? 1ull : 0ull,
                 moved ? (u64)deg : 0ull, (active && dcs.positive) ? 1ull : 0ull, sp.lo, sp.mid, sp.hi};
    const int w = threadIdx.x / WAVE;
#pragma unroll
    for (int q = 0; q < 9; q++) v9[q] = (u64)group_sum64<WAVE>((i64)v9[q]);
    if (threadIdx.x % WAVE == 0) {
#pragma unroll
        for (int q = 0; q < 9; q++) sh.wsum[w][q] = v9[q];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        u64 t[9] = {};
        for (int k = 0; k < 256 / WAVE; k++)
#pragma unroll
            for (int q = 0; q < 9; q++) t[q] += sh.wsum[k][q];
        add_block_totals_split(a.ctl, bucket, t[0], t[1], t[2], t[3], t[4], Split128{t[6], t[7], t[8]}, t[5]);
    }
}

// WIDE: 128-bit gain arithmetic (W * max K >= 2^62); a separate instantiation
// so that the common 64-bit kernels keep their register count.
template <typename OffT, int WK, typename AccT, int G, int CAP, int MODE, bool WIDE>
__global__ void __launch_bounds__(G > 256 ? G : 256) k_move_lds(MoveArgs a, const int32_t* __restrict__ list,
                                                                int32_t count) {
    constexpr int NG = (G > 256 ? G : 256) / G;
    const int32_t* lst = list;
    if (a.dit && (!dev_share(a, a.seg_pre, a.bucket, lst, count) || (int64_t)blockIdx.x * NG >= count)) return;
    __shared__ int32_t s_keys[NG * CAP];
    __shared__ AccT s_vals[NG * CAP];
    __shared__ uint16_t s_list[NG * CAP / 2];
    __shared__ MoveShm sh;
    move_block<OffT, WK, AccT, G, CAP, MODE, WIDE>(a, lst, count, blockIdx.x, a.bucket, s_keys, s_vals, s_list,
                                                   sh);
}

// Buckets 0..3 (all 256-thread blocks) in one launch: block ranges
// [blk_pre[b], blk_pre[b+1]) belong to bucket b; the tables live in dynamic
// LDS sized for the largest of the four.
// Six waves per SIMD fit the unit-weight 64-bit variants in registers (the
// default allocation leaves five); weighted variants would spill to scratch
// memory at six (the weighted 4096^2 grid runs 22% faster at five), so they
// and the 128-bit variants keep the compiler's choice.
template <typename OffT, int WK, typename AccT, int MODE, bool WIDE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu((WIDE || WK != 0) ? 1 : 6, 8)))
k_move_fused(MoveArgs a, FusedLists f) {
    extern __shared__ __align__(16) char dyn[];
    __shared__ MoveShm sh;
    const int64_t b = (int64_t)blockIdx.x;
    int bk = 0;
    while (bk < 3 && b >= f.blk_pre[bk + 1]) bk++;
    const int64_t blk = b - f.blk_pre[bk];
    MoveArgs aa = a;
    aa.seg_pre = f.seg_pre[bk];
    aa.seg_start = f.seg_start[bk];
    aa.seg_cnt = f.seg_cnt[bk];
    const int32_t* list = f.list[bk];
    int32_t count = f.count[bk];
    if (a.dit) {  // device-driven: blocks beyond the true share leave at once
        const int ng = bk == 0 ? 256 / MOVE_G[0] : bk == 1 ? 256 / MOVE_G[1] : bk == 2 ? 256 / MOVE_G[2]
                                                                                     : 256 / MOVE_G[3];
        if (!dev_share(a, f.seg_pre[bk], bk, list, count) || blk * ng >= count) return;
    }
    switch (bk) {
        case 0: {
            static_assert(MOVE_G[0] == 1, "bucket 0 is the lane-per-vertex path");
            using KeyT = typename std::conditional<WIDE, i128, i64>::type;
            move_lanes<OffT, WK, MODE, KeyT>(aa, list, count, blk, 0, sh);
            break;
        }
        case 1: {
            constexpr int NG = 256 / MOVE_G[1];
            constexpr int TB = NG * MOVE_CAP[1];
            move_block<OffT, WK, AccT, MOVE_G[1], MOVE_CAP[1], MODE, WIDE>(
                aa, list, count, blk, 1, (int32_t*)dyn, (AccT*)(dyn + TB * 4),
                (uint16_t*)(dyn + TB * (4 + sizeof(AccT))), sh);
            break;
        }
        case 2: {
            constexpr int NG = 256 / MOVE_G[2];
            constexpr int TB = NG * MOVE_CAP[2];
            move_block<OffT, WK, AccT, MOVE_G[2], MOVE_CAP[2], MODE, WIDE>(
                aa, list, count, blk, 2, (int32_t*)dyn, (AccT*)(dyn + TB * 4),
                (uint16_t*)(dyn + TB * (4 + sizeof(AccT))), sh);
            break;
        }
        default: {
            constexpr int NG = 256 / MOVE_G[3];
            constexpr int TB = NG * MOVE_CAP[3];
            move_block<OffT, WK, AccT, MOVE_G[3], MOVE_CAP[3], MODE, WIDE>(
                aa, list, count, blk, 3, (int32_t*)dyn, (AccT*)(dyn + TB * 4),
                (uint16_t*)(dyn + TB * (4 + sizeof(AccT))), sh);
            break;
        }
    }
}

// ------------------------------------------------------------ hubs
// Vertices above the largest LDS bucket are processed once per iteration,
// before the other buckets, by three launches: (1) chunks of HUB_CH arcs,
// one workgroup each, accumulate K_{i->d} in an LDS table and add it into the
// hub's global table; (2) one workgroup per hub scans its table, decides and
// (ASYNC) applies the move, then clears the table; (3) chunks of the movers'
// rows flag their neighbours.  Queued hubs: all in a sweep (the first
// iteration of a pass, or without pruning), else those flagged by the
// previous iteration.
__device__ __forceinline__ bool hub_queued(const MoveArgs& a, int32_t v) {
    return (a.all_queued || a.fcur[v]) && (!a.gid || a.gact[a.gid[v]]);
}
// largest h in [0, n) with pre[h] - base <= x
__device__ __forceinline__ int32_t owner_of(const int64_t* pre, int32_t n, int64_t base, int64_t x) {
    int32_t lo = 0, hi = n - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (pre[mid] - base <= x) lo = mid; else hi = mid - 1;
    }
    return lo;
}

template <typename OffT, int WK, typename AccT, int MODE>
__global__ void __launch_bounds__(1024) k_hub_insert(MoveArgs a) {
    if (a.dit && a.dit->halt) return;
    constexpr int G = 1024;
    constexpr int L2C = Log2<HUB_LCAP>::v;
    constexpr int PER = HUB_LCAP / G;
    __shared__ int32_t s_keys[HUB_LCAP];
    __shared__ AccT s_vals[HUB_LCAP];
    __shared__ int32_t s_claim[2];  // claimed global slots of this block, their base in the hub's list
    const Graph<OffT, WK> g{(const OffT*)a.off, a.idx, a.w};
    const int32_t ng = a.g_hi - a.g_lo;
    const int64_t chunk_base = a.hch_pre[a.g_lo];
    const int32_t h = a.g_lo + owner_of(a.hch_pre + a.g_lo, ng, chunk_base, blockIdx.x);
    const int32_t v = a.hub_list[h];
    if (!hub_queued(a, v)) return;  // uniform per block
    const int tid = threadIdx.x;
    const int64_t k = (int64_t)blockIdx.x - (a.hch_pre[h] - chunk_base);
    const i64 e0 = (i64)g.off[v] + k * HUB_CH;
    const i64 e1 = min(e0 + (i64)HUB_CH, (i64)g.off[v + 1]);
    for (int s = tid; s < HUB_LCAP; s += G) { s_keys[s] = EMPTY_KEY; s_vals[s] = 0; }
    if (tid == 0) s_claim[0] = 0;
    __syncthreads();
    // U arcs per round: their index loads, then their C' gathers, are issued together.
    constexpr int U = 4;
    for (i64 eb = e0 + tid; eb < e1; eb += U * G) {
        int32_t jj[U], dd[U];
        AccT ww[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
            const i64 e = eb + (i64)u * G;
            jj[u] = e < e1 ? g.idx[e] : v;
            ww[u] = e < e1 ? (AccT)g.weight(e) : (AccT)0;
        }
#pragma unroll
        for (int u = 0; u < U; u++) dd[u] = jj[u] != v ? ld_c<MODE>(&a.Cp[jj[u]]) : EMPTY_KEY;
#pragma unroll
        for (int u = 0; u < U; u++)
            if (dd[u] != EMPTY_KEY) table_add<AccT>(s_keys, s_vals, HUB_LCAP - 1, hash_slot<L2C>(dd[u]), dd[u], ww[u]);
    }
    __syncthreads();
    const int64_t toff = a.hub_pre[h] - a.hub_pre[a.tab_lo];
    const int64_t cap = a.hub_pre[h + 1] - a.hub_pre[h];
    const int log2cap = __ffsll((long long)cap) - 1;
    const uint32_t mask = (uint32_t)(cap - 1);
    int32_t* keys = a.hub_keys + toff;
    AccT* vals = (AccT*)a.hub_vals + toff;
    int32_t* slots = a.hub_slots + toff / 2;  // cap >= 2 * distinct keys, so cap / 2 list entries suffice
    // Merge into the hub's table: the first probes of all of this thread's
    // keys are issued together; a key whose home slot holds another key
    // continues along its probe sequence.
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
    const int mine = nclaim ? atomicAdd(&s_claim[0], nclaim) : 0;
    __syncthreads();
    if (tid == 0) s_claim[1] = s_claim[0] ? atomicAdd(&a.hub_cnt[h], s_claim[0]) : 0;
    __syncthreads();
    if (nclaim) {
        int32_t p = s_claim[1] + mine;
#pragma unroll
        for (int u = 0; u < PER; u++)
            if (got[u] >= 0) slots[p++] = (int32_t)got[u];
    }
}

// Decision of a hub: the hub's occupied slots are split evenly over as many
// blocks as it has insert chunks.  Each block scans its share (gathering
// Sigma of every candidate) and clears it.  A hub with one block decides at
// once; otherwise each block posts a partial best and k_hub_final, launched
// next, combines them (the kernel boundary makes the partials visible on
// every chiplet without fences inside the launch).
template <int MODE, typename KeyT>
__device__ __forceinline__ void hub_finish(const MoveArgs& a, int32_t h, int32_t v, i64 deg, const Best<KeyT>& b,
                                           int lane) {
    const int32_t c = ld_c<MODE>(&a.Cp[v]);
    const i64 Ki = a.K[v];
    const int32_t gv = a.gid ? a.gid[v] : -1;
    const i64 Wv = gv >= 0 ? (i64)a.Wg[gv] : a.W;
    Decision dcs = finish_decision<MODE, KeyT>(a, Wv, true, v, c, Ki, b, ld_s<MODE>(&a.Sig[c]));
    if (lane == 0) {
        a.hub_cnt[h] = 0;
        if constexpr (MODE == M_SYNC) {
            a.sdec[v] = dcs.target;
        } else {
            if (dcs.target >= 0) apply_async<MODE>(a, Wv, v, c, Ki, dcs);
        }
        if (a.Sg && dcs.target >= 0) atomic_add_i128(&a.Sg[2 * gv], &a.Sg[2 * gv + 1], dcs.gain);
        if (a.Pg && dcs.positive) atomicAdd(&a.Pg[gv], 1ull);
        if (a.learn) note_evaluation(a, v, dcs);
        a.gdec[h] = dcs.target;
        add_block_totals(a.ctl, a.bucket, 1, (u64)deg, (u64)dcs.nd, dcs.target >= 0 ? 1 : 0,
                         dcs.target >= 0 ? (u64)deg : 0, dcs.gain, (u64)dcs.positive);
    }
}

template <int MODE, typename KeyT, typename AccT, typename OffT>
__device__ __forceinline__ void hub_decide_block(const MoveArgs& a, int32_t h, int32_t v, int64_t k, int64_t nch,
                                                 KeyT* s_k, int32_t* s_d, i64* s_v, i64* s_t) {
    constexpr int G = 1024;
    const OffT* off = (const OffT*)a.off;
    const int tid = threadIdx.x;
    const int64_t toff = a.hub_pre[h] - a.hub_pre[a.tab_lo];
    const int64_t cap = a.hub_pre[h + 1] - a.hub_pre[h];
    int32_t* keys = a.hub_keys + toff;
    AccT* vals = (AccT*)a.hub_vals + toff;
    const int32_t* slots = a.hub_slots + toff / 2;
    const int64_t nocc = a.hub_cnt[h];
    const int32_t c = ld_c<MODE>(&a.Cp[v]);
    const i64 Ki = a.K[v];
    const int32_t gv = a.gid ? a.gid[v] : -1;
    const i64 Wv = gv >= 0 ? (i64)a.Wg[gv] : a.W;
    Best<KeyT> b;
    if (nocc * 8 >= cap) {
        // a well-filled table (at least 1/8 occupied, as after the first
        // iteration of a pass): scan this block's share of the slots in order,
        // with coalesced loads, and clear it with coalesced stores
        const int64_t t0 = cap * k / nch, t1 = cap * (k + 1) / nch;
        b = scan_table<G, MODE, KeyT, AccT>(a, Wv, keys + t0, vals + t0, t1 - t0, tid, c, Ki, s_k, s_d, s_v, s_t,
                                            (const int32_t*)nullptr, 0);
        for (int64_t x = t0 + tid; x < t1; x += G) {
            keys[x] = EMPTY_KEY;
            vals[x] = 0;
        }
    } else {
        // a sparse table: only the listed occupied slots
        const int64_t lo = nocc * k / nch, hi = nocc * (k + 1) / nch;
        b = scan_table<G, MODE, KeyT, AccT>(a, Wv, keys, vals, cap, tid, c, Ki, s_k, s_d, s_v, s_t, slots + lo,
                                            hi - lo);
        for (int64_t x = lo + tid; x < hi; x += G) {
            const int32_t sl = slots[x];
            keys[sl] = EMPTY_KEY;
            vals[sl] = 0;
        }
    }
    if (nch == 1) {
        hub_finish<MODE, KeyT>(a, h, v, (i64)off[v + 1] - (i64)off[v], b, tid);
    } else if (tid == 0) {
        HubPart* mine = a.hub_part + blockIdx.x;
        const i128 key = (i128)b.bk;
        mine->klo = (i64)(u64)key;
        mine->khi = (i64)(key >> 64);
        mine->v = b.bv;
        mine->kic = b.kic;
        mine->nd = b.nd;
        mine->d = b.bd;
    }
}

template <typename OffT, int WK, typename AccT, int MODE>
__global__ void __launch_bounds__(1024) k_hub_decide(MoveArgs a) {
    if (a.dit && a.dit->halt) return;
    constexpr int G = 1024;
    __shared__ i128 s_k128[G / WAVE];
    __shared__ i64 s_k64[G / WAVE];
    __shared__ int32_t s_d[G / WAVE];
    __shared__ i64 s_v[G / WAVE];
    __shared__ i64 s_t[G / WAVE];
    const int32_t ng = a.g_hi - a.g_lo;
    const int64_t chunk_base = a.hch_pre[a.g_lo];
    const int32_t h = a.g_lo + owner_of(a.hch_pre + a.g_lo, ng, chunk_base, blockIdx.x);
    const int32_t v = a.hub_list[h];
    const int64_t k = (int64_t)blockIdx.x - (a.hch_pre[h] - chunk_base);
    const int64_t nch = a.hch_pre[h + 1] - a.hch_pre[h];
    if (!hub_queued(a, v)) {
        if (k == 0 && threadIdx.x == 0) {
            a.gdec[h] = -1;
            if constexpr (MODE == M_SYNC) a.sdec[v] = -1;
        }
        return;
    }
    if (!a.wide) hub_decide_block<MODE, i64, AccT, OffT>(a, h, v, k, nch, s_k64, s_d, s_v, s_t);
    else hub_decide_block<MODE, i128, AccT, OffT>(a, h, v, k, nch, s_k128, s_d, s_v, s_t);
}

// Iteration 0 of a pass, before any vertex has moved: every neighbour j is its
// own community (C' is the identity), so on a row without repeated neighbours
// K_{i->j} is the arc's weight and the decision is an argmax over the row --
// no table, no atomics.  Blocks take the insert chunks of HUB_CH arcs; a hub
// with several chunks posts partial bests that k_hub_final combines, as the
// table path does.  Valid only while nothing has moved: used for SYNC
// iteration 0, which decides against that snapshot.  (Deciding all ASYNC hubs
// of iteration 0 before the first slice would qualify too, but that schedule
// lowers the modularity reached.)
template <int MODE, typename KeyT, typename OffT, int WK>
__device__ __forceinline__ void hub_direct_block(const MoveArgs& a, int32_t h, int32_t v, int64_t k, int64_t nch,
                                                 KeyT* s_k, int32_t* s_d, i64* s_v, i64* s_t) {
    constexpr int G = 1024;
    const Graph<OffT, WK> g{(const OffT*)a.off, a.idx, a.w};
    const int tid = threadIdx.x;
    const i64 Ki = a.K[v];
    const int32_t gv = a.gid ? a.gid[v] : -1;
    const i64 Wv = gv >= 0 ? (i64)a.Wg[gv] : a.W;
    const i64 e0 = (i64)g.off[v] + k * HUB_CH;
    const i64 e1 = min(e0 + (i64)HUB_CH, (i64)g.off[v + 1]);
    KeyT bk = (sizeof(KeyT) == 8) ? (KeyT)INT64_MIN : (KeyT)(((i128)1) << 127);
    int32_t bd = EMPTY_KEY;
    i64 bv = 0, nd = 0;
    for (i64 e = e0 + tid; e < e1; e += G) {
        const int32_t j = g.idx[e];
        if (j == v) continue;
        const i64 wj = g.weight(e);
        const KeyT key = (KeyT)Wv * wj - (KeyT)Ki * ld_s<MODE>(&a.Sig[j]);
        ++nd;
        if (bd == EMPTY_KEY || better(key, j, bk, bd)) { bk = key; bd = j; bv = wj; }
    }
    reduce_best<G, KeyT>(bk, bd, bv, s_k, s_d, s_v);
    nd = reduce_sum<G>(nd, s_t);
    const Best<KeyT> b{bk, bd, bd != EMPTY_KEY ? bv : 0, 0, nd};
    if (nch == 1) {
        hub_finish<MODE, KeyT>(a, h, v, (i64)g.off[v + 1] - (i64)g.off[v], b, tid);
    } else if (tid == 0) {
        HubPart* mine = a.hub_part + blockIdx.x;
        const i128 key = (i128)b.bk;
        mine->klo = (i64)(u64)key;
        mine->khi = (i64)(key >> 64);
        mine->v = b.bv;
        mine->kic = 0;
        mine->nd = b.nd;
        mine->d = b.bd;
    }
}

template <typename OffT, int WK, int MODE>
__global__ void __launch_bounds__(1024) k_hub_direct(MoveArgs a) {
    if (a.dit && a.dit->halt) return;
    constexpr int G = 1024;
    __shared__ i128 s_k128[G / WAVE];
    __shared__ i64 s_k64[G / WAVE];
    __shared__ int32_t s_d[G / WAVE];
    __shared__ i64 s_v[G / WAVE];
    __shared__ i64 s_t[G / WAVE];
    const int32_t ng = a.g_hi - a.g_lo;
    const int64_t chunk_base = a.hch_pre[a.g_lo];
    const int32_t h = a.g_lo + owner_of(a.hch_pre + a.g_lo, ng, chunk_base, blockIdx.x);
    const int32_t v = a.hub_list[h];
    const int64_t k = (int64_t)blockIdx.x - (a.hch_pre[h] - chunk_base);
    const int64_t nch = a.hch_pre[h + 1] - a.hch_pre[h];
    if (!hub_queued(a, v)) {
        if (k == 0 && threadIdx.x == 0) {
            a.gdec[h] = -1;
            if constexpr (MODE == M_SYNC) a.sdec[v] = -1;
        }
        return;
    }
    if (!a.wide) hub_direct_block<MODE, i64, OffT, WK>(a, h, v, k, nch, s_k64, s_d, s_v, s_t);
    else hub_direct_block<MODE, i128, OffT, WK>(a, h, v, k, nch, s_k128, s_d, s_v, s_t);
}

// Hubs of the launch with more than one decide block: one wave per hub
// combines the partial bests (ties to the smaller community) and decides.
template <int MODE, typename KeyT, typename OffT>
__device__ __forceinline__ void hub_final_wave(const MoveArgs& a, int32_t h, int32_t v, int64_t nch,
                                               const HubPart* parts, int lane) {
    const OffT* off = (const OffT*)a.off;
    KeyT bk = (sizeof(KeyT) == 8) ? (KeyT)INT64_MIN : (KeyT)(((i128)1) << 127);
    int32_t bd = EMPTY_KEY;
    i64 bv = 0, kic = 0, nd = 0;
    for (int64_t x = lane; x < nch; x += WAVE) {
        const HubPart& q = parts[x];
        nd += q.nd;
        kic = q.kic > kic ? q.kic : kic;
        if (q.d == EMPTY_KEY) continue;
        const KeyT key = (KeyT)(((i128)q.khi << 64) | (i128)(u64)q.klo);
        if (bd == EMPTY_KEY || better(key, q.d, bk, bd)) { bk = key; bd = q.d; bv = q.v; }
    }
    if (bd == EMPTY_KEY) bk = (sizeof(KeyT) == 8) ? (KeyT)INT64_MIN : (KeyT)(((i128)1) << 127);
    reduce_best<WAVE, KeyT>(bk, bd, bv, nullptr, nullptr, nullptr);
    kic = reduce_max<WAVE>(kic, nullptr);
    nd = reduce_sum<WAVE>(nd, nullptr);
    hub_finish<MODE, KeyT>(a, h, v, (i64)off[v + 1] - (i64)off[v], Best<KeyT>{bk, bd, bd != EMPTY_KEY ? bv : 0, kic, nd},
                           lane);
}

template <typename OffT, int MODE>
__global__ void __launch_bounds__(256) k_hub_final(MoveArgs a) {
    if (a.dit && a.dit->halt) return;
    const int lane = threadIdx.x % WAVE;
    const int32_t h = a.g_lo + (int32_t)((int64_t)blockIdx.x * (256 / WAVE) + threadIdx.x / WAVE);
    if (h >= a.g_hi) return;  // uniform per wave
    const int64_t nch = a.hch_pre[h + 1] - a.hch_pre[h];
    const int32_t v = a.hub_list[h];
    if (nch <= 1 || !hub_queued(a, v)) return;
    const HubPart* parts = a.hub_part + (a.hch_pre[h] - a.hch_pre[a.g_lo]);
    if (!a.wide) hub_final_wave<MODE, i64, OffT>(a, h, v, nch, parts, lane);
    else hub_final_wave<MODE, i128, OffT>(a, h, v, nch, parts, lane);
}

template <typename OffT>
__global__ void __launch_bounds__(1024) k_hub_mark(MoveArgs a) {
    if (a.dit && a.dit->halt) return;
    const int32_t ng = a.g_hi - a.g_lo;
    const int64_t chunk_base = a.hch_pre[a.g_lo];
    const int32_t h = a.g_lo + owner_of(a.hch_pre + a.g_lo, ng, chunk_base, blockIdx.x);
    if (a.gdec[h] < 0) return;
    const OffT* off = (const OffT*)a.off;
    const int32_t v = a.hub_list[h];
    const int64_t k = (int64_t)blockIdx.x - (a.hch_pre[h] - chunk_base);
    const i64 e0 = (i64)off[v] + k * HUB_CH;
    const i64 e1 = min(e0 + (i64)HUB_CH, (i64)off[v + 1]);
    for (i64 e = e0 + threadIdx.x; e < e1; e += 1024) mark_one(a, v, a.idx[e]);
}

// SYNC: apply the recorded decisions of the iteration's queue together, then
// flag the movers' neighbours for the next iteration (hubs' rows are
// flagged by the chunked hub marking).  One wave per 64 queue entries: each
// lane applies its own vertex's move; the wave then walks each mover's row.
template <typename OffT>
__global__ void __launch_bounds__(256) k_sync_apply(MoveArgs a, const int32_t* __restrict__ list, int64_t count) {
    if (a.dit) {  // device-driven: the whole queue, of the size the last iteration left
        if (a.dit->halt) return;
        count = a.dit->seg[MAX_BUCKETS];
        if ((int64_t)blockIdx.x * 256 >= count) return;
    }
    const int lane = threadIdx.x % WAVE;
    const int64_t k = ((int64_t)blockIdx.x * (256 / WAVE) + threadIdx.x / WAVE) * WAVE + lane;
    const Graph<OffT, 0> g{(const OffT*)a.off, a.idx, nullptr};
    int32_t v = -1, d = -1;
    if (k < count) {
        v = list[k];
        d = a.sdec[v];
        if (d >= 0) {
            const int32_t c = a.Cp[v];
            const i64 Kv = a.K[v];
            atomicAdd((u64*)&a.Sig[c], (u64)(-Kv));
            atomicAdd((u64*)&a.Sig[d], (u64)Kv);
            a.Cp[v] = d;
            if (a.learn) a.f_moved[v] = a.itag;
        }
    }
    if (!(a.prune || a.learn)) return;
    u64 todo = __ballot(d >= 0 && a.vbucket[v] != NB_MOVE);
    while (todo) {
        const int b = __ffsll((long long)todo) - 1;
        todo &= todo - 1;
        const int32_t m = __shfl(v, b, WAVE);
        mark_neighbours<WAVE>(a, g, m, (i64)g.off[m], (i64)g.off[m + 1], lane);
    }
}

}  // namespace

void launch_classify(const LevelView& L, const Buckets& B, uint8_t* vbucket, int32_t* Cp, i64* K, i64* Sig,
                     Ctl* ctl, hipStream_t s) {
    if (L.n <= 0) return;
    const unsigned grid = blocks_for(L.n, 256);
    const bool unit = L.t.wk == 0;
    if (L.t.off64) {
        if (unit) k_classify<int64_t, true><<<grid, 256, 0, s>>>((const int64_t*)L.off, L.n, B, vbucket, Cp, K, Sig, ctl);
        else k_classify<int64_t, false><<<grid, 256, 0, s>>>((const int64_t*)L.off, L.n, B, vbucket, Cp, K, Sig, ctl);
    } else {
        if (unit) k_classify<int32_t, true><<<grid, 256, 0, s>>>((const int32_t*)L.off, L.n, B, vbucket, Cp, K, Sig, ctl);
        else k_classify<int32_t, false><<<grid, 256, 0, s>>>((const int32_t*)L.off, L.n, B, vbucket, Cp, K, Sig, ctl);
    }
}

void bucketize_vertices(int64_t n, const uint8_t* vbucket, const uint8_t* flags, int use_flags, const int32_t* gid,
                        const uint8_t* gact,
                        int32_t* blkcnt, int32_t* blkoff, int32_t* out, int32_t* totals, void* scratch,
                        hipStream_t s, const int32_t* halt) {
    constexpr int NB = NB_MOVE + 1;
    const int64_t nb = bucket_blocks(n);
    if (n <= 0) {
        hipMemsetAsync(totals, 0, NB * sizeof(int32_t), s);
        return;
    }
    if (use_flags) {
        MarkBucket bf{vbucket, flags, gid, gact};
        k_bucket_count<NB><<<(unsigned)nb, BK_TPB, 0, s>>>(bf, n, blkcnt, nb, halt);
        scan_i32_to_i32(blkcnt, blkoff, NB * nb, scratch, s);
        k_bucket_fill<NB><<<(unsigned)nb, BK_TPB, 0, s>>>(bf, n, blkoff, nb, out, halt);
    } else {
        VBucket bf{vbucket};
        k_bucket_count<NB><<<(unsigned)nb, BK_TPB, 0, s>>>(bf, n, blkcnt, nb, halt);
        scan_i32_to_i32(blkcnt, blkoff, NB * nb, scratch, s);
        k_bucket_fill<NB><<<(unsigned)nb, BK_TPB, 0, s>>>(bf, n, blkoff, nb, out, halt);
    }
    k_bucket_totals<<<1, 32, 0, s>>>(blkoff, nb, NB, totals);
}

void launch_rowsum(const LevelView& L, int bucket, const int32_t* list, int32_t count, i64* K, i64* Sig, Ctl* ctl,
                   hipStream_t s) {
    if (count <= 0) return;
    LevelTypes t = L.t;
    t.acc64 = 0;
    dispatch_types(t, [&](auto o, auto w, auto) {
        using OffT = typename decltype(o)::type;
        constexpr int WK = decltype(w)::value;
        Graph<OffT, WK> g{(const OffT*)L.off, L.idx, L.w};
        auto go = [&](auto gtag) {
            constexpr int G = decltype(gtag)::value;
            constexpr int NG = (G > 256 ? G : 256) / G;
            k_rowsum<OffT, WK, G><<<blocks_for(count, NG), (G > 256 ? G : 256), 0, s>>>(g, list, count, K, Sig, ctl);
        };
        switch (bucket) {
            case 0: go(IntTag<MOVE_G[0]>{}); break;
            case 1: go(IntTag<MOVE_G[1]>{}); break;
            case 2: go(IntTag<MOVE_G[2]>{}); break;
            case 3: go(IntTag<MOVE_G[3]>{}); break;
            default: go(IntTag<1024>{}); break;
        }
    });
}

void launch_hub_caps(const LevelView& L, const int32_t* list, int32_t count, int64_t* caps, int64_t* nch,
                     hipStream_t s) {
    if (count <= 0) return;
    if (L.t.off64)
        k_hub_caps<int64_t><<<blocks_for(count, 256), 256, 0, s>>>((const int64_t*)L.off, L.n, list, count, caps, nch);
    else
        k_hub_caps<int32_t><<<blocks_for(count, 256), 256, 0, s>>>((const int32_t*)L.off, L.n, list, count, caps, nch);
}

void launch_move(const LevelView& L, int bucket, int mode, const MoveArgs& a, const int32_t* list, int32_t count,
                 hipStream_t s) {
    if (count <= 0) return;
    dispatch_types(L.t, [&](auto o, auto w, auto ac) {
        using OffT = typename decltype(o)::type;
        constexpr int WK = decltype(w)::value;
        using AccT = typename decltype(ac)::type;
        auto go = [&](auto btag) {
            constexpr int b = decltype(btag)::value;
            constexpr int G = MOVE_G[b], CAP = MOVE_CAP[b];
            constexpr int BLOCK = G > 256 ? G : 256;
            const unsigned grid = blocks_for(count, BLOCK / G);
            auto run = [&](auto wtag) {
                constexpr bool WIDE = decltype(wtag)::value != 0;
                if (mode == M_SYNC)
                    k_move_lds<OffT, WK, AccT, G, CAP, M_SYNC, WIDE><<<grid, BLOCK, 0, s>>>(a, list, count);
                else if (mode == M_ASYNC_CACHED)
                    k_move_lds<OffT, WK, AccT, G, CAP, M_ASYNC_CACHED, WIDE><<<grid, BLOCK, 0, s>>>(a, list, count);
                else k_move_lds<OffT, WK, AccT, G, CAP, M_ASYNC_COHERENT, WIDE><<<grid, BLOCK, 0, s>>>(a, list, count);
            };
            if (a.wide) run(IntTag<1>{});
            else run(IntTag<0>{});
        };
        // buckets 0-3 run in k_move_fused; only the workgroup bucket has its own launch
        if (bucket == 4) go(IntTag<4>{});
    });
}

void launch_hub_insert(const LevelView& L, int mode, const MoveArgs& a, int64_t nchunks, hipStream_t s) {
    if (nchunks <= 0) return;
    dispatch_types(L.t, [&](auto o, auto w, auto ac) {
        using OffT = typename decltype(o)::type;
        constexpr int WK = decltype(w)::value;
        using AccT = typename decltype(ac)::type;
        if (mode == M_SYNC) k_hub_insert<OffT, WK, AccT, M_SYNC><<<(unsigned)nchunks, 1024, 0, s>>>(a);
        else if (mode == M_ASYNC_CACHED) k_hub_insert<OffT, WK, AccT, M_ASYNC_CACHED><<<(unsigned)nchunks, 1024, 0, s>>>(a);
        else k_hub_insert<OffT, WK, AccT, M_ASYNC_COHERENT><<<(unsigned)nchunks, 1024, 0, s>>>(a);
    });
}

void launch_hub_decide(const LevelView& L, int mode, const MoveArgs& a, int64_t nchunks, hipStream_t s) {
    const unsigned nh = (unsigned)nchunks;
    if (nchunks <= 0) return;
    dispatch_types(L.t, [&](auto o, auto w, auto ac) {
        using OffT = typename decltype(o)::type;
        constexpr int WK = decltype(w)::value;
        using AccT = typename decltype(ac)::type;
        if (mode == M_SYNC) k_hub_decide<OffT, WK, AccT, M_SYNC><<<(unsigned)nh, 1024, 0, s>>>(a);
        else if (mode == M_ASYNC_CACHED) k_hub_decide<OffT, WK, AccT, M_ASYNC_CACHED><<<(unsigned)nh, 1024, 0, s>>>(a);
        else k_hub_decide<OffT, WK, AccT, M_ASYNC_COHERENT><<<(unsigned)nh, 1024, 0, s>>>(a);
    });
}

void launch_hub_direct(const LevelView& L, int mode, const MoveArgs& a, int64_t nchunks, hipStream_t s) {
    if (nchunks <= 0) return;
    LevelTypes t = L.t;
    t.acc64 = 0;  // no table
    dispatch_types(t, [&](auto o, auto w, auto) {
        using OffT = typename decltype(o)::type;
        constexpr int WK = decltype(w)::value;
        if (mode == M_SYNC) k_hub_direct<OffT, WK, M_SYNC><<<(unsigned)nchunks, 1024, 0, s>>>(a);
        else if (mode == M_ASYNC_CACHED) k_hub_direct<OffT, WK, M_ASYNC_CACHED><<<(unsigned)nchunks, 1024, 0, s>>>(a);
        else k_hub_direct<OffT, WK, M_ASYNC_COHERENT><<<(unsigned)nchunks, 1024, 0, s>>>(a);
    });
}

void launch_hub_final(const LevelView& L, int mode, const MoveArgs& a, hipStream_t s) {
    const int32_t nh = a.g_hi - a.g_lo;
    if (nh <= 0) return;
    const unsigned grid = (unsigned)((nh + 3) / 4);
    if (L.t.off64) {
        if (mode == M_SYNC) k_hub_final<int64_t, M_SYNC><<<grid, 256, 0, s>>>(a);
        else if (mode == M_ASYNC_CACHED) k_hub_final<int64_t, M_ASYNC_CACHED><<<grid, 256, 0, s>>>(a);
        else k_hub_final<int64_t, M_ASYNC_COHERENT><<<grid, 256, 0, s>>>(a);
    } else {
        if (mode == M_SYNC) k_hub_final<int32_t, M_SYNC><<<grid, 256, 0, s>>>(a);
        else if (mode == M_ASYNC_CACHED) k_hub_final<int32_t, M_ASYNC_CACHED><<<grid, 256, 0, s>>>(a);
        else k_hub_final<int32_t, M_ASYNC_COHERENT><<<grid, 256, 0, s>>>(a);
    }
}

void launch_hub_mark(const LevelView& L, const MoveArgs& a, int64_t nchunks, hipStream_t s) {
    if (nchunks <= 0) return;
    if (L.t.off64) k_hub_mark<int64_t><<<(unsigned)nchunks, 1024, 0, s>>>(a);
    else k_hub_mark<int32_t><<<(unsigned)nchunks, 1024, 0, s>>>(a);
}

void launch_move_fused(const LevelView& L, int mode, const MoveArgs& a, const FusedLists& f, hipStream_t s) {
    const int64_t grid = f.blk_pre[4];
    if (grid <= 0) return;
    dispatch_types(L.t, [&](auto o, auto w, auto ac) {
        using OffT = typename decltype(o)::type;
        constexpr int WK = decltype(w)::value;
        using AccT = typename decltype(ac)::type;
        size_t shm = 0;
        for (int b = 1; b < 4; b++)  // bucket 0 (one vertex per lane) has no table
            shm = std::max(shm, (size_t)(256 / MOVE_G[b]) * MOVE_CAP[b] * (4 + sizeof(AccT) + 1));
        auto run = [&](auto wtag) {
            constexpr bool WIDE = decltype(wtag)::value != 0;
            if (mode == M_SYNC) k_move_fused<OffT, WK, AccT, M_SYNC, WIDE><<<(unsigned)grid, 256, shm, s>>>(a, f);
            else if (mode == M_ASYNC_CACHED)
                k_move_fused<OffT, WK, AccT, M_ASYNC_CACHED, WIDE><<<(unsigned)grid, 256, shm, s>>>(a, f);
            else k_move_fused<OffT, WK, AccT, M_ASYNC_COHERENT, WIDE><<<(unsigned)grid, 256, shm, s>>>(a, f);
        };
        if (a.wide) run(IntTag<1>{});
        else run(IntTag<0>{});
    });
}

void launch_sync_apply(const LevelView& L, const MoveArgs& a, const int32_t* list, int64_t count, hipStream_t s) {
    if (count <= 0) return;
    const unsigned grid = (unsigned)((count + 255) / 256);
    if (L.t.off64) k_sync_apply<int64_t><<<grid, 256, 0, s>>>(a, list, count);
    else k_sync_apply<int32_t><<<grid, 256, 0, s>>>(a, list, count);
}

}  // namespace lv
