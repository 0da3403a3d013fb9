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
// memory pool.  Pruning flags are kept as per-vertex stamps; a vertex whose
// stamp is raised to the next iteration's value is appended to that
// iteration's queue (wave-aggregated atomics per bucket).
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

// Count lanes per bucket with one atomic per bucket per wave.
__device__ __forceinline__ void wave_count(bool want, int b, int32_t* count) {
    const int lane = __lane_id();
    u64 pending = __ballot(want);
    while (pending) {
        int leader = __ffsll((long long)pending) - 1;
        int lb = __shfl(b, leader);
        u64 same = __ballot(want && b == lb);
        if (lane == leader) atomicAdd(&count[lb], __popcll(same));
        pending &= ~same;
    }
}

// Wave-aggregated append of (x, y) pairs to a flat array.
__device__ __forceinline__ void wave_append_pair(bool want, int32_t x, int32_t y, int32_t* out, int32_t* count) {
    const int lane = __lane_id();
    u64 m = __ballot(want);
    if (!m) return;
    int leader = __ffsll((long long)m) - 1;
    int base = 0;
    if (lane == leader) base = atomicAdd(count, __popcll(m));
    base = __shfl(base, leader);
    if (want) {
        int r = base + __popcll(m & ((1ull << lane) - 1ull));
        out[2 * (int64_t)r] = x;
        out[2 * (int64_t)r + 1] = y;
    }
}

// ---------------------------------------------------------- group reductions
// Reductions over a group of G lanes; for G > 64 the group is the whole
// workgroup and the cross-wave step goes through LDS.
template <int G, typename KeyT>
__device__ __forceinline__ void reduce_best(KeyT& key, int32_t& d, KeyT* s_k, int32_t* s_d) {
    constexpr int GW = G < WAVE ? G : WAVE;
    if constexpr (sizeof(KeyT) == 8) group_best64<GW>(*(i64*)&key, d);
    else group_best128<GW>(*(i128*)&key, d);
    if constexpr (G > WAVE) {
        const int w = threadIdx.x / WAVE;
        if (threadIdx.x % WAVE == 0) { s_k[w] = key; s_d[w] = d; }
        __syncthreads();
        key = s_k[0];
        d = s_d[0];
#pragma unroll
        for (int k = 1; k < G / WAVE; k++)
            if (better(s_k[k], s_d[k], key, d)) { key = s_k[k]; d = s_d[k]; }
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

// ------------------------------------------------------------ pass init
template <typename OffT>
__global__ void __launch_bounds__(256) k_classify(const OffT* __restrict__ off, int64_t n, Buckets B,
                                                  uint8_t* __restrict__ vbucket, int32_t* __restrict__ Cp,
                                                  i64* __restrict__ K, i64* __restrict__ Sig, Ctl* ctl) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int b = 255;
    if (v < n) {
        const int64_t deg = (int64_t)off[v + 1] - (int64_t)off[v];
        if (deg > 0) {
            b = B.nb;
            for (int k = 0; k < B.nb; k++)
                if (deg <= B.maxdeg[k]) { b = k; break; }
        }
        vbucket[v] = (uint8_t)b;
        Cp[v] = (int32_t)v;
        K[v] = 0;
        Sig[v] = 0;
    }
    wave_count(v < n && b != 255, b, ctl->bcount);
}

__global__ void __launch_bounds__(256) k_fill_buckets(int64_t n, const uint8_t* __restrict__ vbucket,
                                                      int32_t* __restrict__ blist, const int64_t* __restrict__ seg,
                                                      Ctl* ctl) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int b = v < n ? vbucket[v] : 255;
    wave_enqueue(b != 255, b, (int32_t)v, blist, seg, ctl->bcursor);
}

// K'[i] = sum of i's arc weights (self-loop once); Sigma'[i] = K'[i].
template <typename OffT, int WK, int G>
__global__ void __launch_bounds__(G > 256 ? G : 256) k_rowsum(Graph<OffT, WK> g, const int32_t* __restrict__ list,
                                                              int32_t count, i64* __restrict__ K,
                                                              i64* __restrict__ Sig, Ctl* ctl) {
    constexpr int BLOCK = G > 256 ? G : 256;
    constexpr int NG = BLOCK / G;
    __shared__ i64 s_t[BLOCK / WAVE];
    const int grp = threadIdx.x / G, lane = threadIdx.x % G;
    const int64_t slot = (int64_t)blockIdx.x * NG + grp;
    const bool active = slot < count;
    const int32_t i = active ? list[slot] : 0;
    i64 s = 0;
    if (active)
        for (i64 e = (i64)g.off[i] + lane; e < (i64)g.off[i + 1]; e += G) s += g.weight(e);
    s = reduce_sum<G>(s, s_t);
    if (active && lane == 0) {
        K[i] = s;
        Sig[i] = s;
        atomicMax(&ctl->kmax, (u64)s);
    }
}

// Table capacity of a hub: next power of two >= 2 * (bound on distinct
// neighbour communities) = 2 * min(degree, n).
template <typename OffT>
__global__ void k_hub_caps(const OffT* __restrict__ off, int64_t n, const int32_t* __restrict__ list, int32_t count,
                           int64_t* __restrict__ caps) {
    const int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= count) return;
    const int32_t v = list[h];
    const int64_t deg = (int64_t)off[v + 1] - (int64_t)off[v];
    const uint64_t want = 2 * (uint64_t)(deg < n ? deg : n);
    uint64_t cap = 1;
    while (cap < want) cap <<= 1;
    caps[h] = (int64_t)cap;
}

// ------------------------------------------------------------ local moving
// Per-group decision after the table is filled.  Scans the table slots owned
// by this lane, reduces over the group and returns the move target (or -1)
// with its gain in *gain_out; writes the group's distinct-community count.
template <int G, typename KeyT, typename AccT>
__device__ __forceinline__ int32_t decide(const MoveArgs& a, const int32_t* keys, const AccT* vals, int64_t cap,
                                          int lane, bool active, int32_t i, int32_t c, i64 Ki, KeyT* s_k,
                                          int32_t* s_d, i64* s_t, i128* gain_out, i64* nd_out) {
    KeyT bk = 0;
    int32_t bd = EMPTY_KEY;
    i64 kic = 0, nd = 0;
    for (int64_t s = lane; s < cap; s += G) {
        const int32_t d = keys[s];
        if (d == EMPTY_KEY) continue;
        ++nd;
        const i64 v = (i64)vals[s];
        if (d == c) { kic = v; continue; }
        const KeyT key = (KeyT)a.W * v - (KeyT)Ki * a.Sig[d];
        if (bd == EMPTY_KEY || better(key, d, bk, bd)) { bk = key; bd = d; }
    }
    // Lanes without a candidate must not win: give them the smallest key.
    if (bd == EMPTY_KEY) bk = (sizeof(KeyT) == 8) ? (KeyT)INT64_MIN : (KeyT)(((i128)1) << 127);
    reduce_best<G, KeyT>(bk, bd, s_k, s_d);
    kic = reduce_max<G>(kic, s_t);
    *nd_out = reduce_sum<G>(nd, s_t);
    int32_t target = -1;
    i128 gain = 0;
    if (active && bd != EMPTY_KEY) {
        const i64 Sc = a.Sig[c];
        const KeyT stay = (KeyT)a.W * kic - (KeyT)Ki * (Sc - Ki);
        const KeyT gk = bk - stay;
        if (gk > 0 && (!a.pl || bd < c)) { target = bd; gain = (i128)gk; }
    }
    *gain_out = gain;
    (void)i;
    return target;
}

template <typename OffT, int WK, typename AccT, int G, int CAP, bool SYNC>
__global__ void __launch_bounds__(G > 256 ? G : 256) k_move_lds(MoveArgs a, const int32_t* __restrict__ list,
                                                                int32_t count) {
    constexpr int BLOCK = G > 256 ? G : 256;
    constexpr int NG = BLOCK / G;
    constexpr int L2C = Log2<CAP>::v;
    __shared__ int32_t s_keys[NG * CAP];
    __shared__ AccT s_vals[NG * CAP];
    __shared__ i128 s_k128[BLOCK / WAVE];
    __shared__ i64 s_k64[BLOCK / WAVE];
    __shared__ int32_t s_d[BLOCK / WAVE];
    __shared__ i64 s_t[BLOCK / WAVE];
    __shared__ i128 s_gain[NG];
    __shared__ int32_t s_dec[NG];
    __shared__ i64 s_arcs[NG], s_nd[NG];

    const Graph<OffT, WK> g{(const OffT*)a.off, a.idx, a.w};
    const int grp = threadIdx.x / G, lane = threadIdx.x % G;
    const int64_t slot = (int64_t)blockIdx.x * NG + grp;
    const bool active = slot < count;
    const int32_t i = active ? list[slot] : -1;
    int32_t* keys = s_keys + grp * CAP;
    AccT* vals = s_vals + grp * CAP;
    for (int s = lane; s < CAP; s += G) { keys[s] = EMPTY_KEY; vals[s] = 0; }
    group_sync<G>();

    int32_t c = 0;
    i64 Ki = 0, o0 = 0, o1 = 0;
    if (active) {
        c = a.Cp[i];
        Ki = a.K[i];
        o0 = (i64)g.off[i];
        o1 = (i64)g.off[i + 1];
    }
    for (i64 e = o0 + lane; e < o1; e += G) {
        const int32_t j = g.idx[e];
        if (j == i) continue;
        const int32_t d = a.Cp[j];
        table_add<AccT>(keys, vals, CAP - 1, hash_slot<L2C>(d), d, (AccT)g.weight(e));
    }
    group_sync<G>();

    i128 gain;
    i64 nd;
    int32_t target;
    if (!a.wide)
        target = decide<G, i64, AccT>(a, keys, vals, CAP, lane, active, i, c, Ki, s_k64, s_d, s_t, &gain, &nd);
    else
        target = decide<G, i128, AccT>(a, keys, vals, CAP, lane, active, i, c, Ki, s_k128, s_d, s_t, &gain, &nd);

    if (lane == 0) {
        s_gain[grp] = gain;
        s_dec[grp] = target;
        s_arcs[grp] = active ? (o1 - o0) : -1;
        s_nd[grp] = nd;
    }
    if constexpr (SYNC) {
        wave_append_pair(lane == 0 && target >= 0, i, target, a.movers, &a.ctl->movers);
    } else {
        if (lane == 0 && target >= 0) {
            atomicAdd((u64*)&a.Sig[c], (u64)(-Ki));
            atomicAdd((u64*)&a.Sig[target], (u64)Ki);
            a.Cp[i] = target;
        }
        if (a.prune && target >= 0) {
            for (i64 e = o0 + lane; e < o1; e += G) {
                const int32_t j = g.idx[e];
                bool want = false;
                int b = 0;
                if (j != i && a.mark[j] != a.stamp_next) {
                    b = a.vbucket[j];
                    want = b != 255 && atomicExch(&a.mark[j], a.stamp_next) != a.stamp_next;
                }
                wave_enqueue(want, b, j, a.qnext, a.qseg, a.ctl->qcount);
            }
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        i128 sg = 0;
        u64 nm = 0, ne = 0, na = 0, ndt = 0, nma = 0;
        for (int k = 0; k < NG; k++) {
            if (s_arcs[k] < 0) continue;
            ne++;
            na += (u64)s_arcs[k];
            ndt += (u64)s_nd[k];
            if (s_dec[k] >= 0) { sg += s_gain[k]; nm++; nma += (u64)s_arcs[k]; }
        }
        if (ne) {
            const int b = a.bucket;
            atomicAdd(&a.ctl->b_eval[b], ne);
            atomicAdd(&a.ctl->b_arcs[b], na);
            atomicAdd(&a.ctl->b_distinct[b], ndt);
            if (nm) {
                atomic_add_i128(&a.ctl->s_lo, &a.ctl->s_hi, sg);
                atomicAdd(&a.ctl->moves, nm);
                atomicAdd(&a.ctl->b_moves[b], nm);
                atomicAdd(&a.ctl->b_marcs[b], nma);
            }
        }
    }
}

// Hub path: one 1024-thread workgroup per vertex, table in a global pool.
template <typename OffT, int WK, typename AccT, bool SYNC>
__global__ void __launch_bounds__(HUB_G) k_move_hub(MoveArgs a, const int32_t* __restrict__ list, int32_t count) {
    constexpr int G = HUB_G;
    __shared__ i128 s_k128[G / WAVE];
    __shared__ i64 s_k64[G / WAVE];
    __shared__ int32_t s_d[G / WAVE];
    __shared__ i64 s_t[G / WAVE];
    const Graph<OffT, WK> g{(const OffT*)a.off, a.idx, a.w};
    const int64_t slot = blockIdx.x;
    if (slot >= count) return;
    const int32_t i = list[slot];
    if (a.check_mark && a.mark[i] != a.stamp_cur) return;  // not queued this iteration (uniform per block)
    const int lane = threadIdx.x;
    const int64_t toff = a.hub_off[slot] - a.hub_base;
    const int64_t cap = a.hub_off[slot + 1] - a.hub_off[slot];
    const int log2cap = __ffsll((long long)cap) - 1;
    int32_t* keys = a.hub_keys + toff;
    AccT* vals = (AccT*)a.hub_vals + toff;
    for (int64_t s = lane; s < cap; s += G) { keys[s] = EMPTY_KEY; vals[s] = 0; }
    __syncthreads();
    const int32_t c = a.Cp[i];
    const i64 Ki = a.K[i];
    const i64 o0 = (i64)g.off[i], o1 = (i64)g.off[i + 1];
    for (i64 e = o0 + lane; e < o1; e += G) {
        const int32_t j = g.idx[e];
        if (j == i) continue;
        const int32_t d = a.Cp[j];
        table_add<AccT>(keys, vals, (uint32_t)(cap - 1), hash_slot_rt(d, log2cap), d, (AccT)g.weight(e));
    }
    __syncthreads();
    i128 gain;
    i64 nd;
    int32_t target;
    if (!a.wide)
        target = decide<G, i64, AccT>(a, keys, vals, cap, lane, true, i, c, Ki, s_k64, s_d, s_t, &gain, &nd);
    else
        target = decide<G, i128, AccT>(a, keys, vals, cap, lane, true, i, c, Ki, s_k128, s_d, s_t, &gain, &nd);
    if constexpr (SYNC) {
        wave_append_pair(lane == 0 && target >= 0, i, target, a.movers, &a.ctl->movers);
    } else {
        if (lane == 0 && target >= 0) {
            atomicAdd((u64*)&a.Sig[c], (u64)(-Ki));
            atomicAdd((u64*)&a.Sig[target], (u64)Ki);
            a.Cp[i] = target;
        }
        if (a.prune && target >= 0) {
            for (i64 e = o0 + lane; e < o1; e += G) {
                const int32_t j = g.idx[e];
                bool want = false;
                int b = 0;
                if (j != i && a.mark[j] != a.stamp_next) {
                    b = a.vbucket[j];
                    want = b != 255 && atomicExch(&a.mark[j], a.stamp_next) != a.stamp_next;
                }
                wave_enqueue(want, b, j, a.qnext, a.qseg, a.ctl->qcount);
            }
        }
    }
    if (lane == 0) {
        const int b = a.bucket;
        atomicAdd(&a.ctl->b_eval[b], 1ull);
        atomicAdd(&a.ctl->b_arcs[b], (u64)(o1 - o0));
        atomicAdd(&a.ctl->b_distinct[b], (u64)nd);
        if (target >= 0) {
            atomic_add_i128(&a.ctl->s_lo, &a.ctl->s_hi, gain);
            atomicAdd(&a.ctl->moves, 1ull);
            atomicAdd(&a.ctl->b_moves[b], 1ull);
            atomicAdd(&a.ctl->b_marcs[b], (u64)(o1 - o0));
        }
    }
}

// SYNC: apply the recorded decisions together, then flag the movers'
// neighbours for the next iteration.  One wave per mover.
template <typename OffT>
__global__ void __launch_bounds__(256) k_sync_apply(MoveArgs a) {
    const int32_t nm = *(volatile int32_t*)&a.ctl->movers;
    const int lane = threadIdx.x % WAVE;
    const int64_t nw = (int64_t)gridDim.x * (256 / WAVE);
    const OffT* off = (const OffT*)a.off;
    for (int64_t m = (int64_t)blockIdx.x * (256 / WAVE) + threadIdx.x / WAVE; m < nm; m += nw) {
        const int32_t i = a.movers[2 * m], d = a.movers[2 * m + 1];
        if (lane == 0) {
            const int32_t c = a.Cp[i];
            const i64 Ki = a.K[i];
            atomicAdd((u64*)&a.Sig[c], (u64)(-Ki));
            atomicAdd((u64*)&a.Sig[d], (u64)Ki);
            a.Cp[i] = d;
        }
        if (a.prune) {
            const i64 o0 = (i64)off[i], o1 = (i64)off[i + 1];
            for (i64 e = o0 + lane; e < o1; e += WAVE) {
                const int32_t j = a.idx[e];
                bool want = false;
                int b = 0;
                if (j != i && a.mark[j] != a.stamp_next) {
                    b = a.vbucket[j];
                    want = b != 255 && atomicExch(&a.mark[j], a.stamp_next) != a.stamp_next;
                }
                wave_enqueue(want, b, j, a.qnext, a.qseg, a.ctl->qcount);
            }
        }
    }
}

inline unsigned blocks_for(int64_t items, int per_block) { return (unsigned)((items + per_block - 1) / per_block); }

}  // namespace

void launch_classify(const LevelView& L, const Buckets& B, uint8_t* vbucket, int32_t* Cp, i64* K, i64* Sig,
                     Ctl* ctl, hipStream_t s) {
    if (L.n <= 0) return;
    if (L.t.off64)
        k_classify<int64_t><<<blocks_for(L.n, 256), 256, 0, s>>>((const int64_t*)L.off, L.n, B, vbucket, Cp, K,
                                                                  Sig, ctl);
    else
        k_classify<int32_t><<<blocks_for(L.n, 256), 256, 0, s>>>((const int32_t*)L.off, L.n, B, vbucket, Cp, K,
                                                                  Sig, ctl);
}

void launch_fill_buckets(int64_t n, const uint8_t* vbucket, int32_t* blist, const int64_t* seg, Ctl* ctl,
                         hipStream_t s) {
    if (n <= 0) return;
    k_fill_buckets<<<blocks_for(n, 256), 256, 0, s>>>(n, vbucket, blist, seg, ctl);
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

void launch_hub_caps(const LevelView& L, const int32_t* list, int32_t count, int64_t* caps, hipStream_t s) {
    if (count <= 0) return;
    if (L.t.off64)
        k_hub_caps<int64_t><<<blocks_for(count, 256), 256, 0, s>>>((const int64_t*)L.off, L.n, list, count, caps);
    else
        k_hub_caps<int32_t><<<blocks_for(count, 256), 256, 0, s>>>((const int32_t*)L.off, L.n, list, count, caps);
}

void launch_move(const LevelView& L, int bucket, int sync, const MoveArgs& a, const int32_t* list, int32_t count,
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
            if (sync) k_move_lds<OffT, WK, AccT, G, CAP, true><<<grid, BLOCK, 0, s>>>(a, list, count);
            else k_move_lds<OffT, WK, AccT, G, CAP, false><<<grid, BLOCK, 0, s>>>(a, list, count);
        };
        switch (bucket) {
            case 0: go(IntTag<0>{}); break;
            case 1: go(IntTag<1>{}); break;
            case 2: go(IntTag<2>{}); break;
            case 3: go(IntTag<3>{}); break;
            default: go(IntTag<4>{}); break;
        }
    });
}

void launch_move_hub(const LevelView& L, int sync, const MoveArgs& a, const int32_t* list, int32_t count,
                     hipStream_t s) {
    if (count <= 0) return;
    dispatch_types(L.t, [&](auto o, auto w, auto ac) {
        using OffT = typename decltype(o)::type;
        constexpr int WK = decltype(w)::value;
        using AccT = typename decltype(ac)::type;
        if (sync) k_move_hub<OffT, WK, AccT, true><<<(unsigned)count, HUB_G, 0, s>>>(a, list, count);
        else k_move_hub<OffT, WK, AccT, false><<<(unsigned)count, HUB_G, 0, s>>>(a, list, count);
    });
}

void launch_sync_apply(const LevelView& L, const MoveArgs& a, hipStream_t s) {
    const unsigned grid = (unsigned)std::min<int64_t>(8192, std::max<int64_t>(1, (L.n + 3) / 4));
    if (L.t.off64) k_sync_apply<int64_t><<<grid, 256, 0, s>>>(a);
    else k_sync_apply<int32_t><<<grid, 256, 0, s>>>(a);
}

}  // namespace lv
