// lv_batch.hip -- per-graph bookkeeping for batched runs.
//
// A batch is many independent graphs laid end to end in one CSR: graph g owns
// the vertex range [vbase[g], vbase[g+1]) and no arc leaves its range.  The
// local-moving and aggregation kernels run over the union (a community never
// spans two graphs, and renumbering in ascending id order keeps every graph's
// communities contiguous); these kernels keep the per-graph quantities the
// method needs: the graph id of every vertex of the current level, total
// weights W_g, counts for the aggregation tests, the base of each graph's
// final community ids, and per-graph modularity.
//
// Per-graph sums over vertex ranges use block-level run combining: a block
// covers 256 consecutive vertices, which belong to few graphs, so one thread
// adds up the runs of equal graph id and issues one atomic per run.
#include "lv_internal.h"

namespace lv {
namespace {

constexpr int BT = 256;

// Adds v (one value per thread, graph id g or -1 for none) into out[g], one
// atomic per run of equal g in thread order.
__device__ __forceinline__ void add_by_graph_runs(int32_t g, u64 v, u64* out) {
    __shared__ int32_t s_g[BT];
    __shared__ u64 s_v[BT];
    s_g[threadIdx.x] = g;
    s_v[threadIdx.x] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t cur = -1;
        u64 acc = 0;
        for (int k = 0; k < BT; k++) {
            if (s_g[k] != cur) {
                if (cur >= 0 && acc) atomicAdd(&out[cur], acc);
                cur = s_g[k];
                acc = 0;
            }
            acc += s_v[k];
        }
        if (cur >= 0 && acc) atomicAdd(&out[cur], acc);
    }
}

__global__ void __launch_bounds__(BT) k_gid_init(const int64_t* __restrict__ vbase, int64_t count, int64_t n,
                                                 int32_t* __restrict__ gid) {
    const int64_t v = (int64_t)blockIdx.x * BT + threadIdx.x;
    if (v >= n) return;
    int64_t lo = 0, hi = count - 1;  // largest g with vbase[g] <= v
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (vbase[mid] <= v) lo = mid; else hi = mid - 1;
    }
    gid[v] = (int32_t)lo;
}

// Arcs must stay inside their graph; per-graph total weights W_g.
template <typename OffT, int WK>
__global__ void __launch_bounds__(BT) k_graph_weights(Graph<OffT, WK> g, int64_t n, const int32_t* __restrict__ gid,
                                                      u64* __restrict__ Wg, Ctl* ctl) {
    const int64_t v = (int64_t)blockIdx.x * BT + threadIdx.x;
    u64 sum = 0;
    int32_t gv = -1;
    if (v < n) {
        gv = gid[v];
        bool cross = false;
        for (i64 e = (i64)g.off[v]; e < (i64)g.off[v + 1]; e++) {
            sum += (u64)g.weight(e);
            cross |= gid[g.idx[e]] != gv;
        }
        if (cross) atomicOr(&ctl->err, 8);
    }
    add_by_graph_runs(gv, sum, Wg);
}

// Per-graph count of vertices with at least one arc.
template <typename OffT>
__global__ void __launch_bounds__(BT) k_nonisolated_by_graph(const OffT* __restrict__ off, int64_t n,
                                                             const int32_t* __restrict__ gid, u64* __restrict__ out) {
    const int64_t v = (int64_t)blockIdx.x * BT + threadIdx.x;
    int32_t gv = -1;
    u64 x = 0;
    if (v < n) {
        gv = gid[v];
        x = off[v + 1] > off[v] ? 1 : 0;
    }
    add_by_graph_runs(gv, x, out);
}

// Per-graph count of used community ids (community c belongs to graph gid[c]).
__global__ void __launch_bounds__(BT) k_used_by_graph(const int32_t* __restrict__ used, int64_t n,
                                                      const int32_t* __restrict__ gid, u64* __restrict__ out) {
    const int64_t c = (int64_t)blockIdx.x * BT + threadIdx.x;
    int32_t gv = -1;
    u64 x = 0;
    if (c < n) {
        gv = gid[c];
        x = used[c] ? 1 : 0;
    }
    add_by_graph_runs(gv, x, out);
}

// Graph ids of the next level: community c (used) becomes vertex newid[c].
__global__ void __launch_bounds__(BT) k_gid_next(const int32_t* __restrict__ used, const int32_t* __restrict__ newid,
                                                 int64_t n, const int32_t* __restrict__ gid,
                                                 int32_t* __restrict__ gid_next) {
    const int64_t c = (int64_t)blockIdx.x * BT + threadIdx.x;
    if (c < n && used[c]) gid_next[newid[c]] = gid[c];
}

// Smallest final community id of every graph (ids are dense and contiguous
// per graph), one atomic per run of equal graph id in the block; then rebase
// every graph's ids to start at 0.
__global__ void __launch_bounds__(BT) k_graph_cmin(const int32_t* __restrict__ C, int64_t n,
                                                   const int32_t* __restrict__ gid, int32_t* __restrict__ cmin) {
    __shared__ int32_t s_g[BT], s_c[BT];
    const int64_t v = (int64_t)blockIdx.x * BT + threadIdx.x;
    s_g[threadIdx.x] = v < n ? gid[v] : -1;
    s_c[threadIdx.x] = v < n ? C[v] : 0;
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t cur = -1, m = 0;
        for (int k = 0; k < BT; k++) {
            if (s_g[k] != cur) {
                if (cur >= 0) atomicMin(&cmin[cur], m);
                cur = s_g[k];
                m = s_c[k];
            }
            m = s_c[k] < m ? s_c[k] : m;
        }
        if (cur >= 0) atomicMin(&cmin[cur], m);
    }
}
__global__ void __launch_bounds__(BT) k_rebase(int32_t* __restrict__ C, int64_t n, const int32_t* __restrict__ gid,
                                               const int32_t* __restrict__ cmin) {
    const int64_t v = (int64_t)blockIdx.x * BT + threadIdx.x;
    if (v < n) C[v] -= cmin[gid[v]];
}

// Per-graph modularity numerator sum_c (W_g sigma_c - Sigma_c^2) over the
// union's dense community ids; community c belongs to the graph g with
// cbase[g] <= c < cbase[g+1].
__global__ void __launch_bounds__(BT) k_mod_terms_batch(int64_t ncom, const int32_t* __restrict__ cbase, int64_t count,
                                                        const u64* __restrict__ Wg, const i64* __restrict__ sigin,
                                                        const i64* __restrict__ sigtot, u64* __restrict__ qlohi) {
    const int64_t c = (int64_t)blockIdx.x * BT + threadIdx.x;
    if (c >= ncom) return;
    int64_t lo = 0, hi = count - 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (cbase[mid] <= c) lo = mid; else hi = mid - 1;
    }
    const i128 t = (i128)(i64)Wg[lo] * sigin[c] - (i128)sigtot[c] * sigtot[c];
    if (t != 0) atomic_add_i128(&qlohi[2 * lo], &qlohi[2 * lo + 1], t);
}

// Per-graph counts of one bucket's queue segment (id order, so graphs form
// runs): segcnt[g] += entries of graph g.
// Device-driven iterations (dit): list is the queue's base; bucket b's
// entries and their number come from dit, len is the launch's bound.
__global__ void __launch_bounds__(BT) k_seg_count(const int32_t* __restrict__ list, int64_t len,
                                                  const int32_t* __restrict__ gid, int32_t* __restrict__ segcnt,
                                                  const DevIter* __restrict__ dit, int b) {
    if (dit) {
        if (dit->halt) return;
        list += dit->seg[b];
        len = dit->cnt[b];
        if ((int64_t)blockIdx.x * BT >= len) return;
    }
    const int64_t j = (int64_t)blockIdx.x * BT + threadIdx.x;
    const int32_t key = j < len ? gid[list[j]] : -1;
    __shared__ int32_t s_k[BT];
    s_k[threadIdx.x] = key;
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t cur = -1, acc = 0;
        for (int k = 0; k < BT; k++) {
            if (s_k[k] != cur) {
                if (cur >= 0) atomicAdd(&segcnt[cur], acc);
                cur = s_k[k];
                acc = 0;
            }
            acc++;
        }
        if (cur >= 0) atomicAdd(&segcnt[cur], acc);
    }
}

// For bucket b and slice k: prefall[(b*ns + k)*(count+1) + g] = sum over
// graphs g' < g of their share of slice k.  One block per (b, k) row.
__global__ void __launch_bounds__(1024) k_slice_prefix(const int32_t* __restrict__ segcnt, int64_t count, int ns,
                                                       int32_t* __restrict__ prefall) {
    const int b = blockIdx.x / ns, k = blockIdx.x % ns;
    const int32_t* cnt = segcnt + (int64_t)b * count;
    int32_t* out = prefall + (int64_t)blockIdx.x * (count + 1);
    __shared__ int32_t s_w[1024 / WAVE];
    __shared__ int32_t s_carry;
    if (threadIdx.x == 0) s_carry = 0;
    __syncthreads();
    for (int64_t base = 0; base < count; base += 1024) {
        const int64_t g = base + threadIdx.x;
        int32_t v = 0;
        if (g < count) {
            const int64_t len = cnt[g];
            v = (int32_t)(len * (k + 1) / ns - len * k / ns);
        }
        // block-wide inclusive scan
        int32_t x = v;
        const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
        for (int d = 1; d < WAVE; d <<= 1) {
            const int32_t y = __shfl_up(x, d, WAVE);
            if (lane >= d) x += y;
        }
        if (lane == WAVE - 1) s_w[w] = x;
        __syncthreads();
        int32_t before = s_carry;
        for (int q = 0; q < w; q++) before += s_w[q];
        if (g < count) out[g] = before + x - v;
        __syncthreads();
        if (threadIdx.x == 1023) s_carry = before + x;
        __syncthreads();
    }
    if (threadIdx.x == 0) out[count] = s_carry;
}

}  // namespace

void launch_seg_count(const int32_t* list, int64_t len, const int32_t* gid, int32_t* segcnt, hipStream_t s,
                      const DevIter* dit, int b) {
    if (len > 0) k_seg_count<<<(unsigned)((len + BT - 1) / BT), BT, 0, s>>>(list, len, gid, segcnt, dit, b);
}

void launch_slice_prefix(const int32_t* segcnt, int nbt, int64_t count, int ns, int32_t* prefall, hipStream_t s) {
    if (nbt * ns > 0) k_slice_prefix<<<(unsigned)(nbt * ns), 1024, 0, s>>>(segcnt, count, ns, prefall);
}

void launch_gid_init(const int64_t* vbase, int64_t count, int64_t n, int32_t* gid, hipStream_t s) {
    if (n > 0) k_gid_init<<<(unsigned)((n + BT - 1) / BT), BT, 0, s>>>(vbase, count, n, gid);
}

void launch_graph_weights(const LevelView& L, const int32_t* gid, u64* Wg, Ctl* ctl, hipStream_t s) {
    if (L.n <= 0) return;
    LevelTypes t = L.t;
    t.acc64 = 0;
    const unsigned grid = (unsigned)((L.n + BT - 1) / BT);
    if (t.off64) {
        if (t.wk == 0) k_graph_weights<int64_t, 0><<<grid, BT, 0, s>>>({(const int64_t*)L.off, L.idx, L.w}, L.n, gid, Wg, ctl);
        else k_graph_weights<int64_t, 1><<<grid, BT, 0, s>>>({(const int64_t*)L.off, L.idx, L.w}, L.n, gid, Wg, ctl);
    } else {
        if (t.wk == 0) k_graph_weights<int32_t, 0><<<grid, BT, 0, s>>>({(const int32_t*)L.off, L.idx, L.w}, L.n, gid, Wg, ctl);
        else k_graph_weights<int32_t, 1><<<grid, BT, 0, s>>>({(const int32_t*)L.off, L.idx, L.w}, L.n, gid, Wg, ctl);
    }
}

void launch_nonisolated_by_graph(const LevelView& L, const int32_t* gid, u64* out, hipStream_t s) {
    if (L.n <= 0) return;
    const unsigned grid = (unsigned)((L.n + BT - 1) / BT);
    if (L.t.off64) k_nonisolated_by_graph<int64_t><<<grid, BT, 0, s>>>((const int64_t*)L.off, L.n, gid, out);
    else k_nonisolated_by_graph<int32_t><<<grid, BT, 0, s>>>((const int32_t*)L.off, L.n, gid, out);
}

void launch_used_by_graph(const int32_t* used, int64_t n, const int32_t* gid, u64* out, hipStream_t s) {
    if (n > 0) k_used_by_graph<<<(unsigned)((n + BT - 1) / BT), BT, 0, s>>>(used, n, gid, out);
}

void launch_gid_next(const int32_t* used, const int32_t* newid, int64_t n, const int32_t* gid, int32_t* gid_next,
                     hipStream_t s) {
    if (n > 0) k_gid_next<<<(unsigned)((n + BT - 1) / BT), BT, 0, s>>>(used, newid, n, gid, gid_next);
}

void launch_graph_cmin(const int32_t* C, int64_t n, const int32_t* gid, int32_t* cmin, hipStream_t s) {
    if (n > 0) k_graph_cmin<<<(unsigned)((n + BT - 1) / BT), BT, 0, s>>>(C, n, gid, cmin);
}

void launch_rebase(int32_t* C, int64_t n, const int32_t* gid, const int32_t* cmin, hipStream_t s) {
    if (n > 0) k_rebase<<<(unsigned)((n + BT - 1) / BT), BT, 0, s>>>(C, n, gid, cmin);
}

void launch_mod_terms_batch(int64_t ncom, const int32_t* cbase, int64_t count, const u64* Wg, const i64* sigin,
                            const i64* sigtot, u64* qlohi, hipStream_t s) {
    if (ncom > 0)
        k_mod_terms_batch<<<(unsigned)((ncom + BT - 1) / BT), BT, 0, s>>>(ncom, cbase, count, Wg, sigin, sigtot, qlohi);
}

}  // namespace lv
