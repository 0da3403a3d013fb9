// lv_api.cpp -- C ABI and host driver of the gfx950 Louvain library.
//
// The driver is the pass loop of the paper's Algorithm 1 / Algorithm 4:
//   per pass: K' = row sums, Sigma' = K', C' = identity, all vertices queued;
//   local moving until the iteration's gain sum S satisfies
//     2*S / W^2 <= tau_p = tau_0 / drop^p   (tested exactly in integers)
//   or MAX_ITERATIONS; stop if that took <= 1 iteration; count communities;
//   stop if none merged or |Gamma| / |Gamma_old| > tau_agg; renumber;
//   dendrogram lookup; aggregate; next pass.
//   After the loop: final lookup when it stopped before aggregating.
// Community counts for the shrink test cover vertices with at least one arc.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstddef>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "louvain.h"
#include "lv_bucket.h"
#include "lv_internal.h"

using namespace lv;

namespace {

thread_local std::string g_create_error = "no error";

constexpr size_t ALIGN = 256;
// ASYNC slices of a huge single-graph level hold at most this many queued
// vertices (measured on R-MAT 27: 128 slices with 64 hub groups ran 4.5 %
// faster at higher modularity than 64 with 32; levels of a few million
// vertices keep async_slices, where more slices only add launches).
constexpr int64_t SLICE_SPAN = 1 << 19;

inline size_t align_up(size_t x) { return (x + ALIGN - 1) & ~(ALIGN - 1); }

inline uint64_t next_pow2(uint64_t x) {
    uint64_t p = 1;
    while (p < x) p <<= 1;
    return p;
}

struct Layout {
    size_t ctl, seg, C, Cp, K, Sig, mark, vbucket, blist, qa, qb, sdec, hcaps, hpre;
    size_t used, newid, cnt, coff, cursor, members, cdeg, hoff, cbucket, alist, rowlen;
    size_t hidx, hw, sup_off, sup_idx, sup_w, pool_keys, pool_vals, scan;
    size_t md, mpos, bnch, bchpre, bitmaps, gdec, blkcnt, blkoff;
    size_t f_own, f_adv, f_moved, f_nm, hcnt, hslots, hpart, dit, dshare;
    int64_t part_cap;
    // batched runs (count graphs; absent for a single graph)
    size_t gid[2], gid0, Wg, gact, Sg, Pg, gsweep, gany, gcnt, cmin, vbase, gq, segcnt, segstart, prefall, lig;
    int64_t bitmap_words;
    int64_t pool_entries;
    size_t total;
};

bool make_layout(int64_t n, int64_t m, int64_t count, int slices, Layout* L) {
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o += align_up(bytes > 0 ? bytes : 1); return at; };
    const size_t N = (size_t)n, M = (size_t)m;
    L->ctl = take(sizeof(Ctl));
    L->dit = take(sizeof(DevIter));
    // slice table of device-driven iterations (a huge level may use up to twice `slices`)
    L->dshare = take((size_t)NB_MOVE * 2 * std::max(1, slices) * 8);
    L->seg = take(32 * sizeof(int64_t));
    L->C = take(N * 4);
    L->Cp = take(N * 4);
    L->K = take(N * 8);
    L->Sig = take(N * 8);
    L->mark = take(2 * N);  // two byte flag arrays: this iteration's queue, the next one's
    L->vbucket = take(N);
    L->blist = take(N * 4);
    L->qa = take(N * 4);
    L->qb = take(N * 4);
    L->sdec = take(N * 4);
    L->hcaps = take((N + 1) * 8);
    L->hpre = take((N + 1) * 8);
    L->used = take((N + 1) * 4);
    L->newid = take((N + 1) * 4);
    L->cnt = take((N + 1) * 4);
    L->coff = take((N + 1) * 4);
    L->cursor = take(N * 4);
    L->members = take(N * 4);
    L->cdeg = take((N + 1) * 8);
    L->hoff = take((N + 1) * 8);
    L->cbucket = take(N);
    L->alist = take(N * 4);
    L->rowlen = take((N + 1) * 4);
    L->hidx = take(M * 4);
    L->hw = take(M * 8);
    // One super-graph buffer: level p+1 is compacted over level p, which the
    // hashing into the holey buffer has finished reading by then.
    L->sup_off = take((N + 1) * 8);
    L->sup_idx = take(M * 4);
    L->sup_w = take(M * 8);
    int64_t pool = (int64_t)next_pow2(2 * (uint64_t)(n + 1));
    int64_t want = std::min<int64_t>(std::max<int64_t>(2 * m, (int64_t)1 << 20), (int64_t)1 << 28);
    pool = std::max(pool, want);
    L->pool_entries = pool;
    L->pool_keys = take((size_t)pool * 4);
    L->pool_vals = take((size_t)pool * 8);
    L->hslots = take((size_t)pool / 2 * 4);
    L->hcnt = take((N + 1) * 4);
    // hub-decide partials: a launch never exceeds part_cap blocks, and no hub
    // has more insert chunks than that
    L->part_cap = (int64_t)(M / HUB_CH) + 2;
    L->hpart = take((size_t)L->part_cap * sizeof(HubPart));
    if (count > 0) {
        const size_t G = (size_t)count;
        L->gid[0] = take(N * 4);
        L->gid[1] = take(N * 4);
        L->gid0 = take(N * 4);
        L->Wg = take(G * 8);
        L->gact = take(G);
        L->Sg = take(G * 16);
        L->Pg = take(G * 8);      // per graph: evaluations with a positive best gain
        L->gsweep = take(G);      // per graph: the next iteration is its sweep (learned pruner)
        L->gany = take(G);        // per graph: the learned filter kept a vertex
        L->gcnt = take(G * 16);   // per graph: vertices with arcs, used communities
        L->cmin = take(G * 4);
        L->vbase = take((G + 1) * 8);
        L->gq = take(G * 16);     // per-graph modularity numerators
        const size_t S = (size_t)std::max(1, slices);
        L->segcnt = take((size_t)NB_MOVE * G * 4);
        L->segstart = take((size_t)NB_MOVE * (G + 1) * 4);
        L->prefall = take((size_t)NB_MOVE * S * (G + 1) * 4);
        L->lig = take(G * 4);     // per graph: iterations of the pass (device-driven iterations)
    }
    L->scan = take(scan_scratch_bytes(std::max(n, count) + 2));
    L->gdec = take(N * 4);
    L->blkcnt = take((size_t)(MAX_BUCKETS * (bucket_blocks(n + 1) + 1) + 8) * 4);
    L->blkoff = take((size_t)(MAX_BUCKETS * (bucket_blocks(n + 1) + 1) + 8) * 4);
    L->md = take((N + 1) * 8);
    L->mpos = take((N + 2) * 8);
    L->bnch = take((N + 1) * 8);
    L->bchpre = take((N + 2) * 8);
    L->bitmap_words = (n + 32) / 32;
    L->bitmaps = take((size_t)BIG_EXTRACT_BLOCKS * (size_t)L->bitmap_words * 4);
    L->f_own = take(N * 8);
    L->f_adv = take(N * 8);
    L->f_moved = take(N * 4);
    L->f_nm = take(N * 4);
    L->total = o;
    return true;
}

struct KRec {
    int kind;  // index into kernel name table
    hipEvent_t e0, e1;
    int64_t bytes;
};

enum KName { K_MOVE_FUSED = 0, K_MOVE1, K_MOVE2, K_MOVE3, K_MOVE4, K_MOVE_HUB, K_SYNC_APPLY, K_PASS_INIT, K_AGG_PREP,
             K_AGG0, K_AGG1, K_AGG2, K_AGG3, K_AGG_BIG_INSERT, K_AGG_BIG_EXTRACT, K_COMPACT, K_QUEUE, K_HUB_MARK,
             K_LEARN_FILTER, K_HUB_DECIDE, K_COUNT };
const char* KNAMES[K_COUNT] = {"move_b0_3", "move_unused1", "move_unused2", "move_unused3", "move_b4", "move_hub",
                               "sync_apply",
                               "pass_init", "aggregate_prep", "aggregate_b0", "aggregate_b1", "aggregate_b2",
                               "aggregate_b3", "aggregate_big_insert", "aggregate_big_extract", "compact",
                               "queue_build", "hub_mark", "learn_filter", "hub_decide"};

}  // namespace

struct louvain_s {
    hipStream_t stream = nullptr;
    louvain_graph g{};
    louvain_params p{};
    char* ws = nullptr;
    size_t ws_bytes = 0;
    Layout lay{};
    LevelView L0;
    int64_t W = 0;
    int sup_off64 = 0, sup_wk = 1;
    bool ran = false;
    int64_t ncom = 0;
    // batched runs: number of graphs (0 = a single graph), vertex bases, and
    // per-graph results of the last run
    int64_t nb = 0;
    std::vector<int64_t> vbase;
    std::vector<u64> Wg;
    std::vector<int32_t> b_passes, b_iters;
    std::vector<int64_t> b_comms;
    std::vector<int32_t> b_cbase;  // first final community id of every graph (union numbering)
    louvain_stats st{};
    std::string err = "no error";
    void* pinned = nullptr;  // readback staging
    void* pinned_up = nullptr;  // upload staging
    bool stage_owned = true;    // pinned/pinned_up were allocated by create (else fixed host buffers)
    bool handle_owned = true;   // the handle itself was allocated by create (else placed in fixed storage)
    louvain_iter_fn itfn = nullptr;
    louvain_pass_fn pafn = nullptr;
    void* user = nullptr;
    bool prof = false;
    std::vector<KRec> recs;
    std::vector<hipEvent_t> evpool;
    size_t evnext = 0;
    double kms[K_COUNT] = {};
    int64_t klaunch[K_COUNT] = {};
    int64_t kbytes[K_COUNT] = {};
    uint32_t stamp = 0;
    Buckets mb{}, ab{};
    float* smp_buf = nullptr;  // training samples (borrowed)
    int64_t smp_cap = 0;
    int32_t smp_rate = 0;
    int64_t smp_count = 0;
    int64_t syncs = 0;         // host waits on the stream during the current run
    bool rows_unique0 = false;  // every row of the input strictly ascending (no repeated neighbour)

    template <typename T>
    T* at(size_t off) { return (T*)(ws + off); }
    Ctl* ctl() { return at<Ctl>(lay.ctl); }
};

namespace {

louvain_status fail(louvain_t* h, louvain_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (h) h->err = buf;
    else g_create_error = buf;
    return st;
}

#define HIPCHK(h, x)                                                                            \
    do {                                                                                        \
        hipError_t e_ = (x);                                                                    \
        if (e_ != hipSuccess)                                                                   \
            return fail((h), LOUVAIN_ERR_HIP, "%s failed: %s", #x, hipGetErrorString(e_));     \
    } while (0)

hipEvent_t next_event(louvain_t* h) {
    if (h->evnext >= h->evpool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        h->evpool.push_back(e);
    }
    return h->evpool[h->evnext++];
}

// Time the launches issued by fn() under kernel name `kind` (profiling mode).
template <typename Fn>
void timed(louvain_t* h, int kind, int64_t bytes, Fn&& fn) {
    if (!h->prof) { fn(); return; }
    hipEvent_t a = next_event(h), b = next_event(h);
    if (!a || !b) { fn(); return; }
    (void)hipEventRecord(a, h->stream);
    fn();
    (void)hipEventRecord(b, h->stream);
    h->recs.push_back({kind, a, b, bytes});
}

// Waits for the stream, counted (louvain_stats.host_syncs).
louvain_status sync_stream(louvain_t* h) {
    h->syncs++;
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return LOUVAIN_OK;
}

louvain_status readback(louvain_t* h, void* dst, const void* src, size_t bytes) {
    if (bytes == 0) return LOUVAIN_OK;
    h->syncs++;
    if (bytes <= (1 << 20)) {
        HIPCHK(h, hipMemcpyAsync(h->pinned, src, bytes, hipMemcpyDeviceToHost, h->stream));
        HIPCHK(h, hipStreamSynchronize(h->stream));
        memcpy(dst, h->pinned, bytes);
    } else {
        HIPCHK(h, hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, h->stream));
        HIPCHK(h, hipStreamSynchronize(h->stream));
    }
    return LOUVAIN_OK;
}

Buckets make_buckets(const int32_t* over, int nb, const int* caps, const int* defaults) {
    Buckets B{};
    B.nb = nb;
    for (int k = 0; k < nb; k++) {
        int v = over[k];
        if (v == 0) v = defaults[k];
        else if (v < 0) v = 0;                 // bucket disabled
        B.maxdeg[k] = std::min(v, caps[k] / 2);
    }
    return B;
}

bool converged(unsigned __int128 S, int64_t W, const louvain_params& p, int pass) {
    // 2*S*tol_den*drop^pass <= tol_num * W^2, exactly
    unsigned __int128 rhs = (unsigned __int128)p.tol_num * ((unsigned __int128)W * (unsigned __int128)W);
    unsigned __int128 lhs = 2 * S * (unsigned __int128)p.tol_den;
    for (int k = 0; k < pass; k++) {
        if (lhs > rhs) return false;
        lhs *= (unsigned __int128)p.tol_drop;
    }
    return lhs <= rhs;
}

// Bytes of algorithmic traffic of one evaluation batch (see the roofline model).
int64_t move_alg_bytes(const LevelView& L, uint64_t eval, uint64_t arcs, uint64_t distinct, uint64_t moves,
                       uint64_t marcs, int sync, int learn) {
    const int64_t offb = L.t.off64 ? 8 : 4;
    const int64_t wb = L.t.wk == 0 ? 0 : (L.t.wk == 1 ? 4 : 8);
    int64_t b = (int64_t)eval * (4 + 4 + 8 + 8 + 2 * offb) + (int64_t)arcs * (4 + 4 + wb) + (int64_t)distinct * 8;
    // SYNC: one decision word per evaluated vertex (applied by k_sync_apply);
    // ASYNC: C' write and two Sigma' atomics per move, then per arc of a
    // mover its index and a flag byte
    if (sync) b += (int64_t)eval * 4;
    else b += (int64_t)moves * (4 + 16) + (int64_t)marcs * (4 + 1);
    // learned-pruner state: own/adv per evaluation, moved tag per move, a
    // moved-neighbour count per arc of a mover
    if (learn) b += (int64_t)eval * 16 + (int64_t)moves * 4 + (int64_t)marcs * 4;
    return b;
}

// Bytes of the learned filter: a flag byte per vertex, the feature state of
// each flagged vertex, a cleared flag per dropped vertex, each recorded sample.
int64_t filter_alg_bytes(const LevelView& L, int64_t n, int64_t flagged, int64_t dropped, int64_t samples) {
    const int64_t offb = L.t.off64 ? 8 : 4;
    return n * 1 + flagged * (8 + 8 + 8 + 4 + 4 + 2 * offb) + dropped * 1 + samples * 36;
}

// Sum of the striped per-iteration counters.
struct IterTotals {
    unsigned __int128 S;
    uint64_t moves;
    uint64_t positive;
    int32_t qcount[MAX_BUCKETS];
};
IterTotals sum_iter(const Ctl& c) {
    IterTotals t{};
    for (int k = 0; k < STRIPES; k++) {
        t.S += ((unsigned __int128)c.s_hi[k] << 64) + ((unsigned __int128)c.s_mid[k] << 32) +
               (unsigned __int128)c.s_lo[k];
        t.moves += c.moves[k];
        t.positive += c.positive[k];
    }
    for (int b = 0; b < MAX_BUCKETS; b++) t.qcount[b] = c.qcount[b];
    return t;
}

}  // namespace

extern "C" {

void louvain_params_default(louvain_params* p) {
    if (!p) return;
    memset(p, 0, sizeof(*p));
    p->max_iterations = 20;
    p->max_passes = 10;
    p->tol_num = 1;
    p->tol_den = 100;
    p->tol_drop = 10;
    p->agg_num = 4;
    p->agg_den = 5;
    p->pick_less = 4;
    p->mode = LOUVAIN_ASYNC;
    p->pruner = LOUVAIN_PRUNE_FLAGS;
    p->validate = 1;
    p->async_coherent = 0;
    p->bucket_order = 0;
    p->async_slices = 64;
    p->async_slice_iters = 0;
    p->guard_tolerance = 0;
    p->async_slice_min = 256;
    p->async_hub_groups = 32;
    p->async_min_label = 1;
    p->async_interleave = 0;
    p->table_values_64 = 0;
    p->pruner_weights = nullptr;
    p->pruner_threshold = 0.5;
}

louvain_status louvain_workspace_size(const louvain_graph* g, const louvain_params* p, size_t* bytes) {
    return louvain_workspace_size_batch(g, 0, p, bytes);
}

louvain_status louvain_workspace_size_batch(const louvain_graph* g, int64_t count, const louvain_params* p,
                                            size_t* bytes) {
    if (!g || !p || !bytes) return fail(nullptr, LOUVAIN_ERR_INVALID, "null argument");
    if (g->n < 0 || g->nnz < 0 || g->n > 0x7ffffffeLL)
        return fail(nullptr, LOUVAIN_ERR_INVALID, "n must be in [0, 2^31-2] and nnz >= 0");
    if (count < 0 || count > 0x7ffffffeLL) return fail(nullptr, LOUVAIN_ERR_INVALID, "invalid graph count");
    Layout L;
    make_layout(g->n, g->nnz, count, p->async_slices, &L);
    *bytes = L.total;
    return LOUVAIN_OK;
}

}  // extern "C"

namespace {

// stage/stage_up: fixed host staging buffers (1 MiB and 64 KiB) to use instead
// of allocating pinned ones, or nullptr.
louvain_status create_impl(const louvain_graph* g, const int64_t* vbase, int64_t count, const louvain_params* p,
                           void* stream, void* workspace, size_t workspace_bytes, louvain_t** out,
                           void* stage = nullptr, void* stage_up = nullptr, void* handle_mem = nullptr) {
    if (!out) return fail(nullptr, LOUVAIN_ERR_INVALID, "out is NULL");
    *out = nullptr;
    if (!g || !p) return fail(nullptr, LOUVAIN_ERR_INVALID, "null graph or params");
    if (g->n < 0 || g->nnz < 0 || g->n > 0x7ffffffeLL)
        return fail(nullptr, LOUVAIN_ERR_INVALID, "n must be in [0, 2^31-2] and nnz >= 0");
    if (g->offset_bits != 32 && g->offset_bits != 64)
        return fail(nullptr, LOUVAIN_ERR_INVALID, "offset_bits must be 32 or 64");
    if (g->offset_bits == 32 && g->nnz > 0x7fffffffLL)
        return fail(nullptr, LOUVAIN_ERR_INVALID, "nnz too large for 32-bit offsets");
    if (!g->offsets || (g->nnz > 0 && !g->indices))
        return fail(nullptr, LOUVAIN_ERR_INVALID, "offsets/indices missing");
    if (p->max_iterations < 1 || p->tol_den <= 0 || p->tol_num < 0 || p->tol_drop < 1 || p->agg_den <= 0 ||
        p->agg_num < 0 || p->pick_less < 0 || (p->mode != LOUVAIN_ASYNC && p->mode != LOUVAIN_SYNC) ||
        (p->pruner != LOUVAIN_PRUNE_NONE && p->pruner != LOUVAIN_PRUNE_FLAGS &&
         p->pruner != LOUVAIN_PRUNE_LEARNED) ||
        (p->guard_tolerance != 0 && p->guard_tolerance != 1) ||
        (p->table_values_64 != 0 && p->table_values_64 != 1) || p->async_slices < 0 || p->async_slice_min < 0 ||
        p->async_hub_groups < 0 || (p->device_loop != 0 && p->device_loop != 1))
        return fail(nullptr, LOUVAIN_ERR_INVALID, "invalid parameter value");
    if (p->device_loop && p->pruner == LOUVAIN_PRUNE_LEARNED)
        return fail(nullptr, LOUVAIN_ERR_INVALID, "device_loop does not run the learned pruner");
    if (p->pruner == LOUVAIN_PRUNE_LEARNED && !p->pruner_weights)
        return fail(nullptr, LOUVAIN_ERR_INVALID, "the learned pruner needs pruner_weights");
    if (p->pruner_threshold != p->pruner_threshold)
        return fail(nullptr, LOUVAIN_ERR_INVALID, "pruner_threshold is NaN");
    if (count > 0) {
        if (!vbase) return fail(nullptr, LOUVAIN_ERR_INVALID, "vbase is NULL");
        if (vbase[0] != 0 || vbase[count] != g->n)
            return fail(nullptr, LOUVAIN_ERR_INVALID, "vbase must start at 0 and end at n");
        for (int64_t k = 0; k < count; k++)
            if (vbase[k + 1] < vbase[k]) return fail(nullptr, LOUVAIN_ERR_INVALID, "vbase must be non-decreasing");
    }
    Layout lay;
    make_layout(g->n, g->nnz, count, p->async_slices, &lay);
    if (!workspace || workspace_bytes < lay.total || ((uintptr_t)workspace % ALIGN) != 0)
        return fail(nullptr, LOUVAIN_ERR_WORKSPACE, "workspace must be %zu bytes, 256-byte aligned (got %zu)",
                    lay.total, workspace_bytes);

    louvain_t* h = handle_mem ? new (handle_mem) louvain_s() : new (std::nothrow) louvain_s();
    if (!h) return fail(nullptr, LOUVAIN_ERR_NOMEM, "handle allocation failed");
    h->handle_owned = handle_mem == nullptr;
    h->stream = (hipStream_t)stream;
    h->g = *g;
    h->p = *p;
    h->ws = (char*)workspace;
    h->ws_bytes = workspace_bytes;
    h->lay = lay;
    h->nb = count;
    if (count > 0) h->vbase.assign(vbase, vbase + count + 1);
    h->L0.n = g->n;
    h->L0.nnz = g->nnz;
    h->L0.off = g->offsets;
    h->L0.idx = g->indices;
    h->L0.w = g->weights;
    h->L0.t.off64 = g->offset_bits == 64;
    h->L0.t.wk = g->weights ? 1 : 0;
    h->L0.t.acc64 = 0;
    h->mb = make_buckets(p->bucket_max_degree, NB_MOVE, MOVE_CAP, MOVE_DEFAULT_MAX);
    h->ab = make_buckets(p->agg_bucket_max, NB_AGG, AGG_CAP, AGG_DEFAULT_MAX);
    auto bail = [&](louvain_status st) {
        g_create_error = h->err;
        louvain_destroy(h);
        return st;
    };
    if (stage && stage_up) {
        h->pinned = stage;
        h->pinned_up = stage_up;
        h->stage_owned = false;
    } else if (hipHostMalloc(&h->pinned, 1 << 20, hipHostMallocDefault) != hipSuccess ||
               hipHostMalloc(&h->pinned_up, 1 << 16, hipHostMallocDefault) != hipSuccess) {
        h->err = "pinned host allocation failed";
        return bail(LOUVAIN_ERR_HIP);
    }
    // zero control block, pruning flags and moved-iteration tags
    if (hipMemsetAsync(h->ctl(), 0, sizeof(Ctl), h->stream) != hipSuccess ||
        hipMemsetAsync(h->at<uint8_t>(lay.mark), 0, (size_t)std::max<int64_t>(g->n, 1) * 2, h->stream) !=
            hipSuccess ||
        hipMemsetAsync(h->at<uint32_t>(lay.f_moved), 0, (size_t)std::max<int64_t>(g->n, 1) * 4, h->stream) !=
            hipSuccess) {
        h->err = "workspace initialisation failed";
        return bail(LOUVAIN_ERR_HIP);
    }
    // endpoints of the offsets array
    if (g->n >= 0) {
        int64_t ends[2] = {0, 0};
        const size_t ob = g->offset_bits / 8;
        char tmp[16] = {};
        if (hipMemcpyAsync(tmp, g->offsets, ob, hipMemcpyDeviceToHost, h->stream) != hipSuccess ||
            hipMemcpyAsync(tmp + 8, (const char*)g->offsets + ob * g->n, ob, hipMemcpyDeviceToHost, h->stream) !=
                hipSuccess ||
            hipStreamSynchronize(h->stream) != hipSuccess) {
            h->err = "cannot read offsets";
            return bail(LOUVAIN_ERR_HIP);
        }
        if (ob == 4) { ends[0] = *(int32_t*)tmp; ends[1] = *(int32_t*)(tmp + 8); }
        else { ends[0] = *(int64_t*)tmp; ends[1] = *(int64_t*)(tmp + 8); }
        if (ends[0] != 0 || ends[1] != g->nnz) {
            h->err = "offsets[0] must be 0 and offsets[n] must equal nnz";
            return bail(LOUVAIN_ERR_INVALID);
        }
    }
    // total weight (and validation)
    launch_validate(h->L0, p->validate ? 1 : 0, h->ctl(), h->stream);
    Ctl c;
    if (readback(h, &c, h->ctl(), sizeof(Ctl)) != LOUVAIN_OK) return bail(LOUVAIN_ERR_HIP);
    if (c.err) {
        h->err = std::string("invalid graph:") + ((c.err & 1) ? " offsets not monotone" : "") +
                 ((c.err & 2) ? " index out of range" : "") + ((c.err & 4) ? " non-positive weight" : "");
        return bail(LOUVAIN_ERR_INVALID);
    }
    h->W = (int64_t)c.wsum;
    h->rows_unique0 = c.unsorted == 0;
    if (c.wsum > ((u64)1 << 62)) {
        h->err = "total weight exceeds 2^62";
        return bail(LOUVAIN_ERR_OVERFLOW);
    }
    u64 wmax = c.wsum;
    if (count > 0) {
        // graph ids, per-graph total weights, arcs confined to their graph
        int64_t* vb_dev = h->at<int64_t>(lay.vbase);
        u64* Wg_dev = h->at<u64>(lay.Wg);
        if (hipMemcpyAsync(vb_dev, vbase, (size_t)(count + 1) * 8, hipMemcpyHostToDevice, h->stream) != hipSuccess ||
            hipMemsetAsync(Wg_dev, 0, (size_t)count * 8, h->stream) != hipSuccess) {
            h->err = "batch initialisation failed";
            return bail(LOUVAIN_ERR_HIP);
        }
        launch_gid_init(vb_dev, count, g->n, h->at<int32_t>(lay.gid0), h->stream);
        launch_graph_weights(h->L0, h->at<int32_t>(lay.gid0), Wg_dev, h->ctl(), h->stream);
        h->Wg.resize(count);
        if (readback(h, h->Wg.data(), Wg_dev, (size_t)count * 8) != LOUVAIN_OK ||
            readback(h, &c, h->ctl(), sizeof(Ctl)) != LOUVAIN_OK)
            return bail(LOUVAIN_ERR_HIP);
        if (c.err & 8) {
            h->err = "invalid batch: an arc joins two different graphs";
            return bail(LOUVAIN_ERR_INVALID);
        }
        wmax = 0;
        for (u64 x : h->Wg) wmax = std::max(wmax, x);
    }
    h->sup_off64 = g->nnz > 0x7fffffffLL;
    h->sup_wk = wmax < 0x7fffffffULL ? 1 : 2;
    *out = h;
    return LOUVAIN_OK;
}

}  // namespace

extern "C" {

louvain_status louvain_create(const louvain_graph* g, const louvain_params* p, void* stream, void* workspace,
                              size_t workspace_bytes, louvain_t** out) {
    return create_impl(g, nullptr, 0, p, stream, workspace, workspace_bytes, out);
}

louvain_status louvain_create_batch(const louvain_graph* g, const int64_t* vbase, int64_t count,
                                    const louvain_params* p, void* stream, void* workspace, size_t workspace_bytes,
                                    louvain_t** out) {
    if (count < 1) return fail(nullptr, LOUVAIN_ERR_INVALID, "count must be >= 1");
    return create_impl(g, vbase, count, p, stream, workspace, workspace_bytes, out);
}

}  // extern "C"

namespace {

struct Runner {
    louvain_t* h;
    hipStream_t s;
    louvain_status st = LOUVAIN_OK;
    std::vector<int64_t> hub_pre;

    explicit Runner(louvain_t* hh) : h(hh), s(hh->stream) {}

    Ctl* ctl() { return h->ctl(); }
    template <typename T>
    T* at(size_t off) { return h->at<T>(off); }

    louvain_status memset_ctl_range(size_t off, size_t bytes) {
        HIPCHK(h, hipMemsetAsync((char*)ctl() + off, 0, bytes, s));
        return LOUVAIN_OK;
    }

    // Split the hub list into chunks whose table capacities fit the pool.
    // Fails if one table alone exceeds the pool (cannot happen for
    // capacities bounded by 2 * n, which the pool always holds).
    bool chunks(const std::vector<int64_t>& pre, int64_t pool, std::vector<std::pair<int32_t, int32_t>>* out) {
        out->clear();
        const int32_t cnt = (int32_t)pre.size() - 1;
        int32_t lo = 0;
        while (lo < cnt) {
            if (pre[lo + 1] - pre[lo] > pool) return false;
            int32_t hi = lo + 1;
            while (hi < cnt && pre[hi + 1] - pre[lo] <= pool) hi++;
            out->push_back({lo, hi});
            lo = hi;
        }
        return true;
    }

    louvain_status run();
};

louvain_status Runner::run() {
    louvain_t* H = h;
    const louvain_params& P = H->p;
    const Layout& Y = H->lay;
    const int64_t n0 = H->g.n;
    const int64_t W = H->W;
    const int sync = P.mode == LOUVAIN_SYNC;
    const int prune = P.pruner != LOUVAIN_PRUNE_NONE;
    const int learned = P.pruner == LOUVAIN_PRUNE_LEARNED;
    // learned pruning or sample recording needs the per-vertex feature state
    const int learn = learned || (H->smp_buf && H->smp_rate > 0 && H->smp_cap > 0);
    const float zt = P.pruner_threshold <= 0.0 ? -INFINITY
                     : P.pruner_threshold >= 1.0 ? INFINITY
                     : (float)std::log(P.pruner_threshold / (1.0 - P.pruner_threshold));
    i64* f_own = at<i64>(Y.f_own);
    i64* f_adv = at<i64>(Y.f_adv);
    uint32_t* f_moved = at<uint32_t>(Y.f_moved);
    int32_t* f_nm = at<int32_t>(Y.f_nm);
    int32_t* C = at<int32_t>(Y.C);
    int32_t* Cp = at<int32_t>(Y.Cp);
    i64* K = at<i64>(Y.K);
    i64* Sig = at<i64>(Y.Sig);
    uint8_t* flags = at<uint8_t>(Y.mark);
    uint8_t* vb = at<uint8_t>(Y.vbucket);
    int32_t* blist = at<int32_t>(Y.blist);
    int32_t* qbuf[2] = {at<int32_t>(Y.qa), at<int32_t>(Y.qb)};
    int32_t* gdec = at<int32_t>(Y.gdec);
    int32_t* blkcnt = at<int32_t>(Y.blkcnt);
    int32_t* blkoff = at<int32_t>(Y.blkoff);
    void* scan = at<void>(Y.scan);

    memset(&H->st, 0, sizeof(H->st));
    H->syncs = 0;
    H->smp_count = 0;
    H->recs.clear();
    H->evnext = 0;
    HIPCHK(H, hipMemsetAsync(ctl(), 0, sizeof(Ctl), s));
    iota_i32(C, n0, s);

    LevelView L = H->L0;
    // rows without repeated neighbours: the input when validated so, every
    // super-graph (compacted rows) -- SYNC iteration 0 may then decide hubs
    // straight from their rows
    bool uniq = H->rows_unique0;
    bool stopped_before_aggregate = false;
    bool have_newid = false;
    int64_t ncom_last = 0;
    std::vector<int32_t> hcp;
    std::vector<int64_t> hsig;

    // batched runs: per-graph state (the graphs move in lockstep passes; a
    // graph converged in the current pass, or stopped, is skipped)
    const int64_t nbg = H->nb;
    const bool batch = nbg > 0;
    int32_t* gidb[2] = {batch ? at<int32_t>(Y.gid[0]) : nullptr, batch ? at<int32_t>(Y.gid[1]) : nullptr};
    int gsel = 0;
    uint8_t* gact_dev = batch ? at<uint8_t>(Y.gact) : nullptr;
    u64* Wg_dev = batch ? at<u64>(Y.Wg) : nullptr;
    u64* Sg_dev = batch ? at<u64>(Y.Sg) : nullptr;
    u64* Pg_dev = batch && learned ? at<u64>(Y.Pg) : nullptr;
    u64* gcnt_dev = batch ? at<u64>(Y.gcnt) : nullptr;
    // gsw: graph g sweeps in the current iteration; want: in the next one
    std::vector<uint8_t> alive(nbg, 1), act(nbg, 0), ran(nbg, 0), gsw(nbg, 1), want(nbg, 0), gany(nbg, 0);
    uint8_t* gsweep_dev = batch && learned ? at<uint8_t>(Y.gsweep) : nullptr;
    uint8_t* gany_dev = batch && learned ? at<uint8_t>(Y.gany) : nullptr;
    std::vector<int32_t> li_g(nbg, 0);
    std::vector<int64_t> nver(nbg, 0);
    std::vector<u64> hS(2 * nbg), hcnt(2 * nbg), hP(nbg);
    u64 Wmax = (u64)W;
    if (batch) {
        for (int64_t g = 0; g < nbg; g++) nver[g] = H->vbase[g + 1] - H->vbase[g];
        H->b_passes.assign(nbg, 0);
        H->b_iters.assign(nbg, 0);
        H->b_comms.assign(nbg, 0);
        Wmax = 0;
        for (u64 x : H->Wg) Wmax = std::max(Wmax, x);
        if (n0 > 0) HIPCHK(H, hipMemcpyAsync(gidb[0], at<int32_t>(Y.gid0), (size_t)n0 * 4, hipMemcpyDeviceToDevice, s));
    }
    // per-graph byte arrays to the device (the staging buffer is reused by
    // the next upload, so a pageable or shared one is waited for)
    auto upload_bytes = [&](uint8_t* dev, const std::vector<uint8_t>& src) -> louvain_status {
        if (nbg <= (1 << 16)) {
            if ((st = sync_stream(H)) != LOUVAIN_OK) return st;  // the previous upload has left the staging buffer
            memcpy(H->pinned_up, src.data(), (size_t)nbg);
            HIPCHK(H, hipMemcpyAsync(dev, H->pinned_up, (size_t)nbg, hipMemcpyHostToDevice, s));
            if (!H->stage_owned && (st = sync_stream(H)) != LOUVAIN_OK) return st;
        } else {
            HIPCHK(H, hipMemcpyAsync(dev, src.data(), (size_t)nbg, hipMemcpyHostToDevice, s));
            if ((st = sync_stream(H)) != LOUVAIN_OK) return st;
        }
        return LOUVAIN_OK;
    };
    auto upload_act = [&]() -> louvain_status { return upload_bytes(gact_dev, act); };
    // device-driven iterations: the tests between iterations run in k_iter_end
    const bool devloop = P.device_loop != 0;
    if (devloop && (learn || H->itfn))
        return fail(H, LOUVAIN_ERR_INVALID,
                    "device_loop runs take no learned pruner, sample recording or iteration trace");
    DevIter* dit = devloop ? at<DevIter>(Y.dit) : nullptr;
    int32_t* lig_dev = devloop && batch ? at<int32_t>(Y.lig) : nullptr;

    for (int pass = 0; P.max_passes <= 0 || pass < P.max_passes; pass++) {
        const int64_t n = L.n;
        have_newid = false;
        const int32_t* gid = batch ? gidb[gsel] : nullptr;
        if (batch) {
            for (int64_t g = 0; g < nbg; g++) {
                act[g] = ran[g] = alive[g];
                li_g[g] = P.max_iterations;
                gsw[g] = 1;  // iteration 0 of a pass is every graph's sweep
            }
            if ((st = upload_act()) != LOUVAIN_OK) return st;
            HIPCHK(H, hipMemsetAsync(gcnt_dev, 0, (size_t)nbg * 16, s));
            launch_nonisolated_by_graph(L, gid, gcnt_dev, s);
        }
        // ---------------- pass init: classify, bucket lists, K', Sigma'
        HIPCHK(H, hipMemsetAsync(&ctl()->kmax, 0, sizeof(u64), s));
        const int NBT = NB_MOVE + 1;  // LDS buckets + hub
        int32_t bcount[MAX_BUCKETS] = {};
        timed(H, K_PASS_INIT, 0, [&] {
            launch_classify(L, H->mb, vb, Cp, K, Sig, ctl(), s);
            bucketize_vertices(n, vb, nullptr, 0, nullptr, nullptr, blkcnt, blkoff, blist, ctl()->bcount, scan, s);
        });
        if ((st = readback(H, bcount, ctl()->bcount, NBT * sizeof(int32_t))) != LOUVAIN_OK) return st;
        int64_t segs[MAX_BUCKETS + 1];
        segs[0] = 0;
        for (int b = 0; b < NBT; b++) segs[b + 1] = segs[b] + bcount[b];
        const int64_t nonisolated = segs[NBT];
        if (L.t.wk != 0)  // unit weights: the row sums are the degrees, written by the classification
            timed(H, K_PASS_INIT, 0, [&] {
                for (int b = 0; b < NBT; b++)
                    launch_rowsum(L, b, blist + segs[b], bcount[b], K, Sig, ctl(), s);
            });
        // hub tables and insert chunks over the static hub list (ascending vertex id)
        const int32_t nhub = bcount[NB_MOVE];
        const int32_t* hub_list = blist + segs[NB_MOVE];
        int64_t* hpre = at<int64_t>(Y.hpre);
        int64_t* hchpre = at<int64_t>(Y.bchpre);
        std::vector<int64_t> hch_pre;
        std::vector<std::pair<int32_t, int32_t>> hub_groups;
        if (nhub > 0) {
            launch_hub_caps(L, hub_list, nhub, at<int64_t>(Y.hcaps), at<int64_t>(Y.bnch), s);
            scan_i64_to_i64(at<int64_t>(Y.hcaps), hpre, nhub, scan, s);
            scan_i64_to_i64(at<int64_t>(Y.bnch), hchpre, nhub, scan, s);
            hub_pre.resize(nhub + 1);
            hch_pre.resize(nhub + 1);
            if ((st = readback(H, hub_pre.data(), hpre, (nhub + 1) * sizeof(int64_t))) != LOUVAIN_OK) return st;
            if ((st = readback(H, hch_pre.data(), hchpre, (nhub + 1) * sizeof(int64_t))) != LOUVAIN_OK) return st;
            if (!chunks(hub_pre, Y.pool_entries, &hub_groups))
                return fail(H, LOUVAIN_ERR_WORKSPACE, "hub hash table exceeds the workspace pool");
            int64_t most = 0;
            for (auto& gr : hub_groups) most = std::max(most, hub_pre[gr.second] - hub_pre[gr.first]);
            launch_big_clear(at<int32_t>(Y.pool_keys), at<void>(Y.pool_vals), most, s);
            HIPCHK(H, hipMemsetAsync(at<int32_t>(Y.hcnt), 0, (size_t)nhub * 4, s));
        }
        u64 kmax = 0;
        if ((st = readback(H, &kmax, &ctl()->kmax, sizeof(u64))) != LOUVAIN_OK) return st;
        const bool wide = (unsigned __int128)Wmax * kmax >= ((unsigned __int128)1 << 62);
        LevelView LM = L;
        LM.t.acc64 = P.table_values_64 || kmax >= ((u64)1 << 32);

        // ---------------- local moving
        int32_t li = P.max_iterations;
        int32_t counts[MAX_BUCKETS + 1];
        int64_t csegs[MAX_BUCKETS + 1];
        for (int b = 0; b < NBT; b++) counts[b] = bcount[b];
        for (int b = 0; b <= NBT; b++) csegs[b] = segs[b];
        const int32_t* cur_list = blist;  // iteration 0: every vertex with an arc
        int qsel = 0;
        u64 prev_b[5][MAX_BUCKETS] = {};
        const int mode = sync ? 0 : (P.async_coherent ? 2 : 1);
        bool sweep = learned;          // LEARNED: iteration 0 is a sweep
        int64_t smp_lo = 0, smp_hi = 0;  // samples recorded for the current iteration
        // device-driven iterations: the host uses the pass's bucket sizes as
        // launch bounds (counts/csegs stay those of iteration 0) and reads the
        // pass's state back after chunks of 2, 4, 8, ... iterations
        int32_t chunk_end = 0, chunk_len = 2;
        std::vector<int32_t> seg_ub;  // batched slices: per bucket, a bound on any slice's entries
        int32_t* dshare = devloop ? at<int32_t>(Y.dshare) : nullptr;
        // ASYNC slices of iteration t: at most async_slices, at least
        // async_slice_min queued vertices per slice (device-driven: counted on
        // the pass's first queue, for every iteration of the pass)
        auto slices_of = [&](int t, int64_t queued) {
            const bool slice_now = P.async_slice_iters <= 0 || t < P.async_slice_iters;
            int ns = (!sync && P.async_slices > 1 && slice_now) ? P.async_slices : 1;
            ns = (int)std::max<int64_t>(1, std::min<int64_t>(ns, queued / std::max(1, P.async_slice_min)));
            // a huge single-graph level: at most SLICE_SPAN queued vertices per
            // slice, up to twice async_slices (batched graphs are small)
            if (!batch && ns > 1 && ns == P.async_slices)
                ns = (int)std::min<int64_t>(2 * (int64_t)P.async_slices, std::max<int64_t>(ns, queued / SLICE_SPAN));
            return ns;
        };
        auto interleaved = [&](int ns) { return !sync && P.async_interleave && ns > 1 ? 1 : 0; };
        if (devloop) {
            const int ns0 = slices_of(0, nonisolated);
            launch_iter_setup(dit, ctl()->bcount, NBT, P.max_iterations, dshare, ns0, interleaved(ns0), s);
            if (batch) fill_i32(lig_dev, P.max_iterations, nbg, s);
            chunk_end = std::min(P.max_iterations, chunk_len);
        }
        // profiling: algorithmic bytes of the move launches since the last
        // call, per bucket, from the run's cumulative counters hc->bstat
        auto attribute_move_bytes = [&](const Ctl* hc) {
            for (int b = 0; b < NBT; b++) {
                u64 cur[5];
                for (int q = 0; q < 5; q++) {
                    cur[q] = 0;
                    for (int k = 0; k < STRIPES; k++) cur[q] += hc->bstat[q][b][k];
                }
                const u64 de = cur[0] - prev_b[0][b];
                if (de) {
                    const int64_t bytes = move_alg_bytes(LM, de, cur[1] - prev_b[1][b], cur[2] - prev_b[2][b],
                                                         cur[3] - prev_b[3][b], cur[4] - prev_b[4][b], sync, learn);
                    const int kind = b < 4 ? K_MOVE_FUSED : (b == 4 ? K_MOVE4 : K_MOVE_HUB);
                    for (auto r = H->recs.rbegin(); r != H->recs.rend(); ++r)
                        if (r->kind == kind) { r->bytes += bytes; break; }
                }
                for (int q = 0; q < 5; q++) prev_b[q][b] = cur[q];
            }
        };
        // learned pruner (or sample recording): features and MLP over the
        // vertices flagged by iteration t, then the queue of iteration t + 1
        // from the kept flags (vertices of stopped graphs are left out)
        auto run_filter = [&](int t, uint32_t stamp_next, uint8_t* fnext, const uint8_t* gsw_dev,
                              uint8_t* gany_out) {
            FilterArgs fa{};
            fa.off = L.off;
            fa.n = n;
            fa.K = K;
            fa.own = f_own;
            fa.adv = f_adv;
            fa.moved = f_moved;
            fa.nm = f_nm;
            fa.itag_prev = stamp_next;
            fa.pass = pass;
            fa.t = t + 1;
            fa.flags = fnext;
            fa.all = prune ? 0 : 1;
            fa.learned = learned;
            fa.weights = P.pruner_weights;
            fa.zt = zt;
            fa.samples = H->smp_buf;
            fa.cap = H->smp_buf ? H->smp_cap : 0;
            fa.per_mille = H->smp_buf ? H->smp_rate : 0;
            fa.ctl = ctl();
            fa.gid = gid;
            fa.gsweep = gsw_dev;
            fa.gany = gany_out;
            timed(H, K_LEARN_FILTER, 0, [&] { launch_learn_filter(fa, L.t.off64, s); });
        };
        auto filter_next = [&](int t, uint32_t stamp_next, uint8_t* fnext, int32_t* qnext, IterTotals* itp,
                               int64_t* kept_out, bool filter = true) -> louvain_status {
            Ctl* hc = (Ctl*)H->pinned;
            const int64_t before = H->smp_count;
            if (filter) run_filter(t, stamp_next, fnext, nullptr, nullptr);
            if (prune)
                timed(H, K_QUEUE, 0, [&] {
                    bucketize_vertices(n, vb, fnext, 1, gid, gact_dev, blkcnt, blkoff, qnext, ctl()->qcount, scan, s);
                });
            HIPCHK(H, hipMemcpyAsync(hc, ctl(), CTL_ITER_BYTES, hipMemcpyDeviceToHost, s));
            HIPCHK(H, hipMemcpyAsync(&hc->nsamples, &ctl()->nsamples, sizeof(u64), hipMemcpyDeviceToHost, s));
            if ((st = sync_stream(H)) != LOUVAIN_OK) return st;
            *itp = sum_iter(*hc);
            H->smp_count = std::min<int64_t>((int64_t)hc->nsamples, H->smp_cap);
            smp_lo = before;
            smp_hi = H->smp_count;
            int64_t kept = 0;
            for (int b = 0; b < NBT; b++) kept += itp->qcount[b];
            if (H->prof) {
                const int64_t flagged = prune ? kept + (int64_t)hc->pruned : nonisolated;
                const int64_t bytes = filter_alg_bytes(L, n, flagged, (int64_t)hc->pruned, smp_hi - smp_lo);
                for (auto r = H->recs.rbegin(); r != H->recs.rend(); ++r)
                    if (r->kind == K_LEARN_FILTER) { r->bytes += bytes; break; }
            }
            *kept_out = kept;
            return LOUVAIN_OK;
        };
        for (int t = 0; t < P.max_iterations; t++) {
            const int pl = P.pick_less > 0 && ((t + P.pick_less / 2) % P.pick_less) == 0;
            const uint32_t stamp_next = ++H->stamp;  // unique tag of this iteration
            uint8_t* fnext = flags + (size_t)(stamp_next & 1) * (size_t)n0;
            const uint8_t* fcur = flags + (size_t)((stamp_next + 1) & 1) * (size_t)n0;
            if (devloop) {
                // one zeroing launch, which does nothing once the pass has ended
                ZeroRanges z{};
                z.p[0] = ctl();
                z.bytes[0] = (int64_t)CTL_ITER_BYTES;
                if (batch) { z.p[1] = Sg_dev; z.bytes[1] = nbg * 16; }
                if (prune) { z.p[2] = fnext; z.bytes[2] = n; }
                launch_zero_ranges(dit, z, s);
            } else {
                HIPCHK(H, hipMemsetAsync(ctl(), 0, CTL_ITER_BYTES, s));
                if (learn) HIPCHK(H, hipMemsetAsync(f_nm, 0, (size_t)n * 4, s));
                if (batch) HIPCHK(H, hipMemsetAsync(Sg_dev, 0, (size_t)nbg * 16, s));
                if (Pg_dev) HIPCHK(H, hipMemsetAsync(Pg_dev, 0, (size_t)nbg * 8, s));
                if (prune) HIPCHK(H, hipMemsetAsync(fnext, 0, (size_t)n, s));
            }
            if (sweep) {
                H->st.sweeps++;
            } else if (batch && learned) {
                for (int64_t g = 0; g < nbg; g++)
                    if (act[g] && gsw[g]) { H->st.sweeps++; break; }
            }
            int32_t* qnext = qbuf[qsel];
            MoveArgs a{};
            a.off = L.off;
            a.idx = L.idx;
            a.w = L.w;
            a.Cp = Cp;
            a.Sig = Sig;
            a.K = K;
            a.W = W;
            a.wide = wide;
            a.pl = pl;
            a.min_label = P.async_min_label;
            a.prune = prune;
            a.fnext = fnext;
            a.fcur = fcur;
            a.ctl = ctl();
            a.sdec = at<int32_t>(Y.sdec);
            a.vbucket = vb;
            a.hub_list = hub_list;
            a.hub_pre = hpre;
            a.hch_pre = hchpre;
            a.all_queued = (t == 0 || !prune || sweep) ? 1 : 0;
            a.gdec = gdec;
            a.hub_keys = at<int32_t>(Y.pool_keys);
            a.hub_vals = at<void>(Y.pool_vals);
            a.hub_cnt = at<int32_t>(Y.hcnt);
            a.hub_slots = at<int32_t>(Y.hslots);
            a.hub_part = at<HubPart>(Y.hpart);
            a.gid = gid;
            a.Wg = Wg_dev;
            a.gact = gact_dev;
            a.Sg = Sg_dev;
            a.Pg = Pg_dev;
            a.learn = learn;
            a.itag = stamp_next;
            a.f_own = f_own;
            a.f_adv = f_adv;
            a.f_moved = f_moved;
            a.f_nm = f_nm;
            a.dit = dit;
            a.dshare = dshare;
            // hubs: chunked inserts, one decision per hub, chunked stamping, for
            // the static hub positions [s_lo, s_hi) whose tables share the pool
            // SYNC iteration 0 decides against the identity membership, so hubs
            // decide straight from their rows (no tables)
            const bool hub_direct = sync && t == 0 && uniq && nhub > 0;
            const bool hubs_now = nhub > 0 && (devloop || counts[NB_MOVE] > 0);
            auto hubs_range = [&](int32_t s_lo, int32_t s_hi, bool decide_phase, bool mark_phase) {
                a.bucket = NB_MOVE;
                for (auto& gr : hub_groups) {
                    const int32_t lo = std::max(gr.first, s_lo), hi = std::min(gr.second, s_hi);
                    if (lo >= hi) continue;
                    a.g_lo = lo;
                    a.g_hi = hi;
                    a.tab_lo = lo;
                    const int64_t nchunks = hch_pre[hi] - hch_pre[lo];
                    if (decide_phase) {
                        if (!hub_direct)
                            timed(H, K_MOVE_HUB, 0, [&] { launch_hub_insert(LM, mode, a, nchunks, s); });
                        // decide launches of at most part_cap blocks (all blocks of a hub in one launch)
                        for (int32_t sl = lo; sl < hi;) {
                            int32_t sh = sl + 1;
                            while (sh < hi && hch_pre[sh + 1] - hch_pre[sl] <= Y.part_cap) sh++;
                            MoveArgs ad = a;
                            ad.g_lo = sl;
                            ad.g_hi = sh;
                            timed(H, K_HUB_DECIDE, 0, [&] {
                                if (hub_direct) launch_hub_direct(LM, mode, ad, hch_pre[sh] - hch_pre[sl], s);
                                else launch_hub_decide(LM, mode, ad, hch_pre[sh] - hch_pre[sl], s);
                                launch_hub_final(LM, mode, ad, s);
                            });
                            sl = sh;
                        }
                        a.g_lo = lo;
                        a.g_hi = hi;
                    }
                    if (mark_phase && (prune || learn))
                        timed(H, K_HUB_MARK, 0, [&] { launch_hub_mark(L, a, nchunks, s); });
                }
            };
            // ASYNC: the iteration runs as ns slices in vertex-id order (each
            // bucket's queue is sorted by id; slice sl takes the sl-th share of
            // every bucket), at least async_slice_min queued vertices per slice.
            int64_t queued = 0;
            for (int b = 0; b < NBT; b++) queued += counts[b];
            const int ns = slices_of(t, queued);
            // hub groups: group k covers the static hub positions [k*nhub/hg, (k+1)*nhub/hg)
            // and runs with slice due(k) = (k+1)*ns/hg - 1
            // (a level with more slices than async_slices scales its hub groups alike)
            const int hg = (!sync && P.async_hub_groups > 0)
                               ? (int)std::min<int64_t>(ns, ns > P.async_slices
                                                                ? (int64_t)P.async_hub_groups * ns / P.async_slices
                                                                : P.async_hub_groups)
                               : ns;
            // batched ASYNC: slice sl takes the sl-th share of every graph's part
            // of each bucket's queue (graphs are contiguous id ranges, so plain
            // contiguous slices would hold whole graphs)
            const bool segmented = batch && !sync && ns > 1;
            int32_t* segcnt = segmented ? at<int32_t>(Y.segcnt) : nullptr;
            int32_t* segstart = segmented ? at<int32_t>(Y.segstart) : nullptr;
            int32_t* prefall = segmented ? at<int32_t>(Y.prefall) : nullptr;
            std::vector<int32_t> segtot;
            if (segmented) {
                if (devloop) {
                    ZeroRanges z{};
                    z.p[0] = segcnt;
                    z.bytes[0] = (int64_t)NB_MOVE * nbg * 4;
                    launch_zero_ranges(dit, z, s);
                } else {
                    HIPCHK(H, hipMemsetAsync(segcnt, 0, (size_t)NB_MOVE * nbg * 4, s));
                }
                for (int b = 0; b < NB_MOVE; b++)
                    launch_seg_count(devloop ? cur_list : cur_list + csegs[b], counts[b], gid,
                                     segcnt + (int64_t)b * nbg, s, dit, b);
                for (int b = 0; b < NB_MOVE; b++)
                    scan_i32_to_i32(segcnt + (int64_t)b * nbg, segstart + (int64_t)b * (nbg + 1), nbg, scan, s);
                launch_slice_prefix(segcnt, NB_MOVE, nbg, ns, prefall, s);
                if (!devloop || t == 0) {
                    std::vector<int32_t> hseg((size_t)NB_MOVE * nbg);
                    if ((st = readback(H, hseg.data(), segcnt, hseg.size() * 4)) != LOUVAIN_OK) return st;
                    segtot.assign((size_t)NB_MOVE * ns, 0);
                    seg_ub.assign(NB_MOVE, 0);
                    for (int b = 0; b < NB_MOVE; b++)
                        for (int64_t g = 0; g < nbg; g++) {
                            const int64_t len = hseg[(size_t)b * nbg + g];
                            if (!len) continue;
                            for (int k = 0; k < ns; k++)
                                segtot[(size_t)b * ns + k] += (int32_t)(len * (k + 1) / ns - len * k / ns);
                            // a later queue holds at most len of graph g's entries: at most
                            // ceil(len / ns) of them in any slice
                            seg_ub[b] += (int32_t)((len + ns - 1) / ns);
                        }
                }
                a.seg_n = (int32_t)nbg;
                a.seg_ns = ns;
            }
            for (int sl = 0; sl < ns; sl++) {
                // entries of bucket b in this slice: contiguous share [lo, hi), or
                // (interleaved) every ns-th entry from sl on
                const bool inter = interleaved(ns);
                auto lo_of = [&](int b) { return inter ? 0 : (int32_t)((int64_t)counts[b] * sl / ns); };
                auto hi_of = [&](int b) {
                    return inter ? (counts[b] > sl ? (counts[b] - sl + ns - 1) / ns : 0)
                                 : (int32_t)((int64_t)counts[b] * (sl + 1) / ns);
                };
                a.lstride = inter ? ns : 1;
                a.lphase = inter ? sl : 0;
                a.seg_k = sl;
                a.slice = sl;
                // bucket b's entries of this slice (device-driven: the queue's base
                // and a bound on the count; the kernels find the true share)
                auto share = [&](int b, const int32_t** lst, int32_t* cnt) {
                    if (devloop) {
                        *lst = cur_list;
                        *cnt = segmented ? (t == 0 ? segtot[(size_t)b * ns + sl] : seg_ub[b])
                                         : (int32_t)(((int64_t)counts[b] + ns - 1) / ns);
                    } else {
                        const int32_t lo = segmented ? 0 : lo_of(b);
                        const int32_t hi = segmented ? segtot[(size_t)b * ns + sl] : hi_of(b);
                        *lst = cur_list + csegs[b] + lo;
                        *cnt = hi - lo;
                    }
                };
                auto seg_rows = [&](int b, const int32_t** pre, const int32_t** st0, const int32_t** cnt) {
                    *pre = prefall + ((int64_t)b * ns + sl) * (nbg + 1);
                    *st0 = segstart + (int64_t)b * (nbg + 1);
                    *cnt = segcnt + (int64_t)b * nbg;
                };
                int32_t h_lo = 0, h_hi = 0;  // hub positions due with this slice
                for (int k = 0; k < hg; k++)
                    if ((int)(((int64_t)(k + 1) * ns) / hg) - 1 == sl) {
                        if (h_hi == h_lo) h_lo = (int32_t)((int64_t)nhub * k / hg);
                        h_hi = (int32_t)((int64_t)nhub * (k + 1) / hg);
                    }
                if (P.bucket_order && hubs_now && h_hi > h_lo) hubs_range(h_lo, h_hi, true, !sync);
                FusedLists f{};
                f.blk_pre[0] = 0;
                for (int b = 0; b < 4; b++) {
                    share(b, &f.list[b], &f.count[b]);
                    if (segmented) seg_rows(b, &f.seg_pre[b], &f.seg_start[b], &f.seg_cnt[b]);
                    const int ng = 256 / MOVE_G[b];
                    f.blk_pre[b + 1] = f.blk_pre[b] + (f.count[b] + ng - 1) / ng;
                }
                if (f.blk_pre[4] > 0) timed(H, K_MOVE_FUSED, 0, [&] { launch_move_fused(LM, mode, a, f, s); });
                {
                    const int32_t* l4 = nullptr;
                    int32_t c4 = 0;
                    share(4, &l4, &c4);
                    if (c4 > 0) {
                        a.bucket = 4;
                        MoveArgs a4 = a;
                        if (segmented) seg_rows(4, &a4.seg_pre, &a4.seg_start, &a4.seg_cnt);
                        timed(H, K_MOVE4, 0, [&] { launch_move(LM, 4, mode, a4, l4, c4, s); });
                    }
                }
                if (!P.bucket_order && hubs_now && h_hi > h_lo) hubs_range(h_lo, h_hi, true, !sync);
            }
            if (sync) {
                timed(H, K_SYNC_APPLY, 0, [&] { launch_sync_apply(L, a, cur_list, csegs[NBT], s); });
                if (hubs_now) hubs_range(0, nhub, false, true);
            }
            if (learn) launch_learn_label(H->smp_buf, smp_lo, smp_hi, f_moved, stamp_next, s);
            if (prune && !learn)
                timed(H, K_QUEUE, 0, [&] {
                    bucketize_vertices(n, vb, fnext, 1, gid, gact_dev, blkcnt, blkoff, qnext, ctl()->qcount, scan, s,
                                       devloop ? &dit->halt : nullptr);
                });
            if (devloop) {
                // the tests between iterations, on the device
                IterEndArgs e{};
                e.dit = dit;
                e.ctl = ctl();
                e.t = t;
                e.may_end = sync || !pl;
                e.prune = prune;
                e.max_iterations = P.max_iterations;
                e.nbt = NBT;
                e.W = W;
                e.tol_num = P.tol_num;
                e.tol_den = P.tol_den;
                e.tol_drop = P.tol_drop;
                e.pass = pass;
                e.nbg = batch ? nbg : 0;
                e.Sg = Sg_dev;
                e.Wg = Wg_dev;
                e.gact = gact_dev;
                e.lig = lig_dev;
                e.dshare = dshare;
                e.ns_next = slices_of(t + 1, nonisolated);
                e.interleave = interleaved(e.ns_next);
                launch_iter_end(e, s);
                if (prune) {
                    cur_list = qnext;
                    qsel ^= 1;
                }
                if (t + 1 < chunk_end) continue;
                // end of a chunk: one readback of the pass's state
                Ctl* hc = (Ctl*)H->pinned;
                DevIter* hd = (DevIter*)((char*)H->pinned + (1 << 19));
                if (H->prof)
                    HIPCHK(H, hipMemcpyAsync(&hc->bstat, &ctl()->bstat, sizeof(hc->bstat), hipMemcpyDeviceToHost, s));
                HIPCHK(H, hipMemcpyAsync(hd, dit, sizeof(DevIter), hipMemcpyDeviceToHost, s));
                if ((st = sync_stream(H)) != LOUVAIN_OK) return st;
                if (H->prof) attribute_move_bytes(hc);
                if (!hd->halt && t + 1 < P.max_iterations) {
                    chunk_len *= 2;
                    chunk_end = std::min(P.max_iterations, t + 1 + chunk_len);
                    continue;
                }
                li = hd->halt ? hd->li : P.max_iterations;
                H->st.iterations += hd->ran + hd->extra;
                H->st.moves += (int64_t)hd->moves;
                if (batch && (st = readback(H, li_g.data(), lig_dev, (size_t)nbg * 4)) != LOUVAIN_OK) return st;
                break;
            }
            // read back the iteration's striped totals
            Ctl* hc = (Ctl*)H->pinned;
            HIPCHK(H, hipMemcpyAsync(hc, ctl(), CTL_ITER_BYTES, hipMemcpyDeviceToHost, s));
            if (H->prof) HIPCHK(H, hipMemcpyAsync(&hc->bstat, &ctl()->bstat, sizeof(hc->bstat), hipMemcpyDeviceToHost, s));
            if (batch) HIPCHK(H, hipMemcpyAsync(hS.data(), Sg_dev, (size_t)nbg * 16, hipMemcpyDeviceToHost, s));
            if (Pg_dev) HIPCHK(H, hipMemcpyAsync(hP.data(), Pg_dev, (size_t)nbg * 8, hipMemcpyDeviceToHost, s));
            if ((st = sync_stream(H)) != LOUVAIN_OK) return st;
            IterTotals it = sum_iter(*hc);
            const unsigned __int128 S = it.S;
            H->st.iterations++;
            H->st.moves += (int64_t)it.moves;
            // algorithmic bytes of this iteration's move launches, per bucket
            if (H->prof) attribute_move_bytes(hc);
            if (H->itfn) {
                hcp.resize(n);
                hsig.resize(n);
                if ((st = readback(H, hcp.data(), Cp, n * 4)) != LOUVAIN_OK) return st;
                if ((st = readback(H, hsig.data(), Sig, n * 8)) != LOUVAIN_OK) return st;
                H->itfn(H->user, pass, t, n, hcp.data(), hsig.data(), (int64_t)it.moves, (int64_t)(S >> 64),
                        (uint64_t)S);
            }
            // ASYNC: an iteration under Pick-Less rejects every move to a larger
            // id, so its gain sum says nothing about convergence; only the
            // other iterations may end the pass (SYNC keeps the exact rule)
            const bool may_end = sync || !pl;
            const bool conv = may_end && converged(S, W, P, pass);
            if (batch && learned) {
                // LEARNED, batched: every graph follows its own sweep schedule, as
                // in a lone run.  A graph's pass ends only at one of its sweeps
                // whose exit test passes in that graph (no evaluation with a
                // positive best gain, or the tolerance test).  Its next iteration
                // is a sweep after one of its non-sweep iterations passes the
                // tolerance test, or when the filter keeps none of its vertices;
                // in any other iteration its flagged vertices go through the
                // filter.  A sweep evaluates every vertex of the graph.
                bool changed = false, any = false, all_want = true;
                for (int64_t g = 0; g < nbg; g++) {
                    if (!act[g]) continue;
                    const unsigned __int128 Sg = ((unsigned __int128)hS[2 * g + 1] << 64) + hS[2 * g];
                    const bool conv_g = may_end && converged(Sg, (int64_t)H->Wg[g], P, pass);
                    if (gsw[g] && (P.guard_tolerance ? conv_g : hP[g] == 0)) {
                        li_g[g] = t + 1;
                        act[g] = 0;
                        want[g] = 0;
                        changed = true;
                    } else {
                        any = true;
                        want[g] = !gsw[g] && conv_g;
                        all_want = all_want && want[g];
                    }
                }
                if (!any) { li = t + 1; break; }
                if (changed && (st = upload_act()) != LOUVAIN_OK) return st;
                if (t + 1 >= P.max_iterations) continue;  // the loop ends: no next queue
                if (!all_want) {
                    // filter with the sweeping graphs kept whole, then sweep the
                    // graphs whose filtered queue came out empty
                    if ((st = upload_bytes(gsweep_dev, want)) != LOUVAIN_OK) return st;
                    HIPCHK(H, hipMemsetAsync(gany_dev, 0, (size_t)nbg, s));
                    run_filter(t, stamp_next, fnext, gsweep_dev, gany_dev);
                    if ((st = readback(H, gany.data(), gany_dev, (size_t)nbg)) != LOUVAIN_OK) return st;
                    bool extra = false;
                    all_want = true;
                    for (int64_t g = 0; g < nbg; g++) {
                        if (!act[g]) continue;
                        if (!want[g] && !gany[g]) { want[g] = 1; extra = true; }
                        all_want = all_want && want[g];
                    }
                    if (extra && !all_want) {
                        if ((st = upload_bytes(gsweep_dev, want)) != LOUVAIN_OK) return st;
                        run_filter(t, stamp_next, fnext, gsweep_dev, nullptr);
                    }
                }
                smp_lo = smp_hi = 0;
                if (all_want) {
                    cur_list = blist;
                    for (int b = 0; b < NBT; b++) counts[b] = bcount[b];
                    for (int b = 0; b <= NBT; b++) csegs[b] = segs[b];
                } else {
                    int64_t kept = 0;
                    if ((st = filter_next(t, stamp_next, fnext, qnext, &it, &kept, false)) != LOUVAIN_OK) return st;
                    H->st.pruned += (int64_t)hc->pruned;
                    csegs[0] = 0;
                    for (int b = 0; b < NBT; b++) {
                        counts[b] = it.qcount[b];
                        csegs[b + 1] = csegs[b] + counts[b];
                    }
                    cur_list = qnext;
                    qsel ^= 1;
                }
                for (int64_t g = 0; g < nbg; g++) gsw[g] = act[g] ? want[g] : 0;
                sweep = all_want;
                continue;
            }
            if (batch) {
                // per-graph tolerance tests; converged graphs stop moving for this pass
                bool changed = false, any = false;
                for (int64_t g = 0; g < nbg; g++) {
                    if (!act[g]) continue;
                    const unsigned __int128 Sg = ((unsigned __int128)hS[2 * g + 1] << 64) + hS[2 * g];
                    if (may_end && converged(Sg, (int64_t)H->Wg[g], P, pass)) {
                        li_g[g] = t + 1;
                        act[g] = 0;
                        changed = true;
                    } else {
                        any = true;
                    }
                }
                if (!any) { li = t + 1; break; }
                if (changed && (st = upload_act()) != LOUVAIN_OK) return st;
            } else if (!learn) {
                if (conv) { li = t + 1; break; }
            } else {
                // LEARNED: only a sweep that passes the exit test ends the pass
                if (learned ? (sweep && (P.guard_tolerance ? conv : it.positive == 0)) : conv) { li = t + 1; break; }
                bool next_sweep = learned && !sweep && conv;
                smp_lo = smp_hi = 0;
                if (!next_sweep && t + 1 < P.max_iterations) {
                    int64_t kept = 0;
                    if ((st = filter_next(t, stamp_next, fnext, qnext, &it, &kept)) != LOUVAIN_OK) return st;
                    if (learned) {
                        if (kept == 0) next_sweep = true;  // nothing kept: certify with a sweep
                        else H->st.pruned += (int64_t)hc->pruned;
                    }
                }
                if (!next_sweep && prune && t + 1 < P.max_iterations) {
                    int64_t total = 0;
                    csegs[0] = 0;
                    for (int b = 0; b < NBT; b++) {
                        counts[b] = it.qcount[b];
                        total += counts[b];
                        csegs[b + 1] = csegs[b] + counts[b];
                    }
                    cur_list = qnext;
                    qsel ^= 1;
                    if (total == 0) {
                        // flag pruning with nothing flagged: the next iteration has S = 0 and converges
                        H->st.iterations++;
                        if (H->itfn) H->itfn(H->user, pass, t + 1, n, hcp.data(), hsig.data(), 0, 0, 0);
                        li = t + 2;
                        break;
                    }
                }
                if (next_sweep) {
                    cur_list = blist;
                    for (int b = 0; b < NBT; b++) counts[b] = bcount[b];
                    for (int b = 0; b <= NBT; b++) csegs[b] = segs[b];
                }
                sweep = next_sweep;
                continue;
            }
            // next iteration's queue
            if (prune) {
                int64_t total = 0;
                csegs[0] = 0;
                for (int b = 0; b < NBT; b++) {
                    counts[b] = it.qcount[b];
                    total += counts[b];
                    csegs[b + 1] = csegs[b] + counts[b];
                }
                cur_list = qnext;
                qsel ^= 1;
                if (total == 0) {
                    // nothing flagged: the next iteration has S = 0 and converges
                    if (t + 1 >= P.max_iterations) { li = P.max_iterations; break; }
                    H->st.iterations++;
                    if (H->itfn) H->itfn(H->user, pass, t + 1, n, hcp.data(), hsig.data(), 0, 0, 0);
                    li = t + 2;
                    for (int64_t g = 0; g < nbg; g++)
                        if (act[g]) li_g[g] = t + 2;
                    break;
                }
            }
        }
        H->st.passes++;
        if (pass < 32) H->st.iterations_per_pass[pass] = li;
        stopped_before_aggregate = true;
        if (batch) {
            li = 0;
            for (int64_t g = 0; g < nbg; g++) {
                if (!ran[g]) continue;
                H->b_passes[g]++;
                H->b_iters[g] += li_g[g];
                li = std::max(li, li_g[g]);
                if (li_g[g] <= 1) alive[g] = 0;  // globally converged
            }
        }
        if (li <= 1) break;

        // ---------------- community counts and shrink tests
        int32_t* used = at<int32_t>(Y.used);
        int32_t* newid = at<int32_t>(Y.newid);
        HIPCHK(H, hipMemsetAsync(used, 0, (n + 1) * 4, s));
        timed(H, K_AGG_PREP, 0, [&] {
            launch_mark_used(Cp, n, used, s);
            scan_i32_to_i32(used, newid, n, scan, s);
            if (batch) launch_used_by_graph(used, n, gid, gcnt_dev + nbg, s);
        });
        int32_t gall = 0;
        if ((st = readback(H, &gall, newid + n, 4)) != LOUVAIN_OK) return st;
        have_newid = true;
        ncom_last = gall;
        if (pass < 32) H->st.communities_per_pass[pass] = gall;
        if (batch) {
            // per-graph shrink tests (Gamma over vertices with arcs); every graph is
            // aggregated while any graph continues (a stopped graph's aggregation
            // is its final lookup, and it stays still afterwards)
            if ((st = readback(H, hcnt.data(), gcnt_dev, (size_t)nbg * 16)) != LOUVAIN_OK) return st;
            bool any = false;
            for (int64_t g = 0; g < nbg; g++) {
                const int64_t nonis = (int64_t)hcnt[g], usedg = (int64_t)hcnt[nbg + g];
                if (ran[g] && alive[g]) {
                    const int64_t gamma = usedg - (nver[g] - nonis), gamma_old = nonis;
                    if (gamma == gamma_old ||
                        (unsigned __int128)gamma * (unsigned __int128)P.agg_den >
                            (unsigned __int128)P.agg_num * (unsigned __int128)gamma_old)
                        alive[g] = 0;
                }
                any |= alive[g] != 0;
                nver[g] = usedg;
            }
            if (!any) break;
        } else {
            const int64_t isolated = n - nonisolated;
            const int64_t gamma = gall - isolated, gamma_old = nonisolated;
            if (gamma == gamma_old) break;
            if ((unsigned __int128)gamma * (unsigned __int128)P.agg_den >
                (unsigned __int128)P.agg_num * (unsigned __int128)gamma_old)
                break;
        }

        // ---------------- renumber, dendrogram lookup, community CSR
        const int64_t ncom = gall;
        int32_t* cnt = at<int32_t>(Y.cnt);
        int32_t* coff = at<int32_t>(Y.coff);
        int32_t* cursor = at<int32_t>(Y.cursor);
        int32_t* members = at<int32_t>(Y.members);
        int64_t* cdeg = at<int64_t>(Y.cdeg);
        int64_t* hoff = at<int64_t>(Y.hoff);
        HIPCHK(H, hipMemsetAsync(cnt, 0, (ncom + 1) * 4, s));
        HIPCHK(H, hipMemsetAsync(cursor, 0, (ncom + 1) * 4, s));
        HIPCHK(H, hipMemsetAsync(cdeg, 0, (ncom + 1) * 8, s));
        int32_t* alist = at<int32_t>(Y.alist);
        if (batch) launch_gid_next(used, newid, n, gid, gidb[gsel ^ 1], s);
        timed(H, K_AGG_PREP, 0, [&] {
            launch_relabel(Cp, n, newid, s);
            launch_dendrogram(C, n0, Cp, s);
            launch_comm_count(L, Cp, cnt, cdeg, s);
            scan_i32_to_i32(cnt, coff, ncom, scan, s);
            scan_i64_to_i64(cdeg, hoff, ncom, scan, s);
            launch_comm_fill(n, Cp, coff, cursor, members, s);
            bucketize_communities(ncom, hoff, ncom, H->ab, at<int32_t>(Y.rowlen), blkcnt, blkoff, alist,
                                  ctl()->bcount, scan, s);
        });
        int32_t acount[MAX_BUCKETS] = {};
        const int NBA = NB_AGG + 1;
        if ((st = readback(H, acount, ctl()->bcount, NBA * sizeof(int32_t))) != LOUVAIN_OK) return st;
        int64_t asegs[MAX_BUCKETS + 1];
        asegs[0] = 0;
        for (int b = 0; b < NBA; b++) asegs[b + 1] = asegs[b] + acount[b];

        // ---------------- super-row hashing into the holey buffer
        AggArgs A{};
        A.Cp = Cp;
        A.coff = coff;
        A.members = members;
        A.hoff = hoff;
        A.hidx = at<int32_t>(Y.hidx);
        A.hw = at<void>(Y.hw);
        A.rowlen = at<int32_t>(Y.rowlen);
        A.out_w64 = H->sup_wk == 2;
        // Rows are sorted by neighbour id only when a pass callback receives
        // the super-graphs (the canonical form the traces compare); no
        // decision of the method depends on the order of a row's entries.
        A.sorted = H->pafn != nullptr;
        LevelView LA = L;
        LA.t.acc64 = P.table_values_64 || (u64)W >= ((u64)1 << 32);
        for (int b = 0; b < NB_AGG; b++) {
            if (acount[b] <= 0) continue;
            timed(H, K_AGG0 + b, 0, [&] { launch_aggregate(LA, b, A, alist + asegs[b], acount[b], s); });
        }
        const int32_t nbig = acount[NB_AGG];
        if (nbig > 0) {
            // big communities: virtual-arc positions, chunk and table prefixes
            const int32_t* big_list = alist + asegs[NB_AGG];
            int64_t* md = at<int64_t>(Y.md);
            int64_t* mpos = at<int64_t>(Y.mpos);
            int64_t* bnch = at<int64_t>(Y.bnch);
            int64_t* bchpre = at<int64_t>(Y.bchpre);
            timed(H, K_AGG_PREP, 0, [&] {
                launch_member_deg(L, members, n, md, s);
                scan_i64_to_i64(md, mpos, n, scan, s);
                launch_big_info(big_list, nbig, hoff, ncom, bnch, at<int64_t>(Y.hcaps), s);
                scan_i64_to_i64(bnch, bchpre, nbig, scan, s);
                scan_i64_to_i64(at<int64_t>(Y.hcaps), hpre, nbig, scan, s);
            });
            std::vector<int64_t> chpre(nbig + 1);
            hub_pre.resize(nbig + 1);
            if ((st = readback(H, chpre.data(), bchpre, (nbig + 1) * sizeof(int64_t))) != LOUVAIN_OK) return st;
            if ((st = readback(H, hub_pre.data(), hpre, (nbig + 1) * sizeof(int64_t))) != LOUVAIN_OK) return st;
            std::vector<std::pair<int32_t, int32_t>> groups;
            if (!chunks(hub_pre, Y.pool_entries, &groups))
                return fail(H, LOUVAIN_ERR_WORKSPACE, "community hash table exceeds the workspace pool");
            for (auto& gr : groups) {
                BigArgs B{};
                B.list = big_list + gr.first;
                B.nbig = gr.second - gr.first;
                B.chunk_pre = bchpre + gr.first;
                B.chunk_base = chpre[gr.first];
                B.tab_pre = hpre + gr.first;
                B.tab_base = hub_pre[gr.first];
                B.Cp = Cp;
                B.coff = coff;
                B.members = members;
                B.mpos = mpos;
                B.hoff = hoff;
                B.keys = at<int32_t>(Y.pool_keys);
                B.vals = at<void>(Y.pool_vals);
                B.hidx = A.hidx;
                B.hw = A.hw;
                B.out_w64 = A.out_w64;
                B.rowlen = A.rowlen;
                B.bitmaps = at<uint32_t>(Y.bitmaps);
                B.words = (ncom + 31) / 32;
                B.cnt = at<int32_t>(Y.hcnt) + gr.first;
                B.slots = at<int32_t>(Y.hslots);
                B.sorted = A.sorted;
                const int64_t nchunks = chpre[gr.second] - chpre[gr.first];
                HIPCHK(H, hipMemsetAsync(B.cnt, 0, (size_t)B.nbig * 4, s));
                timed(H, K_AGG_BIG_INSERT, 0, [&] {
                    launch_big_clear(B.keys, B.vals, hub_pre[gr.second] - hub_pre[gr.first], s);
                    launch_big_insert(LA, B, nchunks, s);
                });
                timed(H, K_AGG_BIG_EXTRACT, 0, [&] { launch_big_extract(LA, B, s); });
            }
        }
        // ---------------- compaction into the next super-graph
        void* goff = at<void>(Y.sup_off);
        int32_t* gidx = at<int32_t>(Y.sup_idx);
        void* gw = at<void>(Y.sup_w);
        launch_rowlen_to_offsets(at<int32_t>(Y.rowlen), ncom, goff, H->sup_off64, scan, s);
        int64_t nnz2 = 0;
        if (H->sup_off64) {
            if ((st = readback(H, &nnz2, (int64_t*)goff + ncom, 8)) != LOUVAIN_OK) return st;
        } else {
            int32_t x = 0;
            if ((st = readback(H, &x, (int32_t*)goff + ncom, 4)) != LOUVAIN_OK) return st;
            nnz2 = x;
        }
        timed(H, K_COMPACT, 0, [&] {
            launch_compact(ncom, hoff, A.hidx, A.hw, goff, H->sup_off64, gidx, gw, A.out_w64, s);
        });
        L.n = ncom;
        uniq = true;
        L.nnz = nnz2;
        L.off = goff;
        L.idx = gidx;
        L.w = gw;
        L.t.off64 = H->sup_off64;
        L.t.wk = H->sup_wk;
        L.t.acc64 = 0;
        gsel ^= 1;
        stopped_before_aggregate = false;
        have_newid = false;
        if (H->pafn) {
            std::vector<int64_t> o(ncom + 1);
            std::vector<int32_t> ii(nnz2);
            std::vector<int64_t> ww(nnz2);
            if (H->sup_off64) {
                if ((st = readback(H, o.data(), goff, (ncom + 1) * 8)) != LOUVAIN_OK) return st;
            } else {
                std::vector<int32_t> o32(ncom + 1);
                if ((st = readback(H, o32.data(), goff, (ncom + 1) * 4)) != LOUVAIN_OK) return st;
                for (int64_t k = 0; k <= ncom; k++) o[k] = o32[k];
            }
            if ((st = readback(H, ii.data(), gidx, nnz2 * 4)) != LOUVAIN_OK) return st;
            if (H->sup_wk == 2) {
                if ((st = readback(H, ww.data(), gw, nnz2 * 8)) != LOUVAIN_OK) return st;
            } else {
                std::vector<int32_t> w32(nnz2);
                if ((st = readback(H, w32.data(), gw, nnz2 * 4)) != LOUVAIN_OK) return st;
                for (int64_t k = 0; k < nnz2; k++) ww[k] = w32[k];
            }
            H->pafn(H->user, pass, ncom, o.data(), ii.data(), ww.data(), li);
        }
    }

    // ---------------- final lookup and dense renumbering
    if (stopped_before_aggregate) {
        const int64_t n = L.n;
        int32_t* used = at<int32_t>(Y.used);
        int32_t* newid = at<int32_t>(Y.newid);
        if (!have_newid) {
            HIPCHK(H, hipMemsetAsync(used, 0, (n + 1) * 4, s));
            launch_mark_used(Cp, n, used, s);
            scan_i32_to_i32(used, newid, n, scan, s);
            int32_t gall = 0;
            if ((st = readback(H, &gall, newid + n, 4)) != LOUVAIN_OK) return st;
            ncom_last = gall;
        }
        launch_final_lookup(C, n0, Cp, newid, s);
        H->ncom = ncom_last;
    } else {
        H->ncom = L.n;
    }
    if (batch) {
        // first final community id of every graph (union numbering), kept on
        // the device for membership and modularity
        int32_t* cmin = at<int32_t>(Y.cmin);
        HIPCHK(H, hipMemsetAsync(cmin, 0x7f, (size_t)nbg * 4, s));
        launch_graph_cmin(C, n0, at<int32_t>(Y.gid0), cmin, s);
        H->b_cbase.resize(nbg + 1);
        if ((st = readback(H, H->b_cbase.data(), cmin, (size_t)nbg * 4)) != LOUVAIN_OK) return st;
        H->b_cbase[nbg] = (int32_t)H->ncom;
        for (int64_t g = nbg - 1; g >= 0; g--)  // graphs without vertices: empty range
            if (H->vbase[g + 1] == H->vbase[g]) H->b_cbase[g] = H->b_cbase[g + 1];
        for (int64_t g = 0; g < nbg; g++) H->b_comms[g] = H->b_cbase[g + 1] - H->b_cbase[g];
        HIPCHK(H, hipMemcpyAsync(cmin, H->b_cbase.data(), (size_t)nbg * 4, hipMemcpyHostToDevice, s));
        int32_t mp = 0;
        for (int32_t x : H->b_passes) mp = std::max(mp, x);
        H->st.passes = mp;
    }
    if ((st = sync_stream(H)) != LOUVAIN_OK) return st;
    H->st.communities = H->ncom;
    return LOUVAIN_OK;
}

// After a run: wall time, per-kernel records (profiling), run counters.
louvain_status finish_run(louvain_t* h, louvain_status st, double ms) {
    if (st != LOUVAIN_OK) { h->ran = false; return st; }
    h->st.ms_total = ms;
    // per-kernel timing
    if (h->prof) {
        for (auto& r2 : h->recs) {
            float km = 0;
            if (hipEventElapsedTime(&km, r2.e0, r2.e1) == hipSuccess) h->kms[r2.kind] += km;
            h->klaunch[r2.kind]++;
            h->kbytes[r2.kind] += r2.bytes;
        }
        double mv = 0, ag = 0;
        for (int k = K_MOVE_FUSED; k <= K_SYNC_APPLY; k++) mv += h->kms[k];
        for (int k = K_AGG_PREP; k <= K_COMPACT; k++) ag += h->kms[k];
        h->st.ms_move = mv;
        h->st.ms_aggregate = ag;
    }
    Ctl c;
    if (readback(h, &c, h->ctl(), sizeof(Ctl)) == LOUVAIN_OK) {
        for (int b = 0; b < MAX_BUCKETS; b++)
            for (int k = 0; k < STRIPES; k++) {
                h->st.vertices_evaluated += (int64_t)c.bstat[0][b][k];
                h->st.arcs_scanned += (int64_t)c.bstat[1][b][k];
                h->st.distinct_scanned += (int64_t)c.bstat[2][b][k];
            }
    }
    h->st.host_syncs = h->syncs;
    h->ran = true;
    return LOUVAIN_OK;
}

}  // namespace

extern "C" {

louvain_status louvain_run(louvain_t* h) {
    if (!h) return fail(nullptr, LOUVAIN_ERR_INVALID, "null handle");
    hipEvent_t e0, e1;
    HIPCHK(h, hipEventCreate(&e0));
    HIPCHK(h, hipEventCreate(&e1));
    HIPCHK(h, hipEventRecord(e0, h->stream));
    Runner r(h);
    louvain_status st = r.run();
    (void)hipEventRecord(e1, h->stream);
    h->syncs++;
    (void)hipEventSynchronize(e1);
    float ms = 0;
    (void)hipEventElapsedTime(&ms, e0, e1);
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    return finish_run(h, st, ms);
}

louvain_status louvain_get_membership(louvain_t* h, int32_t* out) {
    if (!h || !out) return fail(h, LOUVAIN_ERR_INVALID, "null argument");
    if (!h->ran) return fail(h, LOUVAIN_ERR_STATE, "louvain_run has not completed");
    if (h->g.n == 0) return LOUVAIN_OK;
    HIPCHK(h, hipMemcpyAsync(out, h->at<int32_t>(h->lay.C), h->g.n * 4, hipMemcpyDeviceToDevice, h->stream));
    if (h->nb > 0)  // per-graph ids 0 .. communities - 1
        launch_rebase(out, h->g.n, h->at<int32_t>(h->lay.gid0), h->at<int32_t>(h->lay.cmin), h->stream);
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return LOUVAIN_OK;
}

louvain_status louvain_modularity_batch(louvain_t* h, double* q, int64_t* num, int64_t* den) {
    if (!h) return fail(nullptr, LOUVAIN_ERR_INVALID, "null handle");
    if (h->nb <= 0) return fail(h, LOUVAIN_ERR_INVALID, "not a batched handle");
    if (!h->ran) return fail(h, LOUVAIN_ERR_STATE, "louvain_run has not completed");
    const int64_t n = h->g.n, G = h->nb;
    i64* sigin = h->at<i64>(h->lay.K);
    i64* sigtot = h->at<i64>(h->lay.Sig);
    u64* gq = h->at<u64>(h->lay.gq);
    if (n > 0) {
        HIPCHK(h, hipMemsetAsync(sigin, 0, n * 8, h->stream));
        HIPCHK(h, hipMemsetAsync(sigtot, 0, n * 8, h->stream));
    }
    HIPCHK(h, hipMemsetAsync(gq, 0, (size_t)G * 16, h->stream));
    launch_modularity_arcs(h->L0, h->at<int32_t>(h->lay.C), sigin, sigtot, h->stream);
    launch_mod_terms_batch(h->ncom, h->at<int32_t>(h->lay.cmin), G, h->at<u64>(h->lay.Wg), sigin, sigtot, gq,
                           h->stream);
    std::vector<u64> hq(2 * G);
    louvain_status st = readback(h, hq.data(), gq, (size_t)G * 16);
    if (st != LOUVAIN_OK) return st;
    for (int64_t g = 0; g < G; g++) {
        const i64 Wg = (i64)h->Wg[g];
        __int128 numv = (__int128)(((unsigned __int128)hq[2 * g + 1] << 64) | hq[2 * g]);
        __int128 denv = Wg == 0 ? (__int128)1 : (__int128)Wg * Wg;
        if (Wg == 0) numv = 0;
        if (num) { num[2 * g] = (int64_t)(numv >> 64); num[2 * g + 1] = (int64_t)(uint64_t)numv; }
        if (den) { den[2 * g] = (int64_t)(denv >> 64); den[2 * g + 1] = (int64_t)(uint64_t)denv; }
        if (q) q[g] = (double)numv / (double)denv;
    }
    return LOUVAIN_OK;
}

louvain_status louvain_batch_results(louvain_t* h, int32_t* passes, int32_t* iterations, int64_t* communities) {
    if (!h) return fail(nullptr, LOUVAIN_ERR_INVALID, "null handle");
    if (h->nb <= 0) return fail(h, LOUVAIN_ERR_INVALID, "not a batched handle");
    if (!h->ran) return fail(h, LOUVAIN_ERR_STATE, "louvain_run has not completed");
    for (int64_t g = 0; g < h->nb; g++) {
        if (passes) passes[g] = h->b_passes[g];
        if (iterations) iterations[g] = h->b_iters[g];
        if (communities) communities[g] = h->b_comms[g];
    }
    return LOUVAIN_OK;
}

louvain_status louvain_modularity(louvain_t* h, double* q, int64_t num[2], int64_t den[2]) {
    if (!h) return fail(nullptr, LOUVAIN_ERR_INVALID, "null handle");
    if (h->nb > 0) return fail(h, LOUVAIN_ERR_INVALID, "batched handle: use louvain_modularity_batch");
    if (!h->ran) return fail(h, LOUVAIN_ERR_STATE, "louvain_run has not completed");
    const int64_t n = h->g.n;
    i64* sigin = h->at<i64>(h->lay.K);
    i64* sigtot = h->at<i64>(h->lay.Sig);
    if (n > 0) {
        HIPCHK(h, hipMemsetAsync(sigin, 0, n * 8, h->stream));
        HIPCHK(h, hipMemsetAsync(sigtot, 0, n * 8, h->stream));
    }
    HIPCHK(h, hipMemsetAsync(&h->ctl()->q_lo, 0, 16, h->stream));
    launch_modularity(h->L0, h->at<int32_t>(h->lay.C), h->ncom, h->W, sigin, sigtot, h->ctl(), h->stream);
    u64 qq[2];
    louvain_status st = readback(h, qq, &h->ctl()->q_lo, 16);
    if (st != LOUVAIN_OK) return st;
    __int128 numv = (__int128)(((unsigned __int128)qq[1] << 64) | qq[0]);
    __int128 denv = h->W == 0 ? (__int128)1 : (__int128)h->W * h->W;
    if (h->W == 0) numv = 0;
    if (num) { num[0] = (int64_t)(numv >> 64); num[1] = (int64_t)(uint64_t)numv; }
    if (den) { den[0] = (int64_t)(denv >> 64); den[1] = (int64_t)(uint64_t)denv; }
    if (q) *q = (double)numv / (double)denv;
    return LOUVAIN_OK;
}

louvain_status louvain_get_stats(louvain_t* h, louvain_stats* s) {
    if (!h || !s) return fail(h, LOUVAIN_ERR_INVALID, "null argument");
    *s = h->st;
    return LOUVAIN_OK;
}

louvain_status louvain_set_profiling(louvain_t* h, int32_t enable) {
    if (!h) return fail(nullptr, LOUVAIN_ERR_INVALID, "null handle");
    h->prof = enable != 0;
    for (int k = 0; k < K_COUNT; k++) { h->kms[k] = 0; h->klaunch[k] = 0; h->kbytes[k] = 0; }
    return LOUVAIN_OK;
}

louvain_status louvain_get_kernel_stats(louvain_t* h, louvain_kernel_stat* out, int32_t max, int32_t* count) {
    if (!h || !count || (max > 0 && !out)) return fail(h, LOUVAIN_ERR_INVALID, "null argument");
    int32_t k = 0;
    for (int i = 0; i < K_COUNT; i++) {
        if (!h->klaunch[i]) continue;
        if (k < max) {
            memset(&out[k], 0, sizeof(out[k]));
            snprintf(out[k].name, sizeof(out[k].name), "%s", KNAMES[i]);
            out[k].launches = h->klaunch[i];
            out[k].ms = h->kms[i];
            out[k].alg_bytes = h->kbytes[i];
        }
        k++;
    }
    *count = k;
    return LOUVAIN_OK;
}

louvain_status louvain_set_trace(louvain_t* h, louvain_iter_fn iter_fn, louvain_pass_fn pass_fn, void* user) {
    if (!h) return fail(nullptr, LOUVAIN_ERR_INVALID, "null handle");
    h->itfn = iter_fn;
    h->pafn = pass_fn;
    h->user = user;
    return LOUVAIN_OK;
}

louvain_status louvain_autotune(louvain_t* h, const int32_t* candidates, int32_t ncand, int32_t reps, int32_t* best,
                                double* ms) {
    if (!h) return fail(nullptr, LOUVAIN_ERR_INVALID, "null handle");
    if (!candidates || ncand < 1 || reps < 1) return fail(h, LOUVAIN_ERR_INVALID, "need ncand >= 1 candidates and reps >= 1");
    // each candidate: the move-bucket degree thresholds of louvain_params.bucket_max_degree
    constexpr int K = 8;
    const Buckets keep = h->mb;
    int32_t keep_deg[K];
    memcpy(keep_deg, h->p.bucket_max_degree, sizeof(keep_deg));
    // modularity of the handle's last run (the batch mean for a batched handle)
    std::vector<double> qb(h->nb > 0 ? (size_t)h->nb : 1);
    auto last_q = [&](double* q) -> louvain_status {
        if (h->nb > 0) {
            const louvain_status st = louvain_modularity_batch(h, qb.data(), nullptr, nullptr);
            if (st != LOUVAIN_OK) return st;
            double m = 0;
            for (double x : qb) m += x;
            *q = m / (double)qb.size();
            return LOUVAIN_OK;
        }
        return louvain_modularity(h, q, nullptr, nullptr);
    };
    // reps timed runs with the current buckets: mean and spread of the times, lowest Q
    auto measure = [&](double* mean, double* spread, double* qmin) -> louvain_status {
        double tot = 0, lo = 0, hi = 0;
        *qmin = 0;
        for (int32_t r = 0; r < reps; r++) {
            louvain_status st = louvain_run(h);
            double q = 0;
            if (st == LOUVAIN_OK) st = last_q(&q);
            if (st != LOUVAIN_OK) return st;
            const double t = h->st.ms_total;
            tot += t;
            lo = r == 0 ? t : std::min(lo, t);
            hi = r == 0 ? t : std::max(hi, t);
            *qmin = r == 0 ? q : std::min(*qmin, q);
        }
        *mean = tot / reps;
        *spread = hi - lo;
        return LOUVAIN_OK;
    };
    auto restore = [&](louvain_status st) {
        h->mb = keep;
        memcpy(h->p.bucket_max_degree, keep_deg, sizeof(keep_deg));
        return st;
    };
    // the handle's own thresholds are the baseline every candidate must beat
    double base_t = 0, base_spread = 0, base_q = 0;
    louvain_status st0 = measure(&base_t, &base_spread, &base_q);
    if (st0 != LOUVAIN_OK) return restore(st0);
    int32_t bi = -1;
    double bt = base_t - base_spread;
    for (int32_t c = 0; c < ncand; c++) {
        const int32_t* cand = candidates + (size_t)c * K;
        h->mb = make_buckets(cand, NB_MOVE, MOVE_CAP, MOVE_DEFAULT_MAX);
        double t = 0, spread = 0, q = 0;
        const louvain_status st = measure(&t, &spread, &q);
        if (st != LOUVAIN_OK) return restore(st);
        if (ms) ms[c] = t;
        // a candidate may not buy its speed with modularity (ASYNC runs can
        // converge early to a worse optimum): at most 0.002 below the baseline
        if (q < base_q - 0.002) continue;
        if (t < bt) { bi = c; bt = t; }
    }
    if (bi < 0) {
        restore(LOUVAIN_OK);
    } else {
        const int32_t* win = candidates + (size_t)bi * K;
        h->mb = make_buckets(win, NB_MOVE, MOVE_CAP, MOVE_DEFAULT_MAX);
        memcpy(h->p.bucket_max_degree, win, sizeof(keep_deg));
    }
    if (best) *best = bi;
    return LOUVAIN_OK;
}

louvain_status louvain_collect_samples(louvain_t* h, float* buffer, int64_t capacity, int32_t sample_per_mille) {
    if (!h) return fail(nullptr, LOUVAIN_ERR_INVALID, "null handle");
    if (buffer && (capacity < 0 || sample_per_mille < 0 || sample_per_mille > 1000))
        return fail(h, LOUVAIN_ERR_INVALID, "capacity must be >= 0 and sample_per_mille in [0, 1000]");
    if (buffer && h->nb > 0) return fail(h, LOUVAIN_ERR_INVALID, "sample recording is not supported on a batched handle");
    h->smp_buf = (buffer && sample_per_mille > 0 && capacity > 0) ? buffer : nullptr;
    h->smp_cap = h->smp_buf ? capacity : 0;
    h->smp_rate = h->smp_buf ? sample_per_mille : 0;
    return LOUVAIN_OK;
}

louvain_status louvain_sample_count(louvain_t* h, int64_t* count) {
    if (!h || !count) return fail(h, LOUVAIN_ERR_INVALID, "null argument");
    *count = h->smp_count;
    return LOUVAIN_OK;
}

// ---------------------------------------------------------- stand-alone MLP

#define MLPCHK(x)                                                                               \
    do {                                                                                        \
        hipError_t e_ = (x);                                                                    \
        if (e_ != hipSuccess)                                                                   \
            return fail(nullptr, LOUVAIN_ERR_HIP, "%s failed: %s", #x, hipGetErrorString(e_));  \
    } while (0)

louvain_status louvain_pruner_init(float* weights, uint64_t seed, void* stream) {
    if (!weights) return fail(nullptr, LOUVAIN_ERR_INVALID, "null weights");
    launch_mlp_init(weights, seed, (hipStream_t)stream);
    MLPCHK(hipGetLastError());
    MLPCHK(hipStreamSynchronize((hipStream_t)stream));
    return LOUVAIN_OK;
}

louvain_status louvain_pruner_predict(const float* weights, const float* features, int64_t count, float* logit,
                                      void* stream) {
    if (count < 0 || (count > 0 && (!weights || !features || !logit)))
        return fail(nullptr, LOUVAIN_ERR_INVALID, "null argument or negative count");
    launch_mlp_predict(weights, features, count, logit, (hipStream_t)stream);
    MLPCHK(hipGetLastError());
    MLPCHK(hipStreamSynchronize((hipStream_t)stream));
    return LOUVAIN_OK;
}

int64_t louvain_pruner_scratch_floats(int32_t batch) {
    (void)batch;  // mini-batch indices are drawn inside the kernels
    return 3 * (int64_t)MLP_PARAMS + 5;  // gradient, two Adam moments, an 8-byte-aligned double
}

namespace {
// The double accumulator sits after 3 * MLP_PARAMS floats, rounded up to 8 bytes.
double* scratch_loss(float* scratch) {
    uintptr_t p = (uintptr_t)(scratch + 3 * MLP_PARAMS);
    return (double*)((p + 7) & ~(uintptr_t)7);
}
}  // namespace

louvain_status louvain_pruner_loss_grad(const float* weights, const float* samples, int64_t count,
                                        float pos_weight, float* grad, double* loss, void* stream) {
    if (!weights || !grad || count < 0 || (count > 0 && !samples))
        return fail(nullptr, LOUVAIN_ERR_INVALID, "null argument or negative count");
    hipStream_t s = (hipStream_t)stream;
    double* acc = nullptr;
    MLPCHK(hipMalloc(&acc, sizeof(double)));
    launch_mlp_zero(grad, MLP_PARAMS, s);
    hipError_t e = hipMemsetAsync(acc, 0, sizeof(double), s);
    if (e == hipSuccess) {
        launch_mlp_loss_grad(weights, samples, count, count, 0, 0, 0, pos_weight, grad, acc, s);
        e = hipGetLastError();
    }
    double hv = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&hv, acc, sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    hipFree(acc);
    if (e != hipSuccess) return fail(nullptr, LOUVAIN_ERR_HIP, "pruner loss: %s", hipGetErrorString(e));
    if (loss) *loss = hv;
    return LOUVAIN_OK;
}

}  // extern "C"

namespace {
// Adam training with the gradient, the two moments and the loss accumulator
// in `scratch` (louvain_pruner_scratch_floats floats); every part that must
// start at zero is cleared here, on the stream, before it is used.
louvain_status train_with_scratch(float* weights, const float* samples, int64_t count, int32_t steps, int32_t batch,
                                  float lr, float pos_weight, uint64_t seed, float* scratch, double* last_loss,
                                  hipStream_t s) {
    float* grad = scratch;
    float* m = scratch + MLP_PARAMS;
    float* v = scratch + 2 * MLP_PARAMS;
    double* acc = scratch_loss(scratch);
    launch_mlp_zero(m, 2 * MLP_PARAMS, s);
    const bool full = batch >= count;
    const int64_t slots = full ? count : batch;
    double b1t = 1.0, b2t = 1.0;
    for (int32_t step = 0; step < steps; step++) {
        launch_mlp_zero(grad, MLP_PARAMS, s);
        launch_mlp_zero((float*)acc, 2, s);
        launch_mlp_loss_grad(weights, samples, count, slots, full ? 0 : batch, seed, step, pos_weight, grad, acc, s);
        b1t *= 0.9;
        b2t *= 0.999;
        launch_adam(weights, grad, m, v, lr, (float)(1.0 - b1t), (float)(1.0 - b2t), s);
    }
    MLPCHK(hipGetLastError());
    double hv = 0;
    if (steps > 0) MLPCHK(hipMemcpyAsync(&hv, acc, sizeof(double), hipMemcpyDeviceToHost, s));
    MLPCHK(hipStreamSynchronize(s));
    if (last_loss) *last_loss = hv;
    return LOUVAIN_OK;
}

// Scratch of louvain_pruner_train_noalloc: a file-scope device array, one
// copy per GPU, kept until the process ends.  Host code never passes the
// array's name to a kernel (on the host it is only a stand-in for the
// symbol); it uses the device address that hipGetSymbolAddress returns,
// looked up once per device with that device current.
constexpr int64_t NOALLOC_SCRATCH_FLOATS = LOUVAIN_NOALLOC_SCRATCH_FLOATS;
__device__ __align__(256) float scratch[NOALLOC_SCRATCH_FLOATS];
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
float* g_scratch_ptr[MAX_DEVICES] = {};

louvain_status noalloc_scratch(hipStream_t s, float** out) {
    int dev = -1;
    MLPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES)
        return fail(nullptr, LOUVAIN_ERR_INVALID, "device ordinal %d beyond the supported %d", dev, MAX_DEVICES);
    if (s) {
        hipDevice_t sd = -1;
        MLPCHK(hipStreamGetDevice(s, &sd));
        if ((int)sd != dev)
            return fail(nullptr, LOUVAIN_ERR_INVALID, "stream belongs to device %d, current device is %d", (int)sd,
                        dev);
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        MLPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        g_scratch_ptr[dev] = (float*)p;
    }
    *out = g_scratch_ptr[dev];
    return LOUVAIN_OK;
}
}  // namespace

extern "C" {

louvain_status louvain_pruner_train(float* weights, const float* samples, int64_t count, int32_t steps,
                                    int32_t batch, float lr, float pos_weight, uint64_t seed, float* scratch,
                                    double* last_loss, void* stream) {
    if (!weights || !scratch || count <= 0 || !samples || steps < 0 || batch <= 0)
        return fail(nullptr, LOUVAIN_ERR_INVALID, "invalid arguments (need samples, count > 0, batch > 0)");
    return train_with_scratch(weights, samples, count, steps, batch, lr, pos_weight, seed, scratch, last_loss,
                              (hipStream_t)stream);
}

louvain_status louvain_pruner_train_noalloc(float* weights, const float* samples, int64_t count, int32_t steps,
                                            int32_t batch, float lr, float pos_weight, uint64_t seed,
                                            double* last_loss, void* stream) {
    if (!weights || count <= 0 || !samples || steps < 0 || batch <= 0)
        return fail(nullptr, LOUVAIN_ERR_INVALID, "invalid arguments (need samples, count > 0, batch > 0)");
    const int64_t need = louvain_pruner_scratch_floats(batch);
    if (need > NOALLOC_SCRATCH_FLOATS)
        return fail(nullptr, LOUVAIN_ERR_INVALID,
                    "training needs %lld scratch floats, beyond the static maximum of %lld",
                    (long long)need, (long long)NOALLOC_SCRATCH_FLOATS);
    float* sp = nullptr;
    const louvain_status st = noalloc_scratch((hipStream_t)stream, &sp);
    if (st != LOUVAIN_OK) return st;
    return train_with_scratch(weights, samples, count, steps, batch, lr, pos_weight, seed, sp, last_loss,
                              (hipStream_t)stream);
}

const char* louvain_last_error(const louvain_t* h) {
    if (!h) return g_create_error.c_str();
    return h->err.c_str();
}

void louvain_destroy(louvain_t* h) {
    if (!h) return;
    if (h->stream) hipStreamSynchronize(h->stream);
    else hipDeviceSynchronize();
    for (auto e : h->evpool) hipEventDestroy(e);
    if (h->stage_owned && h->pinned) hipHostFree(h->pinned);
    if (h->stage_owned && h->pinned_up) hipHostFree(h->pinned_up);
    if (h->handle_owned) delete h;
    else h->~louvain_s();
}

}  // extern "C"
