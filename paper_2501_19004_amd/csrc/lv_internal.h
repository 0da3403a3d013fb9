// lv_internal.h -- host-side interface between the C ABI driver and the
// kernel launchers of the gfx950 Louvain library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lv_common.h"

namespace lv {

// Compiled local-moving variants: G lanes per vertex, CAP LDS table slots per
// vertex (a vertex of degree D needs CAP >= 2*D).  Bucket 0 is one vertex per
// lane with its row in registers (no table; CAP / 2 = 8 is its largest
// degree).  Bucket NB_MOVE is the global-memory ("hub") path.
constexpr int NB_MOVE = 5;
constexpr int MOVE_G[NB_MOVE] = {1, 8, 32, 256, 1024};
constexpr int MOVE_CAP[NB_MOVE] = {16, 64, 256, 1024, 8192};
constexpr int MOVE_DEFAULT_MAX[NB_MOVE] = {8, 32, 128, 512, 4096};
constexpr int HUB_CH = 4096;    // arcs per hub insert chunk (one workgroup)
constexpr int HUB_LCAP = 8192;  // LDS slots of a hub insert chunk

// Aggregation variants (per community; CAP >= 2 * bound on distinct keys).
constexpr int NB_AGG = 4;
constexpr int AGG_G[NB_AGG] = {16, 64, 256, 1024};
constexpr int AGG_CAP[NB_AGG] = {32, 256, 2048, 8192};
constexpr int AGG_DEFAULT_MAX[NB_AGG] = {16, 128, 1024, 4096};

// Type codes of a level graph.
struct LevelTypes {
    int off64;  // offsets int64 (else int32)
    int wk;     // weights: 0 unit, 1 int32, 2 int64
    int acc64;  // hash-table values int64 (else uint32): needed when sums may reach 2^32
};

struct LevelView {
    int64_t n = 0, nnz = 0;
    const void* off = nullptr;
    const int32_t* idx = nullptr;
    const void* w = nullptr;
    LevelTypes t{};
};

// Device-driven iterations (louvain_params.device_loop): the host enqueues a
// pass's iterations without waiting for each one; every launch is sized for
// the pass's largest queue and reads the true queue sizes, and whether the
// pass has ended, from this record, which k_iter_end updates after each
// iteration with the method's convergence tests.
struct DevIter {
    int32_t halt;                  // 1: local moving of this pass has ended; later launches do nothing
    int32_t li;                    // the pass's iteration count (max_iterations until it ends earlier)
    int32_t ran;                   // iterations that ran
    int32_t extra;                 // iterations counted without running (nothing flagged: S = 0)
    int32_t cnt[MAX_BUCKETS];      // current queue: entries per bucket ...
    int32_t seg[MAX_BUCKETS + 1];  // ... and where each bucket's entries start
    int32_t pad;
    u64 moves;                     // moves applied in the pass
};

// Per-iteration arguments of the local-moving kernels.
// Partial best candidate of one hub-decide block (a slice of the hub's
// occupied slots); the hub's last block combines them.
struct HubPart {
    i64 klo, khi;  // key, as a 128-bit value
    i64 v, kic, nd;
    int32_t d, pad;
};

struct MoveArgs {
    const void* off;
    const int32_t* idx;
    const void* w;
    int32_t* Cp;          // level membership C'
    i64* Sig;             // community totals Sigma'
    const i64* K;         // weighted degrees K'
    i64 W;                // total weight (2m)
    int32_t wide;         // 1: 128-bit gain arithmetic
    int32_t pl;           // Pick-Less active this iteration
    int32_t min_label;    // ASYNC: singletons join only singletons of smaller id
    int32_t prune;        // 1: flag neighbours of movers for the next iteration
    uint8_t* fnext;       // flags of the next iteration's queue (cleared before the iteration)
    const uint8_t* fcur;  // flags of this iteration's queue
    Ctl* ctl;
    int32_t* sdec;        // SYNC: per vertex of the queue, its decided target or -1
    int32_t bucket;       // bucket id for per-bucket counters
    int32_t lstride;      // queue entries of this launch: list[slot * lstride + lphase]
    int32_t lphase;
    // batched ASYNC slices: slice seg_k of seg_ns takes, from every graph g's
    // segment of the bucket's queue (start seg_start[g], length seg_cnt[g]),
    // the entries [len*k/ns, len*(k+1)/ns); seg_pre[g] = slots of graphs < g
    const int32_t* seg_pre;
    const int32_t* seg_start;
    const int32_t* seg_cnt;
    int32_t seg_n, seg_k, seg_ns;
    const uint8_t* vbucket;
    // hub path (static hub list of the pass, ascending vertex id)
    const int32_t* hub_list;
    const int64_t* hub_pre;  // prefix of table capacities over the static list
    const int64_t* hch_pre;  // prefix of insert-chunk counts over the static list
    int32_t g_lo, g_hi;      // hubs of this launch (their tables fit the pool together)
    int32_t tab_lo;          // hub whose table starts the pool (tables sit at hub_pre[h] - hub_pre[tab_lo])
    int32_t all_queued;      // 1: every hub is queued (sweep, first iteration or no pruning)
    int32_t* gdec;           // per static hub: applied (ASYNC) or recorded (SYNC) target, or -1
    int32_t* hub_keys;
    void* hub_vals;
    int32_t* hub_cnt;        // per static hub: occupied slots of its table (0 between iterations)
    int32_t* hub_slots;      // occupied slot lists: hub h's list starts at its table offset / 2
    HubPart* hub_part;       // partial decisions, one per decide block of the launch
    // batched runs (gid == nullptr for a single graph): graph id of every
    // vertex of the level, per-graph total weight, graphs still moving in
    // this pass, per-graph 128-bit gain sums (lo, hi)
    const int32_t* gid;
    const u64* Wg;
    const uint8_t* gact;
    u64* Sg;
    u64* Pg;                 // batched learned runs: per-graph evaluations with a positive best gain
    // per-vertex state of the learned pruner's features (learn = 1)
    int32_t learn;
    uint32_t itag;           // tag of this iteration, unique within the run
    i64* f_own;              // K_{v->C'[v]} at v's last evaluation
    i64* f_adv;              // K_{v->d*} - K_{v->C'[v]} at v's last evaluation
    uint32_t* f_moved;       // tag of the last iteration in which v moved
    int32_t* f_nm;           // moved neighbours of v in this iteration (cleared before it)
    // device-driven iterations (nullptr: the host passes exact lists and
    // counts): list arguments are the queue's base and counts are launch
    // bounds; slice `slice` of bucket b starts at dshare[2 * (slice * NB_MOVE
    // + b)] and holds the next entry's count of entries (batched slices:
    // dit->seg[b] and seg_pre[seg_n])
    const DevIter* dit;
    const int32_t* dshare;
    int32_t slice;
};

// Learned-pruner filter of the next iteration's queue (lv_learn.hip).
constexpr int MLP_PARAMS = 32 * 8 + 32 + 32 * 32 + 32 + 32 + 1;
constexpr int SAMPLE_FLOATS = 9;
struct FilterArgs {
    const void* off;
    int64_t n;
    const i64* K;
    const i64* own;
    const i64* adv;
    const uint32_t* moved;
    const int32_t* nm;
    uint32_t itag_prev;   // tag of the iteration that just ended
    int32_t pass, t;      // of the iteration the queue is for
    uint8_t* flags;       // flagged iff flags[v] != 0 ...
    int32_t all;          // ... or, with all = 1, every vertex with an arc
    int32_t learned;      // apply the MLP
    const float* weights;
    float zt;             // keep iff logit >= zt
    float* samples;
    int64_t cap;
    int32_t per_mille;
    Ctl* ctl;
    // batched runs: graph of every vertex; graphs whose next iteration is
    // their own sweep (every vertex with an arc is kept, no MLP); set to 1 for
    // every graph with at least one kept vertex (any of them may be NULL)
    const int32_t* gid;
    const uint8_t* gsweep;
    uint8_t* gany;
};

// Lists of buckets 0..3 for one fused launch; blk_pre[b] is the first block
// of bucket b (blocks of 256 threads hold 256 / MOVE_G[b] vertices).
struct FusedLists {
    const int32_t* list[4];
    int32_t count[4];
    int64_t blk_pre[5];
    const int32_t* seg_pre[4];    // batched slices: per-bucket rows (see MoveArgs)
    const int32_t* seg_start[4];
    const int32_t* seg_cnt[4];
};

struct Buckets {
    int32_t maxdeg[MAX_BUCKETS];  // vertex with degree D goes to the first b with D <= maxdeg[b]; else hub
    int32_t nb;                   // number of LDS buckets in use
};

// ---- launchers: scan / utility (lv_scan.hip)
size_t scan_scratch_bytes(int64_t n);
// out[0..n] = exclusive prefix of in[0..n-1] (out[n] = total).  in and out may not alias.
void scan_i32_to_i32(const int32_t* in, int32_t* out, int64_t n, void* scratch, hipStream_t s);
void scan_i32_to_i64(const int32_t* in, int64_t* out, int64_t n, void* scratch, hipStream_t s);
void scan_i64_to_i64(const int64_t* in, int64_t* out, int64_t n, void* scratch, hipStream_t s);
void fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s);
void iota_i32(int32_t* p, int64_t n, hipStream_t s);

// ---- launchers: pass init and local moving (lv_move.hip)
void launch_classify(const LevelView& L, const Buckets& B, uint8_t* vbucket, int32_t* Cp, i64* K, i64* Sig,
                     Ctl* ctl, hipStream_t s);
// Ordered partition of the level's vertices into NB_MOVE+1 bucket segments
// (all vertices with arcs, or the flagged ones when use_flags); bucket totals
// go to totals[0..NB_MOVE].  blkcnt/blkoff: (NB_MOVE+1) * bucket_blocks(n) (+1).
// halt (may be NULL): when *halt != 0 at run time the count and fill
// launches do nothing (device-driven iterations past the pass's end).
void bucketize_vertices(int64_t n, const uint8_t* vbucket, const uint8_t* flags, int use_flags, const int32_t* gid,
                        const uint8_t* gact,
                        int32_t* blkcnt, int32_t* blkoff, int32_t* out, int32_t* totals, void* scratch,
                        hipStream_t s, const int32_t* halt = nullptr);
void launch_rowsum(const LevelView& L, int bucket, const int32_t* list, int32_t count, i64* K, i64* Sig, Ctl* ctl,
                   hipStream_t s);
void launch_hub_caps(const LevelView& L, const int32_t* list, int32_t count, int64_t* caps, int64_t* nch,
                     hipStream_t s);
// mode: 0 = SYNC, 1 = ASYNC with cached loads, 2 = ASYNC with device-coherent loads/stores
void launch_move(const LevelView& L, int bucket, int mode, const MoveArgs& a, const int32_t* list, int32_t count,
                 hipStream_t s);
void launch_hub_insert(const LevelView& L, int mode, const MoveArgs& a, int64_t nchunks, hipStream_t s);
void launch_hub_decide(const LevelView& L, int mode, const MoveArgs& a, int64_t nchunks, hipStream_t s);
void launch_hub_final(const LevelView& L, int mode, const MoveArgs& a, hipStream_t s);
// SYNC iteration 0 on rows without repeated neighbours: hub decisions
// straight from the rows (C' is the identity snapshot), in place of
// launch_hub_insert + launch_hub_decide (launch_hub_final still combines).
void launch_hub_direct(const LevelView& L, int mode, const MoveArgs& a, int64_t nchunks, hipStream_t s);
void launch_hub_mark(const LevelView& L, const MoveArgs& a, int64_t nchunks, hipStream_t s);
void launch_move_fused(const LevelView& L, int mode, const MoveArgs& a, const FusedLists& f, hipStream_t s);
void launch_sync_apply(const LevelView& L, const MoveArgs& a, const int32_t* list, int64_t count, hipStream_t s);
void launch_learn_filter(const FilterArgs& f, int off64, hipStream_t s);
void launch_learn_label(float* samples, int64_t lo, int64_t hi, const uint32_t* moved, uint32_t itag,
                        hipStream_t s);
void launch_mlp_init(float* w, u64 seed, hipStream_t s);
void launch_mlp_predict(const float* w, const float* X, int64_t count, float* out, hipStream_t s);
void launch_mlp_zero(float* p, int64_t n, hipStream_t s);
void launch_mlp_loss_grad(const float* w, const float* S, int64_t count, int64_t slots, int32_t batch, u64 seed,
                          int64_t step, float pos_weight, float* grad, double* loss, hipStream_t s);
void launch_adam(float* w, const float* g, float* m, float* v, float lr, float bc1, float bc2, hipStream_t s);
// batched slices: per-(bucket, graph) segment counts of the queue, their
// starts, and for every slice the per-graph slot prefixes
// With dit (device-driven iterations): list is the queue's base, the bucket
// b segment is read from dit and len is only the launch's upper bound.
void launch_seg_count(const int32_t* list, int64_t len, const int32_t* gid, int32_t* segcnt, hipStream_t s,
                      const DevIter* dit = nullptr, int b = 0);
void launch_slice_prefix(const int32_t* segcnt, int nbt, int64_t count, int ns, int32_t* prefall, hipStream_t s);
// ---- device-driven iterations (lv_iter.hip)
// Up to 4 byte ranges zeroed by one launch (a kernel, so that the sequence
// can be captured); nothing happens when dit->halt is set.
struct ZeroRanges {
    void* p[4];
    int64_t bytes[4];
};
void launch_zero_ranges(const DevIter* dit, const ZeroRanges& z, hipStream_t s);
// Slices of an iteration: dshare[2 * (k * NB_MOVE + b)] = start of slice k
// of bucket b in the queue, dshare[... + 1] = its entries, for ns slices
// (contiguous shares, or every ns-th entry with interleave).
// Start of a pass: the queue is the pass's bucket lists (bcount), not halted.
void launch_iter_setup(DevIter* dit, const int32_t* bcount, int nbt, int32_t max_iterations, int32_t* dshare,
                       int ns, int interleave, hipStream_t s);
// End of iteration t (see lv_iter.hip for the rules; they are the host
// loop's).  thr: tolerance of the pass as tol_num, tol_den, tol_drop, pass.
struct IterEndArgs {
    DevIter* dit;
    const Ctl* ctl;
    int32_t t, may_end, prune, max_iterations, nbt;
    i64 W;
    int64_t tol_num, tol_den, tol_drop;
    int32_t pass;
    int64_t nbg;          // batched runs: graphs (0: single graph)
    const u64* Sg;        // per-graph gain sums (lo, hi)
    const u64* Wg;
    uint8_t* gact;        // cleared for graphs that converge
    int32_t* lig;         // per-graph iteration count of the pass
    int32_t* dshare;      // slices of the next iteration: ns_next of them
    int32_t ns_next, interleave;
};
void launch_iter_end(const IterEndArgs& e, hipStream_t s);

// ---- batched runs (lv_batch.hip)
void launch_gid_init(const int64_t* vbase, int64_t count, int64_t n, int32_t* gid, hipStream_t s);
void launch_graph_weights(const LevelView& L, const int32_t* gid, u64* Wg, Ctl* ctl, hipStream_t s);
void launch_nonisolated_by_graph(const LevelView& L, const int32_t* gid, u64* out, hipStream_t s);
void launch_used_by_graph(const int32_t* used, int64_t n, const int32_t* gid, u64* out, hipStream_t s);
void launch_gid_next(const int32_t* used, const int32_t* newid, int64_t n, const int32_t* gid, int32_t* gid_next,
                     hipStream_t s);
void launch_graph_cmin(const int32_t* C, int64_t n, const int32_t* gid, int32_t* cmin, hipStream_t s);
void launch_rebase(int32_t* C, int64_t n, const int32_t* gid, const int32_t* cmin, hipStream_t s);
void launch_modularity_arcs(const LevelView& L0, const int32_t* C, i64* sigin, i64* sigtot, hipStream_t s);
void launch_mod_terms_batch(int64_t ncom, const int32_t* cbase, int64_t count, const u64* Wg, const i64* sigin,
                            const i64* sigtot, u64* qlohi, hipStream_t s);

// ---- launchers: aggregation and modularity (lv_aggr.hip)
struct AggArgs {
    const int32_t* Cp;       // dense new community ids of the level's vertices
    const int32_t* coff;     // community-vertex CSR offsets (ncom+1)
    const int32_t* members;  // community-vertex CSR members
    const int64_t* hoff;     // holey offsets (ncom+1)
    int32_t* hidx;           // holey neighbour ids
    void* hw;                // holey weights (int32 or int64, per out_w64)
    int32_t* rowlen;         // distinct count per community
    int32_t out_w64;         // super-graph weights int64
    int32_t sorted;          // 1: rows ascending by neighbour id; 0: in table order
};
void launch_mark_used(const int32_t* Cp, int64_t n, int32_t* used, hipStream_t s);
void launch_relabel(int32_t* Cp, int64_t n, const int32_t* newid, hipStream_t s);
void launch_dendrogram(int32_t* C, int64_t n0, const int32_t* Cp, hipStream_t s);
void launch_final_lookup(int32_t* C, int64_t n0, const int32_t* Cp, const int32_t* newid, hipStream_t s);
void launch_comm_count(const LevelView& L, const int32_t* Cp, int32_t* cnt, int64_t* cdeg, hipStream_t s);
void launch_comm_fill(int64_t n, const int32_t* Cp, const int32_t* coff, int32_t* cursor, int32_t* members,
                      hipStream_t s);
// Ordered partition of communities into NB_AGG LDS buckets + the big path
// (totals to totals[0..NB_AGG]); zeroes rowlen.
void bucketize_communities(int64_t ncom, const int64_t* hoff, int64_t bound_cap, const Buckets& B, int32_t* rowlen,
                           int32_t* blkcnt, int32_t* blkoff, int32_t* out, int32_t* totals, void* scratch,
                           hipStream_t s);
void launch_aggregate(const LevelView& L, int bucket, const AggArgs& a, const int32_t* list, int32_t count,
                      hipStream_t s);

// Big communities: spread over many workgroups (see lv_aggr.hip).
constexpr int BIG_CH = 4096;          // virtual arcs per chunk (one workgroup)
constexpr int BIG_LCAP = 8192;        // LDS table slots per chunk
constexpr int64_t BIG_ARCS = 32768;   // communities with more arcs always take the big path
constexpr int BIG_EXTRACT_BLOCKS = 256;
struct BigArgs {
    const int32_t* list;       // big communities of this group
    int32_t nbig;
    const int64_t* chunk_pre;  // chunk prefix per big community (nbig+1 entries used)
    int64_t chunk_base;
    const int64_t* tab_pre;    // table-capacity prefix (nbig+1 entries used)
    int64_t tab_base;
    const int32_t* Cp;
    const int32_t* coff;
    const int32_t* members;
    const int64_t* mpos;       // exclusive prefix of member degrees, community-vertex order
    const int64_t* hoff;
    int32_t* keys;             // global table pool
    void* vals;
    int32_t* hidx;
    void* hw;
    int32_t out_w64;
    int32_t* rowlen;
    uint32_t* bitmaps;         // BIG_EXTRACT_BLOCKS * words
    int64_t words;             // ceil(ncom / 32)
    int32_t* cnt;              // per big community of the group: occupied table slots (zeroed by the host)
    int32_t* slots;            // occupied slot lists, community h's at its table offset / 2
    int32_t sorted;            // 1: rows ascending by neighbour id; 0: in table order
};
constexpr int BIG_SORT_MAX = 8192;  // rows up to this length are sorted in LDS at extraction
void launch_member_deg(const LevelView& L, const int32_t* members, int64_t n, int64_t* md, hipStream_t s);
void launch_big_info(const int32_t* list, int32_t nbig, const int64_t* hoff, int64_t ncom, int64_t* nch,
                     int64_t* cap, hipStream_t s);
void launch_big_clear(int32_t* keys, void* vals, int64_t count, hipStream_t s);
void launch_big_insert(const LevelView& L, const BigArgs& a, int64_t nchunks, hipStream_t s);
void launch_big_extract(const LevelView& L, const BigArgs& a, hipStream_t s);
void launch_compact(int64_t ncom, const int64_t* hoff, const int32_t* hidx, const void* hw, const void* goff,
                    int goff64, int32_t* gidx, void* gw, int w64, hipStream_t s);
void launch_rowlen_to_offsets(const int32_t* rowlen, int64_t ncom, void* goff, int goff64, void* scratch,
                              hipStream_t s);
void launch_modularity(const LevelView& L0, const int32_t* C, int64_t ncom, i64 W, i64* sigin, i64* sigtot,
                       Ctl* ctl, hipStream_t s);
void launch_validate(const LevelView& L, int check, Ctl* ctl, hipStream_t s);

}  // namespace lv
