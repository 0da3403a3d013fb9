// lv_internal.h -- host-side interface between the C ABI driver and the
// kernel launchers of the gfx950 Louvain library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lv_common.h"

namespace lv {

// Compiled local-moving variants: G lanes per vertex, CAP LDS table slots per
// vertex (a vertex of degree D needs CAP >= 2*D).  Bucket NB_MOVE is the
// global-memory ("hub") path.
constexpr int NB_MOVE = 5;
constexpr int MOVE_G[NB_MOVE] = {8, 16, 64, 256, 1024};
constexpr int MOVE_CAP[NB_MOVE] = {16, 64, 256, 2048, 8192};
constexpr int MOVE_DEFAULT_MAX[NB_MOVE] = {8, 32, 128, 1024, 4096};
constexpr int HUB_G = 1024;

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

// Per-iteration arguments of the local-moving kernels.
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
    int32_t prune;        // 1: mark neighbours of movers for the next iteration
    int32_t check_mark;   // hub path: skip vertices whose mark != stamp_cur
    uint32_t stamp_cur;   // stamp of vertices queued for this iteration
    uint32_t stamp_next;  // stamp for the next iteration's queue
    uint32_t* mark;
    const uint8_t* vbucket;
    int32_t* qnext;
    const int64_t* qseg;  // per-bucket segment start in queues (device)
    Ctl* ctl;
    int32_t* movers;      // SYNC: (vertex, target) pairs
    int32_t bucket;       // bucket id for per-bucket counters
    int32_t log2cap;      // hub path: unused (per-vertex)
    int32_t* hub_keys;    // hub path: table pool
    void* hub_vals;
    const int64_t* hub_off;  // hub path: table offsets (per hub list entry, chunk-relative base subtracted)
    int64_t hub_base;
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
void launch_fill_buckets(int64_t n, const uint8_t* vbucket, int32_t* blist, const int64_t* seg, Ctl* ctl,
                         hipStream_t s);
void launch_rowsum(const LevelView& L, int bucket, const int32_t* list, int32_t count, i64* K, i64* Sig, Ctl* ctl,
                   hipStream_t s);
void launch_hub_caps(const LevelView& L, const int32_t* list, int32_t count, int64_t* caps, hipStream_t s);
void launch_move(const LevelView& L, int bucket, int sync, const MoveArgs& a, const int32_t* list, int32_t count,
                 hipStream_t s);
void launch_move_hub(const LevelView& L, int sync, const MoveArgs& a, const int32_t* list, int32_t count,
                     hipStream_t s);
void launch_sync_apply(const LevelView& L, const MoveArgs& a, hipStream_t s);

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
    int32_t* hub_keys;
    void* hub_vals;
    const int64_t* hub_off;
    int64_t hub_base;
};
void launch_mark_used(const int32_t* Cp, int64_t n, int32_t* used, hipStream_t s);
void launch_relabel(int32_t* Cp, int64_t n, const int32_t* newid, hipStream_t s);
void launch_dendrogram(int32_t* C, int64_t n0, const int32_t* Cp, hipStream_t s);
void launch_final_lookup(int32_t* C, int64_t n0, const int32_t* Cp, const int32_t* newid, hipStream_t s);
void launch_comm_count(const LevelView& L, const int32_t* Cp, int32_t* cnt, int64_t* cdeg, hipStream_t s);
void launch_comm_fill(int64_t n, const int32_t* Cp, const int32_t* coff, int32_t* cursor, int32_t* members,
                      hipStream_t s);
void launch_agg_classify(int64_t ncom, const int64_t* hoff, int64_t bound_cap, const Buckets& B, uint8_t* cbucket,
                         int32_t* rowlen, Ctl* ctl, hipStream_t s);
void launch_agg_fill(int64_t ncom, const uint8_t* cbucket, int32_t* alist, const int64_t* seg, Ctl* ctl,
                     hipStream_t s);
void launch_agg_caps(const int32_t* list, int32_t count, const int64_t* hoff, int64_t bound_cap, int64_t* caps,
                     hipStream_t s);
void launch_aggregate(const LevelView& L, int bucket, const AggArgs& a, const int32_t* list, int32_t count,
                      hipStream_t s);
void launch_aggregate_hub(const LevelView& L, const AggArgs& a, const int32_t* list, int32_t count,
                          hipStream_t s);
void launch_compact(int64_t ncom, const int64_t* hoff, const int32_t* hidx, const void* hw, const void* goff,
                    int goff64, int32_t* gidx, void* gw, int w64, hipStream_t s);
void launch_rowlen_to_offsets(const int32_t* rowlen, int64_t ncom, void* goff, int goff64, void* scratch,
                              hipStream_t s);
void launch_modularity(const LevelView& L0, const int32_t* C, int64_t ncom, i64 W, i64* sigin, i64* sigtot,
                       Ctl* ctl, hipStream_t s);
void launch_validate(const LevelView& L, int check, Ctl* ctl, hipStream_t s);

}  // namespace lv
