/*
 * louvain.h -- C ABI of the MI355X (gfx950) Louvain library.
 *
 * The library runs the two phases of the Louvain method for modularity
 * maximisation -- local moving and aggregation -- on one GPU, as studied in
 * "CPU vs. GPU for Community Detection: Performance Insights from GVE-Louvain
 * and nu-Louvain" (Sahu, 2025).  References below name the paper's sections,
 * equations and algorithms.
 *
 * Conventions shared by every entry point:
 *  - Graphs are undirected, in symmetric CSR form: edge {i, j} with i != j is
 *    stored as the arcs (i, j) and (j, i) with equal weight; a self-loop is one
 *    arc (i, i).  Weights are positive integers.  W = sum of all arc weights is
 *    the paper's 2m (Preliminaries).
 *  - Pointers marked "device" must point to memory of the GPU current when the
 *    handle is created; "host" pointers to ordinary host memory.  The library
 *    never frees caller memory.
 *  - Every call returns a louvain_status; the library never aborts the
 *    process.  After a failure, louvain_last_error(handle) describes it.
 *  - A handle is bound to one HIP stream and is not thread-safe.  Calls that
 *    return results to the host synchronise that stream.
 */
#ifndef LOUVAIN_H
#define LOUVAIN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct louvain_s louvain_t; /* opaque handle */

typedef enum {
    LOUVAIN_OK = 0,
    LOUVAIN_ERR_INVALID = -1,   /* bad argument or malformed graph */
    LOUVAIN_ERR_NOMEM = -2,     /* host allocation failed */
    LOUVAIN_ERR_WORKSPACE = -3, /* workspace missing, misaligned or too small */
    LOUVAIN_ERR_HIP = -4,       /* a HIP runtime call failed */
    LOUVAIN_ERR_OVERFLOW = -5,  /* weights too large for the exact integer path */
    LOUVAIN_ERR_STATE = -6      /* call out of order (e.g. membership before run) */
} louvain_status;

/* Local-moving semantics.
 * ASYNC: one membership vector updated in place while vertices are processed
 *   (the paper's GPU design, Algorithm 5, with Pick-Less every rho
 *   iterations); nondeterministic order, reaches modularity close to the
 *   sequential method.
 * SYNC: every flagged vertex decides against the start-of-iteration state
 *   (C', Sigma'); all moves are then applied together.  Deterministic: the
 *   memberships, Sigma' and super-graphs are identical from run to run. */
typedef enum { LOUVAIN_ASYNC = 0, LOUVAIN_SYNC = 1 } louvain_mode;

/* Which vertices an iteration evaluates.
 * NONE: all vertices every iteration.
 * FLAGS: vertex pruning (Section 4.1, "Vertex pruning"): a vertex is evaluated
 *   again only after a neighbour changed community.
 * LEARNED: FLAGS, with each flagged vertex further filtered by the pruner MLP
 *   below, and a sweep guard: iteration 0 of a pass evaluates every vertex, so
 *   does an iteration whose filtered queue is empty and the iteration after a
 *   non-sweep iteration that passes the tolerance test; a pass ends only at
 *   such a sweep that passes the exit test (guard_tolerance = 0: no evaluated
 *   vertex had a positive best gain, before Pick-Less; 1: the tolerance test)
 *   or at max_iterations. */
typedef enum { LOUVAIN_PRUNE_NONE = 0, LOUVAIN_PRUNE_FLAGS = 1, LOUVAIN_PRUNE_LEARNED = 2 } louvain_pruner;

/* Learned move-pruner: an MLP 8 -> 32 -> 32 -> 1 with ReLU hidden layers, in
 * FP32.  Weight layout (LOUVAIN_MLP_PARAMS floats): W1[32][8], b1[32],
 * W2[32][32], b2[32], w3[32], b3.  Each neuron starts at its bias and adds
 * its inputs in index order by fused multiply-adds (a fully specified FP32
 * result).  A flagged vertex is evaluated iff the output logit z satisfies
 * z >= log(theta / (1 - theta)), i.e. sigmoid(z) >= theta = pruner_threshold
 * (theta <= 0 keeps all, theta >= 1 none).  Features of vertex v of the
 * current level at the start of iteration t of pass p, all FP32 from integers:
 *   f0 = mlog2(1 + deg v) / 16        f1 = own_v / K_v
 *   f2 = mlog2(1 + m_v) / 16          f3 = m_v / deg v
 *   f4 = 1 if v moved in t - 1, else 0
 *   f5 = p / 10                       f6 = t / 20
 *   f7 = adv_v / K_v
 * deg v = row length; m_v = neighbours j != v that moved in iteration t - 1;
 * own_v = K_{v->C'[v]} and adv_v = K_{v->d*} - K_{v->C'[v]} (d* = best
 * candidate, K_{v->d*} = 0 without one), both as of v's last evaluation in
 * the pass (0 before it); a ratio with a zero denominator is 0;
 * mlog2(x) = e + (x - 2^e) / 2^e with e = floor(log2 x) (Mitchell's
 * piecewise-linear logarithm). */
#define LOUVAIN_MLP_IN 8
#define LOUVAIN_MLP_HIDDEN 32
#define LOUVAIN_MLP_PARAMS (32 * 8 + 32 + 32 * 32 + 32 + 32 + 1)
#define LOUVAIN_SAMPLE_FLOATS 9 /* 8 features + label (1 = moved) */

/* Input graph.  offsets: device, n+1 entries of int32 (offset_bits = 32) or
 * int64 (offset_bits = 64), offsets[0] = 0, non-decreasing, offsets[n] = nnz.
 * indices: device, nnz int32 in [0, n).  weights: device, nnz int32 > 0, or
 * NULL for unit weights.  Requires n <= 2^31 - 2. */
typedef struct {
    int64_t n;
    int64_t nnz;
    int32_t offset_bits;
    const void* offsets;
    const int32_t* indices;
    const int32_t* weights;
} louvain_graph;

/* Parameters; louvain_params_default() fills the paper's values
 * (Section 4.3: 20 iterations per pass, 10 passes, tolerance 0.01 dropped
 * 10x per pass, aggregation tolerance 0.8, Pick-Less every 4 iterations,
 * vertex pruning). */
typedef struct {
    int32_t max_iterations;  /* per pass, >= 1 */
    int32_t max_passes;      /* <= 0: until convergence */
    int64_t tol_num;         /* initial tolerance tau_0 = tol_num / tol_den (>= 0) */
    int64_t tol_den;         /* > 0 */
    int64_t tol_drop;        /* tau_{p+1} = tau_p / tol_drop, >= 1 */
    int64_t agg_num;         /* aggregation tolerance tau_agg = agg_num / agg_den: */
    int64_t agg_den;         /*   stop when |Gamma| / |Gamma_old| > tau_agg */
    int32_t pick_less;       /* rho: Pick-Less on when (t + rho/2) mod rho == 0; 0 = off */
    int32_t mode;            /* louvain_mode */
    int32_t pruner;          /* louvain_pruner */
    int32_t validate;        /* 1: check offsets, indices and weights in create */
    /* Degree-bucket overrides (0 = library default).  bucket_max_degree[b] is
     * the largest degree handled by move bucket b; vertices above the last
     * bucket use global-memory hash tables.  Used by tests to force paths. */
    int32_t bucket_max_degree[8];
    int32_t agg_bucket_max[8];
    /* ASYNC only: 1 makes reads and writes of C' and Sigma' in the
     * local-moving kernels device-coherent, so a workgroup sees moves made by
     * workgroups on other chiplets within the same launch; 0 (default) uses
     * cached loads (moves become visible at kernel boundaries, i.e. from one
     * slice to the next). */
    int32_t async_coherent;
    /* Order in which degree buckets are launched within an iteration:
     * 0 = low degree first (default), 1 = high degree first. */
    int32_t bucket_order;
    /* ASYNC only: split every iteration into this many sequential launches
     * over consecutive slices of each bucket's queue (sorted by vertex id);
     * later slices see the moves of earlier ones.  1 = one launch per bucket;
     * default 64.  A single graph's level with more than async_slices x 2^19
     * queued vertices uses one slice per 2^19 of them, up to twice
     * async_slices, and scales async_hub_groups alike. */
    int32_t async_slices;
    /* ASYNC only: apply async_slices to the first this-many iterations of
     * every pass (0 = to every iteration). */
    int32_t async_slice_iters;
    /* LEARNED pruner only: exit test of a sweep (0 strict, the default: no
     * positive-gain move left; 1 tolerance). */
    int32_t guard_tolerance;
    /* ASYNC only: at least this many queued vertices per slice (default 256);
     * an iteration uses min(async_slices, queued / async_slice_min) slices. */
    int32_t async_slice_min;
    /* ASYNC only: the hubs (vertices above the largest LDS bucket) of an
     * iteration are processed in this many id-ordered groups, group k right
     * after slice floor((k + 1) * slices / groups) - 1; 0 = one group per
     * slice; default 32. */
    int32_t async_hub_groups;
    /* ASYNC only: 1 = a vertex alone in its community does not join another
     * single-vertex community of larger id (the pair merges the other way),
     * which prevents concurrent swaps of singletons; 1 = on (default). */
    int32_t async_min_label;
    const float* pruner_weights; /* LEARNED: device, LOUVAIN_MLP_PARAMS floats, read during louvain_run */
    double pruner_threshold;     /* LEARNED: theta */
    /* ASYNC only: 1 = slice s takes every slices-th entry of each bucket's
     * id-sorted queue starting at entry s (each slice samples every part of
     * the id range; in a batch, every graph); 0 = slice s takes the s-th
     * contiguous share (default; closer to the sequential order). */
    int32_t async_interleave;
    /* Width of the hash-table values (the accumulated K_{i->d} of local
     * moving and the merged weights of aggregation): 0 (default) = 32-bit
     * whenever the sums cannot reach 2^32, else 64-bit; 1 = always 64-bit.
     * Results do not depend on it (the paper's "datatype for hashtable
     * values" experiment, Section 4.3, made exact). */
    int32_t table_values_64;
    /* 1 = device-driven iterations: the tolerance test of Alg. 1 (per graph in
     * a batch), the next queue's sizes and the end of a pass's local moving
     * are decided on the device after each iteration, and the host enqueues
     * the iterations of a pass in chunks (2, 4, 8, ...) with one readback per
     * chunk instead of one per iteration; launches are sized for the pass's
     * largest queue and those after the pass's end return at once.  ASYNC
     * slices: every iteration of a pass uses the slice count of its first,
     * counted on the vertices with arcs (see async_slices).  Results: SYNC as
     * with 0.  Not with the LEARNED pruner, sample recording or an
     * iteration trace (LOUVAIN_ERR_INVALID).  0 = host-driven (default). */
    int32_t device_loop;
} louvain_params;

/* Per-run counters, filled by louvain_get_stats after louvain_run. */
typedef struct {
    int32_t passes;             /* passes whose local-moving phase ran */
    int32_t iterations;         /* local-moving iterations, all passes */
    int64_t moves;              /* vertex moves applied */
    int64_t communities;        /* final number of communities */
    int64_t vertices_evaluated; /* vertex evaluations in the local-moving phase */
    int64_t arcs_scanned;       /* arcs read by those evaluations */
    int64_t distinct_scanned;   /* sum over evaluations of distinct neighbour communities */
    double ms_total;            /* wall time of louvain_run */
    double ms_move;             /* local-moving kernels (HIP events; profile_kernels only) */
    double ms_aggregate;        /* aggregation kernels (HIP events; profile_kernels only) */
    int32_t iterations_per_pass[32];
    int64_t communities_per_pass[32];
    int64_t sweeps;             /* LEARNED: iterations that evaluated every vertex */
    int64_t pruned;             /* LEARNED: flagged vertices skipped by the MLP */
    int64_t host_syncs;         /* times louvain_run waited for the stream */
} louvain_stats;

/* Per-kernel timing record (profiling mode). */
typedef struct {
    char name[48];
    int64_t launches;
    double ms;          /* summed HIP-event time of those launches */
    int64_t alg_bytes;  /* algorithmic bytes moved by those launches */
} louvain_kernel_stat;

/* Trace callbacks (host memory; valid only during the call).
 * iter_fn: after every local-moving iteration, the level's membership C'
 *   (n ints) and community totals Sigma' (n int64), the number of moves and
 *   the exact gain sum S of the iteration (Eq. (2) times W^2/2) as hi/lo.
 * pass_fn: after every aggregation, the super-vertex graph in CSR form with
 *   rows sorted by neighbour id (offsets int64[n+1], indices, weights int64). */
typedef void (*louvain_iter_fn)(void* user, int32_t pass, int32_t iter, int64_t n, const int32_t* cprime,
                                const int64_t* sigma, int64_t moves, int64_t gain_hi, uint64_t gain_lo);
typedef void (*louvain_pass_fn)(void* user, int32_t pass, int64_t n, const int64_t* offsets,
                                const int32_t* indices, const int64_t* weights, int32_t iterations);

/* Fill p with the paper's defaults.  p: host, non-NULL. */
void louvain_params_default(louvain_params* p);

/* Bytes of device workspace the handle needs for this graph (upper bound
 * over all passes).  g, p, bytes: host, non-NULL.  Only g->n, g->nnz,
 * g->offset_bits and whether g->weights is NULL are read; no device access. */
louvain_status louvain_workspace_size(const louvain_graph* g, const louvain_params* p, size_t* bytes);

/* Create a handle for graph g on `stream` (a hipStream_t, NULL = default
 * stream).  workspace: device, >= louvain_workspace_size bytes, 256-byte
 * aligned, owned by the caller and borrowed until louvain_destroy, as are
 * the graph arrays (they are not copied).  Computes W and the weighted
 * degrees; with p->validate set, rejects malformed graphs with
 * LOUVAIN_ERR_INVALID.  Returns LOUVAIN_ERR_OVERFLOW when W exceeds 2^62.
 * out: host, receives the handle (NULL on failure). */
louvain_status louvain_create(const louvain_graph* g, const louvain_params* p, void* stream, void* workspace,
                              size_t workspace_bytes, louvain_t** out);

/* Run Louvain: the pass loop of Algorithm 1 / Algorithm 4 with the
 * local-moving phase (Algorithm 2 / 5) and the aggregation phase
 * (Algorithm 3 / 6).  Blocking: returns after the stream has drained.
 * May be called again; each call starts from singleton communities. */
louvain_status louvain_run(louvain_t* h);

/* Copy the final membership to out: device, n int32.  Community ids are
 * dense, 0 .. communities-1, numbered by ascending final label.
 * LOUVAIN_ERR_STATE before the first successful louvain_run. */
louvain_status louvain_get_membership(louvain_t* h, int32_t* out);

/* Modularity of the final membership on the input graph, Eq. (1), computed
 * on the GPU with exact integers: Q = num / den with num = sum_c (W*sigma_c -
 * Sigma_c^2) and den = W^2 (den = 1 when W = 0).  q: host double (may be
 * NULL); num, den: host int64[2] as {hi, lo bits} of a signed 128-bit
 * integer (may be NULL). */
louvain_status louvain_modularity(louvain_t* h, double* q, int64_t num[2], int64_t den[2]);

/* Counters of the last run.  s: host. */
louvain_status louvain_get_stats(louvain_t* h, louvain_stats* s);

/* Degree-bucket autotuner (for callers that run one graph, or one batch,
 * many times).  candidates: host int32[ncand * 8], candidate c in entries
 * [8c, 8c + 8) with the meaning of louvain_params.bucket_max_degree (move
 * buckets; 0 = default, negative = bucket unused, each clamped to the
 * bucket's table size).  The handle's current thresholds are the baseline:
 * they and every candidate are timed over reps runs of louvain_run (the
 * whole method: the timed quantity is the run).  A candidate is eligible if
 * its lowest modularity over its runs (Eq. (1); the mean over the graphs of
 * a batched handle) is at most 0.002 below the baseline's lowest.  The
 * fastest eligible candidate whose mean run time beats the baseline's mean
 * by more than the baseline's own spread (slowest minus fastest of its reps;
 * use reps >= 3 for a meaningful spread) is kept for later runs and its index
 * written to *best; otherwise the thresholds stay as they were and *best =
 * -1.  ms (host double[ncand]) receives each candidate's mean milliseconds.
 * best and ms may be NULL.  SYNC results do not depend on the thresholds;
 * ASYNC results may differ slightly between candidates (another concurrent
 * schedule).  The handle's membership and statistics are those of the last
 * timed run: call louvain_run again for a run with the chosen thresholds.
 * Errors: a run's status (thresholds restored); LOUVAIN_ERR_INVALID for
 * ncand < 1, reps < 1 or NULL candidates. */
louvain_status louvain_autotune(louvain_t* h, const int32_t* candidates, int32_t ncand, int32_t reps, int32_t* best,
                                double* ms);

/* Enable (1) or disable (0) per-kernel HIP-event timing for later runs.
 * Adds two event records per launch; off by default. */
louvain_status louvain_set_profiling(louvain_t* h, int32_t enable);

/* Copy up to max per-kernel records of the last run to out (host) and the
 * record count to *count. */
louvain_status louvain_get_kernel_stats(louvain_t* h, louvain_kernel_stat* out, int32_t max, int32_t* count);

/* Install trace callbacks (either may be NULL).  Tracing copies state to the
 * host after every iteration and pass; it is for testing, not speed. */
louvain_status louvain_set_trace(louvain_t* h, louvain_iter_fn iter_fn, louvain_pass_fn pass_fn, void* user);

/* Batched runs (many independent graphs in one run).  g is the union of
 * `count` graphs laid end to end in one CSR: graph k owns the vertices
 * [vbase[k], vbase[k+1]) (vbase: host array of count+1 entries, vbase[0] = 0,
 * non-decreasing, vbase[count] = n) and every arc of a vertex must stay in its
 * graph (checked in create; LOUVAIN_ERR_INVALID otherwise).  Every graph goes
 * through the method of louvain_run on its own -- its own total weight W_k,
 * tolerance test, iteration count, shrink tests and pass count -- as if run
 * alone; the graphs share every kernel launch.  Every pruner in both modes;
 * with LEARNED each graph follows its own sweep schedule, as in a lone run (a
 * graph sweeps after one of its non-sweep iterations passes the tolerance
 * test or when the filter keeps none of its vertices, and its pass ends only
 * at one of its sweeps whose exit test passes in that graph), so SYNC results
 * equal lone runs graph by graph.  Sample recording is refused on a batched
 * handle.
 * louvain_get_membership writes, for each vertex, its community within its
 * graph (0 .. communities_k - 1, ascending final label); louvain_modularity is
 * refused on a batched handle.  louvain_workspace_size_batch: bytes for a
 * batched handle (count = 0 gives the single-graph size). */
louvain_status louvain_workspace_size_batch(const louvain_graph* g, int64_t count, const louvain_params* p,
                                            size_t* bytes);
louvain_status louvain_create_batch(const louvain_graph* g, const int64_t* vbase, int64_t count,
                                    const louvain_params* p, void* stream, void* workspace, size_t workspace_bytes,
                                    louvain_t** out);
/* Per-graph modularity of the last run (Eq. (1) on each graph with its own
 * W_k): host arrays q[count], num[2*count], den[2*count] (each exact value
 * as a (hi, lo) int64 pair, den = W_k^2; W_k = 0 gives 0/1).  Any may be NULL. */
louvain_status louvain_modularity_batch(louvain_t* h, double* q, int64_t* num, int64_t* den);
/* Per-graph passes, local-moving iterations and final community counts of
 * the last run (host arrays of count entries; any may be NULL). */
louvain_status louvain_batch_results(louvain_t* h, int32_t* passes, int32_t* iterations, int64_t* communities);

/* Record pruner training samples during later runs of h (any mode and
 * pruner): in every iteration t >= 1 that is not a sweep, each vertex v of the
 * iteration's queue with splitmix64(v + 2^32 (p 2^16 + t)) mod 1000 <
 * sample_per_mille (splitmix64: the SplitMix64 output function of one
 * counter value) yields LOUVAIN_SAMPLE_FLOATS floats: its 8 features and the
 * label 1 if v moved in iteration t, else 0.  Samples are appended in no
 * particular order.  buffer: device, capacity * LOUVAIN_SAMPLE_FLOATS floats,
 * borrowed until the next call (buffer = NULL or sample_per_mille = 0
 * disables).  Samples beyond capacity are dropped; the count is reset at the
 * start of every louvain_run.  louvain_sample_count: samples written by the
 * last run (at most capacity). */
louvain_status louvain_collect_samples(louvain_t* h, float* buffer, int64_t capacity, int32_t sample_per_mille);
louvain_status louvain_sample_count(louvain_t* h, int64_t* count);

/* Pruner MLP on its own (no handle).  Pointers are device memory; work is
 * enqueued on `stream` and the calls return after it completes.  Errors:
 * LOUVAIN_ERR_INVALID for bad arguments, LOUVAIN_ERR_HIP for runtime failures
 * (message in louvain_last_error(NULL)).
 * louvain_pruner_init: Glorot-uniform weights, zero biases: parameter k of
 *   the flat layout draws u = (splitmix64(seed + k * 0x9E3779B97F4A7C15) >> 40)
 *   / 2^24 and becomes (2u - 1) * sqrt(6 / (fan_in + fan_out)) in FP32.
 * louvain_pruner_predict: logit[k] = MLP(features[8k .. 8k+7]) (FP32, the
 *   fused order above).
 * louvain_pruner_loss_grad: samples as recorded (8 features + label); loss =
 *   (1/N) sum_k c_k (softplus(z_k) - y_k z_k) with c_k = pos_weight for
 *   y_k = 1, else 1; grad (LOUVAIN_MLP_PARAMS floats) is overwritten with its
 *   gradient, *loss receives the loss.
 * louvain_pruner_train: `steps` Adam updates (Kingma and Ba; beta1 0.9,
 *   beta2 0.999, eps 1e-8, learning rate lr) of the same loss on mini-batches:
 *   slot j of step s uses sample splitmix64(seed + (s * batch + j) *
 *   0x9E3779B97F4A7C15) mod count (all samples, in order, when batch >=
 *   count).  scratch: louvain_pruner_scratch_floats(batch) floats of device
 *   memory (Adam moments, gradient); *last_loss receives the loss of the last
 *   mini-batch before its update. */
louvain_status louvain_pruner_init(float* weights, uint64_t seed, void* stream);
louvain_status louvain_pruner_predict(const float* weights, const float* features, int64_t count, float* logit,
                                      void* stream);
louvain_status louvain_pruner_loss_grad(const float* weights, const float* samples, int64_t count,
                                        float pos_weight, float* grad, double* loss, void* stream);
int64_t louvain_pruner_scratch_floats(int32_t batch);
louvain_status louvain_pruner_train(float* weights, const float* samples, int64_t count, int32_t steps,
                                    int32_t batch, float lr, float pos_weight, uint64_t seed, float* scratch,
                                    double* last_loss, void* stream);

/* louvain_pruner_train without caller scratch and without any device
 * allocation, for callers that cannot allocate (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc).  Same arguments,
 * results and errors as louvain_pruner_train, minus `scratch`: the gradient,
 * Adam moments and loss accumulator live in a static device array of
 * LOUVAIN_NOALLOC_SCRATCH_FLOATS floats (32 KiB), one per GPU, held until the
 * process ends.  Runs on the current device; `stream` must belong to it
 * (LOUVAIN_ERR_INVALID otherwise).  LOUVAIN_ERR_INVALID when
 * louvain_pruner_scratch_floats(batch) exceeds the array.  Every call on a
 * GPU shares that GPU's array (each call clears what it needs at its start):
 * calls that overlap on one GPU, on any streams, race and give undefined
 * weights. */
#define LOUVAIN_NOALLOC_SCRATCH_FLOATS 8192
louvain_status louvain_pruner_train_noalloc(float* weights, const float* samples, int64_t count, int32_t steps,
                                            int32_t batch, float lr, float pos_weight, uint64_t seed,
                                            double* last_loss, void* stream);

/* Last error message of h (or of the last failed create when h is NULL).
 * Never NULL; valid until the next call on h. */
const char* louvain_last_error(const louvain_t* h);

/* Release the handle (not the caller's graph or workspace).  NULL is ok. */
void louvain_destroy(louvain_t* h);

#ifdef __cplusplus
}
#endif

#endif /* LOUVAIN_H */
