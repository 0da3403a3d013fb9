/*
 * louvain_oracle.c -- plain, sequential CPU oracle for the Louvain method.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the correctness reference for the GPU
 * path: only the test suite, the smoke check and the benchmark's CPU-baseline
 * leg may load it.  It shares no code, header or constant with the GPU
 * library.
 *
 * What it computes follows the paper "CPU vs. GPU for Community Detection:
 * Performance Insights from GVE-Louvain and nu-Louvain" (Sahu, 2025):
 *   - modularity Q, Eq. (1) of the Preliminaries (section "Modularity");
 *   - the gain of moving one vertex, Eq. (2), multiplied by 2m^2 so that it is
 *     an exact integer;
 *   - the pass loop of Algorithm 1 / Algorithm 4 (louvain / nu-louvain);
 *   - the local-moving phase of Algorithm 2 (ASYNC mode: one membership
 *     vector updated in place, vertices visited in ascending id order) and a
 *     snapshot variant of Algorithm 5 (SYNC mode: every flagged vertex decides
 *     against the start-of-iteration state, Pick-Less every rho iterations,
 *     then all moves are applied together);
 *   - the aggregation phase of Algorithm 3 / Algorithm 6;
 *   - a learned move-pruner generalising the paper's vertex pruning (its
 *     Optimizations section): an MLP over eight per-vertex features decides
 *     which flagged vertices are evaluated, and a pass may only end after an
 *     unpruned sweep over every vertex passes the exit test.
 *
 * Notation (paper, Preliminaries): W = sum over stored arcs of w = 2m.
 * K_i = weighted degree (a self-loop arc counts once), K_{i->d} = weight from
 * i to the members of d other than i itself, Sigma_d = sum of K over d's
 * members (including i while i is in d), sigma_d = weight of arcs with both
 * ends in d.  c is the current community of i, d a candidate.
 *
 * Integers everywhere: weights are int64, products and sums of gains are
 * __int128.  Parity unpinned: none -- every function is pinned by the CPU
 * tests (brute force, closed forms, invariants, library routines).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef __int128 i128;

typedef struct {
    int64_t n;
    const int64_t* off;   /* n+1 */
    const int32_t* idx;   /* off[n] */
    const int64_t* w;     /* off[n] */
} og_graph;

typedef struct {
    int32_t max_iterations;   /* per pass (paper: 20) */
    int32_t max_passes;       /* <= 0 means unbounded (paper: 10) */
    int64_t tol_num, tol_den; /* initial tolerance tau_0 = tol_num/tol_den (paper: 1/100) */
    int64_t tol_drop;         /* tau_{p+1} = tau_p / tol_drop (paper: 10) */
    int64_t agg_num, agg_den; /* aggregation tolerance tau_agg = agg_num/agg_den (paper: 0.8) */
    int32_t mode;             /* 0 = ASYNC, 1 = SYNC */
    int32_t pick_less;        /* rho for SYNC mode, 0 = off (paper: 4) */
    int32_t prune;            /* 1 = vertex pruning (paper default), 0 = every vertex every iteration,
                                 2 = vertex pruning filtered by the learned MLP, with sweep guard */
    int32_t guard_tolerance;  /* prune 2: a sweep ends the pass if no evaluated vertex has a positive best
                                 gain (0), or if the sweep's gain sum passes the tolerance test (1) */
    const float* mlp;         /* prune 2: OG_MLP_PARAMS weights (layout at mlp_logit) */
    double threshold;         /* prune 2: a flagged vertex is evaluated iff sigmoid(logit) >= threshold */
    int32_t sample_per_mille; /* sample selection rate for the sample callback (0 = none) */
} og_params;

typedef struct {
    int32_t passes;           /* passes whose local-moving phase ran */
    int32_t iterations;       /* local-moving iterations over all passes */
    int64_t moves;            /* vertex moves applied over all passes */
    int64_t communities;      /* final number of communities */
    int64_t sweeps;           /* prune 2: iterations that evaluated every vertex (first ones included) */
    int64_t pruned;           /* prune 2: flagged vertices the MLP skipped */
} og_stats;

/* Per-iteration trace: state after the iteration's moves are applied. */
typedef void (*og_iter_fn)(void* user, int32_t pass, int32_t iter, int64_t n, const int32_t* cprime,
                           const int64_t* sigma, int64_t moves, int64_t gain_hi, uint64_t gain_lo);
/* Training sample: features of an evaluated vertex with at least one arc,
 * before the iteration, and whether it then moved.  Sweeps and iteration 0
 * record none. */
typedef void (*og_sample_fn)(void* user, int32_t pass, int32_t iter, int64_t v, const float* feat, int32_t label);
/* Per-pass trace: the super-vertex graph produced by aggregation. */
typedef void (*og_pass_fn)(void* user, int32_t pass, int64_t n, const int64_t* off, const int32_t* idx,
                           const int64_t* w, int32_t count);

/* ---------------------------------------------------------------- basics */

/* Weighted degree of every vertex (paper: vertexWeights). */
static void vertex_weights(const og_graph* g, int64_t* K) {
    for (int64_t i = 0; i < g->n; i++) {
        int64_t s = 0;
        for (int64_t e = g->off[i]; e < g->off[i + 1]; e++) s += g->w[e];
        K[i] = s;
    }
}

static int64_t total_weight(const og_graph* g) {
    int64_t s = 0;
    for (int64_t e = 0; e < g->off[g->n]; e++) s += g->w[e];
    return s;
}

/*
 * Modularity, Eq. (1), scaled by W^2:  Q * W^2 = sum_c (W*sigma_c - Sigma_c^2).
 * memb[i] must lie in [0, n).  Writes the numerator as (hi, lo) of an int128
 * and the denominator W^2 likewise; for W == 0 the result is 0/1.
 */
int oracle_modularity(int64_t n, const int64_t* off, const int32_t* idx, const int64_t* w,
                      const int32_t* memb, int64_t* num_hi, uint64_t* num_lo, int64_t* den_hi,
                      uint64_t* den_lo) {
    og_graph g = {n, off, idx, w};
    int64_t* sig_in = (int64_t*)calloc((size_t)(n > 0 ? n : 1), sizeof(int64_t));
    int64_t* sig_tot = (int64_t*)calloc((size_t)(n > 0 ? n : 1), sizeof(int64_t));
    if (!sig_in || !sig_tot) { free(sig_in); free(sig_tot); return -1; }
    for (int64_t i = 0; i < n; i++) {
        if (memb[i] < 0 || memb[i] >= n) { free(sig_in); free(sig_tot); return -2; }
        for (int64_t e = off[i]; e < off[i + 1]; e++) {
            sig_tot[memb[i]] += w[e];
            if (memb[idx[e]] == memb[i]) sig_in[memb[i]] += w[e];
        }
    }
    int64_t W = total_weight(&g);
    i128 num = 0;
    for (int64_t c = 0; c < n; c++) num += (i128)W * sig_in[c] - (i128)sig_tot[c] * sig_tot[c];
    i128 den = (W == 0) ? (i128)1 : (i128)W * W;
    if (W == 0) num = 0;
    *num_hi = (int64_t)(num >> 64); *num_lo = (uint64_t)num;
    *den_hi = (int64_t)(den >> 64); *den_lo = (uint64_t)den;
    free(sig_in); free(sig_tot);
    return 0;
}

/* ------------------------------------------------------- local moving */

typedef struct {
    int64_t* acc;      /* dense K_{i->d} scratch, all zero between uses */
    int32_t* touched;  /* communities touched by the current scan */
} scratch;

/*
 * scanCommunities(self = false) of Algorithm 2: K_{i->d} for every community
 * d of a neighbour j != i, accumulated into the dense array s->acc.
 * Returns the number of touched communities (listed in s->touched).
 */
static int64_t scan_communities(const og_graph* g, const int32_t* C, int64_t i, scratch* s) {
    int64_t nt = 0;
    for (int64_t e = g->off[i]; e < g->off[i + 1]; e++) {
        int64_t j = g->idx[e];
        if (j == i) continue;
        int32_t d = C[j];
        if (s->acc[d] == 0) s->touched[nt++] = d;  /* weights are > 0 */
        s->acc[d] += g->w[e];
    }
    return nt;
}

static void clear_scan(scratch* s, int64_t nt) {
    for (int64_t k = 0; k < nt; k++) s->acc[s->touched[k]] = 0;
}

/*
 * Integer form of Eq. (2): gain of moving i from its community c to d,
 * times 2m^2 = W^2/2:
 *     gain = W*(K_{i->d} - K_{i->c}) - K_i*(Sigma_d - Sigma_c + K_i)
 * with Sigma_c including K_i.
 */
static i128 move_gain(int64_t W, int64_t Ki, int64_t Kid, int64_t Kic, int64_t Sd, int64_t Sc) {
    return (i128)W * (Kid - Kic) - (i128)Ki * ((i128)Sd - Sc + Ki);
}

/*
 * Best community for i against the state (C, Sigma): the neighbour community
 * d != C[i] of largest gain, the smallest such d on ties.  Returns 1 and
 * fills (best_d, best_gain) when a candidate exists, 0 otherwise.
 */
static int best_move(const og_graph* g, int64_t W, const int32_t* C, const int64_t* Sig, const int64_t* K,
                     int64_t i, scratch* s, int32_t* best_d, i128* best_gain, int64_t* kic, int64_t* kid) {
    int64_t nt = scan_communities(g, C, i, s);
    int32_t c = C[i];
    int64_t Kic = s->acc[c];
    int found = 0;
    i128 bg = 0;
    int32_t bd = -1;
    int64_t bk = 0;
    for (int64_t k = 0; k < nt; k++) {
        int32_t d = s->touched[k];
        if (d == c) continue;
        i128 gain = move_gain(W, K[i], s->acc[d], Kic, Sig[d], Sig[c]);
        if (!found || gain > bg || (gain == bg && d < bd)) { bg = gain; bd = d; bk = s->acc[d]; found = 1; }
    }
    clear_scan(s, nt);
    *best_d = bd;
    *best_gain = bg;
    *kic = Kic;
    *kid = bk;
    return found;
}

/* ------------------------------------------------ learned move pruner */

#define OG_MLP_IN 8
#define OG_MLP_H 32
#define OG_MLP_PARAMS (OG_MLP_H * OG_MLP_IN + OG_MLP_H + OG_MLP_H * OG_MLP_H + OG_MLP_H + OG_MLP_H + 1)

/* Per-vertex state of the current pass from which the features are formed. */
typedef struct {
    int64_t* own;      /* K_{v->C'[v]} at v's last evaluation */
    int64_t* adv;      /* K_{v->d*} - K_{v->C'[v]} at v's last evaluation, d* = best candidate (K = 0 if none) */
    int32_t* moved_at; /* last iteration of the pass in which v moved, -1 if none */
    int32_t* nm_prev;  /* neighbours of v that moved in the previous iteration */
    int32_t* nm_cur;   /* neighbours of v that moved so far in this iteration */
} learn_state;

/* Piecewise-linear base-2 logarithm of an integer x >= 1 (Mitchell, 1962):
 * with e = floor(log2 x), e + (x - 2^e) / 2^e; exact at powers of two. */
static float mitchell_log2(int64_t x) {
    int e = 0;
    while ((x >> (e + 1)) != 0) e++;
    int64_t p = (int64_t)1 << e;
    float frac = (float)(x - p) / (float)p;
    return (float)e + frac;
}

/* The eight FP32 features of vertex v at the start of iteration t of pass p. */
static void features(const og_graph* g, const int64_t* K, const learn_state* L, int64_t v, int32_t pass,
                     int32_t t, float* f) {
    int64_t deg = g->off[v + 1] - g->off[v];
    int32_t m = L->nm_prev[v];
    f[0] = mitchell_log2(1 + deg) / 16.0f;
    f[1] = K[v] > 0 ? (float)L->own[v] / (float)K[v] : 0.0f;
    f[2] = mitchell_log2(1 + (int64_t)m) / 16.0f;
    f[3] = deg > 0 ? (float)m / (float)deg : 0.0f;
    f[4] = L->moved_at[v] == t - 1 ? 1.0f : 0.0f;
    f[5] = (float)pass / 10.0f;
    f[6] = (float)t / 20.0f;
    f[7] = K[v] > 0 ? (float)L->adv[v] / (float)K[v] : 0.0f;
}

/* MLP 8 -> 32 -> 32 -> 1 with ReLU hidden layers; returns the output logit.
 * Weights: W1[32][8], b1[32], W2[32][32], b2[32], w3[32], b3.  Every
 * neuron starts from its bias and adds its inputs in index order with fused
 * multiply-adds, so the FP32 result is fully specified. */
float oracle_mlp_logit(const float* P, const float* x) {
    const float* W1 = P;
    const float* b1 = W1 + OG_MLP_H * OG_MLP_IN;
    const float* W2 = b1 + OG_MLP_H;
    const float* b2 = W2 + OG_MLP_H * OG_MLP_H;
    const float* w3 = b2 + OG_MLP_H;
    const float b3 = w3[OG_MLP_H];
    float h1[OG_MLP_H], h2[OG_MLP_H];
    for (int k = 0; k < OG_MLP_H; k++) {
        float a = b1[k];
        for (int j = 0; j < OG_MLP_IN; j++) a = fmaf(W1[k * OG_MLP_IN + j], x[j], a);
        h1[k] = a > 0.0f ? a : 0.0f;
    }
    for (int k = 0; k < OG_MLP_H; k++) {
        float a = b2[k];
        for (int j = 0; j < OG_MLP_H; j++) a = fmaf(W2[k * OG_MLP_H + j], h1[j], a);
        h2[k] = a > 0.0f ? a : 0.0f;
    }
    float z = b3;
    for (int j = 0; j < OG_MLP_H; j++) z = fmaf(w3[j], h2[j], z);
    return z;
}

/* sigmoid(z) >= theta  <=>  z >= log(theta / (1 - theta)); theta <= 0 keeps
 * every vertex, theta >= 1 none (short of an infinite logit). */
static float logit_threshold(double theta) {
    if (theta <= 0.0) return -INFINITY;
    if (theta >= 1.0) return INFINITY;
    return (float)log(theta / (1.0 - theta));
}

/* SplitMix64 output function (Steele, Lea, Flood 2014) of one counter value. */
static uint64_t splitmix64(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* Training-sample selection: vertex v at (pass, iteration) is recorded iff
 * splitmix64(key) mod 1000 < per_mille, key = v + 2^32 * (pass * 2^16 + t). */
static int sample_selected(int64_t v, int32_t pass, int32_t t, int32_t per_mille) {
    if (per_mille <= 0) return 0;
    uint64_t key = (uint64_t)v + ((uint64_t)((uint32_t)pass * 65536u + (uint32_t)t) << 32);
    return (int32_t)(splitmix64(key) % 1000u) < per_mille;
}

/* Tolerance test of the local-moving loop: converged iff
 * (2 S / W^2) <= tau_p = tol_num / (tol_den * tol_drop^p),
 * i.e. 2*S*tol_den*tol_drop^p <= tol_num*W^2, evaluated exactly.
 */
static int converged(i128 S, int64_t W, const og_params* P, int32_t pass) {
    i128 lhs = 2 * S * (i128)P->tol_den;
    i128 rhs = (i128)P->tol_num * ((i128)W * W);
    for (int32_t k = 0; k < pass; k++) {
        if (lhs > rhs) return 0;          /* lhs only grows; once above, stays above */
        lhs *= P->tol_drop;
    }
    return lhs <= rhs;
}

/* Record vertex i's outcome in the learned-pruner state: its last
 * evaluation (own-community weight and best-candidate advantage). */
static void note_evaluation(learn_state* L, int64_t i, int found, int64_t kic, int64_t kid) {
    L->own[i] = kic;
    L->adv[i] = (found ? kid : 0) - kic;
}

/* Record a move of i in iteration t: i moved, and each neighbour j != i has
 * one more moved neighbour in this iteration. */
static void note_move(const og_graph* g, learn_state* L, int64_t i, int32_t t) {
    L->moved_at[i] = t;
    for (int64_t e = g->off[i]; e < g->off[i + 1]; e++)
        if (g->idx[e] != i) L->nm_cur[g->idx[e]]++;
}

/*
 * Local-moving phase.  Returns the number of iterations performed.
 *
 * prune = 0: every vertex is evaluated in every iteration.  prune = 1: the
 * paper's vertex pruning -- all vertices start flagged, an evaluated vertex
 * is unflagged, a mover flags its neighbours.  prune = 2: as 1, but in
 * iterations that are not sweeps a flagged vertex is evaluated only if the
 * MLP, given its features at that point, reaches the threshold (else it is
 * unflagged without evaluation); a sweep evaluates every vertex.  Iteration
 * 0 is a sweep; so is an iteration whose pruned queue would be empty, and
 * the iteration after a non-sweep iteration that passes the tolerance test.
 * The pass ends only at a sweep that passes the exit test (guard_tolerance
 * 0: no evaluated vertex had a positive best gain; 1: the tolerance test),
 * or after max_iterations.
 */
static int32_t local_move(const og_graph* g, int64_t W, int32_t* C, int64_t* Sig, const int64_t* K,
                          const og_params* P, int32_t pass, scratch* s, uint8_t* flag, int32_t* dec,
                          i128* gains, learn_state* L, og_stats* st, og_iter_fn it_cb, og_sample_fn sm_cb,
                          void* user) {
    int64_t n = g->n;
    const int learned = P->prune == 2;
    const int track = learned || (sm_cb && P->sample_per_mille > 0);
    const float zt = logit_threshold(P->threshold);
    for (int64_t i = 0; i < n; i++) flag[i] = 1;  /* all unprocessed */
    if (track)
        for (int64_t i = 0; i < n; i++) {
            L->own[i] = L->adv[i] = 0;
            L->moved_at[i] = -1;
            L->nm_prev[i] = L->nm_cur[i] = 0;
        }
    int sweep_next = 1;
    float f[OG_MLP_IN];
    for (int32_t t = 0; t < P->max_iterations; t++) {
        i128 S = 0;
        int64_t moves = 0, positive = 0;
        if (!P->prune)
            for (int64_t i = 0; i < n; i++) flag[i] = 1;
        int sweep = 0;
        if (learned) {
            sweep = sweep_next;
            if (!sweep) {
                int64_t kept = 0;
                for (int64_t i = 0; i < n && !kept; i++) {
                    if (!flag[i]) continue;
                    features(g, K, L, i, pass, t, f);
                    if (oracle_mlp_logit(P->mlp, f) >= zt) kept++;
                }
                if (!kept) sweep = 1;
            }
            if (sweep) {
                for (int64_t i = 0; i < n; i++) flag[i] = 1;
                st->sweeps++;
            }
        }
        /* features are formed for vertices the MLP filters or the sampler records */
        const int need_f = !sweep && t > 0 && (learned || (sm_cb && P->sample_per_mille > 0));
        if (P->mode == 0) {
            /* ASYNC: in place, ascending vertex order. */
            for (int64_t i = 0; i < n; i++) {
                if (!flag[i]) continue;
                flag[i] = 0;
                if (need_f) features(g, K, L, i, pass, t, f);
                if (learned && !sweep && oracle_mlp_logit(P->mlp, f) < zt) { st->pruned++; continue; }
                int32_t d;
                i128 gain;
                int64_t kic, kid;
                int found = best_move(g, W, C, Sig, K, i, s, &d, &gain, &kic, &kid);
                if (track) note_evaluation(L, i, found, kic, kid);
                if (found && gain > 0) positive++;
                int moved = found && gain > 0;
                if (moved) {
                    int32_t c = C[i];
                    Sig[c] -= K[i];
                    Sig[d] += K[i];
                    C[i] = d;
                    S += gain;
                    moves++;
                    for (int64_t e = g->off[i]; e < g->off[i + 1]; e++)
                        if (g->idx[e] != i) flag[g->idx[e]] = 1;
                    if (track) note_move(g, L, i, t);
                }
                if (need_f && sm_cb && g->off[i + 1] > g->off[i] && sample_selected(i, pass, t, P->sample_per_mille))
                    sm_cb(user, pass, t, i, f, moved);
            }
        } else {
            /* SYNC: decide against the snapshot, then apply together. */
            int pl = P->pick_less > 0 && ((t + P->pick_less / 2) % P->pick_less) == 0;
            for (int64_t i = 0; i < n; i++) {
                dec[i] = C[i];
                if (!flag[i]) continue;
                if (need_f) features(g, K, L, i, pass, t, f);
                if (learned && !sweep && oracle_mlp_logit(P->mlp, f) < zt) { st->pruned++; continue; }
                int32_t d;
                i128 gain;
                int64_t kic, kid;
                int found = best_move(g, W, C, Sig, K, i, s, &d, &gain, &kic, &kid);
                if (track) note_evaluation(L, i, found, kic, kid);
                int take = found && gain > 0;
                if (take) positive++;
                if (take && pl && d > C[i]) take = 0;  /* Pick-Less rejects a larger id */
                if (take) {
                    dec[i] = d;
                    gains[i] = gain;
                }
                if (need_f && sm_cb && g->off[i + 1] > g->off[i] && sample_selected(i, pass, t, P->sample_per_mille))
                    sm_cb(user, pass, t, i, f, take);
            }
            for (int64_t i = 0; i < n; i++) flag[i] = 0;
            for (int64_t i = 0; i < n; i++) {
                if (dec[i] == C[i]) continue;
                Sig[C[i]] -= K[i];
                Sig[dec[i]] += K[i];
                S += gains[i];
                moves++;
                for (int64_t e = g->off[i]; e < g->off[i + 1]; e++)
                    if (g->idx[e] != i) flag[g->idx[e]] = 1;
                if (track) note_move(g, L, i, t);
            }
            for (int64_t i = 0; i < n; i++) C[i] = dec[i];
        }
        if (track)
            for (int64_t i = 0; i < n; i++) { L->nm_prev[i] = L->nm_cur[i]; L->nm_cur[i] = 0; }
        st->iterations++;
        st->moves += moves;
        if (it_cb) it_cb(user, pass, t, n, C, Sig, moves, (int64_t)(S >> 64), (uint64_t)S);
        int conv = converged(S, W, P, pass);
        if (learned) {
            if (sweep && (P->guard_tolerance ? conv : positive == 0)) return t + 1;
            sweep_next = !sweep && conv;
        } else if (conv) {
            return t + 1;
        }
    }
    return P->max_iterations;
}

/* -------------------------------------------------------- aggregation */

static int cmp_i32(const void* a, const void* b) {
    int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
    return (x > y) - (x < y);
}

/*
 * Aggregation phase (Algorithm 3): with C holding dense ids in [0, nc),
 * super-vertex c gets an arc to d carrying the sum of w over every arc (i, j, w)
 * of G with C[i] = c and C[j] = d, self-loops included (scanCommunities with
 * self = true).  Rows are sorted by d.  Output arrays are malloc'ed.
 */
static int aggregate(const og_graph* g, const int32_t* C, int64_t nc, int64_t** o_off, int32_t** o_idx,
                     int64_t** o_w) {
    int64_t n = g->n;
    /* community-vertices CSR by counting and an exclusive scan */
    int64_t* coff = (int64_t*)calloc((size_t)nc + 1, sizeof(int64_t));
    int32_t* cmem = (int32_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    for (int64_t i = 0; i < n; i++) coff[C[i] + 1]++;
    for (int64_t c = 0; c < nc; c++) coff[c + 1] += coff[c];
    int64_t* cur = (int64_t*)malloc((size_t)(nc > 0 ? nc : 1) * sizeof(int64_t));
    memcpy(cur, coff, (size_t)nc * sizeof(int64_t));
    for (int64_t i = 0; i < n; i++) cmem[cur[C[i]]++] = (int32_t)i;
    free(cur);

    int64_t cap = g->off[n] > 0 ? g->off[n] : 1;
    int64_t* off = (int64_t*)malloc((size_t)(nc + 1) * sizeof(int64_t));
    int32_t* idx = (int32_t*)malloc((size_t)cap * sizeof(int32_t));
    int64_t* w = (int64_t*)malloc((size_t)cap * sizeof(int64_t));
    int64_t* acc = (int64_t*)calloc((size_t)(nc > 0 ? nc : 1), sizeof(int64_t));
    int32_t* touched = (int32_t*)malloc((size_t)(nc > 0 ? nc : 1) * sizeof(int32_t));
    int64_t pos = 0;
    off[0] = 0;
    for (int64_t c = 0; c < nc; c++) {
        int64_t nt = 0;
        for (int64_t k = coff[c]; k < coff[c + 1]; k++) {
            int64_t i = cmem[k];
            for (int64_t e = g->off[i]; e < g->off[i + 1]; e++) {
                int32_t d = C[g->idx[e]];
                if (acc[d] == 0) touched[nt++] = d;
                acc[d] += g->w[e];
            }
        }
        qsort(touched, (size_t)nt, sizeof(int32_t), cmp_i32);
        for (int64_t k = 0; k < nt; k++) {
            idx[pos] = touched[k];
            w[pos] = acc[touched[k]];
            acc[touched[k]] = 0;
            pos++;
        }
        off[c + 1] = pos;
    }
    free(acc); free(touched); free(coff); free(cmem);
    *o_off = off; *o_idx = idx; *o_w = w;
    return 0;
}

/* Standalone aggregation for tests: C must be dense in [0, nc).  The caller
 * passes output buffers of size nc+1 and off[n] (an upper bound). */
int oracle_aggregate(int64_t n, const int64_t* off, const int32_t* idx, const int64_t* w, const int32_t* C,
                     int64_t nc, int64_t* out_off, int32_t* out_idx, int64_t* out_w) {
    og_graph g = {n, off, idx, w};
    int64_t *o, *ww;
    int32_t* ii;
    for (int64_t i = 0; i < n; i++) if (C[i] < 0 || C[i] >= nc) return -2;
    aggregate(&g, C, nc, &o, &ii, &ww);
    memcpy(out_off, o, (size_t)(nc + 1) * sizeof(int64_t));
    memcpy(out_idx, ii, (size_t)o[nc] * sizeof(int32_t));
    memcpy(out_w, ww, (size_t)o[nc] * sizeof(int64_t));
    free(o); free(ii); free(ww);
    return 0;
}

/* Dense renumbering of labels by ascending old id: map[c] = #used labels < c.
 * Returns the number of distinct labels. */
static int64_t renumber(int64_t n, int32_t* C, int32_t* map) {
    for (int64_t c = 0; c < n; c++) map[c] = 0;
    for (int64_t i = 0; i < n; i++) map[C[i]] = 1;
    int64_t k = 0;
    for (int64_t c = 0; c < n; c++) { int32_t u = map[c]; map[c] = (int32_t)k; k += u; }
    for (int64_t i = 0; i < n; i++) C[i] = map[C[i]];
    return k;
}

/* ------------------------------------------------------------ driver */

/*
 * Louvain (Algorithm 1 / Algorithm 4).  Writes the final membership of the
 * input's n vertices (dense ids, numbered by ascending final label) to memb.
 */
int oracle_louvain_samples(int64_t n, const int64_t* off, const int32_t* idx, const int64_t* w,
                           const og_params* P, int32_t* memb, og_stats* st, og_iter_fn it_cb, og_pass_fn pass_cb,
                           og_sample_fn sm_cb, void* user) {
    memset(st, 0, sizeof(*st));
    int64_t n0 = n;
    for (int64_t v = 0; v < n0; v++) memb[v] = (int32_t)v;
    if (n0 == 0) return 0;
    size_t nn = (size_t)n0;
    int64_t* K = (int64_t*)malloc(nn * sizeof(int64_t));
    int64_t* Sig = (int64_t*)malloc(nn * sizeof(int64_t));
    int32_t* Cp = (int32_t*)malloc(nn * sizeof(int32_t));
    int32_t* dec = (int32_t*)malloc(nn * sizeof(int32_t));
    int32_t* map = (int32_t*)malloc(nn * sizeof(int32_t));
    uint8_t* flag = (uint8_t*)malloc(nn);
    i128* gains = (i128*)malloc(nn * sizeof(i128));
    scratch s;
    s.acc = (int64_t*)calloc(nn, sizeof(int64_t));
    s.touched = (int32_t*)malloc(nn * sizeof(int32_t));
    if (!K || !Sig || !Cp || !dec || !map || !flag || !gains || !s.acc || !s.touched) return -1;
    if (P->prune == 2 && !P->mlp) return -2;
    learn_state L;
    L.own = (int64_t*)malloc(nn * sizeof(int64_t));
    L.adv = (int64_t*)malloc(nn * sizeof(int64_t));
    L.moved_at = (int32_t*)malloc(nn * sizeof(int32_t));
    L.nm_prev = (int32_t*)malloc(nn * sizeof(int32_t));
    L.nm_cur = (int32_t*)malloc(nn * sizeof(int32_t));
    if (!L.own || !L.adv || !L.moved_at || !L.nm_prev || !L.nm_cur) return -1;

    og_graph g = {n0, off, idx, w};
    int64_t *own_off = NULL, *own_w = NULL;
    int32_t* own_idx = NULL;
    int64_t W = total_weight(&g);
    int stopped_before_aggregate = 0;

    for (int32_t p = 0; P->max_passes <= 0 || p < P->max_passes; p++) {
        int64_t nc = g.n;
        vertex_weights(&g, K);
        for (int64_t i = 0; i < nc; i++) { Sig[i] = K[i]; Cp[i] = (int32_t)i; }
        int32_t li = local_move(&g, W, Cp, Sig, K, P, p, &s, flag, dec, gains, &L, st, it_cb, sm_cb, user);
        st->passes++;
        stopped_before_aggregate = 1;
        if (li <= 1) break;  /* globally converged */
        /* community counts over vertices of non-zero weighted degree */
        int64_t gamma_old = 0, gamma = 0;
        for (int64_t i = 0; i < nc; i++) map[i] = 0;
        for (int64_t i = 0; i < nc; i++)
            if (K[i] > 0) { gamma_old++; if (!map[Cp[i]]) { map[Cp[i]] = 1; gamma++; } }
        if (gamma == gamma_old) break;                        /* no merge */
        if (gamma * P->agg_den > P->agg_num * gamma_old) break; /* low shrink */
        int64_t ncom = renumber(nc, Cp, map);
        for (int64_t v = 0; v < n0; v++) memb[v] = Cp[memb[v]];   /* dendrogram lookup */
        int64_t *no, *nw;
        int32_t* ni;
        aggregate(&g, Cp, ncom, &no, &ni, &nw);
        free(own_off); free(own_idx); free(own_w);
        own_off = no; own_idx = ni; own_w = nw;
        g.n = ncom; g.off = no; g.idx = ni; g.w = nw;
        stopped_before_aggregate = 0;
        if (pass_cb) pass_cb(user, p, ncom, no, ni, nw, li);
    }
    if (stopped_before_aggregate)
        for (int64_t v = 0; v < n0; v++) memb[v] = Cp[memb[v]];
    st->communities = renumber(n0, memb, map);

    free(own_off); free(own_idx); free(own_w);
    free(K); free(Sig); free(Cp); free(dec); free(map); free(flag); free(gains);
    free(s.acc); free(s.touched);
    free(L.own); free(L.adv); free(L.moved_at); free(L.nm_prev); free(L.nm_cur);
    return 0;
}

int oracle_louvain(int64_t n, const int64_t* off, const int32_t* idx, const int64_t* w, const og_params* P,
                   int32_t* memb, og_stats* st, og_iter_fn it_cb, og_pass_fn pass_cb, void* user) {
    return oracle_louvain_samples(n, off, idx, w, P, memb, st, it_cb, pass_cb, NULL, user);
}

/* The eight features of vertex v computed from a given state, for tests:
 * deg, K_v, own, adv, nm (moved neighbours), moved_last (0/1), pass, t. */
void oracle_features(int64_t deg, int64_t Kv, int64_t own, int64_t adv, int32_t nm, int32_t moved_last,
                     int32_t pass, int32_t t, float* f) {
    int64_t off2[2] = {0, deg};
    og_graph g = {1, off2, NULL, NULL};
    int64_t K1[1] = {Kv}, o1[1] = {own}, a1[1] = {adv};
    int32_t m1[1] = {moved_last ? t - 1 : -1}, n1[1] = {nm}, z1[1] = {0};
    learn_state L = {o1, a1, m1, n1, z1};
    features(&g, K1, &L, 0, pass, t, f);
}

/* ------------------------------------------------- single-vertex helpers */

/* Gain (Eq. 2 times W^2/2) of moving i from C[i] to community d under the
 * membership C, with K and Sigma recomputed from the graph. */
int oracle_gain(int64_t n, const int64_t* off, const int32_t* idx, const int64_t* w, const int32_t* C,
                int64_t i, int32_t d, int64_t* gain_hi, uint64_t* gain_lo) {
    og_graph g = {n, off, idx, w};
    int64_t* K = (int64_t*)malloc((size_t)n * sizeof(int64_t));
    int64_t* Sig = (int64_t*)calloc((size_t)n, sizeof(int64_t));
    vertex_weights(&g, K);
    for (int64_t v = 0; v < n; v++) Sig[C[v]] += K[v];
    int64_t Kid = 0, Kic = 0;
    for (int64_t e = off[i]; e < off[i + 1]; e++) {
        if (idx[e] == i) continue;
        if (C[idx[e]] == d) Kid += w[e];
        if (C[idx[e]] == C[i]) Kic += w[e];
    }
    i128 gain = move_gain(total_weight(&g), K[i], Kid, Kic, Sig[d], Sig[C[i]]);
    *gain_hi = (int64_t)(gain >> 64); *gain_lo = (uint64_t)gain;
    free(K); free(Sig);
    return 0;
}

/* Decision of one vertex against a given state (C, Sigma): the best
 * neighbour community and its gain, as in best_move above.  K is recomputed
 * for i only.  Returns 1 if a candidate exists. */
int oracle_best_move(int64_t n, const int64_t* off, const int32_t* idx, const int64_t* w, int64_t W,
                     const int32_t* C, const int64_t* Sig, int64_t i, int32_t* best_d, int64_t* gain_hi,
                     uint64_t* gain_lo) {
    og_graph g = {n, off, idx, w};
    int64_t Ki = 0;
    for (int64_t e = off[i]; e < off[i + 1]; e++) Ki += w[e];
    /* sparse scratch sized to the row: communities as keys, linear search */
    int64_t deg = off[i + 1] - off[i];
    int32_t* keys = (int32_t*)malloc((size_t)(deg > 0 ? deg : 1) * sizeof(int32_t));
    int64_t* vals = (int64_t*)malloc((size_t)(deg > 0 ? deg : 1) * sizeof(int64_t));
    int64_t nk = 0, Kic = 0;
    for (int64_t e = off[i]; e < off[i + 1]; e++) {
        if (idx[e] == i) continue;
        int32_t d = C[idx[e]];
        int64_t k = 0;
        while (k < nk && keys[k] != d) k++;
        if (k == nk) { keys[nk] = d; vals[nk] = 0; nk++; }
        vals[k] += w[e];
    }
    for (int64_t k = 0; k < nk; k++) if (keys[k] == C[i]) Kic = vals[k];
    int found = 0;
    i128 bg = 0;
    int32_t bd = -1;
    for (int64_t k = 0; k < nk; k++) {
        if (keys[k] == C[i]) continue;
        i128 gain = move_gain(W, Ki, vals[k], Kic, Sig[keys[k]], Sig[C[i]]);
        if (!found || gain > bg || (gain == bg && keys[k] < bd)) { bg = gain; bd = keys[k]; found = 1; }
    }
    (void)g;
    free(keys); free(vals);
    *best_d = bd;
    *gain_hi = (int64_t)(bg >> 64); *gain_lo = (uint64_t)bg;
    return found;
}
