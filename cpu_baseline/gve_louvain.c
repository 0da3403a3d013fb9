/*
 * gve_louvain.c -- multicore CPU Louvain in the style of GVE-Louvain, for
 * timing the GPU library against all host cores.
 *
 * This is a benchmark baseline, not a reference: its results are checked for
 * validity and modularity, never for equality.  It shares no code with the
 * GPU library or with the sequential oracle.
 *
 * Design (the paper's section on optimisations for multicore Louvain):
 *  - the local-moving phase runs an OpenMP loop over the vertices with a
 *    dynamic schedule of chunk 2048; membership C' and community totals
 *    Sigma' are updated in place (asynchronously), Sigma' by atomic adds;
 *  - each thread owns a collision-free ("Far-KV") table: a dense value array
 *    over all community ids plus the list of ids it touched, cleared after
 *    every vertex;
 *  - vertex pruning: a vertex is processed again only after a neighbour
 *    moved; threshold scaling (tau dropped 10x per pass), at most 20
 *    iterations per pass and 10 passes, aggregation tolerance 0.8;
 *  - aggregation builds the community-vertex CSR with parallel prefix sums,
 *    preallocates every super-row by the community's total degree ("holey"
 *    CSR), fills rows in parallel with the per-thread tables, then compacts.
 *
 * Gains are the integer form of delta-modularity (Eq. 2 times W^2/2),
 *   gain(i: c -> d) = W (K_{i->d} - K_{i->c}) - K_i (Sigma_d - Sigma_c + K_i),
 * with Sigma_c including K_i; sums of gains are 128-bit.  Community counts
 * for the aggregation-tolerance test cover vertices with at least one arc.
 */
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef __int128 i128;

typedef struct {
    int32_t max_iterations, max_passes;
    int64_t tol_num, tol_den, tol_drop, agg_num, agg_den;
} gve_params;

typedef struct {
    int32_t passes, iterations;
    int64_t moves, communities;
} gve_stats;

/* Far-KV table of one thread: dense values over community ids, touched list. */
typedef struct {
    int64_t* val;
    int32_t* keys;
    int64_t nk;
} farkv;

static inline int64_t ld64(const int64_t* p) { return __atomic_load_n(p, __ATOMIC_RELAXED); }
static inline int32_t ld32(const int32_t* p) { return __atomic_load_n(p, __ATOMIC_RELAXED); }

/* Exclusive prefix sum of in[0..n) into out[0..n] (out[n] = total), in parallel. */
static void scan_i64(const int64_t* in, int64_t* out, int64_t n, int nt) {
    int64_t* part = (int64_t*)calloc((size_t)nt + 1, sizeof(int64_t));
    int64_t total = 0;
#pragma omp parallel num_threads(nt)
    {
        const int t = omp_get_thread_num(), T = omp_get_num_threads();
        const int64_t lo = n * t / T, hi = n * (t + 1) / T;
        int64_t s = 0;
        for (int64_t i = lo; i < hi; i++) s += in[i];
        part[t + 1] = s;
#pragma omp barrier
#pragma omp single
        {
            for (int k = 1; k <= T; k++) part[k] += part[k - 1];
            total = part[T];
        }
        s = part[t];
        for (int64_t i = lo; i < hi; i++) {
            const int64_t x = in[i];
            out[i] = s;
            s += x;
        }
    }
    out[n] = total;
    free(part);
}

static int converged(i128 S, int64_t W, const gve_params* P, int pass) {
    /* 2 S / W^2 <= tol_num / (tol_den * drop^pass) */
    unsigned __int128 rhs = (unsigned __int128)P->tol_num * ((unsigned __int128)W * (unsigned __int128)W);
    unsigned __int128 lhs = 2 * (unsigned __int128)S * (unsigned __int128)P->tol_den;
    for (int k = 0; k < pass; k++) {
        if (lhs > rhs) return 0;
        lhs *= (unsigned __int128)P->tol_drop;
    }
    return lhs <= rhs;
}

/* Local-moving phase on one level; returns the iterations run. */
static int32_t local_move(int64_t n, const int64_t* off, const int32_t* idx, const int64_t* w, int64_t W,
                          const int64_t* K, int64_t* Sig, int32_t* Cp, uint8_t* flag, farkv* tabs, int nt,
                          const gve_params* P, int pass, int64_t* moves_out) {
    for (int32_t t = 0; t < P->max_iterations; t++) {
        i128 S = 0;
        int64_t moves = 0;
#pragma omp parallel num_threads(nt) reduction(+ : moves)
        {
            farkv* tb = &tabs[omp_get_thread_num()];
            i128 Sl = 0;
#pragma omp for schedule(dynamic, 2048)
            for (int64_t i = 0; i < n; i++) {
                if (!__atomic_load_n(&flag[i], __ATOMIC_RELAXED)) continue;
                __atomic_store_n(&flag[i], 0, __ATOMIC_RELAXED);
                const int32_t c = ld32(&Cp[i]);
                for (int64_t e = off[i]; e < off[i + 1]; e++) {
                    const int32_t j = idx[e];
                    if (j == i) continue;
                    const int32_t d = ld32(&Cp[j]);
                    if (tb->val[d] == 0) tb->keys[tb->nk++] = d;
                    tb->val[d] += w[e];
                }
                const int64_t Ki = K[i], kic = tb->val[c];
                const int64_t Sc = ld64(&Sig[c]);
                int32_t best = -1;
                i128 bg = 0;
                for (int64_t k = 0; k < tb->nk; k++) {
                    const int32_t d = tb->keys[k];
                    if (d == c) continue;
                    const i128 g = (i128)W * (tb->val[d] - kic) - (i128)Ki * ((i128)ld64(&Sig[d]) - Sc + Ki);
                    if (g > bg || (g == bg && g > 0 && d < best)) { bg = g; best = d; }
                }
                for (int64_t k = 0; k < tb->nk; k++) tb->val[tb->keys[k]] = 0;
                tb->nk = 0;
                if (best >= 0 && bg > 0) {
                    __atomic_fetch_add(&Sig[c], -Ki, __ATOMIC_RELAXED);
                    __atomic_fetch_add(&Sig[best], Ki, __ATOMIC_RELAXED);
                    __atomic_store_n(&Cp[i], best, __ATOMIC_RELAXED);
                    for (int64_t e = off[i]; e < off[i + 1]; e++)
                        if (idx[e] != i) __atomic_store_n(&flag[idx[e]], 1, __ATOMIC_RELAXED);
                    Sl += bg;
                    moves++;
                }
            }
#pragma omp critical
            S += Sl;
        }
        *moves_out += moves;
        if (converged(S, W, P, pass)) return t + 1;
    }
    return P->max_iterations;
}

/* Aggregation of level (n, off, idx, w) by the dense labels Cp (0..nc-1). */
static void aggregate(int64_t n, const int64_t* off, const int32_t* idx, const int64_t* w, const int32_t* Cp,
                      int64_t nc, farkv* tabs, int nt, int64_t** o_off, int32_t** o_idx, int64_t** o_w) {
    int64_t* cnt = (int64_t*)calloc((size_t)nc + 1, sizeof(int64_t));
    int64_t* tdeg = (int64_t*)calloc((size_t)nc + 1, sizeof(int64_t));
#pragma omp parallel for num_threads(nt) schedule(static, 2048)
    for (int64_t i = 0; i < n; i++) {
        __atomic_fetch_add(&cnt[Cp[i]], 1, __ATOMIC_RELAXED);
        __atomic_fetch_add(&tdeg[Cp[i]], off[i + 1] - off[i], __ATOMIC_RELAXED);
    }
    int64_t* coff = (int64_t*)malloc(((size_t)nc + 1) * sizeof(int64_t));
    int64_t* hoff = (int64_t*)malloc(((size_t)nc + 1) * sizeof(int64_t));
    scan_i64(cnt, coff, nc, nt);
    scan_i64(tdeg, hoff, nc, nt);
    int32_t* members = (int32_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    memset(cnt, 0, ((size_t)nc + 1) * sizeof(int64_t));
#pragma omp parallel for num_threads(nt) schedule(static, 2048)
    for (int64_t i = 0; i < n; i++) {
        const int64_t at = __atomic_fetch_add(&cnt[Cp[i]], 1, __ATOMIC_RELAXED);
        members[coff[Cp[i]] + at] = (int32_t)i;
    }
    const int64_t hm = hoff[nc];
    int32_t* hidx = (int32_t*)malloc((size_t)(hm > 0 ? hm : 1) * sizeof(int32_t));
    int64_t* hw = (int64_t*)malloc((size_t)(hm > 0 ? hm : 1) * sizeof(int64_t));
    int64_t* rl = tdeg;  /* reused: distinct entries per super-row */
#pragma omp parallel num_threads(nt)
    {
        farkv* tb = &tabs[omp_get_thread_num()];
#pragma omp for schedule(dynamic, 2048)
        for (int64_t c = 0; c < nc; c++) {
            for (int64_t k = coff[c]; k < coff[c + 1]; k++) {
                const int32_t i = members[k];
                for (int64_t e = off[i]; e < off[i + 1]; e++) {
                    const int32_t d = Cp[idx[e]];
                    if (tb->val[d] == 0) tb->keys[tb->nk++] = d;
                    tb->val[d] += w[e];
                }
            }
            int64_t p = hoff[c];
            for (int64_t k = 0; k < tb->nk; k++) {
                hidx[p] = tb->keys[k];
                hw[p++] = tb->val[tb->keys[k]];
                tb->val[tb->keys[k]] = 0;
            }
            rl[c] = tb->nk;
            tb->nk = 0;
        }
    }
    int64_t* noff = (int64_t*)malloc(((size_t)nc + 1) * sizeof(int64_t));
    scan_i64(rl, noff, nc, nt);
    const int64_t m2 = noff[nc];
    int32_t* nidx = (int32_t*)malloc((size_t)(m2 > 0 ? m2 : 1) * sizeof(int32_t));
    int64_t* nw = (int64_t*)malloc((size_t)(m2 > 0 ? m2 : 1) * sizeof(int64_t));
#pragma omp parallel for num_threads(nt) schedule(static, 2048)
    for (int64_t c = 0; c < nc; c++) {
        memcpy(nidx + noff[c], hidx + hoff[c], (size_t)rl[c] * sizeof(int32_t));
        memcpy(nw + noff[c], hw + hoff[c], (size_t)rl[c] * sizeof(int64_t));
    }
    free(cnt); free(tdeg); free(coff); free(hoff); free(members); free(hidx); free(hw);
    *o_off = noff;
    *o_idx = nidx;
    *o_w = nw;
}

/* Dense relabelling of Cp (0..nc-1 by ascending old label); returns nc. */
static int64_t renumber(int64_t n, int32_t* Cp, int64_t* map, int nt) {
    int64_t* used = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
#pragma omp parallel for num_threads(nt) schedule(static, 4096)
    for (int64_t i = 0; i < n; i++) __atomic_store_n(&used[Cp[i]], 1, __ATOMIC_RELAXED);
    scan_i64(used, map, n, nt);
    const int64_t nc = map[n];
#pragma omp parallel for num_threads(nt) schedule(static, 4096)
    for (int64_t i = 0; i < n; i++) Cp[i] = (int32_t)map[Cp[i]];
    free(used);
    return nc;
}

/* Louvain on (n, off, idx, w); membership: n int32 (output, dense ids).
 * Returns 0, or -1 when memory runs out. */
int gve_louvain(int64_t n, const int64_t* off, const int32_t* idx, const int64_t* w, const gve_params* P,
                int threads, int32_t* membership, gve_stats* st) {
    const int nt = threads > 0 ? threads : omp_get_max_threads();
    memset(st, 0, sizeof(*st));
    int64_t W = 0;
#pragma omp parallel for num_threads(nt) reduction(+ : W) schedule(static, 4096)
    for (int64_t e = 0; e < (n > 0 ? off[n] : 0); e++) W += w[e];
    farkv* tabs = (farkv*)calloc((size_t)nt, sizeof(farkv));
    for (int t = 0; t < nt; t++) {
        tabs[t].val = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
        tabs[t].keys = (int32_t*)malloc(((size_t)n + 1) * sizeof(int32_t));
        if (!tabs[t].val || !tabs[t].keys) return -1;
    }
    int64_t* K = (int64_t*)malloc(((size_t)n + 1) * sizeof(int64_t));
    int64_t* Sig = (int64_t*)malloc(((size_t)n + 1) * sizeof(int64_t));
    int32_t* Cp = (int32_t*)malloc(((size_t)n + 1) * sizeof(int32_t));
    uint8_t* flag = (uint8_t*)malloc((size_t)n + 1);
    int64_t* map = (int64_t*)malloc(((size_t)n + 2) * sizeof(int64_t));
#pragma omp parallel for num_threads(nt) schedule(static, 4096)
    for (int64_t i = 0; i < n; i++) membership[i] = (int32_t)i;
    int64_t cn = n;
    const int64_t* co = off;
    const int32_t* ci = idx;
    const int64_t* cw = w;
    int64_t *own_o = NULL, *own_w = NULL;
    int32_t* own_i = NULL;
    int aggregated_last = 0;
    for (int pass = 0; P->max_passes <= 0 || pass < P->max_passes; pass++) {
        int64_t nonisolated = 0;
#pragma omp parallel for num_threads(nt) reduction(+ : nonisolated) schedule(static, 2048)
        for (int64_t i = 0; i < cn; i++) {
            int64_t s = 0;
            for (int64_t e = co[i]; e < co[i + 1]; e++) s += cw[e];
            K[i] = Sig[i] = s;
            Cp[i] = (int32_t)i;
            flag[i] = 1;
            nonisolated += co[i + 1] > co[i];
        }
        const int32_t li = local_move(cn, co, ci, cw, W, K, Sig, Cp, flag, tabs, nt, P, pass, &st->moves);
        st->passes++;
        st->iterations += li;
        aggregated_last = 0;
        if (li <= 1) break;
        const int64_t nc = renumber(cn, Cp, map, nt);
        const int64_t gamma = nc - (cn - nonisolated);
        if (gamma == nonisolated ||
            (i128)gamma * P->agg_den > (i128)P->agg_num * nonisolated)
            break;
#pragma omp parallel for num_threads(nt) schedule(static, 4096)
        for (int64_t v = 0; v < n; v++) membership[v] = Cp[membership[v]];
        int64_t *no, *nw;
        int32_t* ni;
        aggregate(cn, co, ci, cw, Cp, nc, tabs, nt, &no, &ni, &nw);
        free(own_o); free(own_i); free(own_w);
        own_o = no; own_i = ni; own_w = nw;
        co = no; ci = ni; cw = nw;
        cn = nc;
        aggregated_last = 1;
    }
    if (!aggregated_last) {
        /* the loop stopped before aggregating: look the last level's labels up */
        renumber(cn, Cp, map, nt);
#pragma omp parallel for num_threads(nt) schedule(static, 4096)
        for (int64_t v = 0; v < n; v++) membership[v] = Cp[membership[v]];
    }
    /* final dense ids by ascending label */
    st->communities = renumber(n, membership, map, nt);
    for (int t = 0; t < nt; t++) { free(tabs[t].val); free(tabs[t].keys); }
    free(tabs); free(K); free(Sig); free(Cp); free(flag); free(map);
    free(own_o); free(own_i); free(own_w);
    return 0;
}

int gve_max_threads(void) { return omp_get_max_threads(); }
