/*
 * Seeded synthetic graph generators and a symmetric-CSR builder.
 *
 * This module produces the inputs that both the CPU oracle and the GPU path
 * consume.  It holds no part of the community-detection arithmetic: it only
 * draws random numbers, deduplicates undirected edges and lays them out as a
 * symmetric CSR (each undirected edge stored as two arcs, rows sorted
 * ascending by neighbour id, no self-loops).
 *
 * Randomness is counter-based so that any draw can be recomputed from
 * (seed, stream, counter) alone:
 *   SplitMix64 finaliser (Steele, Lea, Flood, "Fast splittable pseudorandom
 *   number generators", OOPSLA 2014): z += 0x9e3779b97f4a7c15;
 *   z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9; z = (z ^ (z >> 27)) *
 *   0x94d049bb133111eb; return z ^ (z >> 31).
 * A draw is mix(mix(seed ^ mix(stream)) + counter).  Edge weights are a pure
 * function of (seed, min(u,v), max(u,v)), so they never depend on the order
 * in which edges are produced.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static inline uint64_t mix64(uint64_t z) {
    z += 0x9e3779b97f4a7c15ULL;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

uint64_t gg_rand(uint64_t seed, uint64_t stream, uint64_t ctr) {
    return mix64(mix64(seed ^ mix64(stream)) + ctr);
}

/* Uniform double in [0, 1) with 53 random bits. */
static inline double gg_unit(uint64_t seed, uint64_t stream, uint64_t ctr) {
    return (double)(gg_rand(seed, stream, ctr) >> 11) * (1.0 / 9007199254740992.0);
}

enum { ST_RMAT = 1, ST_PERM = 2, ST_WEIGHT = 3, ST_GRID_DEL = 4, ST_GRID_DIAG = 5,
       ST_GRID_DIR = 6, ST_SBM = 7, ST_ERDOS = 8 };

/* Weight of undirected edge {u, v}: uniform integer in [wmin, wmax]. */
static inline int32_t edge_weight(uint64_t seed, int64_t u, int64_t v, int32_t wmin, int32_t wmax) {
    if (wmin >= wmax) return wmin;
    int64_t a = u < v ? u : v, b = u < v ? v : u;
    uint64_t r = gg_rand(seed, ST_WEIGHT, ((uint64_t)a << 32) ^ (uint64_t)b ^ ((uint64_t)a >> 32));
    return wmin + (int32_t)(r % (uint64_t)(wmax - wmin + 1));
}

/* ---------------------------------------------------------------------- */
/* LSD radix sort of 64-bit keys holding `bits` significant bits.          */
/* ---------------------------------------------------------------------- */
static int radix_sort_u64(uint64_t* keys, int64_t m, int bits) {
    if (m <= 1) return 0;
    uint64_t* tmp = (uint64_t*)malloc((size_t)m * sizeof(uint64_t));
    if (!tmp) return -1;
    const int DIG = 11;
    const int64_t R = 1 << DIG;
    int64_t* cnt = (int64_t*)malloc((size_t)R * sizeof(int64_t));
    if (!cnt) { free(tmp); return -1; }
    uint64_t* src = keys;
    uint64_t* dst = tmp;
    int passes = 0;
    for (int shift = 0; shift < bits; shift += DIG) {
        memset(cnt, 0, (size_t)R * sizeof(int64_t));
        for (int64_t i = 0; i < m; i++) cnt[(src[i] >> shift) & (R - 1)]++;
        int64_t s = 0;
        for (int64_t d = 0; d < R; d++) { int64_t c = cnt[d]; cnt[d] = s; s += c; }
        for (int64_t i = 0; i < m; i++) dst[cnt[(src[i] >> shift) & (R - 1)]++] = src[i];
        uint64_t* t = src; src = dst; dst = t;
        passes++;
    }
    if (passes & 1) memcpy(keys, src, (size_t)m * sizeof(uint64_t));
    free(cnt);
    free(tmp);
    return 0;
}

static int bits_for(uint64_t x) {
    int b = 0;
    while (b < 64 && (x >> b)) b++;
    return b;
}

/* Sort keys (u*n + v, u < v), drop duplicates; returns the unique count. */
static int64_t sort_unique(uint64_t* keys, int64_t m, int64_t n) {
    if (radix_sort_u64(keys, m, bits_for((uint64_t)n * (uint64_t)n)) != 0) return -1;
    int64_t k = 0;
    for (int64_t i = 0; i < m; i++)
        if (k == 0 || keys[k - 1] != keys[i]) keys[k++] = keys[i];
    return k;
}

/* Seeded Fisher-Yates permutation of [0, n). */
static void make_perm(int64_t n, uint64_t seed, int32_t* perm) {
    for (int64_t i = 0; i < n; i++) perm[i] = (int32_t)i;
    for (int64_t i = n - 1; i > 0; i--) {
        int64_t j = (int64_t)(gg_rand(seed, ST_PERM, (uint64_t)i) % (uint64_t)(i + 1));
        int32_t t = perm[i]; perm[i] = perm[j]; perm[j] = t;
    }
}

/* Exported permutation (the R-MAT relabelling) for the device generator. */
void gg_perm(int64_t n, uint64_t seed, int32_t* perm) { make_perm(n, seed, perm); }

/*
 * Symmetric CSR from sorted unique keys u*n+v (u < v).  Rows come out sorted:
 * the lower neighbours (keys with v == row) are placed first in key order,
 * which is ascending u, then the upper neighbours in ascending v.
 * off has n+1 entries; idx and w have 2*m entries (w may be NULL).
 */
void gg_csr_from_keys(int64_t n, int64_t m, const uint64_t* keys, uint64_t seed,
                      int32_t wmin, int32_t wmax, int64_t* off, int32_t* idx, int32_t* w) {
    memset(off, 0, (size_t)(n + 1) * sizeof(int64_t));
    for (int64_t e = 0; e < m; e++) {
        int64_t u = (int64_t)(keys[e] / (uint64_t)n), v = (int64_t)(keys[e] % (uint64_t)n);
        off[u + 1]++;
        off[v + 1]++;
    }
    for (int64_t i = 0; i < n; i++) off[i + 1] += off[i];
    int64_t* cur = (int64_t*)malloc((size_t)n * sizeof(int64_t));
    memcpy(cur, off, (size_t)n * sizeof(int64_t));
    for (int64_t e = 0; e < m; e++) {  /* lower neighbours of v */
        int64_t u = (int64_t)(keys[e] / (uint64_t)n), v = (int64_t)(keys[e] % (uint64_t)n);
        int64_t p = cur[v]++;
        idx[p] = (int32_t)u;
        if (w) w[p] = edge_weight(seed, u, v, wmin, wmax);
    }
    for (int64_t e = 0; e < m; e++) {  /* upper neighbours of u */
        int64_t u = (int64_t)(keys[e] / (uint64_t)n), v = (int64_t)(keys[e] % (uint64_t)n);
        int64_t p = cur[u]++;
        idx[p] = (int32_t)v;
        if (w) w[p] = edge_weight(seed, u, v, wmin, wmax);
    }
    free(cur);
}

/* ---------------------------------------------------------------------- */
/* R-MAT (Chakrabarti, Zhan, Faloutsos 2004): each of ntuples edges picks   */
/* one quadrant per level with probabilities a, b, c, 1-a-b-c.  Vertex ids */
/* are then relabelled by a seeded permutation (if permute), self-loops    */
/* dropped and duplicates merged.  keys must hold ntuples entries.         */
/* Returns the number of unique undirected edges, or -1 on failure.        */
/* ---------------------------------------------------------------------- */
int64_t gg_rmat_keys(int scale, int64_t ntuples, double a, double b, double c, uint64_t seed,
                     int permute, uint64_t* keys) {
    int64_t n = (int64_t)1 << scale;
    int32_t* perm = NULL;
    if (permute) {
        perm = (int32_t*)malloc((size_t)n * sizeof(int32_t));
        if (!perm) return -1;
        make_perm(n, seed, perm);
    }
    double ab = a + b, abc = a + b + c;
    int64_t m = 0;
#pragma omp parallel for schedule(static) reduction(+ : m)
    for (int64_t k = 0; k < ntuples; k++) {
        int64_t u = 0, v = 0;
        for (int l = 0; l < scale; l++) {
            double r = gg_unit(seed, ST_RMAT, (uint64_t)k * (uint64_t)scale + (uint64_t)l);
            int bu = 0, bv = 0;
            if (r < a) { }
            else if (r < ab) bv = 1;
            else if (r < abc) bu = 1;
            else { bu = 1; bv = 1; }
            u = (u << 1) | bu;
            v = (v << 1) | bv;
        }
        if (perm) { u = perm[u]; v = perm[v]; }
        if (u == v) { keys[k] = UINT64_MAX; continue; }
        if (u > v) { int64_t t = u; u = v; v = t; }
        keys[k] = (uint64_t)u * (uint64_t)n + (uint64_t)v;
        m += 1;
    }
    free(perm);
    /* Move the self-loop markers out, then sort and deduplicate. */
    int64_t k2 = 0;
    for (int64_t k = 0; k < ntuples; k++)
        if (keys[k] != UINT64_MAX) keys[k2++] = keys[k];
    (void)m;
    return sort_unique(keys, k2, n);
}

/* ---------------------------------------------------------------------- */
/* Road-like grid: rows x cols lattice, 4-neighbour edges each kept with    */
/* probability 1 - p_del; every cell (r, c) with r < rows-1, c < cols-1    */
/* gets a diagonal with probability p_diag, (r,c)-(r+1,c+1) or             */
/* (r,c+1)-(r+1,c) with equal odds.  keys needs 2*rows*cols entries.       */
/* ---------------------------------------------------------------------- */
int64_t gg_grid_keys(int64_t rows, int64_t cols, double p_del, double p_diag, uint64_t seed,
                     uint64_t* keys) {
    int64_t n = rows * cols, m = 0;
    for (int64_t r = 0; r < rows; r++) {
        for (int64_t c = 0; c < cols; c++) {
            int64_t id = r * cols + c;
            if (c + 1 < cols && gg_unit(seed, ST_GRID_DEL, (uint64_t)(2 * id)) >= p_del)
                keys[m++] = (uint64_t)id * (uint64_t)n + (uint64_t)(id + 1);
            if (r + 1 < rows && gg_unit(seed, ST_GRID_DEL, (uint64_t)(2 * id + 1)) >= p_del)
                keys[m++] = (uint64_t)id * (uint64_t)n + (uint64_t)(id + cols);
            if (r + 1 < rows && c + 1 < cols && gg_unit(seed, ST_GRID_DIAG, (uint64_t)id) < p_diag) {
                if (gg_rand(seed, ST_GRID_DIR, (uint64_t)id) & 1)
                    keys[m++] = (uint64_t)(id + 1) * (uint64_t)n + (uint64_t)(id + cols);
                else
                    keys[m++] = (uint64_t)id * (uint64_t)n + (uint64_t)(id + cols + 1);
            }
        }
    }
    return sort_unique(keys, m, n);
}

/* ---------------------------------------------------------------------- */
/* Stochastic block model with k blocks of near-equal size (sizes differ    */
/* by at most one; vertex v belongs to block v*k/n before the optional     */
/* relabelling).  Every pair inside a block is an edge with probability    */
/* p_in, every pair across blocks with p_out.  Pairs are visited by        */
/* geometric skipping (Batagelj and Brandes, Phys. Rev. E 71, 2005), so    */
/* the cost is proportional to the number of edges.                        */
/* Writes block labels (after relabelling) to label[n] when non-NULL.      */
/* keys must hold cap entries; returns the unique count or -1 (overflow).  */
/* ---------------------------------------------------------------------- */
static int64_t block_start(int64_t n, int64_t k, int64_t b) { return (b * n + k - 1) / k; }

int64_t gg_sbm_keys(int64_t n, int64_t k, double p_in, double p_out, uint64_t seed, int permute,
                    uint64_t* keys, int64_t cap, int32_t* label) {
    int32_t* perm = NULL;
    if (permute) {
        perm = (int32_t*)malloc((size_t)n * sizeof(int32_t));
        if (!perm) return -1;
        make_perm(n, seed, perm);
    }
    int64_t m = 0;
    uint64_t ctr = 0;
    for (int64_t ba = 0; ba < k; ba++) {
        int64_t a0 = block_start(n, k, ba), a1 = block_start(n, k, ba + 1);
        for (int64_t bb = ba; bb < k; bb++) {
            int64_t b0 = block_start(n, k, bb), b1 = block_start(n, k, bb + 1);
            double p = (ba == bb) ? p_in : p_out;
            if (p <= 0.0) continue;
            /* candidate pairs, enumerated in a fixed order */
            int64_t na = a1 - a0, nb = b1 - b0;
            int64_t total = (ba == bb) ? na * (na - 1) / 2 : na * nb;
            double lq = (p < 1.0) ? log1p(-p) : 0.0;
            int64_t pos = -1;
            for (;;) {
                if (p >= 1.0) pos += 1;
                else {
                    double r = gg_unit(seed, ST_SBM, ctr++);
                    pos += 1 + (int64_t)floor(log1p(-r) / lq);
                }
                if (pos >= total || pos < 0) break;
                int64_t u, v;
                if (ba == bb) {
                    /* pos -> (x, y) with 0 <= x < y < na, row-major over x */
                    int64_t x = (int64_t)floor((2.0 * na - 1.0 - sqrt((2.0 * na - 1.0) * (2.0 * na - 1.0) - 8.0 * (double)pos)) / 2.0);
                    if (x < 0) x = 0;
                    while (x > 0 && x * (2 * na - x - 1) / 2 > pos) x--;
                    while ((x + 1) * (2 * na - x - 2) / 2 <= pos) x++;
                    int64_t y = pos - x * (2 * na - x - 1) / 2 + x + 1;
                    u = a0 + x; v = a0 + y;
                } else {
                    u = a0 + pos / nb; v = b0 + pos % nb;
                }
                if (perm) { u = perm[u]; v = perm[v]; }
                if (u > v) { int64_t t = u; u = v; v = t; }
                if (m >= cap) { free(perm); return -1; }
                keys[m++] = (uint64_t)u * (uint64_t)n + (uint64_t)v;
            }
        }
    }
    if (label) {
        for (int64_t b = 0; b < k; b++)
            for (int64_t v = block_start(n, k, b); v < block_start(n, k, b + 1); v++)
                label[perm ? perm[v] : v] = (int32_t)b;
    }
    free(perm);
    return sort_unique(keys, m, n);
}

/* ---------------------------------------------------------------------- */
/* Erdos-Renyi G(n, p) with a seeded stream (small random test graphs).    */
/* ---------------------------------------------------------------------- */
int64_t gg_erdos_keys(int64_t n, double p, uint64_t seed, uint64_t* keys, int64_t cap) {
    int64_t m = 0;
    for (int64_t u = 0; u < n; u++)
        for (int64_t v = u + 1; v < n; v++)
            if (gg_unit(seed, ST_ERDOS, (uint64_t)(u * n + v)) < p) {
                if (m >= cap) return -1;
                keys[m++] = (uint64_t)u * (uint64_t)n + (uint64_t)v;
            }
    return m;
}
