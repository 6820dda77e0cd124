/*
 * Seeded synthetic graph generators (input generation only).
 *
 * This file builds the inputs that both the traversal library and the test
 * oracle consume: undirected graphs in CSR form (symmetric, no self loops, no
 * duplicate edges, every adjacency list sorted ascending) plus per-edge
 * integer weights. It contains none of the traversal arithmetic (no BFS, no
 * shortest paths, no colouring); it only draws random numbers and packs
 * edges.
 *
 * Random numbers: SplitMix64 (Steele, Lea and Flood, "Fast Splittable
 * Pseudorandom Number Generators", OOPSLA 2014), used counter-style so every
 * draw is an independent pure function of (seed, stream, index) and can be
 * computed in any order or in parallel. With sm(x) one SplitMix64 step (add
 * the golden gamma G, two xor-shift-multiply rounds, a final xor-shift):
 *     base(seed, stream) = sm(seed ^ (stream << 56))
 *     r(seed, stream, i) = sm(base + i * G)
 * i.e. draw i is output i of a SplitMix64 generator whose state starts at
 * base. (Xoring the seed into the counter instead would make different
 * seeds permute the same aligned block of draws.)
 *
 * Graph families (the paper's inputs are not available, so these stand in):
 *   - Erdos-Renyi G(n, m): endpoint pairs drawn uniformly in counter order;
 *     a pair is accepted unless it is a loop or repeats an accepted edge;
 *     generation stops at m accepted edges, so the average degree is 2m/n.
 *   - R x C 4-neighbour grid: vertex (r, c) has id r*C + c.
 *   - R-MAT (Chakrabarti, Zhan, Faloutsos 2004): ef * 2^scale draws, each
 *     descending `scale` quadrant choices with probabilities (a, b, c, d);
 *     vertex ids are then relabelled by a seeded random permutation; loops
 *     and duplicate edges are dropped.
 *   - Weights belong to the undirected edge {u, v}: uniform integer in
 *     [lo, hi] keyed by (min(u,v) * n + max(u,v)), so both arcs agree.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#define GG_GAMMA 0x9E3779B97F4A7C15ull

enum { GG_STREAM_ER = 1, GG_STREAM_RMAT = 2, GG_STREAM_PERM = 3, GG_STREAM_W = 4,
       GG_STREAM_MISC = 5, GG_STREAM_PTS = 6, GG_STREAM_CENTRES = 7 };

uint64_t gg_splitmix64(uint64_t x) {
    uint64_t z = x + GG_GAMMA;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

uint64_t gg_rand(uint64_t seed, uint32_t stream, uint64_t i) {
    uint64_t base = gg_splitmix64(seed ^ ((uint64_t)stream << 56));
    return gg_splitmix64(base + i * GG_GAMMA);
}

/* Uniform integer in [lo, hi] by rejection (no modulo bias). Attempt a of
 * draw i uses counter i ^ (a << 48); i must stay below 2^48. */
uint64_t gg_uniform(uint64_t seed, uint32_t stream, uint64_t i, uint64_t lo, uint64_t hi) {
    uint64_t range = hi - lo + 1;           /* 0 means the full 2^64 range */
    if (range == 0) return gg_rand(seed, stream, i);
    /* accept r below the largest multiple of range that fits in 2^64 */
    uint64_t limit = (UINT64_MAX / range) * range - 1;
    if (UINT64_MAX % range == range - 1) limit = UINT64_MAX;   /* 2^64 divisible by range */
    for (uint64_t a = 0;; ++a) {
        uint64_t r = gg_rand(seed, stream, i ^ (a << 48));
        if (r <= limit) return lo + r % range;
    }
}

/* Real in [0, 1) from the top 53 bits. */
double gg_real(uint64_t seed, uint32_t stream, uint64_t i) {
    return (double)(gg_rand(seed, stream, i) >> 11) * (1.0 / 9007199254740992.0);
}

/* ---------------------------------------------------------------- sorting */

/* LSD radix sort of 64-bit keys using 8-bit digits; skips digits that are
 * zero in every key. tmp must hold n keys. Histograms for all digits are
 * taken in one read pass. */
static void radix_sort_u64(uint64_t* keys, uint64_t* tmp, uint64_t n) {
    uint64_t all_or = 0;
    uint64_t (*cnt)[256] = (uint64_t (*)[256])calloc(8 * 256, sizeof(uint64_t));
    for (uint64_t i = 0; i < n; ++i) {
        uint64_t k = keys[i];
        all_or |= k;
        for (int d = 0; d < 8; ++d) cnt[d][(k >> (8 * d)) & 0xFF]++;
    }
    uint64_t* src = keys; uint64_t* dst = tmp;
    for (int d = 0; d < 8; ++d) {
        int shift = 8 * d;
        if (((all_or >> shift) & 0xFF) == 0) continue;
        uint64_t s = 0;
        for (int b = 0; b < 256; ++b) { uint64_t c = cnt[d][b]; cnt[d][b] = s; s += c; }
        for (uint64_t i = 0; i < n; ++i) dst[cnt[d][(src[i] >> shift) & 0xFF]++] = src[i];
        uint64_t* t = src; src = dst; dst = t;
    }
    if (src != keys) memcpy(keys, src, sizeof(uint64_t) * n);
    free(cnt);
}

/* Sort canonical keys (u << 32 | v, u < v), drop duplicates, split into
 * endpoint arrays. Returns the number of unique edges. */
static uint64_t unique_edges(uint64_t* keys, uint64_t n, uint32_t* eu, uint32_t* ev) {
    uint64_t* tmp = (uint64_t*)malloc(sizeof(uint64_t) * (n ? n : 1));
    radix_sort_u64(keys, tmp, n);
    free(tmp);
    uint64_t m = 0;
    for (uint64_t i = 0; i < n; ++i) {
        if (i > 0 && keys[i] == keys[i - 1]) continue;
        eu[m] = (uint32_t)(keys[i] >> 32);
        ev[m] = (uint32_t)(keys[i] & 0xFFFFFFFFu);
        ++m;
    }
    return m;
}

/* ------------------------------------------------------------ generators */

/* Erdos-Renyi G(n, m). eu/ev must hold m edges. Returns m, or -1 if m is
 * larger than the number of possible edges. Output is sorted by (u, v). */
int64_t gg_er_edges(uint32_t n, uint64_t m, uint64_t seed, uint32_t* eu, uint32_t* ev) {
    if (n < 2 && m > 0) return -1;
    if (m > (uint64_t)n * (n - 1) / 2) return -1;
    uint64_t cap = 16;
    while (cap < 2 * m + 16) cap <<= 1;
    uint64_t* table = (uint64_t*)calloc(cap, sizeof(uint64_t));   /* 0 = empty, else key + 1 */
    uint64_t* keys = (uint64_t*)malloc(sizeof(uint64_t) * (m ? m : 1));
    uint64_t got = 0;
    for (uint64_t i = 0; got < m; ++i) {
        uint32_t u = (uint32_t)gg_uniform(seed, GG_STREAM_ER, 2 * i, 0, n - 1);
        uint32_t v = (uint32_t)gg_uniform(seed, GG_STREAM_ER, 2 * i + 1, 0, n - 1);
        if (u == v) continue;
        if (u > v) { uint32_t t = u; u = v; v = t; }
        uint64_t key = ((uint64_t)u << 32) | v;
        uint64_t h = gg_splitmix64(key) & (cap - 1);
        int dup = 0;
        while (table[h]) {
            if (table[h] == key + 1) { dup = 1; break; }
            h = (h + 1) & (cap - 1);
        }
        if (dup) continue;
        table[h] = key + 1;
        keys[got++] = key;
    }
    free(table);
    uint64_t mm = unique_edges(keys, m, eu, ev);
    free(keys);
    return (int64_t)mm;
}

/* R x C grid, 4-neighbour. eu/ev must hold R*(C-1) + (R-1)*C edges. */
int64_t gg_grid_edges(uint32_t R, uint32_t C, uint32_t* eu, uint32_t* ev) {
    uint64_t m = 0;
    for (uint32_t r = 0; r < R; ++r)
        for (uint32_t c = 0; c < C; ++c) {
            uint32_t id = r * C + c;
            if (c + 1 < C) { eu[m] = id; ev[m] = id + 1; ++m; }
            if (r + 1 < R) { eu[m] = id; ev[m] = id + C; ++m; }
        }
    return (int64_t)m;   /* already sorted by (u, v) */
}

/* R-MAT with ef * 2^scale draws. eu/ev must hold ef * 2^scale edges.
 * Returns the number of unique undirected non-loop edges. */
int64_t gg_rmat_edges(uint32_t scale, uint32_t ef, double a, double b, double c,
                      uint64_t seed, uint32_t* eu, uint32_t* ev) {
    if (scale < 1 || scale > 30) return -1;
    uint64_t n = 1ull << scale;
    uint64_t draws = (uint64_t)ef * n;
    double ab = a + b, abc = a + b + c;
    /* seeded random permutation of vertex ids (Fisher-Yates, counter-based) */
    uint32_t* perm = (uint32_t*)malloc(sizeof(uint32_t) * n);
    for (uint64_t i = 0; i < n; ++i) perm[i] = (uint32_t)i;
    for (uint64_t i = n - 1; i >= 1; --i) {
        uint64_t j = gg_uniform(seed, GG_STREAM_PERM, i, 0, i);
        uint32_t t = perm[i]; perm[i] = perm[j]; perm[j] = t;
    }
    uint64_t* keys = (uint64_t*)malloc(sizeof(uint64_t) * draws);
    uint64_t kept = 0;
    #pragma omp parallel for schedule(static)
    for (uint64_t i = 0; i < draws; ++i) {
        uint64_t src = 0, dst = 0;
        for (uint32_t l = 0; l < scale; ++l) {
            double p = (double)(gg_rand(seed, GG_STREAM_RMAT, i * scale + l) >> 11) *
                       (1.0 / 9007199254740992.0);
            uint64_t sb, db;
            if (p < a)        { sb = 0; db = 0; }
            else if (p < ab)  { sb = 0; db = 1; }
            else if (p < abc) { sb = 1; db = 0; }
            else              { sb = 1; db = 1; }
            src |= sb << (scale - 1 - l);
            dst |= db << (scale - 1 - l);
        }
        uint32_t u = perm[src], v = perm[dst];
        if (u > v) { uint32_t t = u; u = v; v = t; }
        /* loops are marked with an all-ones key and dropped after sorting */
        keys[i] = (u == v) ? UINT64_MAX : (((uint64_t)u << 32) | v);
    }
    free(perm);
    uint64_t* tmp = (uint64_t*)malloc(sizeof(uint64_t) * draws);
    radix_sort_u64(keys, tmp, draws);
    free(tmp);
    for (uint64_t i = 0; i < draws; ++i) {
        if (keys[i] == UINT64_MAX) break;
        if (i > 0 && keys[i] == keys[i - 1]) continue;
        eu[kept] = (uint32_t)(keys[i] >> 32);
        ev[kept] = (uint32_t)(keys[i] & 0xFFFFFFFFu);
        ++kept;
    }
    free(keys);
    return (int64_t)kept;
}

/* Canonicalise an arbitrary edge list in place: order endpoints, drop loops
 * and duplicates, sort. Returns the new edge count. */
int64_t gg_canonical_edges(uint64_t m, uint32_t* eu, uint32_t* ev) {
    uint64_t* keys = (uint64_t*)malloc(sizeof(uint64_t) * (m ? m : 1));
    uint64_t k = 0;
    for (uint64_t i = 0; i < m; ++i) {
        uint32_t u = eu[i], v = ev[i];
        if (u == v) continue;
        if (u > v) { uint32_t t = u; u = v; v = t; }
        keys[k++] = ((uint64_t)u << 32) | v;
    }
    uint64_t mm = unique_edges(keys, k, eu, ev);
    free(keys);
    return (int64_t)mm;
}

/* --------------------------------------------------------------- packing */

/* Symmetric CSR from canonical edges sorted by (u, v) with u < v.
 * row_ptr holds n + 1 entries, col holds 2m. Because the edge list is sorted
 * by u first, one pass appends every row's smaller neighbours in ascending
 * order before its larger neighbours, so all rows come out sorted. */
int gg_csr(uint32_t n, uint64_t m, const uint32_t* eu, const uint32_t* ev,
           uint32_t* row_ptr, uint32_t* col) {
    if (2 * m > 0xFFFFFFFFull) return -1;
    uint32_t* deg = (uint32_t*)calloc((size_t)n + 1, sizeof(uint32_t));
    for (uint64_t i = 0; i < m; ++i) {
        if (eu[i] >= ev[i] || ev[i] >= n) { free(deg); return -2; }
        deg[eu[i]]++; deg[ev[i]]++;
    }
    uint64_t s = 0;
    for (uint32_t v = 0; v < n; ++v) { row_ptr[v] = (uint32_t)s; s += deg[v]; }
    row_ptr[n] = (uint32_t)s;
    uint32_t* cur = deg;
    for (uint32_t v = 0; v < n; ++v) cur[v] = row_ptr[v];
    for (uint64_t i = 0; i < m; ++i) {
        col[cur[eu[i]]++] = ev[i];
        col[cur[ev[i]]++] = eu[i];
    }
    free(deg);
    return 0;
}

/* Per-arc weights, uniform integer in [lo, hi], keyed by the undirected edge.
 * Requires n <= 2^24 so the key stays below 2^48. */
int gg_weights(uint32_t n, const uint32_t* row_ptr, const uint32_t* col, uint64_t seed,
               uint32_t lo, uint32_t hi, uint32_t* w) {
    if ((uint64_t)n > (1ull << 24) || lo > hi) return -1;
    #pragma omp parallel for schedule(dynamic, 4096)
    for (int64_t v = 0; v < (int64_t)n; ++v) {
        for (uint32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
            uint64_t u = col[e];
            uint64_t a = (uint64_t)v < u ? (uint64_t)v : u;
            uint64_t b = (uint64_t)v < u ? u : (uint64_t)v;
            w[e] = (uint32_t)gg_uniform(seed, GG_STREAM_W, a * n + b, lo, hi);
        }
    }
    return 0;
}

/* Seeded sources: k vertices chosen uniformly among those of degree >= 1
 * (rejection over draw index). Returns the number written (0 if none). */
int64_t gg_sources(uint32_t n, const uint32_t* row_ptr, uint64_t seed, uint32_t k, uint32_t* out) {
    int any = 0;
    for (uint32_t v = 0; v < n && !any; ++v) any = row_ptr[v + 1] > row_ptr[v];
    if (!any) return 0;
    uint64_t i = 0;
    for (uint32_t j = 0; j < k; ++j) {
        for (;; ++i) {
            uint32_t v = (uint32_t)gg_uniform(seed, GG_STREAM_MISC, i, 0, n - 1);
            if (row_ptr[v + 1] > row_ptr[v]) { out[j] = v; ++i; break; }
        }
    }
    return k;
}

/* Seeded points with integer coordinates in [0, 2^21) per axis.
 * kind 0: uniform. kind 1: clustered -- each point picks one of 16 seeded
 * centres and adds, per axis, the sum of three uniform draws in [0, 2^14)
 * minus 3 * 2^13 (a bell-shaped spread of about +-24K), clamped to the
 * cube. Point i uses draws 4i .. 4i+3 of its stream. */
int gg_points(uint32_t n, uint64_t seed, uint32_t kind, uint32_t* x, uint32_t* y, uint32_t* z) {
    const uint64_t side = 1ull << 21;
    if (kind > 1) return -1;
    uint32_t cx[16], cy[16], cz[16];
    for (uint32_t c = 0; c < 16; ++c) {
        cx[c] = (uint32_t)gg_uniform(seed, GG_STREAM_CENTRES, 3 * c, 0, side - 1);
        cy[c] = (uint32_t)gg_uniform(seed, GG_STREAM_CENTRES, 3 * c + 1, 0, side - 1);
        cz[c] = (uint32_t)gg_uniform(seed, GG_STREAM_CENTRES, 3 * c + 2, 0, side - 1);
    }
    for (uint32_t i = 0; i < n; ++i) {
        if (kind == 0) {
            x[i] = (uint32_t)gg_uniform(seed, GG_STREAM_PTS, 4ull * i, 0, side - 1);
            y[i] = (uint32_t)gg_uniform(seed, GG_STREAM_PTS, 4ull * i + 1, 0, side - 1);
            z[i] = (uint32_t)gg_uniform(seed, GG_STREAM_PTS, 4ull * i + 2, 0, side - 1);
        } else {
            const uint32_t c = (uint32_t)gg_uniform(seed, GG_STREAM_PTS, 4ull * i + 3, 0, 15);
            const uint32_t ctr[3] = {cx[c], cy[c], cz[c]};
            uint32_t* out[3] = {x, y, z};
            for (int a = 0; a < 3; ++a) {
                int64_t off = 0;
                /* three disjoint 14-bit fields of one draw */
                const uint64_t r = gg_rand(seed, GG_STREAM_PTS, 4ull * i + a);
                for (int k = 0; k < 3; ++k) off += (int64_t)((r >> (64 - 14 * (k + 1))) & 0x3FFF);
                int64_t v = (int64_t)ctr[a] + off - 3 * 8192;
                if (v < 0) v = 0;
                if (v > (int64_t)side - 1) v = (int64_t)side - 1;
                out[a][i] = (uint32_t)v;
            }
        }
    }
    return 0;
}
