/*
 * All-core CPU baselines for the benchmark's cpu_baseline leg.
 *
 * TEST INFRASTRUCTURE ONLY (like oracle.c): the GPU library never calls
 * this and shares no code with it. It is not the oracle: tests pin it to
 * the oracle (equal output on every graph they try), and the benchmark
 * times it beside the single-threaded oracle so that the GPU figure can be
 * read against every host core, not one.
 *
 *   cpu_bfs_par   level-synchronous BFS with OpenMP: the vertices of level L
 *                 are split over the threads, each thread claims unvisited
 *                 neighbours with a compare-and-swap on their level and
 *                 appends them to a private buffer; the buffers are
 *                 concatenated into level L + 1. The level of every vertex
 *                 is its hop distance, whatever order the claims happen in.
 *   cpu_sssp_par  frontier Bellman-Ford with OpenMP: every round relaxes the
 *                 arcs of the vertices whose distance dropped in the round
 *                 before (atomic minimum on 64-bit distances); it ends after
 *                 a round that lowered nothing. Exact for non-negative weights.
 *
 * Unreached: level 0xFFFFFFFF, distance INT32_MAX. Returns the number of
 * threads used (> 0), or a negative error (-1 bad source, -2 allocation,
 * -6 a distance does not fit in int32).
 */
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define UNREACHED_LEVEL 0xFFFFFFFFu
#define UNREACHED_DIST 0x7FFFFFFF

int cpu_bfs_par(uint32_t n, const uint32_t* row_ptr, const uint32_t* col, uint32_t src, uint32_t* level,
                int threads) {
    if (src >= n) return -1;
    if (threads > 0) omp_set_num_threads(threads);
    uint32_t* cur = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)n);
    uint32_t* next = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)n);
    int nt = omp_get_max_threads();
    uint64_t* counts = (uint64_t*)calloc((size_t)nt + 1, sizeof(uint64_t));
    uint32_t** priv = (uint32_t**)calloc((size_t)nt, sizeof(uint32_t*));
    uint64_t* cap = (uint64_t*)calloc((size_t)nt, sizeof(uint64_t));
    if (!cur || !next || !counts || !priv || !cap) {
        free(cur); free(next); free(counts); free(priv); free(cap);
        return -2;
    }
    int used = 1, fail = 0;
#pragma omp parallel for schedule(static)
    for (uint32_t v = 0; v < n; ++v) level[v] = UNREACHED_LEVEL;
    level[src] = 0;
    cur[0] = src;
    uint64_t ncur = 1;
    uint32_t L = 0;
    while (ncur > 0 && !fail) {
#pragma omp parallel
        {
            const int t = omp_get_thread_num();
#pragma omp single
            used = omp_get_num_threads();
            uint64_t k = 0;
#pragma omp for schedule(dynamic, 256)
            for (uint64_t i = 0; i < ncur; ++i) {
                const uint32_t v = cur[i];
                for (uint32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
                    const uint32_t u = col[e];
                    uint32_t expect = UNREACHED_LEVEL;
                    if (__atomic_load_n(&level[u], __ATOMIC_RELAXED) == UNREACHED_LEVEL &&
                        __atomic_compare_exchange_n(&level[u], &expect, L + 1, 0, __ATOMIC_RELAXED,
                                                    __ATOMIC_RELAXED)) {
                        if (k == cap[t]) {
                            uint64_t nc = cap[t] ? 2 * cap[t] : 1024;
                            uint32_t* p = (uint32_t*)realloc(priv[t], sizeof(uint32_t) * nc);
                            if (!p) { fail = 1; continue; }
                            priv[t] = p;
                            cap[t] = nc;
                        }
                        priv[t][k++] = u;
                    }
                }
            }
            counts[t + 1] = k;
#pragma omp barrier
#pragma omp single
            for (int i = 0; i < used; ++i) counts[i + 1] += counts[i];
            if (k) memcpy(next + counts[t], priv[t], sizeof(uint32_t) * k);
        }
        ncur = counts[used];
        memset(counts, 0, sizeof(uint64_t) * ((size_t)nt + 1));
        uint32_t* tmp = cur; cur = next; next = tmp;
        ++L;
    }
    for (int i = 0; i < nt; ++i) free(priv[i]);
    free(priv); free(cap); free(counts); free(cur); free(next);
    return fail ? -2 : used;
}

int cpu_sssp_par(uint32_t n, const uint32_t* row_ptr, const uint32_t* col, const uint32_t* w, uint32_t src,
                 int32_t* dist, int threads) {
    if (src >= n) return -1;
    if (threads > 0) omp_set_num_threads(threads);
    int64_t* d = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    uint8_t* in_cur = (uint8_t*)calloc((size_t)n, 1);
    uint8_t* in_next = (uint8_t*)calloc((size_t)n, 1);
    if (!d || !in_cur || !in_next) { free(d); free(in_cur); free(in_next); return -2; }
    int used = 1;
#pragma omp parallel for schedule(static)
    for (uint32_t v = 0; v < n; ++v) d[v] = INT64_MAX;
    d[src] = 0;
    in_cur[src] = 1;
    int any = 1;
    while (any) {
        any = 0;
#pragma omp parallel
        {
#pragma omp single
            used = omp_get_num_threads();
#pragma omp for schedule(dynamic, 1024) reduction(| : any)
            for (uint32_t v = 0; v < n; ++v) {
                if (!in_cur[v]) continue;
                in_cur[v] = 0;
                const int64_t dv = __atomic_load_n(&d[v], __ATOMIC_RELAXED);
                for (uint32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
                    const uint32_t u = col[e];
                    const int64_t cand = dv + (int64_t)w[e];
                    int64_t old = __atomic_load_n(&d[u], __ATOMIC_RELAXED);
                    while (cand < old) {
                        if (__atomic_compare_exchange_n(&d[u], &old, cand, 0, __ATOMIC_RELAXED, __ATOMIC_RELAXED)) {
                            __atomic_store_n(&in_next[u], 1, __ATOMIC_RELAXED);
                            any = 1;
                            break;
                        }
                    }
                }
            }
        }
        uint8_t* t = in_cur; in_cur = in_next; in_next = t;
    }
    int rc = used;
    for (uint32_t v = 0; v < n; ++v) {
        if (d[v] == INT64_MAX) dist[v] = UNREACHED_DIST;
        else if (d[v] >= UNREACHED_DIST) { rc = -6; dist[v] = UNREACHED_DIST; }
        else dist[v] = (int32_t)d[v];
    }
    free(d); free(in_cur); free(in_next);
    return rc;
}
