/*
 * CPU oracle for the cooperative graph-traversal path.
 *
 * TEST INFRASTRUCTURE ONLY. Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this library. The GPU library never
 * calls it and shares no code with it.
 *
 * Each function is the plain definition of what the paper's level-by-level
 * graph kernels compute (the traversal loop of the graph-traversal figures in
 * the paper's motivating-examples and programming sections, with the work per
 * node left unspecified there). All results are integers and unique, so the
 * GPU must match them bit for bit whatever kill/fork schedule it ran under
 * (an offer_kill that is ignored and a fork of zero workgroups are always
 * legal, so the never-resizing execution is one of the allowed executions).
 *
 *   oracle_bfs    BFS level of every vertex from one source (textbook FIFO
 *                 queue BFS). Unreached vertices get 0xFFFFFFFF.
 *   oracle_sssp   single-source shortest-path distance (binary-heap Dijkstra
 *                 with 64-bit accumulation). Unreached get INT32_MAX; a
 *                 distance that does not fit in int32 is an error.
 *   oracle_color  greedy colouring in priority order: vertices are taken in
 *                 decreasing key and each gets the smallest colour not used
 *                 by an already coloured (higher-key) neighbour.
 *   oracle_mis    greedy maximal independent set in the same priority order:
 *                 a vertex joins unless a higher-key neighbour already joined.
 *   oracle_cc     connected components, each vertex labelled with the
 *                 smallest vertex id of its component (a FIFO BFS started
 *                 from every still unlabelled vertex in increasing id order;
 *                 the start is then the smallest id the BFS reaches). This is
 *                 the fixed point a label-propagation kernel reaches with
 *                 minimum labels in any schedule, so it is unique.
 *
 * Priority keys: key(v) = (h(v), v) compared lexicographically, higher first,
 * where h(v) is output number v (0-based) of a SplitMix64 generator whose
 * state starts at prio_seed (Steele, Lea and Flood, OOPSLA 2014): the state
 * after v+1 increments by the golden gamma G = 0x9E3779B97F4A7C15 is mixed by
 * z = (z ^ z>>30) * 0xBF58476D1CE4E5B9, z = (z ^ z>>27) * 0x94D049BB133111EB,
 * z ^ z>>31. Including v makes ties impossible.
 *
 * Graphs are CSR: row_ptr[n+1], col[arcs], optional w[arcs], undirected
 * (both arcs present).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_UNREACHED_LEVEL 0xFFFFFFFFu
#define ORACLE_UNREACHED_DIST  0x7FFFFFFF

uint64_t oracle_splitmix64(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* ------------------------------------------------------------------ BFS */

int oracle_bfs(uint32_t n, const uint32_t* row_ptr, const uint32_t* col, uint32_t src,
               uint32_t* level) {
    if (src >= n) return -1;
    for (uint32_t v = 0; v < n; ++v) level[v] = ORACLE_UNREACHED_LEVEL;
    uint32_t* queue = (uint32_t*)malloc(sizeof(uint32_t) * n);
    if (!queue) return -2;
    uint32_t head = 0, tail = 0;
    level[src] = 0;
    queue[tail++] = src;
    while (head < tail) {
        uint32_t v = queue[head++];
        for (uint32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
            uint32_t u = col[e];
            if (level[u] == ORACLE_UNREACHED_LEVEL) {
                level[u] = level[v] + 1;
                queue[tail++] = u;
            }
        }
    }
    free(queue);
    return 0;
}

/* ----------------------------------------------------------------- SSSP */

typedef struct { int64_t d; uint32_t v; } heap_item;

static void heap_push(heap_item* h, uint64_t* size, heap_item it) {
    uint64_t i = (*size)++;
    h[i] = it;
    while (i > 0) {
        uint64_t p = (i - 1) / 2;
        if (h[p].d <= h[i].d) break;
        heap_item t = h[p]; h[p] = h[i]; h[i] = t;
        i = p;
    }
}

static heap_item heap_pop(heap_item* h, uint64_t* size) {
    heap_item top = h[0];
    h[0] = h[--(*size)];
    uint64_t i = 0;
    for (;;) {
        uint64_t l = 2 * i + 1, r = l + 1, m = i;
        if (l < *size && h[l].d < h[m].d) m = l;
        if (r < *size && h[r].d < h[m].d) m = r;
        if (m == i) break;
        heap_item t = h[m]; h[m] = h[i]; h[i] = t;
        i = m;
    }
    return top;
}

/* Returns 0, -1 on a bad source, -2 on allocation failure, -6 if some
 * distance exceeds INT32_MAX - 1 (the sentinel is reserved). */
int oracle_sssp(uint32_t n, const uint32_t* row_ptr, const uint32_t* col, const uint32_t* w,
                uint32_t src, int32_t* dist) {
    if (src >= n) return -1;
    int64_t* d = (int64_t*)malloc(sizeof(int64_t) * n);
    uint64_t arcs = row_ptr[n];
    heap_item* heap = (heap_item*)malloc(sizeof(heap_item) * (arcs + 1));
    if (!d || !heap) { free(d); free(heap); return -2; }
    for (uint32_t v = 0; v < n; ++v) d[v] = INT64_MAX;
    uint64_t hs = 0;
    d[src] = 0;
    heap_item s0 = {0, src};
    heap_push(heap, &hs, s0);
    while (hs > 0) {
        heap_item it = heap_pop(heap, &hs);
        if (it.d != d[it.v]) continue;           /* stale entry */
        for (uint32_t e = row_ptr[it.v]; e < row_ptr[it.v + 1]; ++e) {
            uint32_t u = col[e];
            int64_t nd = it.d + (int64_t)w[e];
            if (nd < d[u]) {
                d[u] = nd;
                heap_item ni = {nd, u};
                heap_push(heap, &hs, ni);
            }
        }
    }
    int rc = 0;
    for (uint32_t v = 0; v < n; ++v) {
        if (d[v] == INT64_MAX) dist[v] = ORACLE_UNREACHED_DIST;
        else if (d[v] >= ORACLE_UNREACHED_DIST) { dist[v] = ORACLE_UNREACHED_DIST; rc = -6; }
        else dist[v] = (int32_t)d[v];
    }
    free(d);
    free(heap);
    return rc;
}

/* ------------------------------------------------------ priority order */

typedef struct { uint64_t h; uint32_t v; } key_item;

static int key_desc(const void* a, const void* b) {
    const key_item* x = (const key_item*)a;
    const key_item* y = (const key_item*)b;
    if (x->h != y->h) return x->h > y->h ? -1 : 1;
    if (x->v != y->v) return x->v > y->v ? -1 : 1;
    return 0;
}

/* Vertices sorted by decreasing key (h(v), v). */
static uint32_t* priority_order(uint32_t n, uint64_t prio_seed) {
    key_item* k = (key_item*)malloc(sizeof(key_item) * (n ? n : 1));
    uint32_t* order = (uint32_t*)malloc(sizeof(uint32_t) * (n ? n : 1));
    if (!k || !order) { free(k); free(order); return NULL; }
    for (uint32_t v = 0; v < n; ++v) {
        k[v].h = oracle_splitmix64(prio_seed + (uint64_t)v * 0x9E3779B97F4A7C15ull);
        k[v].v = v;
    }
    qsort(k, n, sizeof(key_item), key_desc);
    for (uint32_t i = 0; i < n; ++i) order[i] = k[i].v;
    free(k);
    return order;
}

int oracle_priority_order(uint32_t n, uint64_t prio_seed, uint32_t* order_out) {
    uint32_t* order = priority_order(n, prio_seed);
    if (!order) return -2;
    memcpy(order_out, order, sizeof(uint32_t) * n);
    free(order);
    return 0;
}

/* ------------------------------------------------------------ colouring */

int oracle_color(uint32_t n, const uint32_t* row_ptr, const uint32_t* col, uint64_t prio_seed,
                 uint32_t* colour) {
    uint32_t* order = priority_order(n, prio_seed);
    if (!order) return -2;
    uint32_t maxdeg = 0;
    for (uint32_t v = 0; v < n; ++v)
        if (row_ptr[v + 1] - row_ptr[v] > maxdeg) maxdeg = row_ptr[v + 1] - row_ptr[v];
    /* used[c] == stamp marks colour c as taken for the current vertex */
    uint32_t* used = (uint32_t*)calloc((size_t)maxdeg + 2, sizeof(uint32_t));
    uint8_t* done = (uint8_t*)calloc(n ? n : 1, 1);
    if (!used || !done) { free(order); free(used); free(done); return -2; }
    for (uint32_t i = 0; i < n; ++i) {
        uint32_t v = order[i];
        uint32_t stamp = i + 1;
        for (uint32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
            uint32_t u = col[e];
            /* a neighbour already processed has a higher key */
            if (done[u] && colour[u] <= maxdeg + 1) used[colour[u]] = stamp;
        }
        uint32_t c = 0;
        while (used[c] == stamp) ++c;
        colour[v] = c;
        done[v] = 1;
    }
    free(order); free(used); free(done);
    return 0;
}

/* ------------------------------------------------------------------ MIS */

int oracle_mis(uint32_t n, const uint32_t* row_ptr, const uint32_t* col, uint64_t prio_seed,
               uint8_t* in_set) {
    uint32_t* order = priority_order(n, prio_seed);
    if (!order) return -2;
    for (uint32_t v = 0; v < n; ++v) in_set[v] = 0;
    for (uint32_t i = 0; i < n; ++i) {
        uint32_t v = order[i];
        int blocked = 0;
        for (uint32_t e = row_ptr[v]; e < row_ptr[v + 1] && !blocked; ++e)
            blocked = in_set[col[e]];   /* only processed (higher-key) vertices can be in */
        in_set[v] = blocked ? 0 : 1;
    }
    free(order);
    return 0;
}

/* ------------------------------------------------------------- octree */

/* Octree of points with integer coordinates in [0, 2^21) (the work-stealing
 * workload; the paper names the octree build without giving its rules, so
 * these are the readings used): a node at depth d is a cube of side
 * 2^(21 - d); its points go to the 8 child cubes by bit (20 - d) of x, y
 * and z (child = 4 bx + 2 by + bz), keeping their order (a stable split).
 * A node with at most `cap` points, or at depth 21, is a leaf. The code of
 * a node is its path of child indices, 3 bits per level.
 *
 * Output: `out` (4n words) = the points in final order as {x, y, z, index};
 * `leaves` (5 words each, at most max_leaves) = {first, end, depth,
 * code_lo, code_hi} in order of `first`. Returns 0, -1 (too many leaves)
 * or -2 (out of memory). Depth-first with an explicit stack, children in
 * index order, so the leaves come out ordered. */
int oracle_octree(uint32_t n, const uint32_t* x, const uint32_t* y, const uint32_t* z, uint32_t cap,
                  uint32_t* out, uint32_t* leaves, uint64_t max_leaves, uint64_t* nleaves) {
    typedef struct { uint32_t first, end, depth; uint64_t code; } node;
    uint32_t* tmp = (uint32_t*)malloc(sizeof(uint32_t) * 4 * (size_t)(n ? n : 1));
    node* stack = (node*)malloc(sizeof(node) * (7 * 22 + 8));
    if (!tmp || !stack) { free(tmp); free(stack); return -2; }
    for (uint32_t i = 0; i < n; ++i) {
        out[4 * i] = x[i];
        out[4 * i + 1] = y[i];
        out[4 * i + 2] = z[i];
        out[4 * i + 3] = i;
    }
    uint64_t nl = 0;
    int sp = 0;
    stack[sp++] = (node){0, n, 0, 0};
    while (sp > 0) {
        node nd = stack[--sp];
        const uint32_t count = nd.end - nd.first;
        if (count <= cap || nd.depth == 21) {
            if (count == 0) continue;
            if (nl >= max_leaves) { free(tmp); free(stack); return -1; }
            uint32_t* L = leaves + 5 * nl++;
            L[0] = nd.first; L[1] = nd.end; L[2] = nd.depth;
            L[3] = (uint32_t)nd.code; L[4] = (uint32_t)(nd.code >> 32);
            continue;
        }
        /* stable split by the child index at this depth */
        const uint32_t bit = 20 - nd.depth;
        uint32_t cnt[8] = {0}, start[8];
        for (uint32_t i = nd.first; i < nd.end; ++i) {
            const uint32_t* p = out + 4 * (size_t)i;
            const uint32_t c = (((p[0] >> bit) & 1u) << 2) | (((p[1] >> bit) & 1u) << 1) | ((p[2] >> bit) & 1u);
            ++cnt[c];
        }
        uint32_t acc = nd.first;
        for (int c = 0; c < 8; ++c) { start[c] = acc; acc += cnt[c]; }
        uint32_t pos[8];
        for (int c = 0; c < 8; ++c) pos[c] = start[c];
        for (uint32_t i = nd.first; i < nd.end; ++i) {
            const uint32_t* p = out + 4 * (size_t)i;
            const uint32_t c = (((p[0] >> bit) & 1u) << 2) | (((p[1] >> bit) & 1u) << 1) | ((p[2] >> bit) & 1u);
            memcpy(tmp + 4 * (size_t)pos[c]++, p, 16);
        }
        memcpy(out + 4 * (size_t)nd.first, tmp + 4 * (size_t)nd.first, 16 * (size_t)count);
        /* children pushed last-first so child 0 is handled next */
        for (int c = 7; c >= 0; --c)
            if (cnt[c]) stack[sp++] = (node){start[c], start[c] + cnt[c], nd.depth + 1, (nd.code << 3) | (uint64_t)c};
    }
    *nleaves = nl;
    free(tmp);
    free(stack);
    return 0;
}

/* ------------------------------------------------- connected components */

int oracle_cc(uint32_t n, const uint32_t* row_ptr, const uint32_t* col, uint32_t* label) {
    uint32_t* queue = (uint32_t*)malloc(sizeof(uint32_t) * (n ? n : 1));
    if (!queue) return -2;
    for (uint32_t v = 0; v < n; ++v) label[v] = ORACLE_UNREACHED_LEVEL;
    for (uint32_t s = 0; s < n; ++s) {
        if (label[s] != ORACLE_UNREACHED_LEVEL) continue;
        uint32_t head = 0, tail = 0;
        label[s] = s;
        queue[tail++] = s;
        while (head < tail) {
            uint32_t v = queue[head++];
            for (uint32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
                uint32_t u = col[e];
                if (label[u] == ORACLE_UNREACHED_LEVEL) {
                    label[u] = s;
                    queue[tail++] = u;
                }
            }
        }
    }
    free(queue);
    return 0;
}
