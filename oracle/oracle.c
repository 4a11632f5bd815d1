/*
 * ORACLE -- test infrastructure only. Plain, slow, single-threaded C that
 * computes what the partition-centric scatter/gather path must produce, from
 * textbook definitions. Only tests, the smoke check and the benchmark's CPU
 * baseline may load it; the GPU library never does, and this file shares no
 * code, header or table with it.
 *
 *   oracle_bfs_levels   hop distance from one root along out-edges
 *                       (BFS application section; levels, not parents)
 *   oracle_bfs_parents  parent of each reached vertex in the BFS tree of one
 *                       root (the BFS application's output, Algorithm 5):
 *                       the least-id in-neighbour one level closer to the
 *                       root; the root is its own parent
 *   oracle_cc_minlabel  smallest vertex id of each connected component
 *                       (the fixed point of min-label propagation described
 *                       for connected components in the applications section)
 *   oracle_sssp         integer-weight shortest distances from one root
 *                       (the Bellman-Ford SSSP application reaches the same
 *                       unique values; computed here with Dijkstra)
 *   oracle_pagerank     topological PageRank, a fixed number of iterations,
 *                       dangling mass spread uniformly (PageRank application)
 *   oracle_ppr          personalised PageRank with restart to one seed
 *   oracle_nibble       Parallel Nibble (the Nibble application: a seeded
 *                       lazy random walk whose frontier keeps a vertex while
 *                       its mass is at least eps times its out-degree), in
 *                       FP64, with the distance of every frontier decision
 *                       from its threshold
 *
 * Unreachable vertices get 0xFFFFFFFF. Arithmetic is exact for the integer
 * results and FP64 for the PageRank family.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#define INF32 0xFFFFFFFFu

/* FIFO-queue breadth-first search. Returns 0, or -1 on allocation failure. */
int oracle_bfs_levels(uint32_t n, const uint32_t* off, const uint32_t* cols,
                      uint32_t root, uint32_t* level) {
    for (uint32_t v = 0; v < n; ++v) level[v] = INF32;
    if (root >= n) return -1;
    uint32_t* queue = (uint32_t*)malloc((size_t)(n ? n : 1) * sizeof(uint32_t));
    if (!queue) return -1;
    size_t head = 0, tail = 0;
    level[root] = 0;
    queue[tail++] = root;
    while (head < tail) {
        uint32_t u = queue[head++];
        for (uint32_t e = off[u]; e < off[u + 1]; ++e) {
            uint32_t v = cols[e];
            if (level[v] == INF32) {
                level[v] = level[u] + 1;
                queue[tail++] = v;
            }
        }
    }
    free(queue);
    return 0;
}

/* Levels by the FIFO search above, then every edge u -> v with
 * level[u] + 1 == level[v] offers u as the parent of v, and the least offer
 * stays. */
int oracle_bfs_parents(uint32_t n, const uint32_t* off, const uint32_t* cols,
                       uint32_t root, uint32_t* parent) {
    uint32_t* level = (uint32_t*)malloc((size_t)(n ? n : 1) * sizeof(uint32_t));
    if (!level) return -1;
    if (oracle_bfs_levels(n, off, cols, root, level) != 0) {
        free(level);
        return -1;
    }
    for (uint32_t v = 0; v < n; ++v) parent[v] = INF32;
    parent[root] = root;
    for (uint32_t u = 0; u < n; ++u) {
        if (level[u] == INF32) continue;
        for (uint32_t e = off[u]; e < off[u + 1]; ++e) {
            uint32_t v = cols[e];
            if (v != root && level[v] == level[u] + 1 && u < parent[v]) parent[v] = u;
        }
    }
    free(level);
    return 0;
}

static uint32_t uf_find(uint32_t* parent, uint32_t x) {
    uint32_t r = x;
    while (parent[r] != r) r = parent[r];
    while (parent[x] != r) { uint32_t nx = parent[x]; parent[x] = r; x = nx; }
    return r;
}

/* Union-find over every edge (taken as undirected), then the smallest vertex
 * id of each set. On a symmetric graph this is the unique fixed point of
 * min-label propagation. */
int oracle_cc_minlabel(uint32_t n, const uint32_t* off, const uint32_t* cols, uint32_t* label) {
    uint32_t* parent = (uint32_t*)malloc((size_t)(n ? n : 1) * sizeof(uint32_t));
    if (!parent) return -1;
    for (uint32_t v = 0; v < n; ++v) parent[v] = v;
    for (uint32_t u = 0; u < n; ++u)
        for (uint32_t e = off[u]; e < off[u + 1]; ++e) {
            uint32_t a = uf_find(parent, u), b = uf_find(parent, cols[e]);
            if (a != b) parent[a > b ? a : b] = a < b ? a : b;
        }
    for (uint32_t v = 0; v < n; ++v) label[v] = INF32;
    for (uint32_t v = 0; v < n; ++v) {
        uint32_t r = uf_find(parent, v);
        if (v < label[r]) label[r] = v;
    }
    for (uint32_t v = 0; v < n; ++v) label[v] = label[uf_find(parent, v)];
    free(parent);
    return 0;
}

/* Binary min-heap of (distance, vertex) with lazy deletion. */
typedef struct { uint64_t d; uint32_t v; } hent;

static void heap_push(hent* h, size_t* sz, hent x) {
    size_t i = (*sz)++;
    h[i] = x;
    while (i > 0) {
        size_t p = (i - 1) / 2;
        if (h[p].d <= h[i].d) break;
        hent t = h[p]; h[p] = h[i]; h[i] = t;
        i = p;
    }
}

static hent heap_pop(hent* h, size_t* sz) {
    hent top = h[0];
    h[0] = h[--(*sz)];
    size_t i = 0;
    for (;;) {
        size_t l = 2 * i + 1, r = l + 1, m = i;
        if (l < *sz && h[l].d < h[m].d) m = l;
        if (r < *sz && h[r].d < h[m].d) m = r;
        if (m == i) break;
        hent t = h[m]; h[m] = h[i]; h[i] = t;
        i = m;
    }
    return top;
}

/* Dijkstra with uint64 tentative distances; weights NULL means unit weights.
 * Returns 0, -1 on allocation failure, -2 if a distance reaches 2^32 - 1. */
int oracle_sssp(uint32_t n, const uint32_t* off, const uint32_t* cols, const uint8_t* w,
                uint32_t root, uint32_t* dist) {
    for (uint32_t v = 0; v < n; ++v) dist[v] = INF32;
    if (root >= n) return -1;
    uint64_t* d = (uint64_t*)malloc((size_t)(n ? n : 1) * sizeof(uint64_t));
    size_t cap = (size_t)off[n] + 1;
    hent* h = (hent*)malloc(cap * sizeof(hent));
    if (!d || !h) { free(d); free(h); return -1; }
    for (uint32_t v = 0; v < n; ++v) d[v] = UINT64_MAX;
    size_t sz = 0;
    d[root] = 0;
    heap_push(h, &sz, (hent){0, root});
    while (sz) {
        hent t = heap_pop(h, &sz);
        if (t.d != d[t.v]) continue;
        for (uint32_t e = off[t.v]; e < off[t.v + 1]; ++e) {
            uint64_t nd = t.d + (w ? w[e] : 1u);
            uint32_t v = cols[e];
            if (nd < d[v]) { d[v] = nd; heap_push(h, &sz, (hent){nd, v}); }
        }
    }
    int rc = 0;
    for (uint32_t v = 0; v < n; ++v) {
        if (d[v] == UINT64_MAX) continue;
        if (d[v] >= INF32) rc = -2;
        dist[v] = (uint32_t)d[v];
    }
    free(d); free(h);
    return rc;
}

/* x0 = 1/n; for t = 1..iters:
 *   D = sum of x[u] over vertices with out-degree 0
 *   y[v] = sum over edges (u -> v), duplicates counted, of x[u] / outdeg(u)
 *   x[v] = (1 - damping) / n + damping * (y[v] + D / n)            */
int oracle_pagerank(uint32_t n, const uint32_t* off, const uint32_t* cols,
                    double damping, uint32_t iters, double* x) {
    double* y = (double*)malloc((size_t)(n ? n : 1) * sizeof(double));
    if (!y) return -1;
    for (uint32_t v = 0; v < n; ++v) x[v] = 1.0 / n;
    for (uint32_t t = 0; t < iters; ++t) {
        double dang = 0.0;
        for (uint32_t v = 0; v < n; ++v) y[v] = 0.0;
        for (uint32_t u = 0; u < n; ++u) {
            uint32_t deg = off[u + 1] - off[u];
            if (deg == 0) { dang += x[u]; continue; }
            double share = x[u] / deg;
            for (uint32_t e = off[u]; e < off[u + 1]; ++e) y[cols[e]] += share;
        }
        for (uint32_t v = 0; v < n; ++v)
            x[v] = (1.0 - damping) / n + damping * (y[v] + dang / n);
    }
    free(y);
    return 0;
}

/* Personalised PageRank with restart probability alpha to `seed`:
 * x0 = e_seed; for t = 1..iters:
 *   D = sum of x[u] over vertices with out-degree 0 (returned to the seed)
 *   y[v] = sum over edges (u -> v) of x[u] / outdeg(u)
 *   x[v] = alpha [v == seed] + (1 - alpha) (y[v] + D [v == seed])       */
int oracle_ppr(uint32_t n, const uint32_t* off, const uint32_t* cols, double alpha,
               uint32_t iters, uint32_t seed, double* x) {
    if (seed >= n) return -1;
    double* y = (double*)malloc((size_t)n * sizeof(double));
    if (!y) return -1;
    for (uint32_t v = 0; v < n; ++v) x[v] = 0.0;
    x[seed] = 1.0;
    for (uint32_t t = 0; t < iters; ++t) {
        double dang = 0.0;
        for (uint32_t v = 0; v < n; ++v) y[v] = 0.0;
        for (uint32_t u = 0; u < n; ++u) {
            if (x[u] == 0.0) continue;
            uint32_t deg = off[u + 1] - off[u];
            if (deg == 0) { dang += x[u]; continue; }
            double share = x[u] / deg;
            for (uint32_t e = off[u]; e < off[u + 1]; ++e) y[cols[e]] += share;
        }
        for (uint32_t v = 0; v < n; ++v)
            x[v] = (1.0 - alpha) * y[v];
        x[seed] += alpha + (1.0 - alpha) * dang;
    }
    free(y);
    return 0;
}

/* Parallel Nibble (the Nibble application with the iteration of Algorithm 2),
 * FP64. PR = e_seed, frontier A = {seed}. While A is not empty and fewer
 * than max_iter iterations have run:
 *   scatter   every v in A with deg(v) > 0 sends PR[v] / (2 deg(v)) along
 *             each out-edge (duplicate edges send twice); the values are
 *             taken before initFunc changes PR;
 *   initFunc  every v in A: PR[v] = PR[v] / 2, and v stays active iff
 *             PR[v] >= eps deg(v);
 *   gather    every edge message adds its value to PR of its destination,
 *             which becomes active;
 *   filter    every active vertex stays iff PR[v] >= eps deg(v).
 * A vertex without out-edges never stays active (its threshold eps * 0
 * would keep it forever while it has nothing to send); an active seed
 * without out-edges still loses the half initFunc takes.
 *
 * Outputs: PR (n doubles), the frontier size after each iteration
 * (fsize[0 .. *iters)), the iterations run, the least relative distance
 * |PR - eps deg| / (eps deg) over the decisive threshold tests (the filter
 * test of each active vertex after gather, and the initFunc test of a vertex
 * that then receives nothing), and how many of those tests lie closer than
 * `delta` to their threshold. Returns 0, or -1 on a bad seed or allocation
 * failure. */
int oracle_nibble(uint32_t n, const uint32_t* off, const uint32_t* cols, uint32_t seed, double eps,
                  uint32_t max_iter, double delta, double* pr, uint64_t* fsize, uint32_t* iters,
                  double* min_margin, uint64_t* near) {
    *iters = 0;
    *min_margin = 1.0 / 0.0;
    *near = 0;
    if (seed >= n) return -1;
    double* inbox = (double*)calloc(n, sizeof(double));
    uint8_t* got = (uint8_t*)calloc(n, 1);    /* received a message this iteration */
    uint8_t* inA = (uint8_t*)calloc(n, 1);    /* in the next frontier            */
    uint32_t* A = (uint32_t*)malloc((size_t)n * sizeof(uint32_t));
    uint32_t* R = (uint32_t*)malloc((size_t)n * sizeof(uint32_t));
    uint32_t* B = (uint32_t*)malloc((size_t)n * sizeof(uint32_t));
    if (!inbox || !got || !inA || !A || !R || !B) {
        free(inbox); free(got); free(inA); free(A); free(R); free(B);
        return -1;
    }
    for (uint32_t v = 0; v < n; ++v) pr[v] = 0.0;
    pr[seed] = 1.0;
    size_t na = 1;
    A[0] = seed;
#define NIBBLE_TEST(x, d, keep)                                        \
    do {                                                               \
        keep = 0;                                                      \
        if ((d) > 0) {                                                 \
            const double th = eps * (double)(d);                       \
            const double m = fabs((x) - th) / th;                      \
            if (m < *min_margin) *min_margin = m;                      \
            if (m < delta) ++*near;                                    \
            keep = (x) >= th;                                          \
        }                                                              \
    } while (0)
    uint32_t t = 0;
    for (; t < max_iter && na > 0; ++t) {
        size_t nr = 0, nb = 0;
        /* scatter, with the values before initFunc */
        for (size_t i = 0; i < na; ++i) {
            const uint32_t v = A[i], d = off[v + 1] - off[v];
            if (d == 0) continue;
            const double share = pr[v] / (2.0 * (double)d);
            for (uint32_t e = off[v]; e < off[v + 1]; ++e) {
                const uint32_t u = cols[e];
                inbox[u] += share;
                if (!got[u]) { got[u] = 1; R[nr++] = u; }
            }
        }
        /* initFunc: halve; a vertex that fails and receives nothing leaves
         * the frontier here (its test is decisive) */
        for (size_t i = 0; i < na; ++i) {
            const uint32_t v = A[i], d = off[v + 1] - off[v];
            pr[v] *= 0.5;
            if (got[v]) continue;  /* the filter decides after gather */
            int keep;
            NIBBLE_TEST(pr[v], d, keep);
            if (keep && !inA[v]) { inA[v] = 1; B[nb++] = v; }
        }
        /* gather, then filter on the received vertices */
        for (size_t i = 0; i < nr; ++i) {
            const uint32_t u = R[i], d = off[u + 1] - off[u];
            pr[u] += inbox[u];
            inbox[u] = 0.0;
            got[u] = 0;
            int keep;
            NIBBLE_TEST(pr[u], d, keep);
            if (keep && !inA[u]) { inA[u] = 1; B[nb++] = u; }
        }
        for (size_t i = 0; i < nb; ++i) inA[B[i]] = 0;
        fsize[t] = nb;
        uint32_t* tmp = A; A = B; B = tmp;
        na = nb;
    }
#undef NIBBLE_TEST
    *iters = t;
    free(inbox); free(got); free(inA); free(A); free(R); free(B);
    return 0;
}
