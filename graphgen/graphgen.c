/*
 * Seeded synthetic graph inputs: RMAT and Erdos-Renyi edge lists, CSR
 * construction, symmetrisation, edge weights and source selection.
 *
 * This module is shared by the CPU oracle and the GPU path. It holds input
 * preparation only and none of the partition-centric method's arithmetic.
 *
 * Random numbers come from a counter-based use of SplitMix64 (Steele, Lea,
 * Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014): the
 * value for counter c under seed s is mix(s + (c + 1) * 0x9E3779B97F4A7C15),
 * where mix is the SplitMix64 finaliser. Every draw is therefore a pure
 * function of (seed, counter), which makes generation order-free and lets any
 * thread produce any edge.
 *
 * RMAT (Chakrabarti, Zhan, Faloutsos, SDM 2004), the "default settings" the
 * evaluation section uses for its rmat graphs: edge i picks one of four
 * adjacency-matrix quadrants per level, most significant bit first, with
 * probabilities a, b, c, d = 1 - a - b - c; quadrant b sets the destination
 * bit, c the source bit, d both. Level l of edge i uses counter i * 64 + l.
 * No noise, no vertex permutation; duplicates and self-loops are kept.
 *
 * Erdos-Renyi G(n, m): edge i draws source and destination uniformly with
 * replacement from counters 2i and 2i + 1 (multiply-high range reduction).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define GOLDEN 0x9E3779B97F4A7C15ULL

static inline uint64_t sm64_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

uint64_t gg_draw(uint64_t seed, uint64_t counter) {
    return sm64_mix(seed + (counter + 1ULL) * GOLDEN);
}

static inline uint64_t mulhi64(uint64_t a, uint64_t b) {
    return (uint64_t)(((unsigned __int128)a * b) >> 64);
}

/* Quadrant thresholds are compared on the top 53 bits of each draw, i.e. on
 * u = (z >> 11) * 2^-53 against a, a + b, a + b + c in double precision. */
void gg_rmat_edges(int scale, uint64_t m, double a, double b, double c,
                   uint64_t seed, uint32_t* src, uint32_t* dst) {
    const double two53 = 9007199254740992.0;
    const uint64_t ta = (uint64_t)(a * two53);
    const uint64_t tb = (uint64_t)((a + b) * two53);
    const uint64_t tc = (uint64_t)((a + b + c) * two53);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < (int64_t)m; ++i) {
        uint32_t s = 0, d = 0;
        for (int l = 0; l < scale; ++l) {
            uint64_t u = gg_draw(seed, (uint64_t)i * 64ULL + (uint64_t)l) >> 11;
            uint32_t sb, db;
            if (u < ta) { sb = 0; db = 0; }
            else if (u < tb) { sb = 0; db = 1; }
            else if (u < tc) { sb = 1; db = 0; }
            else { sb = 1; db = 1; }
            s = (s << 1) | sb;
            d = (d << 1) | db;
        }
        src[i] = s;
        dst[i] = d;
    }
}

void gg_er_edges(uint64_t n, uint64_t m, uint64_t seed, uint32_t* src, uint32_t* dst) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < (int64_t)m; ++i) {
        src[i] = (uint32_t)mulhi64(gg_draw(seed, 2ULL * (uint64_t)i), n);
        dst[i] = (uint32_t)mulhi64(gg_draw(seed, 2ULL * (uint64_t)i + 1ULL), n);
    }
}

/* Appends the reverse of every edge: out has 2m entries, (s_i, d_i) at i and
 * (d_i, s_i) at m + i. A self-loop therefore appears twice. */
void gg_symmetrize(uint64_t m, const uint32_t* src, const uint32_t* dst,
                   uint32_t* out_src, uint32_t* out_dst) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < (int64_t)m; ++i) {
        out_src[i] = src[i];
        out_dst[i] = dst[i];
        out_src[m + i] = dst[i];
        out_dst[m + i] = src[i];
    }
}

static int cmp_u32(const void* x, const void* y) {
    uint32_t a = *(const uint32_t*)x, b = *(const uint32_t*)y;
    return (a > b) - (a < b);
}

/* LSD radix sort of one row, three 11-bit passes, for long rows. */
static void sort_row(uint32_t* v, uint64_t n, uint32_t* tmp) {
    if (n < 256) { qsort(v, n, sizeof(uint32_t), cmp_u32); return; }
    uint64_t cnt[2049];
    for (int pass = 0; pass < 3; ++pass) {
        int shift = pass * 11;
        memset(cnt, 0, sizeof(cnt));
        for (uint64_t i = 0; i < n; ++i) cnt[((v[i] >> shift) & 0x7FF) + 1]++;
        for (int j = 0; j < 2048; ++j) cnt[j + 1] += cnt[j];
        for (uint64_t i = 0; i < n; ++i) tmp[cnt[(v[i] >> shift) & 0x7FF]++] = v[i];
        memcpy(v, tmp, n * sizeof(uint32_t));
    }
}

/* CSR with rows sorted ascending; duplicates and self-loops kept.
 * offsets has n + 1 entries, cols has m entries. Returns 0, or -1 if an
 * endpoint is out of range or m does not fit the 32-bit offsets. */
int gg_build_csr(uint64_t n, uint64_t m, const uint32_t* src, const uint32_t* dst,
                 uint32_t* offsets, uint32_t* cols) {
    if (m > 0xFFFFFFFFULL) return -1;
    uint64_t* cnt = (uint64_t*)calloc(n + 1, sizeof(uint64_t));
    if (!cnt) return -1;
    for (uint64_t i = 0; i < m; ++i) {
        if (src[i] >= n || dst[i] >= n) { free(cnt); return -1; }
        cnt[src[i] + 1]++;
    }
    for (uint64_t v = 0; v < n; ++v) cnt[v + 1] += cnt[v];
    for (uint64_t v = 0; v <= n; ++v) offsets[v] = (uint32_t)cnt[v];
    for (uint64_t i = 0; i < m; ++i) cols[cnt[src[i]]++] = dst[i];
    free(cnt);
    uint64_t maxrow = 0;
    for (uint64_t v = 0; v < n; ++v) {
        uint64_t len = (uint64_t)offsets[v + 1] - offsets[v];
        if (len > maxrow) maxrow = len;
    }
#pragma omp parallel
    {
        uint32_t* tmp = (uint32_t*)malloc((maxrow ? maxrow : 1) * sizeof(uint32_t));
#pragma omp for schedule(dynamic, 1024)
        for (int64_t v = 0; v < (int64_t)n; ++v)
            sort_row(cols + offsets[v], (uint64_t)offsets[v + 1] - offsets[v], tmp);
        free(tmp);
    }
    return 0;
}

/* Integer weight of CSR entry e: 1 + floor(draw(seed, e) * span / 2^64),
 * uniform on [1, span]. */
void gg_weights(uint64_t m, uint64_t seed, uint32_t span, uint8_t* w) {
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < (int64_t)m; ++e)
        w[e] = (uint8_t)(1 + mulhi64(gg_draw(seed, (uint64_t)e), span));
}

/* Sources: the vertex of highest out-degree (lowest id on ties), then
 * distinct vertices of out-degree > 0 drawn uniformly with counters
 * 0, 1, 2, ... under seed. Writes min(count, #non-isolated) sources and
 * returns how many were written. */
uint32_t gg_sources(uint64_t n, const uint32_t* offsets, uint64_t seed,
                    uint32_t count, uint32_t* out) {
    if (count == 0 || n == 0) return 0;
    uint64_t nonzero = 0, best = 0, bestdeg = 0;
    for (uint64_t v = 0; v < n; ++v) {
        uint64_t d = (uint64_t)offsets[v + 1] - offsets[v];
        if (d > 0) nonzero++;
        if (d > bestdeg) { bestdeg = d; best = v; }
    }
    if (nonzero == 0) return 0;
    uint32_t got = 0;
    out[got++] = (uint32_t)best;
    if (count > nonzero) count = (uint32_t)nonzero;
    for (uint64_t ctr = 0; got < count; ++ctr) {
        uint32_t v = (uint32_t)mulhi64(gg_draw(seed, ctr), n);
        if (offsets[v + 1] == offsets[v]) continue;
        int dup = 0;
        for (uint32_t j = 0; j < got; ++j) dup |= (out[j] == v);
        if (!dup) out[got++] = v;
    }
    return got;
}
