/*
 * Seeded synthetic graph inputs: directed R-MAT edge sampling, a seeded vertex
 * permutation, and conversion of an edge list to a deduplicated in-edge CSR
 * (CSC: row v lists the sources u of edges u->v in ascending order).
 *
 * This module holds no arithmetic of the graph method itself. It is the only
 * code shared by the plain CPU checker and the GPU path: both consume the
 * arrays it produces.
 *
 * R-MAT (Chakrabarti, Zhan, Faloutsos 2004): each edge descends `scale` levels
 * of the adjacency matrix, choosing quadrant (0,0) with probability a, (0,1)
 * with b, (1,0) with c and (1,1) with d = 1-a-b-c. The row bit goes to the
 * source id, the column bit to the destination id. No noise is added.
 *
 * Random numbers come from the SplitMix64 sequence (Steele, Lea, Flood 2014)
 * addressed by counter: value(stream, i) = mix(stream + (i+1)*GAMMA), so that
 * any edge can be generated independently of the others and results do not
 * depend on the thread count.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define GAMMA 0x9E3779B97F4A7C15ULL

static inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* i-th output (0-based) of the SplitMix64 generator seeded with `seed`. */
static inline uint64_t splitmix_at(uint64_t seed, uint64_t i) {
    return mix64(seed + (i + 1) * GAMMA);
}

uint64_t gg_splitmix_at(uint64_t seed, uint64_t i) { return splitmix_at(seed, i); }

/* Stream keys: distinct sub-streams for edge sampling and for the permutation. */
static uint64_t stream_key(uint64_t seed, uint64_t which) {
    return mix64(seed * 0xD1B54A32D192ED03ULL + which * GAMMA + 0x5851F42D4C957F2DULL);
}

/*
 * Sample m = edge_factor * 2^scale directed edges. Thresholds are compared
 * against 32-bit uniforms: quadrant chosen by u < A, u < A+B, u < A+B+C with
 * A = floor(a * 2^32) etc. Each 64-bit draw supplies two levels.
 * If perm != NULL, both endpoints are mapped through it.
 */
void gg_rmat_edges(int scale, int64_t m, double a, double b, double c, uint64_t seed,
                   const int32_t *perm, int32_t *src, int32_t *dst, int nthreads) {
    const uint64_t key = stream_key(seed, 1);
    const uint64_t ta = (uint64_t)(a * 4294967296.0);
    const uint64_t tb = (uint64_t)((a + b) * 4294967296.0);
    const uint64_t tc = (uint64_t)((a + b + c) * 4294967296.0);
    const int words = (scale + 1) / 2;
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m; ++i) {
        uint32_t u = 0, v = 0;
        int level = 0;
        for (int w = 0; w < words; ++w) {
            uint64_t r = splitmix_at(key, (uint64_t)i * 16u + (uint64_t)w);
            for (int h = 0; h < 2 && level < scale; ++h, ++level) {
                uint64_t x = (h == 0) ? (r & 0xFFFFFFFFULL) : (r >> 32);
                uint32_t rowbit, colbit;
                if (x < ta) { rowbit = 0; colbit = 0; }
                else if (x < tb) { rowbit = 0; colbit = 1; }
                else if (x < tc) { rowbit = 1; colbit = 0; }
                else { rowbit = 1; colbit = 1; }
                u = (u << 1) | rowbit;
                v = (v << 1) | colbit;
            }
        }
        if (perm) { u = (uint32_t)perm[u]; v = (uint32_t)perm[v]; }
        src[i] = (int32_t)u;
        dst[i] = (int32_t)v;
    }
}

/* Seeded uniform random permutation of [0, V) (Fisher-Yates, Lemire's
 * multiply-high range reduction). */
void gg_permutation(int32_t V, uint64_t seed, int32_t *perm) {
    const uint64_t key = stream_key(seed, 2);
    for (int32_t i = 0; i < V; ++i) perm[i] = i;
    for (int64_t i = (int64_t)V - 1; i > 0; --i) {
        uint64_t r = splitmix_at(key, (uint64_t)i);
        uint64_t j = (uint64_t)(((unsigned __int128)r * (unsigned __int128)(i + 1)) >> 64);
        int32_t t = perm[i]; perm[i] = perm[j]; perm[j] = t;
    }
}

static void sort_i32(int32_t *a, int64_t n) {
    /* insertion sort for short rows, heap-free radix for long ones */
    if (n <= 48) {
        for (int64_t i = 1; i < n; ++i) {
            int32_t x = a[i]; int64_t j = i - 1;
            while (j >= 0 && a[j] > x) { a[j + 1] = a[j]; --j; }
            a[j + 1] = x;
        }
        return;
    }
    int32_t *tmp = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    int32_t *from = a, *to = tmp;
    for (int shift = 0; shift < 32; shift += 8) {
        int64_t cnt[257];
        memset(cnt, 0, sizeof(cnt));
        for (int64_t i = 0; i < n; ++i) cnt[(((uint32_t)from[i]) >> shift & 0xFF) + 1]++;
        for (int d = 0; d < 256; ++d) cnt[d + 1] += cnt[d];
        for (int64_t i = 0; i < n; ++i) to[cnt[((uint32_t)from[i]) >> shift & 0xFF]++] = from[i];
        int32_t *t = from; from = to; to = t;
    }
    /* after 4 passes the data is back in `a` */
    free(tmp);
}

/*
 * Edge list -> CSC with self-loops dropped (if drop_self) and duplicates
 * removed; each row's sources ascending. in_offsets has V+1 entries;
 * in_sources must hold m entries (the deduplicated count E <= m is returned).
 * Deterministic for any thread count.
 */
int64_t gg_edges_to_csc(int32_t V, int64_t m, const int32_t *src, const int32_t *dst, int drop_self,
                        int32_t *in_offsets, int32_t *in_sources, int nthreads) {
    if (nthreads > 0) omp_set_num_threads(nthreads);
    int64_t *cnt = (int64_t *)calloc((size_t)V + 1, sizeof(int64_t));
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m; ++i) {
        if (drop_self && src[i] == dst[i]) continue;
#pragma omp atomic
        cnt[dst[i] + 1]++;
    }
    for (int64_t v = 0; v < V; ++v) cnt[v + 1] += cnt[v];
    int64_t total = cnt[V];
    int64_t *cursor = (int64_t *)malloc((size_t)V * sizeof(int64_t));
    memcpy(cursor, cnt, (size_t)V * sizeof(int64_t));
    /* placement order within a row depends on timing; rows are sorted below */
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m; ++i) {
        if (drop_self && src[i] == dst[i]) continue;
        int64_t p;
#pragma omp atomic capture
        p = cursor[dst[i]]++;
        in_sources[p] = src[i];
    }
    free(cursor);
    int64_t *newdeg = (int64_t *)calloc((size_t)V + 1, sizeof(int64_t));
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t v = 0; v < V; ++v) {
        int32_t *row = in_sources + cnt[v];
        int64_t n = cnt[v + 1] - cnt[v];
        sort_i32(row, n);
        int64_t w = 0;
        for (int64_t i = 0; i < n; ++i)
            if (i == 0 || row[i] != row[i - 1]) row[w++] = row[i];
        newdeg[v + 1] = w;
    }
    for (int64_t v = 0; v < V; ++v) newdeg[v + 1] += newdeg[v];
    /* compact in place: rows only move left, and a row's destination never
       overlaps a later row's unread source range, so process rows in order */
    for (int64_t v = 0; v < V; ++v) {
        int64_t from = cnt[v], to = newdeg[v], n = newdeg[v + 1] - newdeg[v];
        if (from != to) memmove(in_sources + to, in_sources + from, (size_t)n * sizeof(int32_t));
    }
    (void)total;
    for (int64_t v = 0; v <= V; ++v) in_offsets[v] = (int32_t)newdeg[v];
    int64_t E = newdeg[V];
    free(cnt);
    free(newdeg);
    return E;
}

/* out_degree[u] = number of CSC entries equal to u. */
void gg_out_degree(int32_t V, int64_t E, const int32_t *in_sources, int32_t *out_degree, int nthreads) {
    if (nthreads > 0) omp_set_num_threads(nthreads);
    memset(out_degree, 0, (size_t)V * sizeof(int32_t));
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < E; ++i) {
#pragma omp atomic
        out_degree[in_sources[i]]++;
    }
}

/* CSC -> edge list of the reverse graph plus the graph itself (for symmetrizing):
   writes 2E (src,dst) pairs. */
void gg_csc_both_directions(int32_t V, const int32_t *in_offsets, const int32_t *in_sources,
                            int32_t *src, int32_t *dst, int nthreads) {
    if (nthreads > 0) omp_set_num_threads(nthreads);
    int64_t E = in_offsets[V];
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t v = 0; v < V; ++v) {
        for (int64_t i = in_offsets[v]; i < in_offsets[v + 1]; ++i) {
            src[i] = in_sources[i]; dst[i] = (int32_t)v;
            src[E + i] = (int32_t)v; dst[E + i] = in_sources[i];
        }
    }
}

/* Value of every in-edge of a graph whose edges come in both directions: the
   same value for u -> v and v -> u, 1 + (SplitMix64 output at the unordered
   pair key) mod 5, as a float (synthetic ratings). */
void gg_pair_values(int32_t V, const int32_t *in_offsets, const int32_t *in_sources, uint64_t seed,
                    float *out, int threads) {
#pragma omp parallel for schedule(dynamic, 1024) num_threads(threads)
    for (int32_t v = 0; v < V; ++v) {
        for (int32_t e = in_offsets[v]; e < in_offsets[v + 1]; ++e) {
            uint64_t a = (uint64_t)(uint32_t)in_sources[e], b = (uint64_t)(uint32_t)v;
            uint64_t key = a < b ? (a << 32) | b : (b << 32) | a;
            out[e] = (float)(1 + splitmix_at(seed, key) % 5u);
        }
    }
}
