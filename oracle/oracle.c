/*
 * Plain CPU oracle for the segmented pull traversal of
 * "Making Caches Work for Graph Analytics" (Zhang, Kiriansky, Mendis,
 * Amarasinghe, Zaharia; arXiv 1608.01362).
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product library links, calls or
 * includes this file; only the test-suite, the smoke check and the benchmark's
 * CPU-baseline leg use it. It shares no code, header, table or helper with
 * the GPU path: the two meet only at the input arrays produced by the graph
 * generator.
 *
 * Everything is FP64 (the paper stores PageRank vertex data as double,
 * Section 4, PageRank listing) with plain loops in the order the definitions
 * give. Graphs are in-edge CSR ("CSC"): sources of edges u->v are
 * src[off[v] .. off[v+1]), ascending.
 *
 * OpenMP splits only the loop over destination vertices; every per-vertex sum
 * runs sequentially over ascending sources, and whole-graph sums (dangling
 * mass, L1 residual) are taken over fixed chunks of CHUNK vertices and then
 * over the chunks in order, so results are identical for any thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define CHUNK 65536

static void set_threads(int nthreads) {
    if (nthreads > 0) omp_set_num_threads(nthreads);
}

/* Sum of x[v] over v in [0,V) where mask(v) holds, in fixed chunks. */
static double chunked_sum_dangling(int32_t V, const double *x, const int32_t *outdeg) {
    int64_t nchunks = ((int64_t)V + CHUNK - 1) / CHUNK;
    double *part = (double *)calloc((size_t)(nchunks > 0 ? nchunks : 1), sizeof(double));
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < nchunks; ++c) {
        int64_t lo = c * CHUNK, hi = lo + CHUNK < V ? lo + CHUNK : V;
        double s = 0.0;
        for (int64_t u = lo; u < hi; ++u)
            if (outdeg[u] == 0) s += x[u];
        part[c] = s;
    }
    double tot = 0.0;
    for (int64_t c = 0; c < nchunks; ++c) tot += part[c];
    free(part);
    return tot;
}

static double chunked_l1_diff(int32_t V, const double *a, const double *b) {
    int64_t nchunks = ((int64_t)V + CHUNK - 1) / CHUNK;
    double *part = (double *)calloc((size_t)(nchunks > 0 ? nchunks : 1), sizeof(double));
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < nchunks; ++c) {
        int64_t lo = c * CHUNK, hi = lo + CHUNK < V ? lo + CHUNK : V;
        double s = 0.0;
        for (int64_t v = lo; v < hi; ++v) s += fabs(a[v] - b[v]);
        part[c] = s;
    }
    double tot = 0.0;
    for (int64_t c = 0; c < nchunks; ++c) tot += part[c];
    free(part);
    return tot;
}

/*
 * One pull PageRank step (Section 2, PageRank listing: newRank[v] += rank[u]/degree[u]
 * over the in-edges of v), normalized with teleport (1-d)/V and the dangling
 * mass D = sum of r(u) over vertices without out-edges spread uniformly:
 *   r'(v) = (1-d)/V + d * ( sum_{u->v} r(u)/outdeg(u) + D/V ).
 * Returns D.
 */
static double pagerank_step(int32_t V, const int32_t *off, const int32_t *src, const int32_t *outdeg,
                            double d, const double *r, double *rn) {
    double D = chunked_sum_dangling(V, r, outdeg);
    double base = (1.0 - d) / (double)V + d * D / (double)V;
#pragma omp parallel for schedule(dynamic, 4096)
    for (int64_t v = 0; v < V; ++v) {
        double acc = 0.0;
        for (int64_t i = off[v]; i < off[v + 1]; ++i) {
            int32_t u = src[i];
            acc += r[u] / (double)outdeg[u];
        }
        rn[v] = base + d * acc;
    }
    return D;
}

/*
 * PageRank for `iters` iterations from r0 (NULL: uniform 1/V).
 * resid[t] = || r_{t+1} - r_t ||_1 for t < iters (may be NULL).
 * If tol > 0, stops after the first t with resid[t] < tol; returns the number
 * of iterations run.
 */
int oracle_pagerank(int32_t V, const int32_t *off, const int32_t *src, const int32_t *outdeg, double d,
                    int iters, double tol, const double *r0, double *r_out, double *resid, int nthreads) {
    set_threads(nthreads);
    double *r = (double *)malloc((size_t)V * sizeof(double));
    double *rn = (double *)malloc((size_t)V * sizeof(double));
    for (int64_t v = 0; v < V; ++v) r[v] = r0 ? r0[v] : 1.0 / (double)V;
    int t = 0;
    for (t = 0; t < iters; ++t) {
        pagerank_step(V, off, src, outdeg, d, r, rn);
        double rho = chunked_l1_diff(V, rn, r);
        if (resid) resid[t] = rho;
        double *tmp = r; r = rn; rn = tmp;
        if (tol > 0.0 && rho < tol) { ++t; break; }
    }
    memcpy(r_out, r, (size_t)V * sizeof(double));
    free(r);
    free(rn);
    return t;
}

/* One step evaluated only at the listed vertices (for spot checks on graphs too
 * large to iterate here): out[j] = r'(vertices[j]) given the full vector r. */
void oracle_pagerank_step_at(int32_t V, const int32_t *off, const int32_t *src, const int32_t *outdeg,
                             double d, const double *r, int64_t n, const int32_t *vertices, double *out,
                             int nthreads) {
    set_threads(nthreads);
    double D = chunked_sum_dangling(V, r, outdeg);
    double base = (1.0 - d) / (double)V + d * D / (double)V;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t j = 0; j < n; ++j) {
        int32_t v = vertices[j];
        double acc = 0.0;
        for (int64_t i = off[v]; i < off[v + 1]; ++i) acc += r[src[i]] / (double)outdeg[src[i]];
        out[j] = base + d * acc;
    }
}

/* Dangling mass sum_{outdeg(u)=0} r(u), fixed chunk order. */
double oracle_dangling_mass(int32_t V, const int32_t *outdeg, const double *r, int nthreads) {
    set_threads(nthreads);
    return chunked_sum_dangling(V, r, outdeg);
}

/*
 * The PageRank listing of Section 4 taken literally (no teleport
 * normalization, no dangling handling): R_0 = 1, R'(v) = 0.15 + 0.85 * sum R(u)/outdeg(u).
 * Only meaningful on graphs where every vertex has out-edges.
 */
void oracle_pagerank_paper_mode(int32_t V, const int32_t *off, const int32_t *src, const int32_t *outdeg,
                                int iters, double *R_out) {
    double *R = (double *)malloc((size_t)V * sizeof(double));
    double *Rn = (double *)malloc((size_t)V * sizeof(double));
    for (int64_t v = 0; v < V; ++v) R[v] = 1.0;
    for (int t = 0; t < iters; ++t) {
        for (int64_t v = 0; v < V; ++v) {
            double acc = 0.0;
            for (int64_t i = off[v]; i < off[v + 1]; ++i) acc += R[src[i]] / (double)outdeg[src[i]];
            Rn[v] = 0.15 + 0.85 * acc;
        }
        double *tmp = R; R = Rn; Rn = tmp;
    }
    memcpy(R_out, R, (size_t)V * sizeof(double));
    free(R);
    free(Rn);
}

/*
 * Personalized PageRank with a single restart vertex s (restart probability
 * 1-d): r_0 = e_s; r'(v) = (1-d)[v==s] + d*( sum_{u->v} r(u)/outdeg(u) + D*[v==s] ),
 * dangling mass D returned to the restart vertex.
 */
void oracle_ppr(int32_t V, const int32_t *off, const int32_t *src, const int32_t *outdeg, double d,
                int32_t seed_vertex, int iters, double *r_out, int nthreads) {
    set_threads(nthreads);
    double *r = (double *)calloc((size_t)V, sizeof(double));
    double *rn = (double *)malloc((size_t)V * sizeof(double));
    r[seed_vertex] = 1.0;
    for (int t = 0; t < iters; ++t) {
        double D = chunked_sum_dangling(V, r, outdeg);
#pragma omp parallel for schedule(dynamic, 4096)
        for (int64_t v = 0; v < V; ++v) {
            double acc = 0.0;
            for (int64_t i = off[v]; i < off[v + 1]; ++i) acc += r[src[i]] / (double)outdeg[src[i]];
            rn[v] = d * acc + (v == seed_vertex ? (1.0 - d) + d * D : 0.0);
        }
        double *tmp = r; r = rn; rn = tmp;
    }
    memcpy(r_out, r, (size_t)V * sizeof(double));
    free(r);
    free(rn);
}

/*
 * Label propagation (named in the evaluation, Section 6; integer labels): on
 * an undirected graph stored with both edge directions, synchronous
 * min-label updates l'(v) = min(l(v), min_{u in N(v)} l(u)) from l_0(v) = v,
 * run until an iteration changes nothing. Returns the number of iterations
 * executed, including the final one that changed nothing.
 */
int oracle_labelprop(int32_t V, const int32_t *off, const int32_t *src, int max_iters, int32_t *labels_out,
                     int nthreads) {
    set_threads(nthreads);
    int32_t *l = (int32_t *)malloc((size_t)V * sizeof(int32_t));
    int32_t *ln = (int32_t *)malloc((size_t)V * sizeof(int32_t));
    for (int64_t v = 0; v < V; ++v) l[v] = (int32_t)v;
    int t = 0;
    for (t = 0; t < max_iters;) {
        int64_t changed = 0;
#pragma omp parallel for schedule(dynamic, 4096) reduction(+ : changed)
        for (int64_t v = 0; v < V; ++v) {
            int32_t m = l[v];
            for (int64_t i = off[v]; i < off[v + 1]; ++i)
                if (l[src[i]] < m) m = l[src[i]];
            ln[v] = m;
            if (m != l[v]) changed++;
        }
        int32_t *tmp = l; l = ln; ln = tmp;
        ++t;
        if (changed == 0) break;
    }
    memcpy(labels_out, l, (size_t)V * sizeof(int32_t));
    free(l);
    free(ln);
    return t;
}

/* ------------------------------------------------------------------------ */
/* CSR segmenting (Section 3)                                                */
/* ------------------------------------------------------------------------ */

/*
 * Preprocessing (Section 3.1, preprocessing algorithm), with segment id of an
 * in-edge = source / N. For every destination v in ascending order and each of
 * its in-edges (ascending source), the edge is appended to subgraph src/N.
 * Within a subgraph, edges are then grouped by destination (already the case:
 * destinations arrive in ascending order), giving per subgraph a CSR whose
 * rows are the distinct destinations.
 *
 * Layout written (all subgraphs concatenated, subgraph s first, s ascending):
 *   seg_row_begin[k+1]   first row of subgraph s
 *   row_ptr[Q+1]         first edge of each row
 *   row_dst[Q]           idxMap: global destination id of each row
 *   edge_src[E]          source id minus s*N (local index into the segment)
 *   block_ptr[(nb+1)*k]  block_ptr[b*k + s] = first row of subgraph s whose
 *                        destination is >= b*B (row index into the concatenation);
 *                        the block index of the cache-aware merge (Section 3.3).
 * Call with row_ptr == NULL to get only Q (returned).
 */
int64_t oracle_segment(int32_t V, const int32_t *off, const int32_t *src, int32_t N, int32_t B,
                       int32_t *seg_row_begin, int32_t *row_ptr, int32_t *row_dst, int32_t *edge_src,
                       int32_t *block_ptr) {
    int64_t k = ((int64_t)V + N - 1) / N;
    int64_t nb = ((int64_t)V + B - 1) / B;
    int64_t *rows = (int64_t *)calloc((size_t)k, sizeof(int64_t));
    int64_t *edges = (int64_t *)calloc((size_t)k, sizeof(int64_t));
    int64_t *last_dst = (int64_t *)malloc((size_t)k * sizeof(int64_t));
    for (int64_t s = 0; s < k; ++s) last_dst[s] = -1;
    /* first pass: sizes of each subgraph */
    for (int64_t v = 0; v < V; ++v) {
        for (int64_t i = off[v]; i < off[v + 1]; ++i) {
            int64_t s = src[i] / N;
            edges[s]++;
            if (last_dst[s] != v) { rows[s]++; last_dst[s] = v; }
        }
    }
    int64_t Q = 0;
    for (int64_t s = 0; s < k; ++s) Q += rows[s];
    if (!row_ptr) { free(rows); free(edges); free(last_dst); return Q; }

    int64_t *row_cursor = (int64_t *)malloc((size_t)k * sizeof(int64_t));
    int64_t *edge_cursor = (int64_t *)malloc((size_t)k * sizeof(int64_t));
    int64_t r = 0, e = 0;
    for (int64_t s = 0; s < k; ++s) {
        seg_row_begin[s] = (int32_t)r;
        row_cursor[s] = r;
        edge_cursor[s] = e;
        r += rows[s];
        e += edges[s];
        last_dst[s] = -1;
    }
    seg_row_begin[k] = (int32_t)r;
    /* second pass: addInEdge(v, src) to subgraph src/N */
    for (int64_t v = 0; v < V; ++v) {
        for (int64_t i = off[v]; i < off[v + 1]; ++i) {
            int64_t s = src[i] / N;
            if (last_dst[s] != v) {
                int64_t row = row_cursor[s]++;
                row_dst[row] = (int32_t)v;
                row_ptr[row] = (int32_t)edge_cursor[s];
                last_dst[s] = v;
            }
            edge_src[edge_cursor[s]++] = (int32_t)(src[i] - s * N);
        }
    }
    row_ptr[Q] = (int32_t)e;
    /* block index: for each subgraph and block, the first row with dst >= b*B */
    for (int64_t s = 0; s < k; ++s) {
        int64_t rr = seg_row_begin[s], rend = seg_row_begin[s + 1];
        for (int64_t b = 0; b <= nb; ++b) {
            int64_t lim = b * (int64_t)B;
            while (rr < rend && row_dst[rr] < lim) ++rr;
            block_ptr[b * k + s] = (int32_t)rr;
        }
    }
    free(rows); free(edges); free(last_dst); free(row_cursor); free(edge_cursor);
    return Q;
}

/*
 * Parallel segment processing (Section 3.2) with the PageRank update
 * (Section 4: EdgeUpdate adds the source value into the buffer): for each
 * subgraph s, each of its rows, partial[row] = sum of x[s*N + local source] over
 * the row's edges, ascending. op 0: sum (FP64); op 1: min (labels, as double
 * holding exact integers; identity +inf is never produced since rows are non-empty).
 */
void oracle_segment_gather(int64_t k, int32_t N, const int32_t *seg_row_begin, const int32_t *row_ptr,
                           const int32_t *edge_src, const double *x, int op, double *partial) {
    for (int64_t s = 0; s < k; ++s) {
        for (int64_t row = seg_row_begin[s]; row < seg_row_begin[s + 1]; ++row) {
            double acc = op == 0 ? 0.0 : INFINITY;
            for (int64_t i = row_ptr[row]; i < row_ptr[row + 1]; ++i) {
                double val = x[s * (int64_t)N + edge_src[i]];
                if (op == 0) acc += val;
                else if (val < acc) acc = val;
            }
            partial[row] = acc;
        }
    }
}

/*
 * Cache-aware merge (Section 3.3, merge algorithm): for each block of B
 * destination ids, for each subgraph in order, the buffer entries in
 * [block_ptr[b*k+s], block_ptr[(b+1)*k+s]) are combined into out[row_dst[i]].
 * out starts at the identity (0 for sum, +inf for min).
 */
void oracle_merge(int32_t V, int64_t k, int32_t B, const int32_t *row_dst, const int32_t *block_ptr,
                  const double *partial, int op, double *out) {
    int64_t nb = ((int64_t)V + B - 1) / B;
    for (int64_t v = 0; v < V; ++v) out[v] = op == 0 ? 0.0 : INFINITY;
    for (int64_t b = 0; b < nb; ++b) {
        for (int64_t s = 0; s < k; ++s) {
            int64_t lo = block_ptr[b * k + s], hi = block_ptr[(b + 1) * k + s];
            for (int64_t i = lo; i < hi; ++i) {
                if (op == 0) out[row_dst[i]] += partial[i];
                else if (partial[i] < out[row_dst[i]]) out[row_dst[i]] = partial[i];
            }
        }
    }
}
