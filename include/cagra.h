/*
 * cagra.h -- C ABI of the MI355X (gfx950) CSR-segmenting library.
 *
 * Implements the pull-direction edge traversal of "Making Caches Work for
 * Graph Analytics" (arXiv 1608.01362): CSR segmenting preprocessing
 * (Section 3.1), per-segment gather into sequential buffers (Section 3.2),
 * the cache-aware merge (Section 3.3), and the PageRank / label-propagation
 * iterations built from them (Section 4 programming abstraction; Section 6
 * applications).
 *
 * Conventions shared by every entry point
 *   - Pointers are DEVICE pointers unless the parameter name starts with host_.
 *   - The caller owns all memory; the library never allocates or frees device
 *     memory. Sizes of caller buffers are given by the *_bytes helpers.
 *   - Work is enqueued on `stream` and is asynchronous, except where a function
 *     states that it synchronizes the stream.
 *   - Every argument is validated on the host before any HIP call; invalid
 *     arguments return a negative status and enqueue nothing. A description of
 *     the last error on the calling thread is available from cagra_last_error().
 *   - All results are deterministic: repeated calls on the same inputs produce
 *     bit-identical outputs.
 *   - Graphs are in-edge CSR ("CSC"): the sources of the edges u->v are
 *     in_sources[in_offsets[v] .. in_offsets[v+1]), strictly ascending, with no
 *     self-loops and no duplicates; E < 2^31.
 */
#ifndef CAGRA_H
#define CAGRA_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CAGRA_ABI_VERSION 2

typedef enum {
    CAGRA_OK = 0,
    CAGRA_E_INVALID = -1,   /* null pointer, bad size, unknown enum value */
    CAGRA_E_OVERFLOW = -2,  /* a count would not fit in int32 */
    CAGRA_E_CAPACITY = -3,  /* parameter beyond a kernel capacity (LDS bytes, segment count) */
    CAGRA_E_BUFFER = -4,    /* workspace too small or misaligned */
    CAGRA_E_HIP = -5,       /* a HIP runtime call or kernel launch failed */
    CAGRA_E_NOT_CONVERGED = -6, /* an iteration cap was reached before the stopping rule held */
    CAGRA_E_RANGE = -7      /* values outside the range the exact fixed-point merge sums
                               (non-finite, or an absolute buffer mass of 64 or more in one
                               merge block); the results of that iteration are not exact */
} cagra_status;

/* Element types of vertex values gathered by the segment processing step. */
enum { CAGRA_F32 = 0, CAGRA_BF16 = 1, CAGRA_I32 = 2 };

/* Combine operators (the paper's user-supplied Merge, Section 4). */
enum {
    CAGRA_SUM_F32 = 0,       /* float sum, identity 0 */
    CAGRA_MIN_I32 = 1,       /* int32 minimum, identity INT32_MAX */
    CAGRA_SUM_F32_COMP = 2   /* float sum with Neumaier compensation (merge only) */
};

/* LDS per workgroup on gfx950. */
#define CAGRA_LDS_BYTES 163840
/* A segment's values are staged in LDS when N * element bytes <=
   CAGRA_STAGE_BYTES (32,768 FP32 or 65,536 BF16 / int32 32,768 values); larger
   segments are gathered through the cache hierarchy (L2- or Infinity-Cache-
   sized segments). The rest of the LDS collects finished rows for coalesced
   buffer writes. */
#define CAGRA_STAGE_BYTES 131072
/* Segments of at most this many vertices store 16-bit edge words: a local
   source index needs 15 bits and bit 15 marks a row start. This halves the
   dominant edge stream of segment processing. */
#define CAGRA_EDGE16_MAX_N 32768
/* Waves (64 lanes) that share one staged segment in the gather kernel. */
#define CAGRA_TILE_WAVES 16

typedef struct {
    int32_t V;                  /* vertices */
    int64_t E;                  /* edges, < 2^31 */
    const int32_t *in_offsets;  /* [V+1] */
    const int32_t *in_sources;  /* [E] */
    const int32_t *out_degree;  /* [V] out-degree of each vertex (for PageRank) */
} cagra_graph;

/*
 * Segmented graph (Section 3.1). Subgraph s holds the in-edges whose source is
 * in [s*N, min((s+1)*N, V)); its rows are the distinct destinations of those
 * edges in ascending order, and a row's edges keep ascending source order.
 * All subgraphs are concatenated, s ascending. Q = total number of rows.
 *
 *   seg_row_begin[k+1]   first row of subgraph s; seg_row_begin[k] = Q
 *   row_ptr[Q+1]         first edge of each row; row_ptr[Q] = E
 *   row_dst[Q]           global destination of each row (the paper's idxMap)
 *   edge_src[E]          edge words: the local source index u - s*N plus a
 *                        row-start flag on the first edge of every row. Word
 *                        width depends on N: uint16 when N <= CAGRA_EDGE16_MAX_N
 *                        (flag = bit 15, index = bits 0-14), int32 otherwise
 *                        (flag = bit 31, index = bits 0-30)
 *   block_ptr[(nb+1)*k]  merge block index: block_ptr[b*k + s] = first row of
 *                        subgraph s whose destination is >= b*B (Section 3.3's
 *                        block starts; block b of subgraph s ends at
 *                        block_ptr[(b+1)*k + s])
 *   tile_edge[ntiles+1]  gather work units: tile t covers edges
 *                        [tile_edge[t], tile_edge[t+1]), starts and ends on row
 *                        boundaries and lies within subgraph tile_seg[t]
 *   tile_seg[ntiles]
 *   tile_span_row[ntiles*CAGRA_TILE_WAVES]  for each tile, the first row that
 *                        starts at or after each wave's share of the tile
 *   row_dst_lo[Q]        row_dst mod B as uint16: the destination's offset in
 *                        its merge block (what the fused merges read)
 *   block_items[nb+1]    merge work items of the fused PageRank merge: block b
 *                        is merged by items [block_items[b], block_items[b+1]),
 *                        which split its entries (flattened over subgraphs)
 *                        into equal parts. A block is split when it holds more
 *                        than four times the mean number of entries per block
 *                        (destinations of very high in-degree, e.g. after
 *                        clustering); at most max_items items in all
 *
 * edge_src must be 16-byte aligned and hold E * cagra_edge_word_bytes(N)
 * bytes. All arrays are caller-allocated device memory of the sizes the query
 * call reports.
 */
typedef struct {
    /* parameters (set by the caller before the query call) */
    int32_t N;            /* vertices per segment, >= 1 */
    int32_t B;            /* merge block size in vertices, 1 <= B <= cagra_max_merge_block() */
    int32_t tile_edges;   /* nominal edges per gather tile, >= 64 */
    /* sizes (filled by the query call) */
    int32_t V, k, nb, ntiles;
    int64_t E, Q;
    size_t build_workspace_bytes;
    int32_t max_items;    /* bound on block_items[nb]; a caller may lower it to
                             block_items[nb] once the build has run (no split
                             block then saves the merge's slot pass). Set to
                             nb, every block is merged whole by one work item.
                             Between nb and block_items[nb] it is invalid: the
                             PageRank merge then merges nothing and its scalars
                             come out NaN */
    /* device arrays */
    int32_t *seg_row_begin;
    int32_t *row_ptr;
    int32_t *row_dst;
    void *edge_src;
    int32_t *block_ptr;
    int32_t *tile_edge;
    int32_t *tile_seg;
    int32_t *tile_span_row;
    uint16_t *row_dst_lo;
    int32_t *block_items;
} cagra_segments;

int cagra_abi_version(void);
const char *cagra_status_string(int status);
/* Thread-local description of the last non-OK status returned on this thread. */
const char *cagra_last_error(void);
/* Largest merge block B accepted (LDS capacity of the merge kernel). */
int32_t cagra_max_merge_block(void);

/* Bytes per edge word of a segmentation with segment size N: 2 when
   N <= CAGRA_EDGE16_MAX_N, else 4 (0 for N < 1). */
int32_t cagra_edge_word_bytes(int32_t N);

/*
 * Frequency-based clustering (Section 5), applied to the whole graph before
 * segmenting. Vertices whose out-degree is strictly above the average degree
 * E / V are moved to the front, ordered by out-degree from high to low; the
 * order is stable (equal out-degrees keep their original order), and every
 * other vertex follows in its original order. The graph is relabelled: old
 * vertex perm[i] becomes vertex i, and each in-edge row lists its sources
 * ascending under the new ids. PageRank on the result, read through perm,
 * equals PageRank on the input.
 *
 *   g           input graph (device arrays; out_degree required)
 *   perm        device int32[V], written: old id of each new vertex
 *   in_offsets  device int32[V+1], written: new row offsets
 *   in_sources  device int32[E], written: new sources (may be NULL when E = 0)
 *   out_degree  device int32[V], written: new out-degrees
 *   hot         device int32[1] or NULL, written: number of clustered vertices
 *   workspace   device memory of cagra_cluster_workspace_bytes(V, E) bytes
 *               (about 16 bytes per edge; the caller owns it)
 * Outputs must not alias the inputs. Errors: CAGRA_E_INVALID / _OVERFLOW for
 * bad arguments, CAGRA_E_BUFFER for a missing or small workspace, nothing
 * launched in those cases. Asynchronous on `stream`.
 */
size_t cagra_cluster_workspace_bytes(int32_t V, int64_t E);
int cagra_cluster(const cagra_graph *g, int32_t *perm, int32_t *in_offsets, int32_t *in_sources,
                  int32_t *out_degree, int32_t *hot, void *workspace, size_t workspace_bytes, hipStream_t stream);

/* Latent factors per vertex of the collaborative-filtering step. */
#define CAGRA_CF_FACTORS 64

/*
 * Edge values in the segmented edge order: seg_values[p] = in_values[e] where
 * p is the position that in-edge e (CSC order, as in g) takes in the
 * segmented edge array of seg. in_values and seg_values are device float[E],
 * not aliased. Asynchronous; no workspace.
 */
cagra_status cagra_segment_edge_values(const cagra_graph *g, const cagra_segments *seg, const float *in_values,
                                       float *seg_values, hipStream_t stream);

/* Device workspace of cagra_cf_iter (one FP64 value per gather tile). */
size_t cagra_cf_workspace_bytes(const cagra_segments *seg);

/*
 * One collaborative-filtering step on a rating graph (every rating an edge in
 * both directions; Section 4's update function with access to the old
 * destination value), as gradient descent on
 *   F(X) = 1/2 sum_ratings (r - <x_u, x_i>)^2 + lambda/2 sum_v |x_v|^2:
 *   g_v      = sum over in-edges u -> v of (r_uv - <x_u, x_v>) x_u
 *   x_out[v] = x_in[v] + gamma * (g_v - lambda * x_in[v])
 *   sq_out[0] = sum over in-edges of (r_uv - <x_u, x_v>)^2 at x_in (FP64)
 * x_in, x_out: device float[V][CAGRA_CF_FACTORS] (row-major, not aliased);
 * seg_values: the ratings in the segmented edge order
 * (cagra_segment_edge_values); partial: float[Q][CAGRA_CF_FACTORS] scratch.
 * The merge adds the subgraphs' buffers in ascending order (FP32). Requires
 * seg->B <= 512.
 */
cagra_status cagra_cf_iter(const cagra_graph *g, const cagra_segments *seg, const float *seg_values, double gamma,
                           double lambda, const float *x_in, float *partial, float *x_out, double *sq_out,
                           void *workspace, size_t workspace_bytes, hipStream_t stream);

/*
 * Betweenness centrality from a start vertex (Brandes' algorithm) as
 * level-synchronous segmented pulls with an active frontier (Section 4
 * EdgeMap): a forward level adds sigma[u] over in-edges u -> v from the
 * vertices u at depth d into every unvisited v, which then gets depth d + 1
 * and that sum as sigma[v]; a backward level, run on the segmentation of the
 * reverse graph (seg_t), sets delta[u] = sigma[u] * sum over out-edges u -> w
 * with depth d + 1 of (1 + delta[w]) / sigma[w] for the vertices u at depth d
 * and adds delta[u] to bc[u] unless u is the start. Segments without a
 * frontier vertex are skipped in both phases. FP32 values, FP32 merges in
 * subgraph order.
 *
 *   depth  device int32[V]  (-1 = unreached)      sigma, delta, bc  device float[V]
 *   vals, sums  device float[V] scratch            partial  device float[Q] scratch
 *   count  device int32[1]: size of the new frontier after a forward level
 *   workspace: cagra_bc_workspace_bytes(seg) bytes (the frontier's segment bits)
 * cagra_bc_start sets depth = -1, sigma = delta = 0, then depth[source] = 0 and
 * sigma[source] = 1. A start's forward levels run for d = 0, 1, ... until the
 * count is 0; its backward levels then run for d = deepest - 1 down to 0.
 */
size_t cagra_bc_workspace_bytes(const cagra_segments *seg);
cagra_status cagra_bc_start(int32_t V, int32_t source, int32_t *depth, float *sigma, float *delta,
                            hipStream_t stream);
cagra_status cagra_bc_forward_level(const cagra_segments *seg, int32_t d, int32_t *depth, float *sigma, float *vals,
                                    float *partial, float *sums, int32_t *count, void *workspace,
                                    size_t workspace_bytes, hipStream_t stream);
cagra_status cagra_bc_backward_level(const cagra_segments *seg_t, int32_t d, int32_t source, const int32_t *depth,
                                     const float *sigma, float *delta, float *bc, float *vals, float *partial,
                                     float *sums, void *workspace, size_t workspace_bytes, hipStream_t stream);

/*
 * Push-direction segmenting: the out-edge traversal cut into segments (the
 * alternative to the in-edge pull that Section 3 mentions and Section 4's
 * EdgeMap allows). seg_t is the segmentation of the REVERSE graph (built with
 * cagra_build_segments from the out-edge lists written as a CSC; for an
 * undirected graph that is the graph itself): its subgraph s holds the edges
 * u -> v with v in segment s, rows are sources u. An iteration
 *   1. expands: vals[i] = x[row_dst[i]] for every row i of seg_t, block by
 *      block of sources (the merge's access pattern run backwards),
 *   2. scatters: one workgroup per piece (a run of one subgraph's tiles)
 *      adds each edge's row value to its destination's accumulator in LDS,
 *      then writes the accumulators to the piece's slot,
 *   3. updates each vertex from its segment's slots.
 * Sums are exact (each FP32 value truncated toward zero to a multiple of
 * 2^-56, added as int64; |values| and |sums| < 64), minima exact, so results are bit-identical run to run.
 * Requirements: the scatter keeps N accumulators in LDS, 8 bytes each for
 * PageRank (N <= 20,480) and 4 for label propagation (N <= 40,960); and
 * 4*B + 8*(k+1) + 320 <= CAGRA_LDS_BYTES for the expand. The workspace (plan, per-block sums
 * and one slot of N 8-byte accumulators per piece) carries no state between
 * calls.
 */
size_t cagra_push_workspace_bytes(const cagra_segments *seg_t);

/*
 * One PageRank iteration in the push direction: same formula, scalars and
 * start (cagra_pagerank_init with CAGRA_F32) as cagra_pagerank_iter; FP32
 * contributions. g is the graph itself (out_degree), seg_t the segmentation
 * of its reverse; vals is float[seg_t->Q] scratch. scalars_out[3] carries
 * scalars_in[3] unchanged: the push scatter does not check the range of its
 * values.
 */
cagra_status cagra_pagerank_push_iter(const cagra_graph *g, const cagra_segments *seg_t, double damping,
                                      const float *rank_in, const float *contrib_in, const double *scalars_in,
                                      float *vals, float *rank_out, float *contrib_out, double *scalars_out,
                                      void *workspace, size_t workspace_bytes, hipStream_t stream);

/*
 * One min-label propagation step in the push direction (same result as
 * cagra_labelprop_iter): every edge u -> v offers labels_in[u] to v.
 * vals is int32[seg_t->Q] scratch; *changed_out = number of labels changed.
 */
cagra_status cagra_labelprop_push_iter(const cagra_segments *seg_t, const int32_t *labels_in, int32_t *vals,
                                       int32_t *labels_out, int32_t *changed_out, void *workspace,
                                       size_t workspace_bytes, hipStream_t stream);

/*
 * Device check of a graph against the CSC rules at the top of this file:
 * in_offsets[0] == 0, in_offsets[V] == E, offsets non-decreasing; every source
 * in [0, V); sources strictly ascending within each row (no duplicates); no
 * self-loops. The offsets are checked first and the edges only when the
 * offsets are sound, so a corrupt graph is never read out of bounds. Returns
 * CAGRA_OK, or CAGRA_E_INVALID naming the first offending vertex or edge of
 * the first violated rule in cagra_last_error(). SYNCHRONIZES the stream.
 * workspace: device memory of cagra_validate_workspace_bytes() bytes.
 */
size_t cagra_validate_workspace_bytes(void);
cagra_status cagra_validate_graph(const cagra_graph *g, void *workspace, size_t workspace_bytes,
                                  hipStream_t stream);

/* Device workspace needed by the query call of cagra_build_segments. */
size_t cagra_query_workspace_bytes(int32_t V, int64_t E, int32_t N);

/*
 * Section 3.1 preprocessing on the GPU. Two calls:
 *  1. Query: seg->N, seg->B, seg->tile_edges set, seg->row_dst == NULL,
 *     workspace >= cagra_query_workspace_bytes(). Counts rows and per-segment
 *     edges, SYNCHRONIZES the stream, and fills seg->{V,E,k,nb,Q,ntiles,
 *     build_workspace_bytes}.
 *  2. Build: every array of *seg allocated at the reported sizes, workspace >=
 *     seg->build_workspace_bytes. Fills all arrays; asynchronous.
 * Requirements: k = ceil(V/N) <= 32768; CSC as described at the top of this file.
 */
cagra_status cagra_build_segments(const cagra_graph *g, cagra_segments *seg, void *workspace,
                                  size_t workspace_bytes, hipStream_t stream);

/* Device workspace of the per-iteration calls below: per-block FP64 partial
   sums, then one int64 slot of B values for each work item of a split merge
   block (2 * (max_items - nb) slots). It carries no state between calls. */
size_t cagra_iter_workspace_bytes(const cagra_segments *seg);

/*
 * Segment processing (Section 3.2) on its own: for every row r of every
 * subgraph s, partial[r] = op over the row's edges of values[s*N + local src].
 *   op CAGRA_SUM_F32: values are CAGRA_F32 or CAGRA_BF16 (value_type), partial is float[Q]
 *   op CAGRA_MIN_I32: values are CAGRA_I32, partial is int32[Q]
 * Segments with N * element bytes <= CAGRA_STAGE_BYTES are staged in LDS.
 */
cagra_status cagra_segment_gather(const cagra_segments *seg, int32_t op, int32_t value_type, const void *values,
                                  void *partial, hipStream_t stream);

/*
 * Cache-aware merge (Section 3.3): out[v] = op over subgraphs s, strictly in
 * ascending order, of the buffer entries whose row_dst is v (FP32 sums are
 * rounded after every addition in that order, as the paper's merge loop does);
 * vertices without entries get the identity. op CAGRA_SUM_F32 or
 * CAGRA_SUM_F32_COMP (Neumaier-compensated; partial/out float) or
 * CAGRA_MIN_I32 (int32).
 */
cagra_status cagra_merge(const cagra_segments *seg, int32_t op, const void *partial, void *out,
                         hipStream_t stream);

/*
 * PageRank start: contrib_out[v] = rank[v] / out_degree[v] (0 where the
 * out-degree is 0) stored as contrib_type (CAGRA_F32 or CAGRA_BF16, round to
 * nearest even); scalars_out[0] = dangling mass sum_{out_degree=0} rank (FP64),
 * scalars_out[1] = 0, scalars_out[2] = sum of rank (FP64), scalars_out[3] =
 * number of non-finite rank values (the range count, see cagra_pagerank_iter).
 * The workspace needs 32*ceil(V/16384) + 256 bytes (the iteration workspace
 * of any segmentation of the graph is large enough).
 */
cagra_status cagra_pagerank_init(const cagra_graph *g, int32_t contrib_type, const float *rank, void *contrib_out,
                                 double *scalars_out, void *workspace, size_t workspace_bytes,
                                 hipStream_t stream);

/*
 * One PageRank iteration through segmenting (Section 4 PageRank: EdgeMap with
 * a summing EdgeUpdate and Merge, then VertexMap), normalized with teleport and
 * uniform redistribution of the dangling mass (restart_vertex = -1):
 *   rank_out[v] = (1-d)/V + d * ( sum_{u->v} contrib_in[u] + scalars_in[0]/V )
 * or personalized to one restart vertex s = restart_vertex in [0, V), where the
 * teleport and the dangling mass return to s:
 *   rank_out[v] = d * sum_{u->v} contrib_in[u] + [v == s] * ((1-d) + d * scalars_in[0])
 *   contrib_out[v] = rank_out[v] / out_degree[v] (0 if out_degree is 0)
 *   scalars_out[0] = dangling mass of rank_out, scalars_out[1] = ||rank_out - rank_in||_1,
 *   scalars_out[2] = sum of rank_out,
 *   scalars_out[3] = range count: scalars_in[3] plus the number of merge blocks
 *                    whose buffer values were non-finite or summed to 64 or more in
 *                    absolute value   (all FP64)
 * partial is float[Q] scratch for the per-subgraph buffers. The merge adds the
 * FP32 buffer values exactly (each truncated toward zero to a multiple of 2^-56 and summed
 * as int64), so its result does not depend on the order of the additions.
 * That is exact while each merge block's buffer values sum to less than 64 in
 * absolute value, which holds for non-negative rank vectors of mass at most 1;
 * every block outside that range is counted in scalars_out[3], which carries
 * over from iteration to iteration, so a non-zero count after any number of
 * iterations means some iteration was not exact (cagra_pagerank_solve then
 * returns CAGRA_E_RANGE). contrib_in is read with contrib_type, contrib_out
 * written with it. scalars_in must not alias scalars_out. Requires
 * 8*B + 8*(k+1) + 320 <= CAGRA_LDS_BYTES.
 */
cagra_status cagra_pagerank_iter(const cagra_graph *g, const cagra_segments *seg, double damping,
                                 int32_t restart_vertex, int32_t contrib_type, const float *rank_in,
                                 const void *contrib_in, const double *scalars_in, float *partial, float *rank_out,
                                 void *contrib_out, double *scalars_out, void *workspace, size_t workspace_bytes,
                                 hipStream_t stream);

/*
 * cagra_pagerank_iter without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc). The iteration's scratch (per-block FP64
 * partial sums, split-block slots) lives in a static device array of
 * CAGRA_NOALLOC_SCRATCH_BYTES per GPU, held until the process ends; the call
 * allocates nothing. Iterations whose workspace (cagra_iter_workspace_bytes)
 * exceeds that size are rejected with CAGRA_E_CAPACITY before any launch.
 * Every call on one GPU shares that GPU's array: calls that overlap in time on
 * one GPU (other streams, other threads) race and must not be issued. Same
 * arguments otherwise, same kernels, bit-identical results.
 */
#define CAGRA_NOALLOC_SCRATCH_BYTES (64u << 20)
size_t cagra_noalloc_scratch_bytes(void);
cagra_status cagra_pagerank_iter_noalloc(const cagra_graph *g, const cagra_segments *seg, double damping,
                                         int32_t restart_vertex, int32_t contrib_type, const float *rank_in,
                                         const void *contrib_in, const double *scalars_in, float *partial,
                                         float *rank_out, void *contrib_out, double *scalars_out,
                                         hipStream_t stream);

/*
 * The merge half of cagra_pagerank_iter on its own: cache-aware merge of an
 * already gathered partial[Q] (Section 3.3) followed by the vertex update
 * (Section 4 VertexMap). cagra_pagerank_iter == cagra_segment_gather(SUM_F32,
 * contrib_type) + cagra_pagerank_merge; same arguments, same results.
 */
cagra_status cagra_pagerank_merge(const cagra_graph *g, const cagra_segments *seg, double damping,
                                  int32_t restart_vertex, int32_t contrib_type, const float *rank_in,
                                  const double *scalars_in, const float *partial, float *rank_out, void *contrib_out,
                                  double *scalars_out, void *workspace, size_t workspace_bytes, hipStream_t stream);

/*
 * PageRank power iteration to a residual threshold (the Section 4 program's
 * loop of EdgeMap and VertexMap, run until the L1 change falls below tol),
 * driven from the host: cagra_pagerank_init, then cagra_pagerank_iter steps;
 * after every check_every-th step the scalars are read back and the loop stops
 * at the first L1 residual below tol. The start vector's scalars are read
 * synchronously; after that the step following a check is queued before the
 * host waits for the check's scalars (through pinned host memory), unless the
 * residual trend predicts that the check may end the loop or switch the
 * precision. When a check ends the loop or switches, the step queued past it
 * is dropped: every result (iterate, counts, scalars) is the one a loop that
 * waited at each check would give; only the other buffer of each pair may hold
 * the dropped step's values. The call SYNCHRONIZES the stream before it
 * returns. The read-back uses 4 KiB of pinned host memory and two events per
 * concurrent solve, allocated on a device's first solve and kept until the
 * process ends.
 *   rank0, rank1       float[V] pair; rank0 holds the start vector on entry
 *   contrib0, contrib1 contribution pair: float[V] for CAGRA_F32 or when
 *                      switch_tol > 0, uint16[V] for CAGRA_BF16 otherwise
 *   scalars            double[8]: the two scalar sets of the pair
 *   partial, workspace as for cagra_pagerank_iter
 * BF16 finishing switch: with contrib_type CAGRA_BF16 and switch_tol > 0, the
 * first residual read below switch_tol rebuilds the contributions as FP32 from
 * the current ranks (cagra_pagerank_init) and the remaining iterations gather
 * FP32, so the answer is no longer limited by BF16 rounding.
 * The result is in rank[host_result->final_buf] and contrib[...] (the latter in
 * FP32 once switched). Returns CAGRA_OK when the residual fell below tol,
 * CAGRA_E_NOT_CONVERGED when max_iters steps ran without that (host_result
 * still describes the last iterate), CAGRA_E_RANGE when a read-back range count
 * (scalars[3]) is non-zero, or the status of a failed step.
 */
typedef struct {
    double damping;        /* d in [0, 1] */
    double tol;            /* stopping threshold on the L1 residual, > 0 */
    double switch_tol;     /* CAGRA_BF16 only: residual below which to finish in FP32 (0: never) */
    int32_t restart_vertex;/* -1: uniform teleport; else personalized to this vertex (see
                              cagra_pagerank_iter; the caller's start vector is used as given) */
    int32_t max_iters;     /* iteration cap, >= 1 */
    int32_t check_every;   /* read the residual back every this many iterations, >= 1 */
    int32_t contrib_type;  /* CAGRA_F32 or CAGRA_BF16 */
} cagra_pr_params;
typedef struct {
    int32_t iters;         /* iterations run */
    int32_t iters_bf16;    /* of which gathered BF16 contributions */
    int32_t final_buf;     /* 0 or 1: which buffer of each pair holds the result */
    double residual;       /* last L1 residual read back (inf before the first) */
    double scalars[4];     /* last scalars read back (as cagra_pagerank_iter) */
} cagra_pr_result;
cagra_status cagra_pagerank_solve(const cagra_graph *g, const cagra_segments *seg, const cagra_pr_params *params,
                                  float *rank0, float *rank1, void *contrib0, void *contrib1, double *scalars,
                                  float *partial, void *workspace, size_t workspace_bytes,
                                  cagra_pr_result *host_result, hipStream_t stream);

/*
 * One synchronous min-label propagation step on a segmented undirected graph
 * (both edge directions present). Label propagation is one of the paper's
 * applications (Section 6.1: it reads one integer label per vertex and needs no
 * activeness check); it runs as the Section 4 program with EdgeUpdate = take
 * the source's label, Merge = minimum, VertexMap = keep the smaller of the
 * merged and the own label:
 *   labels_out[v] = min(labels_in[v], min over in-neighbours u of labels_in[u])
 * The segment processing (Section 3.2) gathers minima per subgraph row into
 * partial, int32[Q] scratch; the cache-aware merge (Section 3.3) combines them
 * with int32 minimum (exact, order-free). *changed_out (device int32) = number
 * of v whose label changed. Repeated until no label changes, the labels reach
 * the smallest vertex id of each connected component.
 */
cagra_status cagra_labelprop_iter(const cagra_segments *seg, const int32_t *labels_in, int32_t *partial,
                                  int32_t *labels_out, int32_t *changed_out, void *workspace,
                                  size_t workspace_bytes, hipStream_t stream);

/*
 * Label propagation to its fixed point (the Section 4 program repeated until
 * no label changes): cagra_labelprop_iter steps from labels0, with the change
 * count read back after every check_every-th step; the loop stops at the
 * first check that reads 0, or after max_iters steps. The host loop is the one
 * of cagra_pagerank_solve: the step after a check is queued before the check
 * is read back (unless the change counts predict that the check may read 0),
 * and when the check ends the loop that step is dropped, so the labels and
 * the count are those of a loop that waited at every check. The stream is
 * synchronized before the call returns.
 *   labels0, labels1   int32[V] pair; labels0 holds the start labels on entry
 *                      (the vertex ids for connected components)
 *   partial, workspace as for cagra_labelprop_iter; changed: device int32[1]
 * The result is in labels[host_result->final_buf]. Returns CAGRA_OK when a
 * check read no change (host_result->iters counts that last step),
 * CAGRA_E_NOT_CONVERGED when max_iters steps ran without that, or the status
 * of a failed step.
 */
typedef struct {
    int32_t iters;         /* steps run, the last (unchanged) one included */
    int32_t final_buf;     /* 0 or 1: which buffer of the pair holds the result */
    int32_t changed;       /* change count of the last check read back (-1 before the first) */
} cagra_lp_result;
cagra_status cagra_labelprop_solve(const cagra_segments *seg, int32_t max_iters, int32_t check_every,
                                   int32_t *labels0, int32_t *labels1, int32_t *partial, int32_t *changed,
                                   void *workspace, size_t workspace_bytes, cagra_lp_result *host_result,
                                   hipStream_t stream);

/*
 * The fixed-point loops of cagra_pagerank_solve and cagra_labelprop_solve
 * with push-direction steps (cagra_pagerank_push_iter,
 * cagra_labelprop_push_iter): same loop, same stopping rules, same results
 * as a loop of those steps that waits at every check; the stream is
 * synchronized before the call returns. cagra_pagerank_push_solve takes
 * cagra_pr_params with contrib_type CAGRA_F32, switch_tol 0 and
 * restart_vertex -1 (the push iteration has FP32 contributions and the
 * uniform teleport); its contribution pair is float[V] and vals, workspace
 * are those of the push steps (the workspace must also hold the
 * cagra_pagerank_init temporaries). The result is in buffer
 * host_result->final_buf of each pair.
 */
cagra_status cagra_pagerank_push_solve(const cagra_graph *g, const cagra_segments *seg_t, const cagra_pr_params *params,
                                       float *rank0, float *rank1, float *contrib0, float *contrib1, double *scalars,
                                       float *vals, void *workspace, size_t workspace_bytes,
                                       cagra_pr_result *host_result, hipStream_t stream);
cagra_status cagra_labelprop_push_solve(const cagra_segments *seg_t, int32_t max_iters, int32_t check_every,
                                        int32_t *labels0, int32_t *labels1, int32_t *vals, int32_t *changed,
                                        void *workspace, size_t workspace_bytes, cagra_lp_result *host_result,
                                        hipStream_t stream);

/* ------------------------------------------------------------------------ */
/* Personalized PageRank for many restart vertices (segmented SpMM)          */
/* ------------------------------------------------------------------------ */

/* Columns per vertex row of the batched calls: vertex values are [V][64] float,
   column j of vertex v at v*64 + j; columns >= ncols are kept at zero. */
#define CAGRA_PPR_COLS 64

/* Device workspace of cagra_ppr_init / cagra_ppr_iter for these segments
   (FP64 per-column partial sums). */
size_t cagra_ppr_workspace_bytes(const cagra_segments *seg);

/*
 * Start vectors r_0(v, j) = [v == seeds[j]] for j < ncols (1 <= ncols <= 64;
 * seeds: device int32[ncols], each in [0, V)), contributions r/out_degree, and
 * per column j: scalars_out[4j] = dangling mass, [4j+2] = mass (FP64).
 */
cagra_status cagra_ppr_init(const cagra_graph *g, int32_t ncols, const int32_t *seeds, float *rank_out,
                            float *contrib_out, double *scalars_out, void *workspace, size_t workspace_bytes,
                            hipStream_t stream);

/*
 * One iteration for all columns at once: segment processing of the [V][64]
 * contributions into partial[Q][64] (rows gathered through the cache
 * hierarchy, one 256-byte source row per edge), the cache-aware merge in the
 * paper's order (subgraphs ascending, FP32), and the personalized update
 *   rank_out(v, j) = d * sum_{u->v} contrib_in(u, j) + [v == seeds[j]] * ((1-d) + d * D_j)
 * with D_j = scalars_in[4j] the dangling mass of column j (returned to the
 * seed). scalars_out per column: [4j] dangling mass, [4j+1] L1 residual,
 * [4j+2] mass. Requires seg->B <= 512 (the merge keeps B x 64 floats in LDS).
 */
cagra_status cagra_ppr_iter(const cagra_graph *g, const cagra_segments *seg, double damping, int32_t ncols,
                            const int32_t *seeds, const float *rank_in, const float *contrib_in,
                            const double *scalars_in, float *partial, float *rank_out, float *contrib_out,
                            double *scalars_out, void *workspace, size_t workspace_bytes, hipStream_t stream);

/*
 * Batched personalized PageRank to a residual threshold (the Section 4 loop,
 * every column at once): cagra_ppr_init from the seeds, then cagra_ppr_iter
 * steps until every column's L1 residual (scalars [4j+1]) read back after a
 * check is below tol. The host loop is the one of cagra_pagerank_solve (one
 * iteration queued past each check; results as if it waited at every check;
 * the stream is synchronized before the call returns).
 *   rank0, rank1, contrib0, contrib1   float[V][64] pairs (rank0 and contrib0
 *                                      receive the start vectors)
 *   scalars            double[2 * 64 * 4]: the two scalar sets of the pair
 *   seeds, partial, workspace as for cagra_ppr_iter (workspace of
 *                      cagra_ppr_workspace_bytes)
 * The result is in rank[host_result->final_buf] (and contrib[...]). Returns
 * CAGRA_OK when every column converged, CAGRA_E_NOT_CONVERGED when max_iters
 * steps ran without that (host_result still describes the last iterate), or
 * the status of a failed step.
 */
typedef struct {
    double damping;        /* d in [0, 1] */
    double tol;            /* stopping threshold on every column's L1 residual, > 0 */
    int32_t max_iters;     /* iteration cap, >= 1 */
    int32_t check_every;   /* read the residuals back every this many iterations, >= 1 */
} cagra_ppr_params;
typedef struct {
    int32_t iters;         /* iterations run */
    int32_t final_buf;     /* 0 or 1: which buffer of each pair holds the result */
    double residual;       /* largest column residual of the last read-back (inf before the first) */
} cagra_ppr_result;
cagra_status cagra_ppr_solve(const cagra_graph *g, const cagra_segments *seg, const cagra_ppr_params *params,
                             int32_t ncols, const int32_t *seeds, float *rank0, float *rank1, float *contrib0,
                             float *contrib1, double *scalars, float *partial, void *workspace,
                             size_t workspace_bytes, cagra_ppr_result *host_result, hipStream_t stream);

/* ------------------------------------------------------------------------ */
/* Many independent graphs in one launch per kernel                          */
/* ------------------------------------------------------------------------ */

/*
 * Plan for running PageRank on many graphs at once. Every graph keeps its own
 * segments (built with cagra_build_segments, N * 4 <= CAGRA_STAGE_BYTES); the
 * vectors of all graphs live in shared pools, graph i's at the running offset
 * of the earlier graphs' V (rank, contrib) and Q (partial). Persistent
 * workgroups stride over the global tile and merge-block lists, so each
 * iteration of all graphs is three kernel launches without host
 * synchronization (capturable into one HIP graph).
 */
typedef struct {
    int32_t ngraphs;
    int32_t max_k, max_B;            /* filled by cagra_multi_query */
    int64_t total_V, total_Q, total_tiles, total_blocks;
    size_t desc_bytes;
    void *desc;                      /* device, desc_bytes, caller-allocated */
    float *rank[2], *contrib[2];     /* device pools, total_V each */
    double *scalars[2];              /* device, 4 * ngraphs each: per graph the
                                        cagra_pagerank_iter scalars */
    float *partial;                  /* device, total_Q */
    double *blk;                     /* device, 4 * total_blocks */
    int32_t grid_gather, grid_merge; /* filled by cagra_multi_setup */
} cagra_multi;

/* Host only: validates the host arrays graphs[ngraphs], segs[ngraphs] (device
   pointers inside) and fills the sizes of *m. */
cagra_status cagra_multi_query(int32_t ngraphs, const cagra_graph *graphs, const cagra_segments *segs,
                               cagra_multi *m);
/* Writes the per-graph descriptors into m->desc (pools must be set);
   SYNCHRONIZES the stream once. */
cagra_status cagra_multi_setup(cagra_multi *m, const cagra_graph *graphs, const cagra_segments *segs,
                               hipStream_t stream);
/* Uniform start vectors of every graph into pools [0]. */
cagra_status cagra_multi_pagerank_start(const cagra_multi *m, hipStream_t stream);
/* One PageRank iteration (as cagra_pagerank_iter, FP32 contributions) of every
   graph: reads pools [parity], writes pools [1 - parity]. Each graph's range
   count scalars[.][3] carries over from step to step, as in cagra_pagerank_iter
   (the start vectors set it to 0). */
cagra_status cagra_multi_pagerank_step(const cagra_multi *m, int32_t parity, double damping, hipStream_t stream);

/* ------------------------------------------------------------------------ */
/* Learned warm start of the PageRank power iteration                        */
/* ------------------------------------------------------------------------ */

/* Parameters of the 3 -> 64 -> 64 -> 1 GELU network: W1[64][3], b1[64],
   W2[64][64] (row j = output j), b2[64], w3[64], b3. */
#define CAGRA_MLP_PARAMS 4481

size_t cagra_features_workspace_bytes(const cagra_segments *seg);
/*
 * Per-vertex features (row-major [V][3] float): log(1 + in-degree),
 * log(1 + out-degree), and the mean over in-neighbours u of log(1 + out-degree(u))
 * (0 without in-neighbours). The last one is a segmented pull: the segment
 * gather of log(1 + out-degree) over `seg` and an order-free merge (int64
 * fixed point, 2^-24 resolution). Requires 8*B + 8*(k+1) + 320 <= CAGRA_LDS_BYTES.
 */
cagra_status cagra_degree_features(const cagra_graph *g, const cagra_segments *seg, float *features,
                                   void *workspace, size_t workspace_bytes, hipStream_t stream);

/*
 * y[r] = network(standardized features[r]) for r < n. weights: BF16
 * [CAGRA_MLP_PARAMS]; norm: float[6] = mean[3], 1/std[3]. GELU with erf from
 * Abramowitz & Stegun 7.1.26 (|error| <= 1.5e-7); FP32 arithmetic. The 64 x 64
 * hidden product runs on the matrix cores with the BF16 weights and each FP32
 * activation split into two BF16 parts (hi + lo, within 2^-17 relative),
 * accumulated in FP32.
 */
cagra_status cagra_mlp_forward(const float *features, int64_t n, const uint16_t *weights, const float *norm,
                               float *y, hipStream_t stream);

size_t cagra_mlp_grad_workspace_bytes(void);
/*
 * Mean squared error over n rows and its gradient with respect to all
 * parameters (float[CAGRA_MLP_PARAMS]); *loss (device double). FP32
 * activations throughout. Deterministic: fixed row-to-workgroup assignment and
 * fixed-order reductions.
 */
cagra_status cagra_mlp_grad(const float *features, const float *targets, int64_t n, const uint16_t *weights,
                            const float *norm, float *grad, double *loss, void *workspace, size_t workspace_bytes,
                            hipStream_t stream);

/* One Adam step (bias-corrected; step >= 1) on FP32 master weights, which are
   then rounded to nearest even into the BF16 copy. */
cagra_status cagra_adam_step(float *master, uint16_t *weights, float *m, float *v, const float *grad, int32_t step,
                             float lr, float beta1, float beta2, float eps, hipStream_t stream);

/* Regression targets of the network: targets[v] = log(V * max(rank[v], 1e-30))
   (float[V]; the network predicts log-ranks relative to the uniform 1/V). */
cagra_status cagra_mlp_targets(const float *rank, int32_t V, float *targets, hipStream_t stream);

/* Feature standardization for cagra_mlp_forward / cagra_mlp_grad: norm (device
   float[6]) = per-column mean of features[n][3], then 1 / max(s, 1e-6) with s
   the sample standard deviation (n - 1). FP64 sums in a fixed order. */
size_t cagra_feature_norm_workspace_bytes(int64_t n);
cagra_status cagra_feature_norm(const float *features, int64_t n, float *norm, void *workspace,
                                size_t workspace_bytes, hipStream_t stream);

/* Minibatch draw `draw` of `batch` rows with replacement from (features[n][3],
   targets[n]): row i is floor(h * n / 2^64) with h = SplitMix64 of the counter
   draw * batch + i under `seed`. Deterministic; outputs features_out[batch][3],
   targets_out[batch]. */
cagra_status cagra_sample_rows(const float *features, const float *targets, int64_t n, uint64_t seed, int64_t draw,
                               int32_t batch, float *features_out, float *targets_out, hipStream_t stream);

/*
 * Learned start vector in one call: cagra_degree_features, the network on every
 * vertex (cagra_mlp_forward), and cagra_warm_start_vector, with the same
 * results bit for bit. A vertex without in-edges has the features
 * (0, log(1 + out-degree), 0), so its output depends on its out-degree alone:
 * the network runs once per out-degree below 1024 for such vertices (about half
 * of an R-MAT graph's) and every other vertex is evaluated on its own.
 * scalars_out as cagra_warm_start_vector. Requirements as cagra_degree_features.
 */
size_t cagra_learned_start_workspace_bytes(const cagra_segments *seg);
cagra_status cagra_learned_start(const cagra_graph *g, const cagra_segments *seg, const uint16_t *weights,
                                 const float *norm, float *rank0, double *scalars_out, void *workspace,
                                 size_t workspace_bytes, hipStream_t stream);

size_t cagra_warm_start_workspace_bytes(int32_t V);
/*
 * Start vector r0 = exp(y) / sum(exp(y)) over V vertices (FP64 sums, fixed
 * order). scalars_out (device double[4]): max(y), number of non-finite y,
 * sum of exp(y - max), 0. The caller falls back to the uniform start when the
 * count is non-zero or the sum is not a positive finite number.
 */
cagra_status cagra_warm_start_vector(const float *y, int32_t V, float *rank0, double *scalars_out,
                                     void *workspace, size_t workspace_bytes, hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* CAGRA_H */
