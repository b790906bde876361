// C ABI entry points: host-side validation, then kernel launches.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <set>
#include <utility>
#include <vector>

#include "common.h"
#include "solve_loop.h"

namespace cagra {

cagra_status ensure_dynamic_lds(const void *fn) {
    int dev = 0;
    const hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(CAGRA_E_HIP, "hipGetDevice failed: %s", hipGetErrorString(e));
    static std::mutex mu;
    static std::set<std::pair<int, const void *>> done;  // (device, kernel) pairs already set
    std::lock_guard<std::mutex> lock(mu);
    if (done.count({dev, fn})) return CAGRA_OK;
    const cagra_status s = allow_dynamic_lds(fn);
    if (s == CAGRA_OK) done.insert({dev, fn});
    return s;
}

static thread_local char g_last_error[512] = "";

cagra_status fail(cagra_status st, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
    va_end(ap);
    return st;
}

// defined in builder.hip / gather.hip / merge.hip
size_t query_workspace_bytes(int32_t V, int64_t E, int32_t N);
cagra_status query_segments(const cagra_graph *g, cagra_segments *seg, void *ws, size_t ws_bytes, hipStream_t st);
cagra_status build_segments(const cagra_graph *g, cagra_segments *seg, void *ws, size_t ws_bytes, hipStream_t st);
bool gather_staged(int32_t N, int32_t value_type);
cagra_status cluster_workspace_bytes(int32_t V, int64_t E, size_t *bytes);
size_t bc_mask_words(const cagra_segments *seg);
cagra_status launch_bc_start(int32_t V, int32_t source, int32_t *depth, float *sigma, float *delta, hipStream_t st);
cagra_status launch_bc_forward(const cagra_segments *seg, int32_t d, int32_t *depth, float *sigma, float *vals,
                               float *partial, float *sums, int32_t *count, uint32_t *mask, hipStream_t st);
cagra_status launch_bc_backward(const cagra_segments *seg_t, int32_t d, int32_t source, const int32_t *depth,
                                const float *sigma, float *delta, float *bc, float *vals, float *partial,
                                float *sums, uint32_t *mask, hipStream_t st);
cagra_status launch_edge_values(const cagra_graph *g, const cagra_segments *seg, const float *in_values,
                                 float *seg_values, hipStream_t st);
cagra_status launch_cf_iter(const cagra_segments *seg, const float *seg_values, double gamma, double lambda,
                            const float *x_in, float *partial, float *x_out, double *sq_out, double *tile_sq,
                            hipStream_t st);
cagra_status cluster_graph(const cagra_graph *g, int32_t *perm, int32_t *in_offsets_new, int32_t *in_sources_new,
                           int32_t *outdeg_new, int32_t *hot, void *ws, size_t ws_bytes, hipStream_t st);
cagra_status launch_gather(const cagra_segments *seg, int32_t op, int32_t value_type, const void *values,
                           void *partial, hipStream_t st);
size_t merge_ordered_lds_bytes(int32_t B, int32_t op);
size_t merge_fused_lds_total(int32_t B, int32_t k, int acc_bytes);
cagra_status launch_merge(const cagra_segments *seg, int32_t op, const void *partial, void *out, hipStream_t st);
int32_t init_blocks(int32_t V);
cagra_status launch_pr_init(const cagra_graph *g, int32_t contrib_type, const float *rank, void *contrib_out,
                            double *scalars_out, void *ws, hipStream_t st);
size_t ws_blk_bytes(int32_t V, int32_t nb);
size_t ws_item_bytes(const cagra_segments *seg);
size_t ws_slot_bytes(const cagra_segments *seg);
cagra_status launch_merge_pr(const cagra_graph *g, const cagra_segments *seg, double damping, int32_t seed,
                             int32_t contrib_type,
                             const float *rank_in, const double *scalars_in, const float *partial, float *rank_out,
                             void *contrib_out, double *scalars_out, void *ws, hipStream_t st);
cagra_status launch_merge_lp(const cagra_segments *seg, const int32_t *labels_in, const int32_t *partial,
                             int32_t *labels_out, int32_t *changed_out, void *ws, hipStream_t st);

int32_t ppr_init_blocks(int32_t V);
size_t ppr_merge_lds_bytes(int32_t B);
cagra_status launch_ppr_init(const cagra_graph *g, int32_t ncols, const int32_t *seeds, float *rank_out,
                             float *contrib_out, double *scalars_out, double *blk, hipStream_t st);
cagra_status launch_ppr_iter(const cagra_graph *g, const cagra_segments *seg, double damping, int32_t ncols,
                             const int32_t *seeds, const float *rank_in, const float *contrib_in,
                             const double *scalars_in, float *partial, float *rank_out, float *contrib_out,
                             double *scalars_out, double *blk, hipStream_t st);

size_t features_ws_bytes(const cagra_segments *seg);
cagra_status launch_features(const cagra_graph *g, const cagra_segments *seg, float *feats, void *ws,
                             hipStream_t st);
cagra_status launch_mlp_forward(const float *feats, int64_t n, const uint16_t *wb, const float *norm, float *y,
                                hipStream_t st);
size_t mlp_grad_ws_bytes();
cagra_status launch_mlp_grad(const float *feats, const float *target, int64_t n, const uint16_t *wb,
                             const float *norm, float *grad, double *loss, void *ws, hipStream_t st);
cagra_status launch_adam(float *master, uint16_t *wb, float *m, float *v, const float *g, int32_t step, float lr,
                         float b1, float b2, float eps, hipStream_t st);
size_t softmax_ws_bytes(int32_t V);
cagra_status launch_targets(const float *rank, int32_t V, float *t, hipStream_t st);
size_t norm_ws_bytes(int64_t n);
cagra_status launch_feature_norm(const float *f, int64_t n, float *norm, void *ws, hipStream_t st);
cagra_status launch_sample_rows(const float *f, const float *t, int64_t n, uint64_t seed, int64_t draw, int32_t batch,
                                float *fo, float *to, hipStream_t st);
size_t learned_start_ws_bytes(const cagra_segments *seg);
cagra_status launch_learned_start(const cagra_graph *g, const cagra_segments *seg, const uint16_t *wb,
                                  const float *norm, float *rank0, double *scal, void *ws, hipStream_t st);
cagra_status launch_softmax(const float *y, int32_t V, float *r0, double *scal, void *ws, hipStream_t st);

size_t push_ws_bytes(const cagra_segments *seg);
size_t validate_ws_bytes();
cagra_status validate_graph(const cagra_graph *g, void *ws, hipStream_t st);
size_t push_expand_lds_total(int32_t B, int32_t k);
size_t push_scatter_lds_bytes(int32_t N, int acc_bytes);
int64_t push_max_pieces(const cagra_segments *seg);
cagra_status launch_pr_push(const cagra_graph *g, const cagra_segments *seg, double damping, const float *rank_in,
                            const float *contrib_in, const double *scalars_in, float *vals, float *rank_out,
                            float *contrib_out, double *scalars_out, void *workspace, hipStream_t st);
cagra_status launch_lp_push(const cagra_segments *seg, const int32_t *labels_in, int32_t *vals, int32_t *labels_out,
                            int32_t *changed_out, void *workspace, hipStream_t st);

static constexpr int32_t kMaxSegments = 32768;
static constexpr int32_t kMaxPprBlock = 512;
static constexpr int32_t kMaxMergeBlock = 16384;

static cagra_status check_graph(const cagra_graph *g, bool need_outdeg) {
    if (!g) return fail(CAGRA_E_INVALID, "graph is NULL");
    if (g->V < 1) return fail(CAGRA_E_INVALID, "V must be >= 1 (got %d)", g->V);
    if (g->E < 0) return fail(CAGRA_E_INVALID, "E must be >= 0");
    if (g->E > (int64_t)INT32_MAX - 1) return fail(CAGRA_E_OVERFLOW, "E=%lld does not fit int32", (long long)g->E);
    if (!g->in_offsets) return fail(CAGRA_E_INVALID, "in_offsets is NULL");
    if (g->E > 0 && !g->in_sources) return fail(CAGRA_E_INVALID, "in_sources is NULL");
    if (need_outdeg && !g->out_degree) return fail(CAGRA_E_INVALID, "out_degree is NULL");
    return CAGRA_OK;
}

static cagra_status check_params(const cagra_segments *seg, int32_t V) {
    if (!seg) return fail(CAGRA_E_INVALID, "segments is NULL");
    if (seg->N < 1) return fail(CAGRA_E_INVALID, "N must be >= 1 (got %d)", seg->N);
    if (seg->B < 1 || seg->B > kMaxMergeBlock)
        return fail(CAGRA_E_INVALID, "B must be in [1, %d] (got %d)", kMaxMergeBlock, seg->B);
    if (seg->tile_edges < 64) return fail(CAGRA_E_INVALID, "tile_edges must be >= 64 (got %d)", seg->tile_edges);
    int64_t k = ceil_div(V, seg->N);
    if (k > kMaxSegments) return fail(CAGRA_E_CAPACITY, "k=%lld segments exceeds %d", (long long)k, kMaxSegments);
    return CAGRA_OK;
}

// A segments struct filled by a successful build (sizes consistent, arrays present).
static cagra_status check_built(const cagra_segments *seg) {
    if (!seg) return fail(CAGRA_E_INVALID, "segments is NULL");
    if (seg->V < 1 || seg->N < 1 || seg->B < 1 || seg->k != (int32_t)ceil_div(seg->V, seg->N) ||
        seg->nb != (int32_t)ceil_div(seg->V, seg->B) || seg->Q < 0 || seg->Q > seg->E || seg->ntiles < 0 ||
        seg->max_items < seg->nb)
        return fail(CAGRA_E_INVALID, "segments sizes are inconsistent (not built?)");
    if (!seg->seg_row_begin || !seg->row_ptr || !seg->row_dst || !seg->edge_src || !seg->block_ptr ||
        !seg->tile_edge || !seg->tile_seg || !seg->tile_span_row || !seg->row_dst_lo || !seg->block_items)
        return fail(CAGRA_E_INVALID, "a segments array is NULL");
    if (((uintptr_t)seg->edge_src & 15) != 0) return fail(CAGRA_E_INVALID, "edge_src must be 16-byte aligned");
    return CAGRA_OK;
}

static size_t iter_ws_bytes(const cagra_segments *seg) {
    return ws_blk_bytes(seg->V, seg->nb) + ws_item_bytes(seg) + ws_slot_bytes(seg) + 256;
}

}  // namespace cagra

using namespace cagra;

extern "C" {

int cagra_abi_version(void) { return CAGRA_ABI_VERSION; }

const char *cagra_status_string(int status) {
    switch (status) {
        case CAGRA_OK: return "CAGRA_OK";
        case CAGRA_E_INVALID: return "CAGRA_E_INVALID";
        case CAGRA_E_OVERFLOW: return "CAGRA_E_OVERFLOW";
        case CAGRA_E_CAPACITY: return "CAGRA_E_CAPACITY";
        case CAGRA_E_BUFFER: return "CAGRA_E_BUFFER";
        case CAGRA_E_HIP: return "CAGRA_E_HIP";
        case CAGRA_E_NOT_CONVERGED: return "CAGRA_E_NOT_CONVERGED";
        case CAGRA_E_RANGE: return "CAGRA_E_RANGE";
        default: return "CAGRA_E_UNKNOWN";
    }
}

const char *cagra_last_error(void) { return g_last_error; }

int32_t cagra_max_merge_block(void) { return kMaxMergeBlock; }

cagra_status cagra_segment_edge_values(const cagra_graph *g, const cagra_segments *seg, const float *in_values,
                                       float *seg_values, hipStream_t stream) {
    cagra_status s;
    if ((s = check_graph(g, false)) != CAGRA_OK) return s;
    if ((s = check_built(seg)) != CAGRA_OK) return s;
    if (seg->V != g->V || seg->E != g->E) return fail(CAGRA_E_INVALID, "segments belong to a different graph");
    if (g->E > 0 && (!in_values || !seg_values)) return fail(CAGRA_E_INVALID, "in_values or seg_values is NULL");
    if (g->E > 0 && (const void *)in_values == (const void *)seg_values)
        return fail(CAGRA_E_INVALID, "in_values and seg_values must not alias");
    return launch_edge_values(g, seg, in_values, seg_values, stream);
}

size_t cagra_cf_workspace_bytes(const cagra_segments *seg) {
    if (!seg || seg->ntiles < 0) return 0;
    return (size_t)(seg->ntiles > 0 ? seg->ntiles : 1) * sizeof(double) + 256;
}

cagra_status cagra_cf_iter(const cagra_graph *g, const cagra_segments *seg, const float *seg_values, double gamma,
                           double lambda, const float *x_in, float *partial, float *x_out, double *sq_out,
                           void *workspace, size_t workspace_bytes, hipStream_t stream) {
    cagra_status s;
    if ((s = check_graph(g, false)) != CAGRA_OK) return s;
    if ((s = check_built(seg)) != CAGRA_OK) return s;
    if (seg->V != g->V || seg->E != g->E) return fail(CAGRA_E_INVALID, "segments belong to a different graph");
    if (seg->B > kMaxPprBlock) return fail(CAGRA_E_CAPACITY, "the CF merge needs B <= %d (got %d)", kMaxPprBlock, seg->B);
    if (!x_in || !x_out || !sq_out || (seg->Q > 0 && (!partial || !seg_values)))
        return fail(CAGRA_E_INVALID, "a vector argument is NULL");
    if ((const void *)x_in == (const void *)x_out) return fail(CAGRA_E_INVALID, "x_in and x_out must not alias");
    if (!(gamma >= 0.0) || !(lambda >= 0.0)) return fail(CAGRA_E_INVALID, "gamma and lambda must be >= 0");
    if (!workspace || workspace_bytes < cagra_cf_workspace_bytes(seg))
        return fail(CAGRA_E_BUFFER, "workspace needs %zu bytes (got %zu)", cagra_cf_workspace_bytes(seg),
                    workspace_bytes);
    return launch_cf_iter(seg, seg_values, gamma, lambda, x_in, partial, x_out, sq_out, (double *)workspace, stream);
}

size_t cagra_bc_workspace_bytes(const cagra_segments *seg) {
    if (!seg || seg->k < 1) return 0;
    return bc_mask_words(seg) * sizeof(uint32_t) + 256;
}

cagra_status cagra_bc_start(int32_t V, int32_t source, int32_t *depth, float *sigma, float *delta,
                            hipStream_t stream) {
    if (V < 1) return fail(CAGRA_E_INVALID, "V must be >= 1 (got %d)", V);
    if (source < 0 || source >= V) return fail(CAGRA_E_INVALID, "source %d outside [0, %d)", source, V);
    if (!depth || !sigma || !delta) return fail(CAGRA_E_INVALID, "depth, sigma or delta is NULL");
    return launch_bc_start(V, source, depth, sigma, delta, stream);
}

static cagra_status check_bc(const cagra_segments *seg, const void *depth, const void *sigma, const void *vals,
                             const void *partial, const void *sums, const void *workspace, size_t workspace_bytes) {
    cagra_status s;
    if ((s = check_built(seg)) != CAGRA_OK) return s;
    if (!depth || !sigma || !vals || !sums || (seg->Q > 0 && !partial))
        return fail(CAGRA_E_INVALID, "a vector argument is NULL");
    if (merge_ordered_lds_bytes(seg->B, CAGRA_SUM_F32) > CAGRA_LDS_BYTES)
        return fail(CAGRA_E_CAPACITY, "merge block B=%d too large", seg->B);
    if (!workspace || workspace_bytes < cagra_bc_workspace_bytes(seg))
        return fail(CAGRA_E_BUFFER, "workspace needs %zu bytes (got %zu)", cagra_bc_workspace_bytes(seg),
                    workspace_bytes);
    return CAGRA_OK;
}

cagra_status cagra_bc_forward_level(const cagra_segments *seg, int32_t d, int32_t *depth, float *sigma, float *vals,
                                    float *partial, float *sums, int32_t *count, void *workspace,
                                    size_t workspace_bytes, hipStream_t stream) {
    cagra_status s;
    if ((s = check_bc(seg, depth, sigma, vals, partial, sums, workspace, workspace_bytes)) != CAGRA_OK) return s;
    if (!count) return fail(CAGRA_E_INVALID, "count is NULL");
    if (d < 0) return fail(CAGRA_E_INVALID, "level %d < 0", d);
    return launch_bc_forward(seg, d, depth, sigma, vals, partial, sums, count, (uint32_t *)workspace, stream);
}

cagra_status cagra_bc_backward_level(const cagra_segments *seg_t, int32_t d, int32_t source, const int32_t *depth,
                                     const float *sigma, float *delta, float *bc, float *vals, float *partial,
                                     float *sums, void *workspace, size_t workspace_bytes, hipStream_t stream) {
    cagra_status s;
    if ((s = check_bc(seg_t, depth, sigma, vals, partial, sums, workspace, workspace_bytes)) != CAGRA_OK) return s;
    if (!delta || !bc) return fail(CAGRA_E_INVALID, "delta or bc is NULL");
    if (d < 0) return fail(CAGRA_E_INVALID, "level %d < 0", d);
    if (source < 0 || source >= seg_t->V) return fail(CAGRA_E_INVALID, "source %d outside [0, %d)", source, seg_t->V);
    return launch_bc_backward(seg_t, d, source, depth, sigma, delta, bc, vals, partial, sums, (uint32_t *)workspace,
                              stream);
}

size_t cagra_cluster_workspace_bytes(int32_t V, int64_t E) {
    if (V < 1 || E < 0 || E > (int64_t)INT32_MAX - 1) return 0;
    size_t b = 0;
    return cluster_workspace_bytes(V, E, &b) == CAGRA_OK ? b : 0;
}

int cagra_cluster(const cagra_graph *g, int32_t *perm, int32_t *in_offsets, int32_t *in_sources, int32_t *out_degree,
                  int32_t *hot, void *workspace, size_t workspace_bytes, hipStream_t stream) {
    cagra_status s;
    if ((s = check_graph(g, true)) != CAGRA_OK) return s;
    if (!perm || !in_offsets || !out_degree || (g->E > 0 && !in_sources))
        return fail(CAGRA_E_INVALID, "a clustering output array is NULL");
    if ((const void *)in_offsets == (const void *)g->in_offsets ||
        (in_sources && (const void *)in_sources == (const void *)g->in_sources) ||
        (const void *)out_degree == (const void *)g->out_degree)
        return fail(CAGRA_E_INVALID, "clustering outputs must not alias the input graph");
    if (!workspace || workspace_bytes == 0) return fail(CAGRA_E_BUFFER, "clustering workspace is NULL");
    return cluster_graph(g, perm, in_offsets, in_sources, out_degree, hot, workspace, workspace_bytes, stream);
}

int32_t cagra_edge_word_bytes(int32_t N) { return N < 1 ? 0 : (edge16(N) ? 2 : 4); }

size_t cagra_query_workspace_bytes(int32_t V, int64_t E, int32_t N) {
    if (V < 1 || N < 1 || E < 0) return 0;
    return query_workspace_bytes(V, E, N);
}

cagra_status cagra_build_segments(const cagra_graph *g, cagra_segments *seg, void *workspace,
                                  size_t workspace_bytes, hipStream_t stream) {
    cagra_status s;
    if ((s = check_graph(g, false)) != CAGRA_OK) return s;
    if ((s = check_params(seg, g->V)) != CAGRA_OK) return s;
    if (seg->row_dst == nullptr) {
        size_t need = query_workspace_bytes(g->V, g->E, seg->N);
        if (!workspace || workspace_bytes < need)
            return fail(CAGRA_E_BUFFER, "query workspace needs %zu bytes (got %zu)", need, workspace_bytes);
        return query_segments(g, seg, workspace, workspace_bytes, stream);
    }
    if (seg->V != g->V || seg->E != g->E)
        return fail(CAGRA_E_INVALID, "segments were queried for a different graph");
    if ((s = check_built(seg)) != CAGRA_OK) return s;
    if (!workspace || workspace_bytes < seg->build_workspace_bytes)
        return fail(CAGRA_E_BUFFER, "build workspace needs %zu bytes (got %zu)", seg->build_workspace_bytes,
                    workspace_bytes);
    return build_segments(g, seg, workspace, workspace_bytes, stream);
}

size_t cagra_iter_workspace_bytes(const cagra_segments *seg) {
    if (!seg || seg->V < 1 || seg->nb < 1 || seg->max_items < seg->nb) return 0;
    return iter_ws_bytes(seg);
}

cagra_status cagra_segment_gather(const cagra_segments *seg, int32_t op, int32_t value_type, const void *values,
                                  void *partial, hipStream_t stream) {
    cagra_status s;
    if ((s = check_built(seg)) != CAGRA_OK) return s;
    if (!(op == CAGRA_SUM_F32 && (value_type == CAGRA_F32 || value_type == CAGRA_BF16)) &&
        !(op == CAGRA_MIN_I32 && value_type == CAGRA_I32))
        return fail(CAGRA_E_INVALID, "unsupported gather op %d with value type %d", op, value_type);
    if (!values || (seg->Q > 0 && !partial)) return fail(CAGRA_E_INVALID, "values or partial is NULL");
    return launch_gather(seg, op, value_type, values, partial, stream);
}

cagra_status cagra_merge(const cagra_segments *seg, int32_t op, const void *partial, void *out, hipStream_t stream) {
    cagra_status s;
    if ((s = check_built(seg)) != CAGRA_OK) return s;
    if (op != CAGRA_SUM_F32 && op != CAGRA_SUM_F32_COMP && op != CAGRA_MIN_I32)
        return fail(CAGRA_E_INVALID, "unknown merge op %d", op);
    if (!out || (seg->Q > 0 && !partial)) return fail(CAGRA_E_INVALID, "partial or out is NULL");
    if (merge_ordered_lds_bytes(seg->B, op) > CAGRA_LDS_BYTES)
        return fail(CAGRA_E_CAPACITY, "merge block B=%d too large for op %d", seg->B, op);
    return launch_merge(seg, op, partial, out, stream);
}

cagra_status cagra_pagerank_init(const cagra_graph *g, int32_t contrib_type, const float *rank, void *contrib_out,
                                 double *scalars_out, void *workspace, size_t workspace_bytes, hipStream_t stream) {
    cagra_status s;
    if ((s = check_graph(g, true)) != CAGRA_OK) return s;
    if (contrib_type != CAGRA_F32 && contrib_type != CAGRA_BF16)
        return fail(CAGRA_E_INVALID, "contrib_type must be CAGRA_F32 or CAGRA_BF16");
    if (!rank || !contrib_out || !scalars_out) return fail(CAGRA_E_INVALID, "rank, contrib_out or scalars_out is NULL");
    size_t need = (size_t)init_blocks(g->V) * 4 * sizeof(double) + 256;
    if (!workspace || workspace_bytes < need)
        return fail(CAGRA_E_BUFFER, "workspace needs %zu bytes (got %zu)", need, workspace_bytes);
    return launch_pr_init(g, contrib_type, rank, contrib_out, scalars_out, workspace, stream);
}

static cagra_status check_pagerank_core(const cagra_graph *g, const cagra_segments *seg, double damping,
                                        int32_t contrib_type) {
    cagra_status s;
    if ((s = check_graph(g, true)) != CAGRA_OK) return s;
    if ((s = check_built(seg)) != CAGRA_OK) return s;
    if (seg->V != g->V || seg->E != g->E) return fail(CAGRA_E_INVALID, "segments belong to a different graph");
    if (!(damping >= 0.0 && damping <= 1.0)) return fail(CAGRA_E_INVALID, "damping must be in [0, 1]");
    if (contrib_type != CAGRA_F32 && contrib_type != CAGRA_BF16)
        return fail(CAGRA_E_INVALID, "contrib_type must be CAGRA_F32 or CAGRA_BF16");
    if (merge_fused_lds_total(seg->B, seg->k, 8) > CAGRA_LDS_BYTES)
        return fail(CAGRA_E_CAPACITY, "B=%d with k=%d exceeds the merge kernel's LDS", seg->B, seg->k);
    return CAGRA_OK;
}

static cagra_status check_pagerank(const cagra_graph *g, const cagra_segments *seg, double damping,
                                   int32_t contrib_type, size_t workspace_bytes, const void *workspace) {
    cagra_status s;
    if ((s = check_pagerank_core(g, seg, damping, contrib_type)) != CAGRA_OK) return s;
    if (!workspace || workspace_bytes < iter_ws_bytes(seg))
        return fail(CAGRA_E_BUFFER, "workspace needs %zu bytes (got %zu)", iter_ws_bytes(seg),
                    workspace_bytes);
    return CAGRA_OK;
}

static cagra_status check_restart(const cagra_graph *g, int32_t restart_vertex) {
    if (restart_vertex < -1 || restart_vertex >= g->V)
        return fail(CAGRA_E_INVALID, "restart_vertex %d outside [-1, %d)", restart_vertex, g->V);
    return CAGRA_OK;
}

cagra_status cagra_pagerank_merge(const cagra_graph *g, const cagra_segments *seg, double damping,
                                  int32_t restart_vertex, int32_t contrib_type, const float *rank_in,
                                  const double *scalars_in, const float *partial, float *rank_out, void *contrib_out,
                                  double *scalars_out, void *workspace, size_t workspace_bytes, hipStream_t stream) {
    cagra_status s;
    if ((s = check_pagerank(g, seg, damping, contrib_type, workspace_bytes, workspace)) != CAGRA_OK) return s;
    if ((s = check_restart(g, restart_vertex)) != CAGRA_OK) return s;
    if (!rank_in || !scalars_in || !rank_out || !contrib_out || !scalars_out || (seg->Q > 0 && !partial))
        return fail(CAGRA_E_INVALID, "a vector argument is NULL");
    return launch_merge_pr(g, seg, damping, restart_vertex, contrib_type, rank_in, scalars_in, partial, rank_out,
                           contrib_out, scalars_out, workspace, stream);
}

}  // extern "C"

namespace cagra {
// Arguments of one PageRank iteration apart from its workspace.
cagra_status check_pagerank_args(const cagra_graph *g, const cagra_segments *seg, double damping,
                                 int32_t restart_vertex, int32_t contrib_type, const void *rank_in,
                                 const void *contrib_in, const void *scalars_in, const void *partial,
                                 const void *rank_out, const void *contrib_out, const void *scalars_out) {
    cagra_status s;
    if ((s = check_pagerank_core(g, seg, damping, contrib_type)) != CAGRA_OK) return s;
    if ((s = check_restart(g, restart_vertex)) != CAGRA_OK) return s;
    if (!rank_in || !contrib_in || !scalars_in || !rank_out || !contrib_out || !scalars_out ||
        (seg->Q > 0 && !partial))
        return fail(CAGRA_E_INVALID, "a vector argument is NULL");
    return CAGRA_OK;
}
}  // namespace cagra

extern "C" {

cagra_status cagra_pagerank_iter(const cagra_graph *g, const cagra_segments *seg, double damping,
                                 int32_t restart_vertex, int32_t contrib_type, const float *rank_in,
                                 const void *contrib_in, const double *scalars_in, float *partial, float *rank_out,
                                 void *contrib_out, double *scalars_out, void *workspace, size_t workspace_bytes,
                                 hipStream_t stream) {
    cagra_status s;
    if ((s = check_pagerank_args(g, seg, damping, restart_vertex, contrib_type, rank_in, contrib_in, scalars_in,
                                 partial, rank_out, contrib_out, scalars_out)) != CAGRA_OK)
        return s;
    if ((s = check_pagerank(g, seg, damping, contrib_type, workspace_bytes, workspace)) != CAGRA_OK) return s;
    if ((s = launch_gather(seg, CAGRA_SUM_F32, contrib_type, contrib_in, partial, stream)) != CAGRA_OK) return s;
    return launch_merge_pr(g, seg, damping, restart_vertex, contrib_type, rank_in, scalars_in, partial, rank_out,
                           contrib_out, scalars_out, workspace, stream);
}

// Reads the four FP64 scalars of one iteration back to the host (synchronizes).
static cagra_status read_scalars(const double *d_scalars, double (&h)[4], hipStream_t stream) {
    CAGRA_HIP_CHECK(hipMemcpyAsync(h, d_scalars, sizeof(h), hipMemcpyDeviceToHost, stream));
    CAGRA_HIP_CHECK(hipStreamSynchronize(stream));
    return CAGRA_OK;
}

}  // extern "C"

namespace cagra {
// The PageRank parts of the pipelined solve: iterations of cagra_pagerank_iter
// on the buffer pairs, the residual and range count of its scalars, and the
// BF16-to-FP32 switch.
struct PageRankSolveOps {
    struct State {
        int32_t iters, iters_bf16, cur, ct;
    };
    const cagra_graph *g;
    const cagra_segments *seg;
    const cagra_pr_params *p;
    float *rank[2];
    void *contrib[2];
    double *sc[2];
    float *partial;
    void *ws;
    hipStream_t st;
    cagra_pr_result *res;
    State at{0, 0, 0, CAGRA_F32};
    bool push = false;  // push direction: seg is the reverse graph's segmentation, partial its vals

    State state() const { return at; }
    void restore(const State &s) { at = s; }
    int32_t iters() const { return at.iters; }
    cagra_status step() {
        cagra_status s;
        const int c = at.cur;
        if (push) {
            if ((s = launch_pr_push(g, seg, p->damping, rank[c], static_cast<const float *>(contrib[c]), sc[c], partial,
                                    rank[1 - c], static_cast<float *>(contrib[1 - c]), sc[1 - c], ws, st)) != CAGRA_OK)
                return s;
            at.cur = 1 - c;
            ++at.iters;
            return CAGRA_OK;
        }
        if ((s = launch_gather(seg, CAGRA_SUM_F32, at.ct, contrib[c], partial, st)) != CAGRA_OK) return s;
        if ((s = launch_merge_pr(g, seg, p->damping, p->restart_vertex, at.ct, rank[c], sc[c], partial, rank[1 - c],
                                 contrib[1 - c], sc[1 - c], ws, st)) != CAGRA_OK)
            return s;
        at.cur = 1 - c;
        ++at.iters;
        if (at.ct == CAGRA_BF16) ++at.iters_bf16;
        return CAGRA_OK;
    }
    const void *dev_check() const { return sc[at.cur]; }
    size_t check_bytes() const { return 4 * sizeof(double); }
    bool switch_pending(int32_t ct) const { return ct == CAGRA_BF16 && p->switch_tol > 0.0; }
    CheckOutcome decide(const State &a, const void *hv, double *resid, cagra_status *err) const {
        const double *h = static_cast<const double *>(hv);
        for (int c = 0; c < 4; ++c) res->scalars[c] = h[c];
        res->residual = *resid = h[1];
        if (h[3] != 0.0) {
            *err = fail(CAGRA_E_RANGE, "iteration %d: %g merge blocks held non-finite buffer values or an absolute "
                        "buffer mass beyond the exact fixed-point range", a.iters, h[3]);
            return CheckOutcome::kError;
        }
        if (h[1] < p->tol) return CheckOutcome::kConverged;
        if (switch_pending(a.ct) && h[1] < p->switch_tol) return CheckOutcome::kSwitch;
        return CheckOutcome::kContinue;
    }
    bool may_end(double pred) const {
        return pred < 2.0 * p->tol || (switch_pending(at.ct) && pred < 2.0 * p->switch_tol);
    }
    cagra_status switch_precision() {
        // finish in FP32: contributions rebuilt from the current ranks
        at.ct = CAGRA_F32;
        return launch_pr_init(g, at.ct, rank[at.cur], contrib[at.cur], sc[at.cur], ws, st);
    }
};
}  // namespace cagra

extern "C" {

cagra_status cagra_pagerank_solve(const cagra_graph *g, const cagra_segments *seg, const cagra_pr_params *p,
                                  float *rank0, float *rank1, void *contrib0, void *contrib1, double *scalars,
                                  float *partial, void *workspace, size_t workspace_bytes,
                                  cagra_pr_result *host_result, hipStream_t stream) {
    cagra_status s;
    if (!p || !host_result) return fail(CAGRA_E_INVALID, "params or host_result is NULL");
    if ((s = check_pagerank(g, seg, p->damping, p->contrib_type, workspace_bytes, workspace)) != CAGRA_OK) return s;
    if ((s = check_restart(g, p->restart_vertex)) != CAGRA_OK) return s;
    if (!(p->tol > 0.0)) return fail(CAGRA_E_INVALID, "tol must be > 0");
    if (p->max_iters < 1 || p->check_every < 1) return fail(CAGRA_E_INVALID, "max_iters and check_every must be >= 1");
    if (!(p->switch_tol >= 0.0)) return fail(CAGRA_E_INVALID, "switch_tol must be >= 0");
    if (p->switch_tol > 0.0 && p->contrib_type != CAGRA_BF16)
        return fail(CAGRA_E_INVALID, "switch_tol applies to CAGRA_BF16 contributions only");
    if (!rank0 || !rank1 || !contrib0 || !contrib1 || !scalars || (seg->Q > 0 && !partial))
        return fail(CAGRA_E_INVALID, "a vector argument is NULL");
    if (rank0 == rank1 || contrib0 == contrib1) return fail(CAGRA_E_INVALID, "the two buffers of a pair must differ");
    *host_result = cagra_pr_result{};
    PageRankSolveOps ops{g, seg, p, {rank0, rank1}, {contrib0, contrib1}, {scalars, scalars + 4}, partial, workspace,
                         stream, host_result};
    ops.at.ct = p->contrib_type;
    if ((s = launch_pr_init(g, ops.at.ct, rank0, contrib0, scalars, workspace, stream)) != CAGRA_OK) return s;
    double h[4];
    if ((s = read_scalars(scalars, h, stream)) != CAGRA_OK) return s;
    for (int c = 0; c < 4; ++c) host_result->scalars[c] = h[c];
    host_result->residual = INFINITY;
    if (h[3] != 0.0) return fail(CAGRA_E_RANGE, "the start vector holds %.0f non-finite values", h[3]);
    s = pipelined_solve(ops, p->max_iters, p->check_every, stream);
    host_result->iters = ops.at.iters;
    host_result->iters_bf16 = ops.at.iters_bf16;
    host_result->final_buf = ops.at.cur;
    if (s == CAGRA_E_NOT_CONVERGED)
        return fail(CAGRA_E_NOT_CONVERGED, "no L1 residual below %g within %d iterations (last %g)", p->tol,
                    p->max_iters, host_result->residual);
    return s;
}

cagra_status cagra_labelprop_iter(const cagra_segments *seg, const int32_t *labels_in, int32_t *partial,
                                  int32_t *labels_out, int32_t *changed_out, void *workspace,
                                  size_t workspace_bytes, hipStream_t stream) {
    cagra_status s;
    if ((s = check_built(seg)) != CAGRA_OK) return s;
    if (!labels_in || !labels_out || !changed_out || (seg->Q > 0 && !partial))
        return fail(CAGRA_E_INVALID, "a vector argument is NULL");
    if (merge_fused_lds_total(seg->B, seg->k, 4) > CAGRA_LDS_BYTES)
        return fail(CAGRA_E_CAPACITY, "B=%d with k=%d exceeds the merge kernel's LDS", seg->B, seg->k);
    if (!workspace || workspace_bytes < iter_ws_bytes(seg))
        return fail(CAGRA_E_BUFFER, "workspace needs %zu bytes (got %zu)", iter_ws_bytes(seg),
                    workspace_bytes);
    if ((s = launch_gather(seg, CAGRA_MIN_I32, CAGRA_I32, labels_in, partial, stream)) != CAGRA_OK) return s;
    return launch_merge_lp(seg, labels_in, partial, labels_out, changed_out, workspace, stream);
}

}  // extern "C"

namespace cagra {
// The label-propagation parts of the pipelined solve: steps of
// cagra_labelprop_iter on the label pair; a check converges when the step
// changed no label (its count, read back, is zero).
struct LabelpropSolveOps {
    struct State {
        int32_t iters, cur;
    };
    const cagra_segments *seg;
    int32_t *lab[2];
    int32_t *partial;
    int32_t *changed;
    void *ws;
    hipStream_t st;
    cagra_lp_result *res;
    State at{0, 0};
    bool push = false;  // push direction: seg is the reverse graph's segmentation, partial its vals

    State state() const { return at; }
    void restore(const State &s) { at = s; }
    int32_t iters() const { return at.iters; }
    cagra_status step() {
        const int c = at.cur;
        if (push) {
            cagra_status s = launch_lp_push(seg, lab[c], partial, lab[1 - c], changed, ws, st);
            if (s != CAGRA_OK) return s;
            at.cur = 1 - c;
            ++at.iters;
            return CAGRA_OK;
        }
        cagra_status s = launch_gather(seg, CAGRA_MIN_I32, CAGRA_I32, lab[c], partial, st);
        if (s != CAGRA_OK) return s;
        if ((s = launch_merge_lp(seg, lab[c], partial, lab[1 - c], changed, ws, st)) != CAGRA_OK) return s;
        at.cur = 1 - c;
        ++at.iters;
        return CAGRA_OK;
    }
    const void *dev_check() const { return changed; }
    size_t check_bytes() const { return sizeof(int32_t); }
    CheckOutcome decide(const State &, const void *hv, double *resid, cagra_status *) const {
        const int32_t n = *static_cast<const int32_t *>(hv);
        res->changed = n;
        *resid = (double)n;
        return n == 0 ? CheckOutcome::kConverged : CheckOutcome::kContinue;
    }
    bool may_end(double pred) const { return pred < 2.0; }
    cagra_status switch_precision() { return CAGRA_OK; }
};
}  // namespace cagra

extern "C" {

cagra_status cagra_labelprop_solve(const cagra_segments *seg, int32_t max_iters, int32_t check_every,
                                   int32_t *labels0, int32_t *labels1, int32_t *partial, int32_t *changed,
                                   void *workspace, size_t workspace_bytes, cagra_lp_result *host_result,
                                   hipStream_t stream) {
    cagra_status s;
    if (!host_result) return fail(CAGRA_E_INVALID, "host_result is NULL");
    if ((s = check_built(seg)) != CAGRA_OK) return s;
    if (max_iters < 1 || check_every < 1) return fail(CAGRA_E_INVALID, "max_iters and check_every must be >= 1");
    if (!labels0 || !labels1 || !changed || (seg->Q > 0 && !partial))
        return fail(CAGRA_E_INVALID, "a vector argument is NULL");
    if (labels0 == labels1) return fail(CAGRA_E_INVALID, "the two label buffers must differ");
    if (merge_fused_lds_total(seg->B, seg->k, 4) > CAGRA_LDS_BYTES)
        return fail(CAGRA_E_CAPACITY, "B=%d with k=%d exceeds the merge kernel's LDS", seg->B, seg->k);
    if (!workspace || workspace_bytes < iter_ws_bytes(seg))
        return fail(CAGRA_E_BUFFER, "workspace needs %zu bytes (got %zu)", iter_ws_bytes(seg),
                    workspace_bytes);
    *host_result = cagra_lp_result{};
    host_result->changed = -1;
    LabelpropSolveOps ops{seg, {labels0, labels1}, partial, changed, workspace, stream, host_result};
    s = pipelined_solve(ops, max_iters, check_every, stream);
    host_result->iters = ops.at.iters;
    host_result->final_buf = ops.at.cur;
    if (s == CAGRA_E_NOT_CONVERGED)
        return fail(CAGRA_E_NOT_CONVERGED, "labels still changed (%d) after %d iterations", host_result->changed,
                    max_iters);
    return s;
}

size_t cagra_features_workspace_bytes(const cagra_segments *seg) {
    if (!seg || seg->V < 1) return 0;
    return features_ws_bytes(seg);
}

cagra_status cagra_degree_features(const cagra_graph *g, const cagra_segments *seg, float *features,
                                   void *workspace, size_t workspace_bytes, hipStream_t stream) {
    cagra_status s;
    if ((s = check_graph(g, true)) != CAGRA_OK) return s;
    if ((s = check_built(seg)) != CAGRA_OK) return s;
    if (seg->V != g->V || seg->E != g->E) return fail(CAGRA_E_INVALID, "segments belong to a different graph");
    if (!features) return fail(CAGRA_E_INVALID, "features is NULL");
    if (merge_fused_lds_total(seg->B, seg->k, 8) > CAGRA_LDS_BYTES)
        return fail(CAGRA_E_CAPACITY, "B=%d with k=%d exceeds the merge kernel's LDS", seg->B, seg->k);
    if (!workspace || workspace_bytes < features_ws_bytes(seg))
        return fail(CAGRA_E_BUFFER, "workspace needs %zu bytes (got %zu)", features_ws_bytes(seg), workspace_bytes);
    return launch_features(g, seg, features, workspace, stream);
}

cagra_status cagra_mlp_forward(const float *features, int64_t n, const uint16_t *weights, const float *norm,
                               float *y, hipStream_t stream) {
    if (n < 0) return fail(CAGRA_E_INVALID, "n must be >= 0");
    if (n > 0 && (!features || !weights || !norm || !y)) return fail(CAGRA_E_INVALID, "a vector argument is NULL");
    return launch_mlp_forward(features, n, weights, norm, y, stream);
}

size_t cagra_mlp_grad_workspace_bytes(void) { return mlp_grad_ws_bytes(); }

cagra_status cagra_mlp_grad(const float *features, const float *targets, int64_t n, const uint16_t *weights,
                            const float *norm, float *grad, double *loss, void *workspace, size_t workspace_bytes,
                            hipStream_t stream) {
    if (n < 1) return fail(CAGRA_E_INVALID, "n must be >= 1");
    if (!features || !targets || !weights || !norm || !grad || !loss)
        return fail(CAGRA_E_INVALID, "a vector argument is NULL");
    if (!workspace || workspace_bytes < mlp_grad_ws_bytes())
        return fail(CAGRA_E_BUFFER, "workspace needs %zu bytes (got %zu)", mlp_grad_ws_bytes(), workspace_bytes);
    return launch_mlp_grad(features, targets, n, weights, norm, grad, loss, workspace, stream);
}

cagra_status cagra_adam_step(float *master, uint16_t *weights, float *m, float *v, const float *grad, int32_t step,
                             float lr, float beta1, float beta2, float eps, hipStream_t stream) {
    if (!master || !weights || !m || !v || !grad) return fail(CAGRA_E_INVALID, "a vector argument is NULL");
    if (step < 1) return fail(CAGRA_E_INVALID, "step must be >= 1");
    if (!(beta1 >= 0.0f && beta1 < 1.0f && beta2 >= 0.0f && beta2 < 1.0f && eps > 0.0f && lr >= 0.0f))
        return fail(CAGRA_E_INVALID, "bad Adam hyper-parameters");
    return launch_adam(master, weights, m, v, grad, step, lr, beta1, beta2, eps, stream);
}

size_t cagra_warm_start_workspace_bytes(int32_t V) { return V < 1 ? 0 : softmax_ws_bytes(V); }

cagra_status cagra_mlp_targets(const float *rank, int32_t V, float *targets, hipStream_t stream) {
    if (V < 1) return fail(CAGRA_E_INVALID, "V must be >= 1");
    if (!rank || !targets) return fail(CAGRA_E_INVALID, "rank or targets is NULL");
    return launch_targets(rank, V, targets, stream);
}

size_t cagra_feature_norm_workspace_bytes(int64_t n) { return n < 1 ? 0 : norm_ws_bytes(n); }

cagra_status cagra_feature_norm(const float *features, int64_t n, float *norm, void *workspace,
                                size_t workspace_bytes, hipStream_t stream) {
    if (n < 1) return fail(CAGRA_E_INVALID, "n must be >= 1");
    if (!features || !norm) return fail(CAGRA_E_INVALID, "features or norm is NULL");
    if (!workspace || workspace_bytes < norm_ws_bytes(n))
        return fail(CAGRA_E_BUFFER, "workspace needs %zu bytes (got %zu)", norm_ws_bytes(n), workspace_bytes);
    return launch_feature_norm(features, n, norm, workspace, stream);
}

cagra_status cagra_sample_rows(const float *features, const float *targets, int64_t n, uint64_t seed, int64_t draw,
                               int32_t batch, float *features_out, float *targets_out, hipStream_t stream) {
    if (n < 1 || batch < 0 || draw < 0) return fail(CAGRA_E_INVALID, "n must be >= 1, batch and draw >= 0");
    if (batch > 0 && (!features || !targets || !features_out || !targets_out))
        return fail(CAGRA_E_INVALID, "a vector argument is NULL");
    if (batch == 0) return CAGRA_OK;
    return launch_sample_rows(features, targets, n, seed, draw, batch, features_out, targets_out, stream);
}

size_t cagra_learned_start_workspace_bytes(const cagra_segments *seg) {
    if (!seg || seg->V < 1) return 0;
    return learned_start_ws_bytes(seg);
}

cagra_status cagra_learned_start(const cagra_graph *g, const cagra_segments *seg, const uint16_t *weights,
                                 const float *norm, float *rank0, double *scalars_out, void *workspace,
                                 size_t workspace_bytes, hipStream_t stream) {
    cagra_status s;
    if ((s = check_graph(g, true)) != CAGRA_OK) return s;
    if ((s = check_built(seg)) != CAGRA_OK) return s;
    if (seg->V != g->V || seg->E != g->E) return fail(CAGRA_E_INVALID, "segments belong to a different graph");
    if (!weights || !norm || !rank0 || !scalars_out) return fail(CAGRA_E_INVALID, "a vector argument is NULL");
    if (merge_fused_lds_total(seg->B, seg->k, 8) > CAGRA_LDS_BYTES)
        return fail(CAGRA_E_CAPACITY, "B=%d with k=%d exceeds the merge kernel's LDS", seg->B, seg->k);
    if (!workspace || workspace_bytes < learned_start_ws_bytes(seg))
        return fail(CAGRA_E_BUFFER, "workspace needs %zu bytes (got %zu)", learned_start_ws_bytes(seg),
                    workspace_bytes);
    return launch_learned_start(g, seg, weights, norm, rank0, scalars_out, workspace, stream);
}

cagra_status cagra_warm_start_vector(const float *y, int32_t V, float *rank0, double *scalars_out,
                                     void *workspace, size_t workspace_bytes, hipStream_t stream) {
    if (V < 1) return fail(CAGRA_E_INVALID, "V must be >= 1");
    if (!y || !rank0 || !scalars_out) return fail(CAGRA_E_INVALID, "a vector argument is NULL");
    if (!workspace || workspace_bytes < softmax_ws_bytes(V))
        return fail(CAGRA_E_BUFFER, "workspace needs %zu bytes (got %zu)", softmax_ws_bytes(V), workspace_bytes);
    return launch_softmax(y, V, rank0, scalars_out, workspace, stream);
}

size_t cagra_ppr_workspace_bytes(const cagra_segments *seg) {
    if (!seg || seg->V < 1) return 0;
    int64_t n = seg->nb > ppr_init_blocks(seg->V) ? seg->nb : ppr_init_blocks(seg->V);
    return (size_t)n * CAGRA_PPR_COLS * 4 * sizeof(double) + 256;
}

cagra_status cagra_ppr_init(const cagra_graph *g, int32_t ncols, const int32_t *seeds, float *rank_out,
                            float *contrib_out, double *scalars_out, void *workspace, size_t workspace_bytes,
                            hipStream_t stream) {
    cagra_status s;
    if ((s = check_graph(g, true)) != CAGRA_OK) return s;
    if (ncols < 1 || ncols > CAGRA_PPR_COLS) return fail(CAGRA_E_INVALID, "ncols must be in [1, %d]", CAGRA_PPR_COLS);
    if (!seeds || !rank_out || !contrib_out || !scalars_out) return fail(CAGRA_E_INVALID, "a vector argument is NULL");
    size_t need = (size_t)ppr_init_blocks(g->V) * CAGRA_PPR_COLS * 4 * sizeof(double) + 256;
    if (!workspace || workspace_bytes < need)
        return fail(CAGRA_E_BUFFER, "workspace needs %zu bytes (got %zu)", need, workspace_bytes);
    return launch_ppr_init(g, ncols, seeds, rank_out, contrib_out, scalars_out, (double *)workspace, stream);
}

cagra_status cagra_ppr_iter(const cagra_graph *g, const cagra_segments *seg, double damping, int32_t ncols,
                            const int32_t *seeds, const float *rank_in, const float *contrib_in,
                            const double *scalars_in, float *partial, float *rank_out, float *contrib_out,
                            double *scalars_out, void *workspace, size_t workspace_bytes, hipStream_t stream) {
    cagra_status s;
    if ((s = check_graph(g, true)) != CAGRA_OK) return s;
    if ((s = check_built(seg)) != CAGRA_OK) return s;
    if (seg->V != g->V || seg->E != g->E) return fail(CAGRA_E_INVALID, "segments belong to a different graph");
    if (!(damping >= 0.0 && damping <= 1.0)) return fail(CAGRA_E_INVALID, "damping must be in [0, 1]");
    if (ncols < 1 || ncols > CAGRA_PPR_COLS) return fail(CAGRA_E_INVALID, "ncols must be in [1, %d]", CAGRA_PPR_COLS);
    if (seg->B > kMaxPprBlock) return fail(CAGRA_E_CAPACITY, "batched merge needs B <= %d (got %d)", kMaxPprBlock, seg->B);
    if (!seeds || !rank_in || !contrib_in || !scalars_in || !rank_out || !contrib_out || !scalars_out ||
        (seg->Q > 0 && !partial))
        return fail(CAGRA_E_INVALID, "a vector argument is NULL");
    if (!workspace || workspace_bytes < cagra_ppr_workspace_bytes(seg))
        return fail(CAGRA_E_BUFFER, "workspace needs %zu bytes (got %zu)", cagra_ppr_workspace_bytes(seg),
                    workspace_bytes);
    return launch_ppr_iter(g, seg, damping, ncols, seeds, rank_in, contrib_in, scalars_in, partial, rank_out,
                           contrib_out, scalars_out, (double *)workspace, stream);
}

}  // extern "C"

namespace cagra {
// The batched personalized PageRank parts of the pipelined solve: iterations
// of cagra_ppr_iter on the buffer pairs; a check converges when every
// column's L1 residual is below tol (a NaN residual never is).
struct PprSolveOps {
    struct State {
        int32_t iters, cur;
    };
    const cagra_graph *g;
    const cagra_segments *seg;
    const cagra_ppr_params *p;
    int32_t ncols;
    const int32_t *seeds;
    float *rank[2];
    float *contrib[2];
    double *sc[2];
    float *partial;
    double *ws;
    hipStream_t st;
    cagra_ppr_result *res;
    State at{0, 0};

    State state() const { return at; }
    void restore(const State &s) { at = s; }
    int32_t iters() const { return at.iters; }
    cagra_status step() {
        const int c = at.cur;
        cagra_status s = launch_ppr_iter(g, seg, p->damping, ncols, seeds, rank[c], contrib[c], sc[c], partial,
                                         rank[1 - c], contrib[1 - c], sc[1 - c], ws, st);
        if (s != CAGRA_OK) return s;
        at.cur = 1 - c;
        ++at.iters;
        return CAGRA_OK;
    }
    const void *dev_check() const { return sc[at.cur]; }
    size_t check_bytes() const { return (size_t)ncols * 4 * sizeof(double); }
    CheckOutcome decide(const State &, const void *hv, double *resid, cagra_status *) const {
        const double *h = static_cast<const double *>(hv);
        double worst = 0.0;
        for (int j = 0; j < ncols; ++j) {
            const double r = h[j * 4 + 1];
            if (!(r <= worst)) worst = r;  // NaN sticks
            if (isnan(r)) break;
        }
        res->residual = *resid = worst;
        return worst < p->tol ? CheckOutcome::kConverged : CheckOutcome::kContinue;
    }
    bool may_end(double pred) const { return pred < 2.0 * p->tol; }
    cagra_status switch_precision() { return CAGRA_OK; }
};
}  // namespace cagra

extern "C" {

cagra_status cagra_ppr_solve(const cagra_graph *g, const cagra_segments *seg, const cagra_ppr_params *p,
                             int32_t ncols, const int32_t *seeds, float *rank0, float *rank1, float *contrib0,
                             float *contrib1, double *scalars, float *partial, void *workspace,
                             size_t workspace_bytes, cagra_ppr_result *host_result, hipStream_t stream) {
    cagra_status s;
    if (!p || !host_result) return fail(CAGRA_E_INVALID, "params or host_result is NULL");
    if ((s = check_graph(g, true)) != CAGRA_OK) return s;
    if ((s = check_built(seg)) != CAGRA_OK) return s;
    if (seg->V != g->V || seg->E != g->E) return fail(CAGRA_E_INVALID, "segments belong to a different graph");
    if (!(p->damping >= 0.0 && p->damping <= 1.0)) return fail(CAGRA_E_INVALID, "damping must be in [0, 1]");
    if (!(p->tol > 0.0)) return fail(CAGRA_E_INVALID, "tol must be > 0");
    if (p->max_iters < 1 || p->check_every < 1) return fail(CAGRA_E_INVALID, "max_iters and check_every must be >= 1");
    if (ncols < 1 || ncols > CAGRA_PPR_COLS) return fail(CAGRA_E_INVALID, "ncols must be in [1, %d]", CAGRA_PPR_COLS);
    if (seg->B > kMaxPprBlock) return fail(CAGRA_E_CAPACITY, "batched merge needs B <= %d (got %d)", kMaxPprBlock, seg->B);
    if (!seeds || !rank0 || !rank1 || !contrib0 || !contrib1 || !scalars || (seg->Q > 0 && !partial))
        return fail(CAGRA_E_INVALID, "a vector argument is NULL");
    if (rank0 == rank1 || contrib0 == contrib1) return fail(CAGRA_E_INVALID, "the two buffers of a pair must differ");
    if (!workspace || workspace_bytes < cagra_ppr_workspace_bytes(seg))
        return fail(CAGRA_E_BUFFER, "workspace needs %zu bytes (got %zu)", cagra_ppr_workspace_bytes(seg),
                    workspace_bytes);
    *host_result = cagra_ppr_result{};
    host_result->residual = INFINITY;
    PprSolveOps ops{g, seg, p, ncols, seeds, {rank0, rank1}, {contrib0, contrib1},
                    {scalars, scalars + CAGRA_PPR_COLS * 4}, partial, (double *)workspace, stream, host_result};
    if ((s = launch_ppr_init(g, ncols, seeds, rank0, contrib0, scalars, (double *)workspace, stream)) != CAGRA_OK)
        return s;
    s = pipelined_solve(ops, p->max_iters, p->check_every, stream);
    host_result->iters = ops.at.iters;
    host_result->final_buf = ops.at.cur;
    if (s == CAGRA_E_NOT_CONVERGED)
        return fail(CAGRA_E_NOT_CONVERGED, "a column's L1 residual is still %g >= %g after %d iterations",
                    host_result->residual, p->tol, p->max_iters);
    return s;
}

size_t cagra_push_workspace_bytes(const cagra_segments *seg_t) {
    if (!seg_t || seg_t->V < 1 || seg_t->N < 1 || seg_t->k < 1 || seg_t->E < 0) return 0;
    return push_ws_bytes(seg_t);
}

static cagra_status check_push(const cagra_segments *seg, int acc_bytes, const void *vals, size_t workspace_bytes,
                               const void *workspace) {
    cagra_status s;
    if ((s = check_built(seg)) != CAGRA_OK) return s;
    if (seg->N > CAGRA_LDS_BYTES || push_scatter_lds_bytes(seg->N, acc_bytes) > CAGRA_LDS_BYTES)
        return fail(CAGRA_E_CAPACITY, "push accumulators of N=%d vertices (%d bytes each) exceed the LDS", seg->N,
                    acc_bytes);
    if (push_expand_lds_total(seg->B, seg->k) > CAGRA_LDS_BYTES)
        return fail(CAGRA_E_CAPACITY, "B=%d with k=%d exceeds the expand kernel's LDS", seg->B, seg->k);
    if (push_max_pieces(seg) > INT32_MAX / 2) return fail(CAGRA_E_OVERFLOW, "too many push pieces");
    if (seg->Q > 0 && !vals) return fail(CAGRA_E_INVALID, "vals is NULL");
    if (!workspace || workspace_bytes < push_ws_bytes(seg))
        return fail(CAGRA_E_BUFFER, "workspace needs %zu bytes (got %zu)", push_ws_bytes(seg), workspace_bytes);
    return CAGRA_OK;
}

cagra_status cagra_pagerank_push_iter(const cagra_graph *g, const cagra_segments *seg_t, double damping,
                                      const float *rank_in, const float *contrib_in, const double *scalars_in,
                                      float *vals, float *rank_out, float *contrib_out, double *scalars_out,
                                      void *workspace, size_t workspace_bytes, hipStream_t stream) {
    cagra_status s;
    if ((s = check_graph(g, true)) != CAGRA_OK) return s;
    if ((s = check_push(seg_t, 8, vals, workspace_bytes, workspace)) != CAGRA_OK) return s;
    if (seg_t->V != g->V || seg_t->E != g->E)
        return fail(CAGRA_E_INVALID, "segments belong to a graph of another size");
    if (!(damping >= 0.0 && damping <= 1.0)) return fail(CAGRA_E_INVALID, "damping must be in [0, 1]");
    if (!rank_in || !contrib_in || !scalars_in || !rank_out || !contrib_out || !scalars_out)
        return fail(CAGRA_E_INVALID, "a vector argument is NULL");
    return launch_pr_push(g, seg_t, damping, rank_in, contrib_in, scalars_in, vals, rank_out, contrib_out,
                          scalars_out, workspace, stream);
}

cagra_status cagra_labelprop_push_iter(const cagra_segments *seg_t, const int32_t *labels_in, int32_t *vals,
                                       int32_t *labels_out, int32_t *changed_out, void *workspace,
                                       size_t workspace_bytes, hipStream_t stream) {
    cagra_status s;
    if ((s = check_push(seg_t, 4, vals, workspace_bytes, workspace)) != CAGRA_OK) return s;
    if (!labels_in || !labels_out || !changed_out) return fail(CAGRA_E_INVALID, "a vector argument is NULL");
    return launch_lp_push(seg_t, labels_in, vals, labels_out, changed_out, workspace, stream);
}

cagra_status cagra_pagerank_push_solve(const cagra_graph *g, const cagra_segments *seg_t, const cagra_pr_params *p,
                                       float *rank0, float *rank1, float *contrib0, float *contrib1, double *scalars,
                                       float *vals, void *workspace, size_t workspace_bytes,
                                       cagra_pr_result *host_result, hipStream_t stream) {
    cagra_status s;
    if (!p || !host_result) return fail(CAGRA_E_INVALID, "params or host_result is NULL");
    if ((s = check_graph(g, true)) != CAGRA_OK) return s;
    if ((s = check_push(seg_t, 8, vals, workspace_bytes, workspace)) != CAGRA_OK) return s;
    if (seg_t->V != g->V || seg_t->E != g->E)
        return fail(CAGRA_E_INVALID, "segments belong to a graph of another size");
    if (!(p->damping >= 0.0 && p->damping <= 1.0)) return fail(CAGRA_E_INVALID, "damping must be in [0, 1]");
    if (!(p->tol > 0.0)) return fail(CAGRA_E_INVALID, "tol must be > 0");
    if (p->max_iters < 1 || p->check_every < 1) return fail(CAGRA_E_INVALID, "max_iters and check_every must be >= 1");
    if (p->contrib_type != CAGRA_F32 || p->switch_tol != 0.0 || p->restart_vertex != -1)
        return fail(CAGRA_E_INVALID, "the push solve runs FP32 contributions, no switch, uniform teleport");
    if (!rank0 || !rank1 || !contrib0 || !contrib1 || !scalars)
        return fail(CAGRA_E_INVALID, "a vector argument is NULL");
    if (rank0 == rank1 || contrib0 == contrib1) return fail(CAGRA_E_INVALID, "the two buffers of a pair must differ");
    const size_t need_init = (size_t)init_blocks(g->V) * 4 * sizeof(double) + 256;
    if (workspace_bytes < need_init)
        return fail(CAGRA_E_BUFFER, "workspace needs %zu bytes (got %zu)", need_init, workspace_bytes);
    *host_result = cagra_pr_result{};
    PageRankSolveOps ops{g, seg_t, p, {rank0, rank1}, {contrib0, contrib1}, {scalars, scalars + 4}, vals, workspace,
                         stream, host_result};
    ops.push = true;
    if ((s = launch_pr_init(g, CAGRA_F32, rank0, contrib0, scalars, workspace, stream)) != CAGRA_OK) return s;
    double h[4];
    if ((s = read_scalars(scalars, h, stream)) != CAGRA_OK) return s;
    for (int c = 0; c < 4; ++c) host_result->scalars[c] = h[c];
    host_result->residual = INFINITY;
    if (h[3] != 0.0) return fail(CAGRA_E_RANGE, "the start vector holds %.0f non-finite values", h[3]);
    s = pipelined_solve(ops, p->max_iters, p->check_every, stream);
    host_result->iters = ops.at.iters;
    host_result->final_buf = ops.at.cur;
    if (s == CAGRA_E_NOT_CONVERGED)
        return fail(CAGRA_E_NOT_CONVERGED, "no L1 residual below %g within %d iterations (last %g)", p->tol,
                    p->max_iters, host_result->residual);
    return s;
}

cagra_status cagra_labelprop_push_solve(const cagra_segments *seg_t, int32_t max_iters, int32_t check_every,
                                        int32_t *labels0, int32_t *labels1, int32_t *vals, int32_t *changed,
                                        void *workspace, size_t workspace_bytes, cagra_lp_result *host_result,
                                        hipStream_t stream) {
    cagra_status s;
    if (!host_result) return fail(CAGRA_E_INVALID, "host_result is NULL");
    if ((s = check_push(seg_t, 4, vals, workspace_bytes, workspace)) != CAGRA_OK) return s;
    if (max_iters < 1 || check_every < 1) return fail(CAGRA_E_INVALID, "max_iters and check_every must be >= 1");
    if (!labels0 || !labels1 || !changed) return fail(CAGRA_E_INVALID, "a vector argument is NULL");
    if (labels0 == labels1) return fail(CAGRA_E_INVALID, "the two label buffers must differ");
    *host_result = cagra_lp_result{};
    host_result->changed = -1;
    LabelpropSolveOps ops{seg_t, {labels0, labels1}, vals, changed, workspace, stream, host_result};
    ops.push = true;
    s = pipelined_solve(ops, max_iters, check_every, stream);
    host_result->iters = ops.at.iters;
    host_result->final_buf = ops.at.cur;
    if (s == CAGRA_E_NOT_CONVERGED)
        return fail(CAGRA_E_NOT_CONVERGED, "labels still changed (%d) after %d iterations", host_result->changed,
                    max_iters);
    return s;
}

size_t cagra_validate_workspace_bytes(void) { return validate_ws_bytes(); }

cagra_status cagra_validate_graph(const cagra_graph *g, void *workspace, size_t workspace_bytes,
                                  hipStream_t stream) {
    cagra_status s;
    if ((s = check_graph(g, false)) != CAGRA_OK) return s;
    if (!workspace || workspace_bytes < validate_ws_bytes())
        return fail(CAGRA_E_BUFFER, "workspace needs %zu bytes (got %zu)", validate_ws_bytes(), workspace_bytes);
    return validate_graph(g, workspace, stream);
}

}  // extern "C"
