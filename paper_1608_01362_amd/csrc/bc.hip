// Betweenness centrality from sampled starts (Brandes) as level-synchronous
// segmented pulls: EdgeMap with an active frontier (Section 4). A forward level
// gathers sigma over in-edges from the vertices at depth d; a backward level
// gathers (1 + delta) / sigma over the reverse graph from the vertices at depth
// d + 1. The frontier enters as a bitmask of active segments: tiles and merge
// ranges of segments without a frontier vertex are skipped, so the sparse
// levels at both ends of a BFS cost little.
#include "common.h"

namespace cagra {

cagra_status launch_gather_active(const cagra_segments *seg, int32_t op, int32_t value_type, const void *values,
                                  void *partial, const uint32_t *seg_active, hipStream_t st);
cagra_status launch_merge_active(const cagra_segments *seg, int32_t op, const void *partial, void *out,
                                 const uint32_t *seg_active, hipStream_t st);

constexpr int kBcThreads = 256;

__global__ void k_bc_start(int32_t V, int32_t source, int32_t *__restrict__ depth, float *__restrict__ sigma,
                           float *__restrict__ delta) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= V) return;
    depth[v] = v == source ? 0 : -1;
    sigma[v] = v == source ? 1.0f : 0.0f;
    delta[v] = 0.0f;
}

__global__ void k_zero_words(uint32_t *__restrict__ w, int32_t n) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) w[i] = 0u;
}

// Marks the segment of every active vertex: one atomic per wave when the wave's
// 64 vertices lie in one segment, else one per active lane.
__device__ __forceinline__ void mark_segment(uint32_t *mask, int64_t v, int32_t N, bool active) {
    const uint64_t any = __ballot(active);
    if (!any) return;
    const int64_t v0 = v - __lane_id();
    const int32_t s0 = (int32_t)(v0 / N), s1 = (int32_t)((v0 + kWave - 1) / N);
    if (s0 == s1) {
        if (__lane_id() == 0) atomicOr(&mask[s0 >> 5], 1u << (s0 & 31));
    } else if (active) {
        const int32_t s = (int32_t)(v / N);
        atomicOr(&mask[s >> 5], 1u << (s & 31));
    }
}

// vals[u] = sigma[u] for the frontier (depth d), else 0; frontier segments marked.
__global__ __launch_bounds__(kBcThreads) void k_bc_fwd_values(int32_t V, int32_t N, int32_t d,
                                                              const int32_t *__restrict__ depth,
                                                              const float *__restrict__ sigma,
                                                              float *__restrict__ vals, uint32_t *__restrict__ mask,
                                                              int32_t *__restrict__ count) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v == 0) *count = 0;  // next frontier size, counted by k_bc_fwd_update
    const bool in = v < V && depth[v] == d;
    if (v < V) vals[v] = in ? sigma[v] : 0.0f;
    mark_segment(mask, v, N, in);
}

// Unvisited vertices reached at this level: depth d + 1, sigma = the sum.
__global__ __launch_bounds__(kBcThreads) void k_bc_fwd_update(int32_t V, int32_t d, const float *__restrict__ sums,
                                                              int32_t *__restrict__ depth,
                                                              float *__restrict__ sigma,
                                                              int32_t *__restrict__ count) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool reached = false;
    if (v < V && depth[v] < 0) {
        const float x = sums[v];
        if (x > 0.0f) {
            depth[v] = d + 1;
            sigma[v] = x;
            reached = true;
        }
    }
    const uint64_t b = __ballot(reached);
    if (__lane_id() == 0 && b) atomicAdd(count, (int32_t)__popcll(b));
}

// vals[w] = (1 + delta[w]) / sigma[w] for the vertices at depth d + 1, else 0;
// their segments (in the reverse graph's segmentation) marked.
__global__ __launch_bounds__(kBcThreads) void k_bc_bwd_values(int32_t V, int32_t N, int32_t d,
                                                              const int32_t *__restrict__ depth,
                                                              const float *__restrict__ sigma,
                                                              const float *__restrict__ delta,
                                                              float *__restrict__ vals, uint32_t *__restrict__ mask) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool in = v < V && depth[v] == d + 1;
    if (v < V) vals[v] = in ? (1.0f + delta[v]) / sigma[v] : 0.0f;
    mark_segment(mask, v, N, in);
}

// Vertices at depth d: delta = sigma * sum; the centrality of every vertex
// other than the start accumulates delta.
__global__ __launch_bounds__(kBcThreads) void k_bc_bwd_update(int32_t V, int32_t d, int32_t source,
                                                              const float *__restrict__ sums,
                                                              const int32_t *__restrict__ depth,
                                                              const float *__restrict__ sigma,
                                                              float *__restrict__ delta, float *__restrict__ bc) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= V || depth[v] != d) return;
    const float dl = sigma[v] * sums[v];
    delta[v] = dl;
    if (v != source) bc[v] += dl;
}

static unsigned blocks_for(int64_t n) { return (unsigned)ceil_div(n > 0 ? n : 1, kBcThreads); }

size_t bc_mask_words(const cagra_segments *seg) { return (size_t)ceil_div(seg->k, 32); }

cagra_status launch_bc_start(int32_t V, int32_t source, int32_t *depth, float *sigma, float *delta, hipStream_t st) {
    k_bc_start<<<blocks_for(V), kBcThreads, 0, st>>>(V, source, depth, sigma, delta);
    CAGRA_LAUNCH_CHECK();
    return CAGRA_OK;
}

cagra_status launch_bc_forward(const cagra_segments *seg, int32_t d, int32_t *depth, float *sigma, float *vals,
                               float *partial, float *sums, int32_t *count, uint32_t *mask, hipStream_t st) {
    const int32_t V = seg->V, words = (int32_t)bc_mask_words(seg);
    k_zero_words<<<(unsigned)ceil_div(words, 256), 256, 0, st>>>(mask, words);
    CAGRA_LAUNCH_CHECK();
    k_bc_fwd_values<<<blocks_for(V), kBcThreads, 0, st>>>(V, seg->N, d, depth, sigma, vals, mask, count);
    CAGRA_LAUNCH_CHECK();
    cagra_status s;
    if ((s = launch_gather_active(seg, CAGRA_SUM_F32, CAGRA_F32, vals, partial, mask, st)) != CAGRA_OK) return s;
    if ((s = launch_merge_active(seg, CAGRA_SUM_F32, partial, sums, mask, st)) != CAGRA_OK) return s;
    k_bc_fwd_update<<<blocks_for(V), kBcThreads, 0, st>>>(V, d, sums, depth, sigma, count);
    CAGRA_LAUNCH_CHECK();
    return CAGRA_OK;
}

cagra_status launch_bc_backward(const cagra_segments *seg_t, int32_t d, int32_t source, const int32_t *depth,
                                const float *sigma, float *delta, float *bc, float *vals, float *partial,
                                float *sums, uint32_t *mask, hipStream_t st) {
    const int32_t V = seg_t->V, words = (int32_t)bc_mask_words(seg_t);
    k_zero_words<<<(unsigned)ceil_div(words, 256), 256, 0, st>>>(mask, words);
    CAGRA_LAUNCH_CHECK();
    k_bc_bwd_values<<<blocks_for(V), kBcThreads, 0, st>>>(V, seg_t->N, d, depth, sigma, delta, vals, mask);
    CAGRA_LAUNCH_CHECK();
    cagra_status s;
    if ((s = launch_gather_active(seg_t, CAGRA_SUM_F32, CAGRA_F32, vals, partial, mask, st)) != CAGRA_OK) return s;
    if ((s = launch_merge_active(seg_t, CAGRA_SUM_F32, partial, sums, mask, st)) != CAGRA_OK) return s;
    k_bc_bwd_update<<<blocks_for(V), kBcThreads, 0, st>>>(V, d, source, sums, depth, sigma, delta, bc);
    CAGRA_LAUNCH_CHECK();
    return CAGRA_OK;
}

}  // namespace cagra
