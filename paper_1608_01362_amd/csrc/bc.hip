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

// The vertex kernels give each workgroup a contiguous span of vertices. The
// segments of its frontier vertices are first marked in an LDS bitmask that
// covers only the span's segments, then OR-ed into the global mask, one atomic
// per non-zero word; the new-frontier count is reduced in the workgroup and
// added once. (One global atomic per wave on a handful of words serialises:
// half a million of them took 1.5-1.9 ms per level at scale 25.)
constexpr int kBcSpan = 16384;                    // vertices per workgroup
constexpr int kBcMaskWords = kBcSpan / 32 + 2;    // segments of a span, in 32-bit words, for N >= 1

struct SpanMask {
    int64_t v0, v1;     // the workgroup's vertices [v0, v1)
    int32_t w_lo, w_hi; // global mask words covering their segments
};

__device__ __forceinline__ SpanMask span_begin(int32_t V, int32_t N, uint32_t *lmask) {
    SpanMask m;
    m.v0 = (int64_t)blockIdx.x * kBcSpan;
    m.v1 = m.v0 + kBcSpan < V ? m.v0 + kBcSpan : V;
    m.w_lo = (int32_t)(m.v0 / N) >> 5;
    m.w_hi = (int32_t)((m.v1 - 1) / N) >> 5;
    for (int i = threadIdx.x; i <= m.w_hi - m.w_lo; i += kBcThreads) lmask[i] = 0u;
    __syncthreads();
    return m;
}

// Marks v's segment in the span's LDS mask: one LDS atomic per wave when the
// wave's active vertices share a segment.
__device__ __forceinline__ void mark_segment(uint32_t *lmask, int32_t w_lo, int64_t v, int32_t N, bool active) {
    const uint64_t any = __ballot(active);
    if (!any) return;
    const int32_t s = active ? (int32_t)(v / N) : 0;
    const int first = (int)__builtin_ctzll(any);
    const int32_t s0 = __builtin_amdgcn_readlane(s, first);
    if (__ballot(active && s != s0) == 0) {
        if (__lane_id() == first) atomicOr(&lmask[(s0 >> 5) - w_lo], 1u << (s0 & 31));
    } else if (active) {
        atomicOr(&lmask[(s >> 5) - w_lo], 1u << (s & 31));
    }
}

__device__ __forceinline__ void span_flush(const SpanMask &m, const uint32_t *lmask, uint32_t *mask) {
    __syncthreads();
    for (int i = threadIdx.x; i <= m.w_hi - m.w_lo; i += kBcThreads) {
        const uint32_t bits = lmask[i];
        if (bits) atomicOr(&mask[m.w_lo + i], bits);
    }
}

// vals[u] = sigma[u] for the frontier (depth d), else 0; frontier segments marked.
__global__ __launch_bounds__(kBcThreads) void k_bc_fwd_values(int32_t V, int32_t N, int32_t d,
                                                              const int32_t *__restrict__ depth,
                                                              const float *__restrict__ sigma,
                                                              float *__restrict__ vals, uint32_t *__restrict__ mask,
                                                              int32_t *__restrict__ count) {
    __shared__ uint32_t lmask[kBcMaskWords];
    const SpanMask m = span_begin(V, N, lmask);
    if (blockIdx.x == 0 && threadIdx.x == 0) *count = 0;  // next frontier size, counted by k_bc_fwd_update
    for (int64_t v0 = m.v0; v0 < m.v1; v0 += kBcThreads) {
        const int64_t v = v0 + threadIdx.x;
        const bool in = v < m.v1 && depth[v] == d;
        if (v < m.v1) vals[v] = in ? sigma[v] : 0.0f;
        mark_segment(lmask, m.w_lo, v, N, in);
    }
    span_flush(m, lmask, mask);
}

// Unvisited vertices reached at this level: depth d + 1, sigma = the sum.
__global__ __launch_bounds__(kBcThreads) void k_bc_fwd_update(int32_t V, int32_t d, const float *__restrict__ sums,
                                                              int32_t *__restrict__ depth,
                                                              float *__restrict__ sigma,
                                                              int32_t *__restrict__ count) {
    __shared__ int32_t red[kBcThreads / kWave];
    const int64_t v0 = (int64_t)blockIdx.x * kBcSpan;
    const int64_t v1 = v0 + kBcSpan < V ? v0 + kBcSpan : V;
    int32_t reached = 0;
    for (int64_t v = v0 + threadIdx.x; v < v1; v += kBcThreads) {
        if (depth[v] < 0) {
            const float x = sums[v];
            if (x > 0.0f) {
                depth[v] = d + 1;
                sigma[v] = x;
                ++reached;
            }
        }
    }
    for (int o = 32; o >= 1; o >>= 1) reached += __shfl_down(reached, o, 64);
    if (__lane_id() == 0) red[threadIdx.x >> 6] = reached;
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t t = 0;
        for (int i = 0; i < kBcThreads / kWave; ++i) t += red[i];
        if (t) atomicAdd(count, t);
    }
}

// vals[w] = (1 + delta[w]) / sigma[w] for the vertices at depth d + 1, else 0;
// their segments (in the reverse graph's segmentation) marked.
__global__ __launch_bounds__(kBcThreads) void k_bc_bwd_values(int32_t V, int32_t N, int32_t d,
                                                              const int32_t *__restrict__ depth,
                                                              const float *__restrict__ sigma,
                                                              const float *__restrict__ delta,
                                                              float *__restrict__ vals, uint32_t *__restrict__ mask) {
    __shared__ uint32_t lmask[kBcMaskWords];
    const SpanMask m = span_begin(V, N, lmask);
    for (int64_t v0 = m.v0; v0 < m.v1; v0 += kBcThreads) {
        const int64_t v = v0 + threadIdx.x;
        const bool in = v < m.v1 && depth[v] == d + 1;
        if (v < m.v1) vals[v] = in ? (1.0f + delta[v]) / sigma[v] : 0.0f;
        mark_segment(lmask, m.w_lo, v, N, in);
    }
    span_flush(m, lmask, mask);
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

static unsigned spans_for(int64_t V) { return (unsigned)ceil_div(V > 0 ? V : 1, kBcSpan); }

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
    k_bc_fwd_values<<<spans_for(V), kBcThreads, 0, st>>>(V, seg->N, d, depth, sigma, vals, mask, count);
    CAGRA_LAUNCH_CHECK();
    cagra_status s;
    if ((s = launch_gather_active(seg, CAGRA_SUM_F32, CAGRA_F32, vals, partial, mask, st)) != CAGRA_OK) return s;
    if ((s = launch_merge_active(seg, CAGRA_SUM_F32, partial, sums, mask, st)) != CAGRA_OK) return s;
    k_bc_fwd_update<<<spans_for(V), kBcThreads, 0, st>>>(V, d, sums, depth, sigma, count);
    CAGRA_LAUNCH_CHECK();
    return CAGRA_OK;
}

cagra_status launch_bc_backward(const cagra_segments *seg_t, int32_t d, int32_t source, const int32_t *depth,
                                const float *sigma, float *delta, float *bc, float *vals, float *partial,
                                float *sums, uint32_t *mask, hipStream_t st) {
    const int32_t V = seg_t->V, words = (int32_t)bc_mask_words(seg_t);
    k_zero_words<<<(unsigned)ceil_div(words, 256), 256, 0, st>>>(mask, words);
    CAGRA_LAUNCH_CHECK();
    k_bc_bwd_values<<<spans_for(V), kBcThreads, 0, st>>>(V, seg_t->N, d, depth, sigma, delta, vals, mask);
    CAGRA_LAUNCH_CHECK();
    cagra_status s;
    if ((s = launch_gather_active(seg_t, CAGRA_SUM_F32, CAGRA_F32, vals, partial, mask, st)) != CAGRA_OK) return s;
    if ((s = launch_merge_active(seg_t, CAGRA_SUM_F32, partial, sums, mask, st)) != CAGRA_OK) return s;
    k_bc_bwd_update<<<blocks_for(V), kBcThreads, 0, st>>>(V, d, source, sums, depth, sigma, delta, bc);
    CAGRA_LAUNCH_CHECK();
    return CAGRA_OK;
}

}  // namespace cagra
