// Collaborative filtering on a rating graph through segmenting: the edge
// update reads the source's and the destination's latent vectors (the old
// destination value of Section 4's interface), EdgeUpdate (r - <x_u, x_v>) x_u,
// Merge = vector sum, VertexUpdate x_v + gamma (g_v - lambda x_v): gradient
// descent on 1/2 sum_ratings (r - <x_u, x_i>)^2 + lambda/2 sum |x|^2.
//
// Layout as for batched personalized PageRank: [V][64] FP32 vertex vectors.
// In the gather a 16-lane group handles one edge at a time, lane i owning
// factors 4i..4i+3, so each source row is one 16-byte load per lane and each
// buffer row one 16-byte store per lane; the dot product of an edge is four
// FMAs and a DPP reduction across the group's 16 lanes. In the merge lane j of
// a wave owns factor j. Segments are sized for L2 or the Infinity Cache
// (256 bytes per vertex). Edge values travel in the segmented edge order,
// produced once by k_edge_values.
#include "common.h"
#include "rowgroup.h"

namespace cagra {

constexpr int kCfK = CAGRA_CF_FACTORS;
constexpr int kCfWaves = CAGRA_TILE_WAVES;
constexpr int kCfThreads = kCfWaves * kWave;
constexpr int kCfMergeBatch = 8;    // merge rows / vertices per wave whose loads are in flight together
constexpr int kEdgesPerThread = 16;  // edge-value permutation

static_assert(kCfK == kWave, "one factor per lane");

// ---------------------------------------------------------------- edge values

// Last r in [lo, hi) with a[r] <= x (a ascending, a[lo] <= x).
__device__ __forceinline__ int32_t last_le(const int32_t *a, int32_t lo, int32_t hi, int64_t x) {
    while (hi - lo > 1) {
        const int32_t mid = lo + ((hi - lo) >> 1);
        if ((int64_t)a[mid] <= x) lo = mid;
        else hi = mid;
    }
    return lo;
}

// First r in [lo, hi) with a[r] >= x (hi if none).
__device__ __forceinline__ int32_t first_ge(const int32_t *a, int32_t lo, int32_t hi, int64_t x) {
    while (lo < hi) {
        const int32_t mid = lo + ((hi - lo) >> 1);
        if ((int64_t)a[mid] < x) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// seg_values[p] = in_values[e], p = position of in-edge e (CSC order) in the
// segmented edge order: row r = (subgraph of the source, destination), p =
// row_ptr[r] + rank of e among the row's edges (sources ascending in both).
__global__ void k_edge_values(const int32_t *__restrict__ in_offsets, const int32_t *__restrict__ in_sources,
                              int32_t V, int64_t E, int32_t N, const int32_t *__restrict__ seg_row_begin,
                              const int32_t *__restrict__ row_ptr, const int32_t *__restrict__ row_dst,
                              const float *__restrict__ in_values, float *__restrict__ seg_values) {
    const int64_t e0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * kEdgesPerThread;
    if (e0 >= E) return;
    const int64_t e1 = e0 + kEdgesPerThread < E ? e0 + kEdgesPerThread : E;
    int32_t v = last_le(in_offsets, 0, V, e0);  // non-empty row holding e0
    int32_t run_s = -1, run_start = 0, row = 0;
    for (int64_t e = e0; e < e1; ++e) {
        while ((int64_t)in_offsets[v + 1] <= e) {
            ++v;
            run_s = -1;
        }
        const int32_t s = in_sources[e] / N;
        if (s != run_s) {  // first edge of this (segment, destination) run seen by the thread
            run_s = s;
            run_start = first_ge(in_sources, in_offsets[v], in_offsets[v + 1], (int64_t)s * N);
            row = first_ge(row_dst, seg_row_begin[s], seg_row_begin[s + 1], v);
        }
        seg_values[(int64_t)row_ptr[row] + (e - run_start)] = in_values[e];
    }
}

cagra_status launch_edge_values(const cagra_graph *g, const cagra_segments *seg, const float *in_values,
                                 float *seg_values, hipStream_t st) {
    if (g->E == 0) return CAGRA_OK;
    const int64_t threads = ceil_div(g->E, kEdgesPerThread);
    k_edge_values<<<(unsigned)ceil_div(threads, 256), 256, 0, st>>>(g->in_offsets, g->in_sources, g->V, g->E, seg->N,
                                                                    seg->seg_row_begin, seg->row_ptr, seg->row_dst,
                                                                    in_values, seg_values);
    CAGRA_LAUNCH_CHECK();
    return CAGRA_OK;
}

// ---------------------------------------------------------------- gather

constexpr int kCfGroups = kCfWaves * kGroupsPerWave;
constexpr int kGroupBatch = 4;  // edges per window: source rows a group loads together
static_assert(kCfK == kGroup * 4, "four factors per lane of a group");

// Sum over the 16 lanes of a DPP row, returned to each of them: pairs, quads
// (quad_perm), halves (row_half_mirror), the row (row_mirror).
__device__ __forceinline__ float row16_sum(float x) {
    x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0xB1, 0xf, 0xf, false));   // [1,0,3,2]
    x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x4E, 0xf, 0xf, false));   // [2,3,0,1]
    x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x141, 0xf, 0xf, false));  // half mirror
    x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x140, 0xf, 0xf, false));  // mirror
    return x;
}

__device__ __forceinline__ float dot4(float4 a, float4 b) {
    return fmaf(a.w, b.w, fmaf(a.z, b.z, fmaf(a.y, b.y, a.x * b.x)));
}

// One tile per workgroup; each wave takes an equal share of the tile's edges
// and each of its four 16-lane groups an equal part of the share, walked one
// edge at a time (lane i holds factors 4i..4i+3). A row's partial gradient is
// written when the row closes inside the part; rows that continue across parts
// are completed after a barrier in part order. The row open at a part's start
// is the share's open row advanced by the row starts before the part.
template <typename W>
__global__ __launch_bounds__(kCfThreads) void k_cf_gather(
    const W *__restrict__ edge_src, const float *__restrict__ vals, const int32_t *__restrict__ tile_edge,
    const int32_t *__restrict__ tile_seg, const int32_t *__restrict__ span_row, const int32_t *__restrict__ row_dst,
    const float *__restrict__ X, int32_t N, int32_t ntiles, float *__restrict__ partial,
    double *__restrict__ tile_sq) {
    __shared__ float4 fix_head[kCfGroups][kGroup];
    __shared__ float4 fix_last[kCfGroups][kGroup];
    __shared__ int32_t fix_row[kCfGroups];
    __shared__ int32_t fix_has[kCfGroups];
    __shared__ double red_sq[kCfGroups];

    const int t = xcd_remap(blockIdx.x, ntiles);
    const int64_t e0 = tile_edge[t], e1 = tile_edge[t + 1];
    if (e0 >= e1) {  // an empty tile (uniform over the workgroup): nothing to read
        if (threadIdx.x == 0) tile_sq[t] = 0.0;
        return;
    }
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int g = lane >> 4, sub = lane & 15, G = w * kGroupsPerWave + g;
    const int64_t vbase = (int64_t)tile_seg[t] * N;
    const int64_t sl = (e1 - e0 + kCfWaves - 1) / kCfWaves;
    int64_t w0 = e0 + w * sl;
    if (w0 > e1) w0 = e1;
    int64_t w1 = w0 + sl;
    if (w1 > e1) w1 = e1;
    const GroupPart part = group_part<W>(edge_src, w0, w1, g, lane);
    const int64_t a = part.a, b = part.b, gl = part.len;
    const int32_t before = part.before;
    int32_t row = span_row[(int64_t)t * kCfWaves + w] - 1 + before;  // row open at the part's start
    int32_t seen = 0;
    float4 acc = make_float4(0.0f, 0.0f, 0.0f, 0.0f), xv = acc;
    float sqf = 0.0f;
    double sq = 0.0;
    const float4 *X4 = reinterpret_cast<const float4 *>(X);
    // the part starts inside a row (never the case for the tile's first part: tiles start on rows)
    if (a < b && !((uint32_t)edge_src[a] & EdgeWord<W>::kFlag)) xv = X4[(int64_t)row_dst[row] * kGroup + sub];
    const float4 *xs = X4 + vbase * kGroup + sub;

    // lane j < kGroupBatch of the group holds the word and rating of edge
    // o + j of the current window; the next window's are loaded one window ahead
    static_assert(kGroupBatch == 4, "windows of four edges (group_window_edge, group_bcast4)");
    int64_t ecur = group_window_edge(part, 0, sub, e0, e1);
    int32_t word = (int32_t)(uint32_t)edge_src[ecur];
    float val = vals[ecur];
    for (int64_t o = 0; o < gl; o += kGroupBatch) {
        const int64_t enxt = group_window_edge(part, o + kGroupBatch, sub, e0, e1);
        const int32_t word_n = (int32_t)(uint32_t)edge_src[enxt];
        const float val_n = vals[enxt];
        uint32_t wv[kGroupBatch];
        float rv[kGroupBatch];
        float4 x[kGroupBatch];
        const int32_t vi = __float_as_int(val);
#pragma unroll
        for (int j = 0; j < kGroupBatch; ++j) {
            wv[j] = (uint32_t)group_bcast4(word, j);
            rv[j] = __int_as_float(group_bcast4(vi, j));
            x[j] = xs[(int64_t)(wv[j] & EdgeWord<W>::kIndex) * kGroup];
        }
#pragma unroll
        for (int j = 0; j < kGroupBatch; ++j) {
            if (a + o + j < b) {
                if (wv[j] & EdgeWord<W>::kFlag) {  // a row starts: the open row is complete
                    if (seen) reinterpret_cast<float4 *>(partial)[(int64_t)row * kGroup + sub] = acc;
                    else fix_head[G][sub] = acc;  // the part's head: the row open at its start
                    seen = 1;
                    ++row;
                    acc = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                    xv = X4[(int64_t)row_dst[row] * kGroup + sub];
                }
                const float err = rv[j] - row16_sum(dot4(x[j], xv));
                acc.x = fmaf(err, x[j].x, acc.x);
                acc.y = fmaf(err, x[j].y, acc.y);
                acc.z = fmaf(err, x[j].z, acc.z);
                acc.w = fmaf(err, x[j].w, acc.w);
                sqf = fmaf(err, err, sqf);
            }
        }
        sq += (double)sqf;  // FP32 over at most kGroupBatch errors, FP64 across windows
        sqf = 0.0f;
        word = word_n;
        val = val_n;
    }
    if (!seen) fix_head[G][sub] = acc;  // no row closed: all of it continues the open row
    fix_last[G][sub] = acc;
    if (sub == 0) {
        fix_row[G] = row;
        fix_has[G] = seen;
        red_sq[G] = sq;
    }
    __syncthreads();
    if (fix_has[G]) {
        float4 tot = fix_last[G][sub];
        for (int x2 = G + 1; x2 < kCfGroups; ++x2) {
            const float4 h = fix_head[x2][sub];
            tot.x += h.x;
            tot.y += h.y;
            tot.z += h.z;
            tot.w += h.w;
            if (fix_has[x2]) break;
        }
        reinterpret_cast<float4 *>(partial)[(int64_t)fix_row[G] * kGroup + sub] = tot;
    }
    if (threadIdx.x == 0) {
        double s2 = 0.0;
        for (int x2 = 0; x2 < kCfGroups; ++x2) s2 += red_sq[x2];
        tile_sq[t] = s2;
    }
}

// ---------------------------------------------------------------- merge + update

// Paper-order merge of block b (subgraphs ascending; within a subgraph the
// waves take distinct rows, hence distinct destinations), then
// x_v' = x_v + gamma * (g_v - lambda * x_v).
__global__ __launch_bounds__(kCfThreads) void k_merge_cf(const int32_t *__restrict__ row_dst,
                                                         const int32_t *__restrict__ block_ptr,
                                                         const float *__restrict__ partial, int32_t V, int32_t k,
                                                         int32_t B, int32_t nb, float gamma, float lambda,
                                                         const float *__restrict__ x_in, float *__restrict__ x_out) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    float *acc = reinterpret_cast<float *>(smem);  // [B][kCfK]
    const int b = xcd_remap(blockIdx.x, nb);
    const int64_t vb = (int64_t)b * B;
    const int32_t nv = (int32_t)((int64_t)V - vb < B ? (int64_t)V - vb : B);
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    for (int i = threadIdx.x; i < nv * kCfK; i += kCfThreads) acc[i] = 0.0f;
    __syncthreads();
    // kCfMergeBatch rows (then vertices) per wave and pass, their loads issued
    // before any is used (past the range: its first row again, unused); a
    // subgraph's rows have distinct destinations, and the barrier after each
    // subgraph keeps the subgraphs in ascending order for every destination
    for (int32_t s = 0; s < k; ++s) {
        const int32_t lo = block_ptr[(int64_t)b * k + s], hi = block_ptr[(int64_t)(b + 1) * k + s];
        for (int32_t i0 = lo + w; i0 < hi; i0 += kCfWaves * kCfMergeBatch) {
            int32_t d[kCfMergeBatch];
            float x[kCfMergeBatch];
#pragma unroll
            for (int j = 0; j < kCfMergeBatch; ++j) {
                const int32_t i = i0 + j * kCfWaves;
                const int32_t ii = i < hi ? i : lo;
                d[j] = row_dst[ii];
                x[j] = partial[(int64_t)ii * kCfK + lane];
            }
#pragma unroll
            for (int j = 0; j < kCfMergeBatch; ++j)
                if (i0 + j * kCfWaves < hi) acc[(int32_t)(d[j] - vb) * kCfK + lane] += x[j];
        }
        __syncthreads();
    }
    for (int i0 = w; i0 < nv; i0 += kCfWaves * kCfMergeBatch) {
        float xo[kCfMergeBatch];
#pragma unroll
        for (int j = 0; j < kCfMergeBatch; ++j) {
            const int i = i0 + j * kCfWaves;
            xo[j] = x_in[(vb + (i < nv ? i : 0)) * kCfK + lane];
        }
#pragma unroll
        for (int j = 0; j < kCfMergeBatch; ++j) {
            const int i = i0 + j * kCfWaves;
            if (i >= nv) break;
            x_out[(vb + i) * kCfK + lane] = xo[j] + gamma * (acc[i * kCfK + lane] - lambda * xo[j]);
        }
    }
}

// Fixed-order sum of the tiles' squared errors.
__global__ __launch_bounds__(256) void k_sum_tiles(const double *__restrict__ tile_sq, int32_t n,
                                                   double *__restrict__ out) {
    __shared__ double red[4];
    double a = 0.0;
    for (int32_t j = threadIdx.x; j < n; j += 256) a += tile_sq[j];
    a = block_sum_f64<256>(a, red);
    if (threadIdx.x == 0) out[0] = a;
}

size_t cf_merge_lds_bytes(int32_t B) { return (size_t)B * kCfK * sizeof(float); }

cagra_status launch_cf_iter(const cagra_segments *seg, const float *seg_values, double gamma, double lambda,
                            const float *x_in, float *partial, float *x_out, double *sq_out, double *tile_sq,
                            hipStream_t st) {
    if (seg->ntiles > 0) {
        if (edge16(seg->N))
            k_cf_gather<uint16_t><<<seg->ntiles, kCfThreads, 0, st>>>(
                static_cast<const uint16_t *>(seg->edge_src), seg_values, seg->tile_edge, seg->tile_seg,
                seg->tile_span_row, seg->row_dst, x_in, seg->N, seg->ntiles, partial, tile_sq);
        else
            k_cf_gather<uint32_t><<<seg->ntiles, kCfThreads, 0, st>>>(
                static_cast<const uint32_t *>(seg->edge_src), seg_values, seg->tile_edge, seg->tile_seg,
                seg->tile_span_row, seg->row_dst, x_in, seg->N, seg->ntiles, partial, tile_sq);
        CAGRA_LAUNCH_CHECK();
    }
    if (cagra_status a_ = ensure_dynamic_lds((const void *)k_merge_cf)) return a_;
    k_merge_cf<<<seg->nb, kCfThreads, cf_merge_lds_bytes(seg->B), st>>>(
        seg->row_dst, seg->block_ptr, partial, seg->V, seg->k, seg->B, seg->nb, (float)gamma, (float)lambda, x_in,
        x_out);
    CAGRA_LAUNCH_CHECK();
    k_sum_tiles<<<1, 256, 0, st>>>(tile_sq, seg->ntiles, sq_out);
    CAGRA_LAUNCH_CHECK();
    return CAGRA_OK;
}

}  // namespace cagra
