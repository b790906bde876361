// Personalized PageRank for many restart vertices at once: the segmented pull
// of Sections 3.2-3.3 applied to a [V x 64] block of vertex values (a segmented
// sparse-times-dense product). Lane j of a wave owns column j, so every gathered
// source row is one 256-byte load and every buffer row one 256-byte store.
//
// With 256 bytes per vertex, a segment that fits LDS would hold only 512
// vertices and q would approach the average degree; the natural segment sizes
// here are L2- or Infinity-Cache-sized (Section 3.4's trade-off with a larger
// vertex record), and the gathers read whole cache lines through that level.
//
// The merge keeps the paper's order exactly: for each block of destinations,
// subgraphs in ascending order, each subgraph's rows spread over the waves
// (distinct destinations), FP32 accumulators in LDS.
#include <math.h>

#include "common.h"

namespace cagra {

constexpr int kCols = CAGRA_PPR_COLS;
constexpr int kPprWaves = CAGRA_TILE_WAVES;
constexpr int kPprThreads = kPprWaves * kWave;
constexpr int kBatch = 16;  // source rows loaded ahead per wave
constexpr int kMergeBatch = 8;  // merge rows / vertices per wave whose loads are in flight together

template <typename W>
__global__ __launch_bounds__(kPprThreads) void k_gather_cols(const W *__restrict__ edge_src, int64_t E,
                                                             const int32_t *__restrict__ tile_edge,
                                                             const int32_t *__restrict__ tile_seg,
                                                             const int32_t *__restrict__ span_row,
                                                             const float *__restrict__ values, int32_t N,
                                                             int32_t ntiles, float *__restrict__ partial) {
    __shared__ float fix_head[kPprWaves][kCols];
    __shared__ float fix_last[kPprWaves][kCols];
    __shared__ int32_t fix_row[kPprWaves];
    __shared__ int32_t fix_has[kPprWaves];

    const int t = xcd_remap(blockIdx.x, ntiles);
    const int64_t e0 = tile_edge[t], e1 = tile_edge[t + 1];
    if (e0 >= e1) return;
    const int64_t vbase = (int64_t)tile_seg[t] * N;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int64_t sl = (e1 - e0 + kPprWaves - 1) / kPprWaves;
    int64_t w0 = e0 + w * sl;
    if (w0 > e1) w0 = e1;
    int64_t w1 = w0 + sl;
    if (w1 > e1) w1 = e1;
    int32_t row = span_row[(int64_t)t * kPprWaves + w] - 1;  // row open at the share's start
    int32_t seen = 0;
    // Neumaier-compensated row sums: rows of L2/Infinity-Cache-sized segments
    // can hold thousands of terms
    float acc = 0.0f, comp = 0.0f, head = 0.0f;
    const float *vals = values + vbase * kCols + lane;

    for (int64_t b0 = w0; b0 < w1; b0 += kWave) {
        const int64_t e = b0 + lane;
        const uint32_t word = e < w1 ? (uint32_t)edge_src[e] : 0u;
        const int n = (int)(w1 - b0 < kWave ? w1 - b0 : kWave);
        for (int jb = 0; jb < n; jb += kBatch) {
            uint32_t wv[kBatch];
            float x[kBatch];
#pragma unroll
            for (int u = 0; u < kBatch; ++u) {
                wv[u] = (uint32_t)__builtin_amdgcn_readlane((int32_t)word, jb + u);
                x[u] = vals[(int64_t)(wv[u] & EdgeWord<W>::kIndex) * kCols];
            }
#pragma unroll
            for (int u = 0; u < kBatch; ++u) {
                if (jb + u < n) {
                    if (wv[u] & EdgeWord<W>::kFlag) {  // a row starts: the open row is complete
                        if (seen) partial[(int64_t)row * kCols + lane] = acc + comp;
                        else head = acc + comp;
                        seen = 1;
                        ++row;
                        acc = 0.0f;
                        comp = 0.0f;
                    }
                    const float tsum = acc + x[u];
                    comp += fabsf(acc) >= fabsf(x[u]) ? (acc - tsum) + x[u] : (x[u] - tsum) + acc;
                    acc = tsum;
                }
            }
        }
    }
    fix_head[w][lane] = seen ? head : acc + comp;
    fix_last[w][lane] = acc + comp;
    if (lane == 0) {
        fix_row[w] = row;
        fix_has[w] = seen;
    }
    __syncthreads();
    if (fix_has[w]) {
        float tot = fix_last[w][lane];
        for (int x2 = w + 1; x2 < kPprWaves; ++x2) {
            tot += fix_head[x2][lane];
            if (fix_has[x2]) break;
        }
        partial[(int64_t)fix_row[w] * kCols + lane] = tot;
    }
}

// Merge in the paper's order plus the personalized vertex update:
//   r'(v, j) = d * sum_rows(v, j) + [v == seed_j] * ((1 - d) + d * D_j)
__global__ __launch_bounds__(kPprThreads) void k_merge_ppr(
    const int32_t *__restrict__ row_dst, const int32_t *__restrict__ block_ptr, const float *__restrict__ partial,
    int32_t V, int32_t k, int32_t B, int32_t nb, int32_t ncols, const int32_t *__restrict__ seeds,
    const float *__restrict__ rank_in, const int32_t *__restrict__ outdeg, const double *__restrict__ scalars_in,
    double damping, float *__restrict__ rank_out, float *__restrict__ contrib_out, double *__restrict__ blk) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    float *acc = reinterpret_cast<float *>(smem);  // [B][kCols]
    __shared__ double red[kPprWaves][kCols];
    const int b = xcd_remap(blockIdx.x, nb);
    const int64_t vb = (int64_t)b * B;
    const int32_t nv = (int32_t)((int64_t)V - vb < B ? (int64_t)V - vb : B);
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    for (int i = threadIdx.x; i < nv * kCols; i += kPprThreads) acc[i] = 0.0f;
    __syncthreads();
    // kMergeBatch rows per wave and pass, their loads issued before any is
    // applied (rows past the range re-read its first row, unused); a
    // subgraph's rows have distinct destinations, and the barrier after each
    // subgraph keeps the subgraphs in ascending order for every destination
    for (int32_t s = 0; s < k; ++s) {
        const int32_t lo = block_ptr[(int64_t)b * k + s], hi = block_ptr[(int64_t)(b + 1) * k + s];
        for (int32_t i0 = lo + w; i0 < hi; i0 += kPprWaves * kMergeBatch) {
            int32_t d[kMergeBatch];
            float x[kMergeBatch];
#pragma unroll
            for (int j = 0; j < kMergeBatch; ++j) {
                const int32_t i = i0 + j * kPprWaves;
                const int32_t ii = i < hi ? i : lo;
                d[j] = row_dst[ii];
                x[j] = partial[(int64_t)ii * kCols + lane];
            }
#pragma unroll
            for (int j = 0; j < kMergeBatch; ++j)
                if (i0 + j * kPprWaves < hi) acc[(int32_t)(d[j] - vb) * kCols + lane] += x[j];
        }
        __syncthreads();
    }
    const double dd = damping;
    const bool live = lane < ncols;
    const int32_t seed = live ? seeds[lane] : -1;
    const double Dj = live ? scalars_in[lane * 4 + 0] : 0.0;
    double dang = 0.0, res = 0.0, mass = 0.0;
    // kMergeBatch vertices per wave and pass, their loads issued together
    // (vertices past the block re-read its first, unused); the sums keep the
    // vertex order
    for (int i0 = w; i0 < nv; i0 += kPprWaves * kMergeBatch) {
        float rin[kMergeBatch];
        int32_t odv[kMergeBatch];
#pragma unroll
        for (int j = 0; j < kMergeBatch; ++j) {
            const int i = i0 + j * kPprWaves;
            const int64_t v = vb + (i < nv ? i : 0);
            rin[j] = rank_in[v * kCols + lane];
            odv[j] = outdeg[v];
        }
#pragma unroll
        for (int j = 0; j < kMergeBatch; ++j) {
            const int i = i0 + j * kPprWaves;
            if (i >= nv) break;
            const int64_t v = vb + i;
            double r = dd * (double)acc[i * kCols + lane];
            if (v == seed) r += (1.0 - dd) + dd * Dj;
            const float rf = live ? (float)r : 0.0f;
            rank_out[v * kCols + lane] = rf;
            const int32_t od = odv[j];
            contrib_out[v * kCols + lane] = od > 0 ? rf / (float)od : 0.0f;
            if (od == 0) dang += (double)rf;
            res += fabs((double)rf - (double)rin[j]);
            mass += (double)rf;
        }
    }
    // per-column partial sums over the waves, in wave order
    double *out = blk + (int64_t)b * kCols * 4;
    red[w][lane] = dang;
    __syncthreads();
    if (w == 0) {
        double s0 = 0.0;
        for (int x = 0; x < kPprWaves; ++x) s0 += red[x][lane];
        out[lane * 4 + 0] = s0;
    }
    __syncthreads();
    red[w][lane] = res;
    __syncthreads();
    if (w == 0) {
        double s1 = 0.0;
        for (int x = 0; x < kPprWaves; ++x) s1 += red[x][lane];
        out[lane * 4 + 1] = s1;
    }
    __syncthreads();
    red[w][lane] = mass;
    __syncthreads();
    if (w == 0) {
        double s2 = 0.0;
        for (int x = 0; x < kPprWaves; ++x) s2 += red[x][lane];
        out[lane * 4 + 2] = s2;
        out[lane * 4 + 3] = 0.0;
    }
}

// r_0(v, j) = [v == seed_j]; contributions and per-column dangling mass.
constexpr int kPprInitSpan = 256;  // vertices per init block
__global__ __launch_bounds__(256) void k_ppr_init(int32_t V, int32_t ncols, const int32_t *__restrict__ seeds,
                                                  const int32_t *__restrict__ outdeg, float *__restrict__ rank_out,
                                                  float *__restrict__ contrib_out, double *__restrict__ blk) {
    __shared__ double red[4][kCols][2];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const bool live = lane < ncols;
    const int32_t seed = live ? seeds[lane] : -1;
    double dang = 0.0, mass = 0.0;
    const int64_t lo = (int64_t)blockIdx.x * kPprInitSpan;
    for (int64_t v = lo + w; v < lo + kPprInitSpan && v < V; v += 4) {
        const float r = (v == seed) ? 1.0f : 0.0f;
        rank_out[v * kCols + lane] = r;
        const int32_t od = outdeg[v];
        contrib_out[v * kCols + lane] = od > 0 ? r / (float)od : 0.0f;
        if (od == 0) dang += r;
        mass += r;
    }
    red[w][lane][0] = dang;
    red[w][lane][1] = mass;
    __syncthreads();
    if (w == 0) {
        double* out = blk + (int64_t)blockIdx.x * kCols * 4;
        out[lane * 4 + 0] = red[0][lane][0] + red[1][lane][0] + red[2][lane][0] + red[3][lane][0];
        out[lane * 4 + 1] = 0.0;
        out[lane * 4 + 2] = red[0][lane][1] + red[1][lane][1] + red[2][lane][1] + red[3][lane][1];
        out[lane * 4 + 3] = 0.0;
    }
}

// Fixed-order sums over n blocks of [kCols][4] partials: one workgroup per column.
__global__ __launch_bounds__(256) void k_reduce_cols(const double *__restrict__ blk, int32_t n,
                                                     double *__restrict__ out) {
    __shared__ double red[4];
    const int j = blockIdx.x;
    double a[4] = {0.0, 0.0, 0.0, 0.0};
    for (int32_t b = threadIdx.x; b < n; b += 256)
        for (int c = 0; c < 4; ++c) a[c] += blk[((int64_t)b * kCols + j) * 4 + c];
    for (int c = 0; c < 4; ++c) {
        double t = block_sum_f64<256>(a[c], red);
        if (threadIdx.x == 0) out[j * 4 + c] = t;
    }
}

int32_t ppr_init_blocks(int32_t V) { return (int32_t)ceil_div(V, kPprInitSpan); }

size_t ppr_merge_lds_bytes(int32_t B) { return (size_t)B * kCols * sizeof(float); }

cagra_status launch_ppr_init(const cagra_graph *g, int32_t ncols, const int32_t *seeds, float *rank_out,
                             float *contrib_out, double *scalars_out, double *blk, hipStream_t st) {
    const int32_t nblk = ppr_init_blocks(g->V);
    k_ppr_init<<<nblk, 256, 0, st>>>(g->V, ncols, seeds, g->out_degree, rank_out, contrib_out, blk);
    CAGRA_LAUNCH_CHECK();
    k_reduce_cols<<<kCols, 256, 0, st>>>(blk, nblk, scalars_out);
    CAGRA_LAUNCH_CHECK();
    return CAGRA_OK;
}

cagra_status launch_ppr_iter(const cagra_graph *g, const cagra_segments *seg, double damping, int32_t ncols,
                             const int32_t *seeds, const float *rank_in, const float *contrib_in,
                             const double *scalars_in, float *partial, float *rank_out, float *contrib_out,
                             double *scalars_out, double *blk, hipStream_t st) {
    if (seg->ntiles > 0) {
        if (edge16(seg->N))
            k_gather_cols<uint16_t><<<seg->ntiles, kPprThreads, 0, st>>>(
                static_cast<const uint16_t *>(seg->edge_src), seg->E, seg->tile_edge, seg->tile_seg,
                seg->tile_span_row, contrib_in, seg->N, seg->ntiles, partial);
        else
            k_gather_cols<uint32_t><<<seg->ntiles, kPprThreads, 0, st>>>(
                static_cast<const uint32_t *>(seg->edge_src), seg->E, seg->tile_edge, seg->tile_seg,
                seg->tile_span_row, contrib_in, seg->N, seg->ntiles, partial);
        CAGRA_LAUNCH_CHECK();
    }
    if (cagra_status a_ = ensure_dynamic_lds((const void *)k_merge_ppr)) return a_;
    k_merge_ppr<<<seg->nb, kPprThreads, ppr_merge_lds_bytes(seg->B), st>>>(
        seg->row_dst, seg->block_ptr, partial, seg->V, seg->k, seg->B, seg->nb, ncols, seeds, rank_in, g->out_degree,
        scalars_in, damping, rank_out, contrib_out, blk);
    CAGRA_LAUNCH_CHECK();
    k_reduce_cols<<<kCols, 256, 0, st>>>(blk, seg->nb, scalars_out);
    CAGRA_LAUNCH_CHECK();
    return CAGRA_OK;
}

}  // namespace cagra
