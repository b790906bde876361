// Push-direction segmenting: the out-edge traversal cut into segments, the
// option Section 3 leaves open next to the pull (in-edge) version it builds.
//
// The segmentation of the reverse graph is the push layout of the graph:
// subgraph s holds every edge u -> v whose destination v lies in segment s,
// in rows of ascending source u (row_dst[i] = u), and each edge word carries
// the local destination v - s*N. One iteration has three steps:
//
//  1. Expand, the mirror image of the cache-aware merge (Section 3.3): every
//     row takes its source's value, vals[i] = x[row_dst[i]]. Sources are cut
//     into blocks of B vertices; a block's values are staged in LDS once and
//     each subgraph's rows of that block are written sequentially, so x is
//     read once and the random reads hit LDS.
//  2. Scatter, the mirror image of segment processing (Section 3.2): a
//     workgroup takes a piece (a run of consecutive tiles of one subgraph) and
//     keeps the accumulators of that subgraph's destination segment in LDS;
//     each edge adds its row's value to its destination with an LDS atomic.
//     Sums are int64 fixed point (every FP32 value truncated toward zero to a
//     multiple of 2^-56) and minima are exact, so no result depends on the order of the
//     atomics. A piece's finished accumulators leave as one sequential slot.
//  3. Update: each vertex combines the slots of its segment's pieces and
//     applies the vertex update (PageRank, or label propagation).
//
// Pieces: a subgraph with E_s edges is cut into ceil(E_s / cap) runs of its
// tiles (at most one per tile); cap is twice the mean subgraph size, capped so
// that a small graph still yields about 1024 pieces. The plan is rebuilt by
// one small kernel at the start of every call, so the workspace holds no
// state between calls.
#include <math.h>

#include "blockwalk.h"
#include "common.h"
#include "wave.h"

namespace cagra {

cagra_status launch_reduce4(const double *blk, int32_t n, double *out, const double *carry, hipStream_t st);
cagra_status launch_reduce_i32(const int32_t *blk, int32_t n, int32_t *out, hipStream_t st);

constexpr int kPushWaves = CAGRA_TILE_WAVES;  // tiles carry one starting row per wave
constexpr int kPushThreads = kPushWaves * kWave;
constexpr int kPushEPT = 8;                   // edges per lane per chunk
constexpr int kPushChunk = kWave * kPushEPT;
constexpr int kPushStages = 4;                // chunk buffers of edge words per wave
static_assert(kPushStages % 2 == 0, "the two value sets alternate with the chunk index inside one ring pass");
constexpr int kPlanThreads = 1024;
constexpr int kUpdSpan = 4096;                // vertices per update workgroup
constexpr int kUpdThreads = 256;
// expand items per XCD group (R-MAT 25 push iteration: 4 -> 2.814, 8 -> 2.790,
// 16 -> 2.783 ms; fewer block boundaries cross XCDs)
constexpr int32_t kExpandGroup = 16;
constexpr int kExpandStage = 8;    // staged source values per thread per batch
// windows per pass of the expand (R-MAT 25 push iteration, N = 20,480: 8 -> 2.786,
// 16 -> 2.731 ms with the batched staging; non-temporal stores of the values
// 3.15 ms; 32 windows need more than 64 VGPRs and halve the occupancy)
constexpr int kExpandUnroll = 16;

typedef int32_t v4i __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------------ plan

// First tile of subgraph s or later (tile_seg is non-decreasing); ntiles if none.
__device__ __forceinline__ int32_t first_tile_of(const int32_t *__restrict__ tile_seg, int32_t ntiles, int32_t s) {
    int32_t lo = 0, hi = ntiles;
    while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if (tile_seg[mid] < s) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

struct PieceRange {
    int32_t t0, nt, np;
};

__device__ __forceinline__ PieceRange pieces_of(const int32_t *__restrict__ tile_seg,
                                                const int32_t *__restrict__ tile_edge, int32_t ntiles, int32_t s,
                                                int64_t cap) {
    PieceRange r;
    r.t0 = first_tile_of(tile_seg, ntiles, s);
    const int32_t t1 = first_tile_of(tile_seg, ntiles, s + 1);
    r.nt = t1 - r.t0;
    r.np = 0;
    if (r.nt > 0) {
        const int64_t es = (int64_t)tile_edge[t1] - tile_edge[r.t0];
        int64_t p = (es + cap - 1) / cap;
        if (p < 1) p = 1;
        if (p > r.nt) p = r.nt;
        r.np = (int32_t)p;
    }
    return r;
}

// One workgroup: pfirst[s] = first piece of subgraph s (pfirst[k] = piece
// count), and per piece its first tile and subgraph; piece_tile[count] =
// ntiles closes the last piece. Subgraphs without tiles get no piece.
__global__ __launch_bounds__(kPlanThreads) void k_push_plan(const int32_t *__restrict__ tile_seg,
                                                            const int32_t *__restrict__ tile_edge, int32_t ntiles,
                                                            int32_t k, int64_t cap, int32_t *__restrict__ pfirst,
                                                            int32_t *__restrict__ piece_tile,
                                                            int32_t *__restrict__ piece_seg) {
    __shared__ int32_t tmp[kPlanThreads / kWave];
    const int32_t per = (k + kPlanThreads - 1) / kPlanThreads;
    const int32_t lo = threadIdx.x * per, hi = min(lo + per, k);
    int32_t sum = 0;
    for (int32_t s = lo; s < hi; ++s) sum += pieces_of(tile_seg, tile_edge, ntiles, s, cap).np;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int32_t incl = sum;
    for (int d = 1; d < kWave; d <<= 1) {
        const int32_t o = __shfl_up(incl, d, 64);
        if (lane >= d) incl += o;
    }
    if (lane == 63) tmp[w] = incl;
    __syncthreads();
    int32_t base = incl - sum;
    for (int i = 0; i < w; ++i) base += tmp[i];
    for (int32_t s = lo; s < hi; ++s) {
        const PieceRange r = pieces_of(tile_seg, tile_edge, ntiles, s, cap);
        pfirst[s] = base;
        for (int32_t j = 0; j < r.np; ++j) {
            piece_tile[base + j] = r.t0 + (int32_t)((int64_t)r.nt * j / r.np);
            piece_seg[base + j] = s;
        }
        base += r.np;
    }
    if (threadIdx.x == kPlanThreads - 1) {
        int32_t total = 0;
        for (int i = 0; i < kPlanThreads / kWave; ++i) total += tmp[i];
        pfirst[k] = total;
        piece_tile[total] = ntiles;
    }
}

// ------------------------------------------------------------------ expand

// vals[i] = x[row_dst[i]] for the rows of source block b, item j of its S
// items (the block's rows flattened over subgraphs, cut into S equal parts).
template <bool WIDE>
__global__ __launch_bounds__(kMergeThreads) void k_push_expand(const uint16_t *__restrict__ row_dst_lo,
                                                               const int32_t *__restrict__ block_ptr,
                                                               const int32_t *__restrict__ block_items,
                                                               const uint32_t *__restrict__ x, int32_t V, int32_t k,
                                                               int32_t B, int32_t nb, uint32_t *__restrict__ vals) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    __shared__ int32_t tmp[16];
    const int32_t total = block_items[nb];
    if ((int32_t)blockIdx.x >= total) return;  // the grid is the bound max_items
    // neighbouring blocks share the cache lines at the ends of their row ranges:
    // groups of them run on one XCD at once, so partial lines meet in its L2
    const ItemPlace ip = place_item(block_items, nb, total, xcd_group_map(blockIdx.x, total, kExpandGroup));
    const int32_t b = ip.b, j = ip.j, S = ip.S;
    uint32_t *xs = reinterpret_cast<uint32_t *>(smem);
    int32_t *ofs = reinterpret_cast<int32_t *>(smem + align_up((size_t)B * 4, 16));
    int32_t *pre = ofs + k;

    const int64_t vb = (int64_t)b * B;
    const int32_t nv = (int32_t)((int64_t)V - vb < B ? (int64_t)V - vb : B);
    // all of a thread's loads are issued before its first LDS write (nv >= 1)
    for (int i0 = 0; i0 < nv; i0 += kExpandStage * kMergeThreads) {
        uint32_t v[kExpandStage];
#pragma unroll
        for (int u = 0; u < kExpandStage; ++u) v[u] = x[vb + min(i0 + u * kMergeThreads + (int)threadIdx.x, nv - 1)];
#pragma unroll
        for (int u = 0; u < kExpandStage; ++u) {
            const int i = i0 + u * kMergeThreads + (int)threadIdx.x;
            if (i < nv) xs[i] = v[u];
        }
    }
    // the barrier inside load_block_ranges also publishes the staged values
    const int32_t P = load_block_ranges(block_ptr, b, k, ofs, pre, tmp);
    const int32_t F0 = (int32_t)((int64_t)P * j / S), F1 = (int32_t)((int64_t)P * (j + 1) / S);

    // the wave's share, walked in windows of 64 rows as in the merge
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int32_t share = ((((F1 - F0) + 15) / 16) + 63) & ~63;
    const int32_t fa = min(F0 + w * share, F1), fb = min(fa + share, F1);
    if (fa >= fb) return;  // uniform over the wave
    int32_t sw = __builtin_amdgcn_readfirstlane(run_of(pre, k, fa));
    int32_t i_safe = __builtin_amdgcn_readfirstlane(ofs[sw]) + fa;
    for (int32_t f0 = fa; f0 < fb; f0 += kWave * kExpandUnroll) {
        int32_t idx[kExpandUnroll], d[kExpandUnroll];
        int32_t sl = WIDE ? run_of(pre, k, f0) : 0;
#pragma unroll
        for (int u = 0; u < kExpandUnroll; ++u) {
            const int32_t fs = f0 + u * kWave;
            const int32_t f = fs + lane;
            const bool valid = f < fb;
            int32_t i;
            if (WIDE) {
                const int32_t ff = valid ? f : f0;
                sl = advance<true>(pre, k, sl, ff);
                i = ofs[sl] + ff;
            } else if (fs < fb) {  // uniform
                const int32_t ii = window_index(ofs, pre, sw, fs, min(fs + kWave - 1, fb - 1), f);
                i_safe = __builtin_amdgcn_readfirstlane(ii);
                i = valid ? ii : i_safe;
            } else {
                i = i_safe;
            }
            d[u] = (int32_t)row_dst_lo[i];
            idx[u] = valid ? i : -1;
        }
#pragma unroll
        for (int u = 0; u < kExpandUnroll; ++u)
            if (idx[u] >= 0) vals[idx[u]] = xs[d[u]];
    }
}

// ------------------------------------------------------------------ scatter

// Sums: every FP32 value x becomes trunc(x * 2^56) as a two's-complement
// int64 (exact for |x| < 64; the truncation error is below 2^-56 per term) and
// the int64 adds are exact, so the order of the atomics does not matter.
struct PushSum {
    using A = unsigned long long;
    static constexpr bool kSum = true;
    static __device__ __forceinline__ A identity() { return 0ull; }
    static __device__ __forceinline__ uint64_t magnitude(uint32_t u) { return fix56_magnitude(u); }
};
// Minima of int32 values.
struct PushMin {
    using A = int32_t;
    static constexpr bool kSum = false;
    static __device__ __forceinline__ A identity() { return 0x7fffffff; }
};

template <typename W>
constexpr int kPushLoads = kPushEPT * (int)sizeof(W) / 16;

template <typename W>
__device__ __forceinline__ void push_load_chunk(v4i (&r)[kPushLoads<W>], __amdgpu_buffer_rsrc_t ein, uint32_t off) {
#pragma unroll
    for (int j = 0; j < kPushLoads<W>; ++j)
        r[j] = __builtin_amdgcn_raw_buffer_load_b128(ein, off + 16 * j, 0, kNonTemporal);
}

// Values of one chunk in flight: loaded per edge, applied one chunk later so
// that the loads overlap the previous chunk's atomics.
struct PushPend {
    uint32_t xv[kPushEPT];  // the edge's row value (0 outside the share)
    int32_t d[kPushEPT];    // local destination (0 outside the share)
    uint32_t valid;         // bit i: edge i lies in the share
};

// Issue step of one chunk (this lane: kPushEPT consecutive edge words). rel0 =
// the chunk's first edge relative to the share (negative for a first chunk
// that starts before it); FULL chunks lie entirely inside the share. nfl = row
// starts seen in earlier chunks. The row of an edge is row_before + (row
// starts in the share up to and including it); vin is addressed relative to
// base_row (row_off = row_before - base_row). Edges outside the share read 0
// (buffer bounds) and target accumulator 0, so the apply step needs no branch.
template <typename W, bool FULL>
__device__ __forceinline__ void push_issue(const v4i (&wv)[kPushLoads<W>], int32_t rel0, int32_t share,
                                           int32_t row_off, __amdgpu_buffer_rsrc_t vin, int32_t &nfl, PushPend &P) {
    constexpr int kFlagShift = (int)sizeof(W) * 8 - 1;
    const int lane = threadIdx.x & 63;
    uint32_t wd[kPushEPT];
    if constexpr (sizeof(W) == 4) {
#pragma unroll
        for (int j = 0; j < kPushLoads<W>; ++j)
#pragma unroll
            for (int c = 0; c < 4; ++c) wd[4 * j + c] = (uint32_t)wv[j][c];
    } else {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            wd[2 * c] = (uint32_t)wv[0][c] & 0xffffu;
            wd[2 * c + 1] = (uint32_t)wv[0][c] >> 16;
        }
    }
    const int32_t rel = rel0 + lane * kPushEPT;
    bool valid[kPushEPT];
    int32_t f[kPushEPT], nf = 0;
    P.valid = 0u;
#pragma unroll
    for (int i = 0; i < kPushEPT; ++i) {
        valid[i] = FULL || (uint32_t)(rel + i) < (uint32_t)share;
        f[i] = valid[i] ? (int32_t)(wd[i] >> kFlagShift) : 0;
        nf += f[i];
        P.valid |= valid[i] ? (1u << i) : 0u;
    }
    const int32_t incl = wave_incl_sum(nf);
    const int32_t chunk_nf = __builtin_amdgcn_readlane(incl, 63);
    int32_t r = row_off + nfl + (incl - nf);  // row of the edge before this lane's first, relative to base_row
#pragma unroll
    for (int i = 0; i < kPushEPT; ++i) {
        r += f[i];
        const uint32_t off = valid[i] ? (uint32_t)r * 4u : kOutOfRange;
        P.xv[i] = (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(vin, off, 0, 0);
        P.d[i] = valid[i] ? (int32_t)(wd[i] & EdgeWord<W>::kIndex) : 0;
    }
    nfl += chunk_nf;
}

// Apply step: the chunk's atomics into the segment's LDS accumulators.
template <class PO>
__device__ __forceinline__ void push_apply(const PushPend &P, typename PO::A *acc) {
    if constexpr (PO::kSum) {
        uint32_t any = 0;
#pragma unroll
        for (int i = 0; i < kPushEPT; ++i) any |= P.xv[i];
        if (__ballot((int32_t)any < 0)) {  // uniform: a negative value in the wave
#pragma unroll
            for (int i = 0; i < kPushEPT; ++i) {
                const uint64_t m = PushSum::magnitude(P.xv[i]);
                atomicAdd(&acc[P.d[i]], (P.xv[i] >> 31) ? (unsigned long long)(-(int64_t)m) : (unsigned long long)m);
            }
        } else {
#pragma unroll
            for (int i = 0; i < kPushEPT; ++i) atomicAdd(&acc[P.d[i]], (unsigned long long)PushSum::magnitude(P.xv[i]));
        }
    } else {
#pragma unroll
        for (int i = 0; i < kPushEPT; ++i)
            atomicMin(&acc[P.d[i]], ((P.valid >> i) & 1u) ? (int32_t)P.xv[i] : PO::identity());
    }
}

template <typename W>
__device__ __forceinline__ void push_issue_any(const v4i (&wv)[kPushLoads<W>], int32_t rel0, int32_t share,
                                               int32_t row_off, __amdgpu_buffer_rsrc_t vin, int32_t &nfl,
                                               PushPend &P) {
    if (rel0 >= 0 && rel0 + kPushChunk <= share) push_issue<W, true>(wv, rel0, share, row_off, vin, nfl, P);
    else push_issue<W, false>(wv, rel0, share, row_off, vin, nfl, P);
}

// One workgroup per piece: accumulate the piece's edges into the destination
// segment's LDS accumulators, then write them to the piece's slot.
template <class PO, typename W>
__global__ __launch_bounds__(kPushThreads) void k_push_scatter(
    const W *__restrict__ edge_src, int64_t Q, const int32_t *__restrict__ tile_edge,
    const int32_t *__restrict__ span_row, const uint32_t *__restrict__ vals, int32_t V, int32_t N,
    const int32_t *__restrict__ pfirst, int32_t k, const int32_t *__restrict__ piece_tile,
    const int32_t *__restrict__ piece_seg, typename PO::A *__restrict__ slots) {
    using A = typename PO::A;
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    A *acc = reinterpret_cast<A *>(smem);
    const int32_t np = pfirst[k];
    const int32_t p = blockIdx.x;
    if (p >= np) return;  // the grid is a bound on the piece count
    const int32_t s = piece_seg[p], t0 = piece_tile[p], t1 = piece_tile[p + 1];
    const int64_t vbase = (int64_t)s * N;
    const int32_t n = (int32_t)((int64_t)V - vbase < N ? (int64_t)V - vbase : N);
    for (int i = threadIdx.x; i < n; i += kPushThreads) acc[i] = PO::identity();
    __syncthreads();

    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    constexpr int kWB = (int)sizeof(W);
    const uint32_t lane_off = (uint32_t)(lane * kPushEPT * kWB);
    for (int32_t t = t0; t < t1; ++t) {
        const int64_t e0 = tile_edge[t], e1 = tile_edge[t + 1];
        const int64_t sl = (e1 - e0 + kPushWaves - 1) / kPushWaves;
        int64_t w0 = e0 + w * sl;
        if (w0 > e1) w0 = e1;
        int64_t w1 = w0 + sl;
        if (w1 > e1) w1 = e1;
        if (w0 >= w1) continue;  // uniform over the wave
        // the share's edges before its first row start belong to row row_before
        const int32_t row_before = span_row[(int64_t)t * kPushWaves + w] - 1;
        const int32_t base_row = row_before > 0 ? row_before : 0;
        const int32_t share = (int32_t)(w1 - w0);
        const int64_t ebase = w0 & ~(int64_t)(16 / kWB - 1);
        const __amdgpu_buffer_rsrc_t ein = __builtin_amdgcn_make_buffer_rsrc(
            (void *)(edge_src + ebase), 0, (int32_t)align_up((size_t)(w1 - ebase) * kWB, 4), kBufFlags);
        // rows of the share: row_before .. row_before + share
        int64_t nrows = Q - base_row;
        if (nrows > (int64_t)share + 1) nrows = (int64_t)share + 1;
        const __amdgpu_buffer_rsrc_t vin = __builtin_amdgcn_make_buffer_rsrc(
            (void *)(vals + base_row), 0, (int32_t)(nrows * 4), kBufFlags);
        const int32_t row_off = row_before - base_row;  // -1 or 0
        const int64_t len = w1 - ebase;
        int32_t nfl = 0;
        // edge words kPushStages - 1 chunks ahead of the chunk whose loads are
        // issued, which runs one chunk ahead of the chunk applied
        v4i R[kPushStages][kPushLoads<W>];
        PushPend P[2];
#pragma unroll
        for (int c = 0; c < kPushStages - 1; ++c)
            push_load_chunk<W>(R[c], ein, (uint32_t)(c * kPushChunk * kWB) + lane_off);
        push_issue_any<W>(R[0], (int32_t)(ebase - w0), share, row_off, vin, nfl, P[0]);
        for (int64_t cc = 0; cc < len; cc += kPushStages * kPushChunk) {
#pragma unroll
            for (int c = 0; c < kPushStages; ++c) {
                const int64_t ci = cc + c * kPushChunk;
                if (ci >= len) break;  // uniform
                push_load_chunk<W>(R[(c + kPushStages - 1) % kPushStages], ein,
                                   (uint32_t)((ci + (kPushStages - 1) * kPushChunk) * kWB) + lane_off);
                if (ci + kPushChunk < len)
                    push_issue_any<W>(R[(c + 1) % kPushStages], (int32_t)(ebase + ci + kPushChunk - w0), share,
                                      row_off, vin, nfl, P[(c + 1) & 1]);
                push_apply<PO>(P[c & 1], acc);
            }
        }
    }
    __syncthreads();
    A *out = slots + (int64_t)p * N;
    for (int i = threadIdx.x; i < n; i += kPushThreads) out[i] = acc[i];
}

// ------------------------------------------------------------------ update

__global__ __launch_bounds__(kUpdThreads) void k_push_pr_update(
    const unsigned long long *__restrict__ slots, const int32_t *__restrict__ pfirst, int32_t V, int32_t N,
    const float *__restrict__ rank_in, const int32_t *__restrict__ outdeg, const double *__restrict__ scalars_in,
    double damping, float *__restrict__ rank_out, float *__restrict__ contrib_out, double *__restrict__ blk) {
    __shared__ double red[kUpdThreads / kWave];
    const double dd = damping;
    const double base = (1.0 - dd) / (double)V + dd * scalars_in[0] / (double)V;
    const int64_t lo = (int64_t)blockIdx.x * kUpdSpan;
    const int64_t hi = lo + kUpdSpan < V ? lo + kUpdSpan : V;
    double dang = 0.0, res = 0.0, mass = 0.0;
    for (int64_t v = lo + threadIdx.x; v < hi; v += kUpdThreads) {
        const int32_t s = (int32_t)(v / N);
        const int64_t i = v - (int64_t)s * N;
        unsigned long long a = 0ull;
        for (int32_t p = pfirst[s]; p < pfirst[s + 1]; ++p) a += slots[(int64_t)p * N + i];
        const double sum = (double)(long long)a * kFixInv;
        const float r = (float)(base + dd * sum);
        rank_out[v] = r;
        const int32_t od = outdeg[v];
        contrib_out[v] = od > 0 ? r / (float)od : 0.0f;
        if (od == 0) dang += (double)r;
        res += fabs((double)r - (double)rank_in[v]);
        mass += (double)r;
    }
    dang = block_sum_f64<kUpdThreads>(dang, red);
    res = block_sum_f64<kUpdThreads>(res, red);
    mass = block_sum_f64<kUpdThreads>(mass, red);
    if (threadIdx.x == 0) {
        blk[(int64_t)blockIdx.x * 4 + 0] = dang;
        blk[(int64_t)blockIdx.x * 4 + 1] = res;
        blk[(int64_t)blockIdx.x * 4 + 2] = mass;
        blk[(int64_t)blockIdx.x * 4 + 3] = 0.0;
    }
}

__global__ __launch_bounds__(kUpdThreads) void k_push_lp_update(const int32_t *__restrict__ slots,
                                                                const int32_t *__restrict__ pfirst, int32_t V,
                                                                int32_t N, const int32_t *__restrict__ labels_in,
                                                                int32_t *__restrict__ labels_out,
                                                                int32_t *__restrict__ blk) {
    __shared__ int32_t red[kUpdThreads / kWave];
    const int64_t lo = (int64_t)blockIdx.x * kUpdSpan;
    const int64_t hi = lo + kUpdSpan < V ? lo + kUpdSpan : V;
    int32_t changed = 0;
    for (int64_t v = lo + threadIdx.x; v < hi; v += kUpdThreads) {
        const int32_t s = (int32_t)(v / N);
        const int64_t i = v - (int64_t)s * N;
        const int32_t old = labels_in[v];
        int32_t m = old;
        for (int32_t p = pfirst[s]; p < pfirst[s + 1]; ++p) m = min(m, slots[(int64_t)p * N + i]);
        labels_out[v] = m;
        changed += m != old ? 1 : 0;
    }
    for (int d = 32; d >= 1; d >>= 1) changed += __shfl_down(changed, d, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = changed;
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t t = 0;
        for (int i = 0; i < kUpdThreads / kWave; ++i) t += red[i];
        blk[blockIdx.x] = t;
    }
}

// ------------------------------------------------------------------ host side

int64_t push_piece_cap(const cagra_segments *seg) {
    int64_t cap = ceil_div(2 * seg->E, seg->k);
    const int64_t fill = ceil_div(seg->E, 1024);
    if (fill < cap) cap = fill;
    if (cap < 4096) cap = 4096;
    return cap;
}
int64_t push_max_pieces(const cagra_segments *seg) { return (int64_t)seg->k + ceil_div(seg->E, push_piece_cap(seg)); }
int32_t push_update_blocks(int32_t V) { return (int32_t)ceil_div(V, kUpdSpan); }

// LDS of the expand kernel: staged block values and the block's range starts
// and prefix (plus the static scan scratch).
size_t push_expand_lds_bytes(int32_t B, int32_t k) {
    return align_up((size_t)B * 4, 16) + (size_t)(2 * (int64_t)k + 2) * sizeof(int32_t) + 64;
}
size_t push_expand_lds_total(int32_t B, int32_t k) { return push_expand_lds_bytes(B, k) + 256; }

// Workspace: plan (pfirst, piece_tile, piece_seg), per-block partials of the
// update, then the piece slots (8 bytes per vertex of a piece's segment).
struct PushWs {
    int32_t *pfirst, *piece_tile, *piece_seg;
    void *blk;
    void *slots;
};

static size_t push_layout(const cagra_segments *seg, char *base, PushWs *ws) {
    const int64_t maxp = push_max_pieces(seg);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + bytes, 256);
        return base ? (void *)(base + o) : nullptr;
    };
    void *pf = take((size_t)(seg->k + 1) * 4);
    void *pt = take((size_t)(maxp + 1) * 4);
    void *ps = take((size_t)maxp * 4);
    void *bk = take((size_t)push_update_blocks(seg->V) * 4 * sizeof(double));
    void *sl = take((size_t)maxp * (size_t)seg->N * 8);
    if (ws) *ws = PushWs{(int32_t *)pf, (int32_t *)pt, (int32_t *)ps, bk, sl};
    return off + 256;
}
size_t push_ws_bytes(const cagra_segments *seg) { return push_layout(seg, nullptr, nullptr); }

// LDS of the scatter kernel: the segment's accumulators.
size_t push_scatter_lds_bytes(int32_t N, int acc_bytes) { return (size_t)N * (size_t)acc_bytes; }

template <class PO>
static cagra_status launch_scatter(const cagra_segments *seg, const void *vals, const PushWs &ws, hipStream_t st) {
    const size_t lds = push_scatter_lds_bytes(seg->N, (int)sizeof(typename PO::A));
    const unsigned grid = (unsigned)push_max_pieces(seg);
    if (edge16(seg->N)) {
        if (cagra_status a_ = ensure_dynamic_lds((const void *)k_push_scatter<PO, uint16_t>)) return a_;
        k_push_scatter<PO, uint16_t><<<grid, kPushThreads, lds, st>>>(
            static_cast<const uint16_t *>(seg->edge_src), seg->Q, seg->tile_edge, seg->tile_span_row,
            static_cast<const uint32_t *>(vals), seg->V, seg->N, ws.pfirst, seg->k, ws.piece_tile, ws.piece_seg,
            static_cast<typename PO::A *>(ws.slots));
    } else {
        if (cagra_status a_ = ensure_dynamic_lds((const void *)k_push_scatter<PO, uint32_t>)) return a_;
        k_push_scatter<PO, uint32_t><<<grid, kPushThreads, lds, st>>>(
            static_cast<const uint32_t *>(seg->edge_src), seg->Q, seg->tile_edge, seg->tile_span_row,
            static_cast<const uint32_t *>(vals), seg->V, seg->N, ws.pfirst, seg->k, ws.piece_tile, ws.piece_seg,
            static_cast<typename PO::A *>(ws.slots));
    }
    CAGRA_LAUNCH_CHECK();
    return CAGRA_OK;
}

// Plan, expand and scatter: the common part of both push iterations.
template <class PO>
static cagra_status push_edges(const cagra_segments *seg, const void *x, void *vals, const PushWs &ws,
                               hipStream_t st) {
    k_push_plan<<<1, kPlanThreads, 0, st>>>(seg->tile_seg, seg->tile_edge, seg->ntiles, seg->k, push_piece_cap(seg),
                                           ws.pfirst, ws.piece_tile, ws.piece_seg);
    CAGRA_LAUNCH_CHECK();
    if (seg->Q > 0) {
        const size_t lds = push_expand_lds_bytes(seg->B, seg->k);
        const bool wide = seg->Q < (int64_t)kWave * seg->k * seg->nb;
        if (cagra_status a_ = ensure_dynamic_lds((const void *)k_push_expand<true>)) return a_;
        if (cagra_status a_ = ensure_dynamic_lds((const void *)k_push_expand<false>)) return a_;
        if (wide)
            k_push_expand<true><<<seg->max_items, kMergeThreads, lds, st>>>(
                seg->row_dst_lo, seg->block_ptr, seg->block_items, static_cast<const uint32_t *>(x), seg->V, seg->k,
                seg->B, seg->nb, static_cast<uint32_t *>(vals));
        else
            k_push_expand<false><<<seg->max_items, kMergeThreads, lds, st>>>(
                seg->row_dst_lo, seg->block_ptr, seg->block_items, static_cast<const uint32_t *>(x), seg->V, seg->k,
                seg->B, seg->nb, static_cast<uint32_t *>(vals));
        CAGRA_LAUNCH_CHECK();
    }
    return launch_scatter<PO>(seg, vals, ws, st);
}

cagra_status launch_pr_push(const cagra_graph *g, const cagra_segments *seg, double damping, const float *rank_in,
                            const float *contrib_in, const double *scalars_in, float *vals, float *rank_out,
                            float *contrib_out, double *scalars_out, void *workspace, hipStream_t st) {
    PushWs ws;
    push_layout(seg, static_cast<char *>(workspace), &ws);
    if (cagra_status s = push_edges<PushSum>(seg, contrib_in, vals, ws, st)) return s;
    const int32_t nblk = push_update_blocks(seg->V);
    k_push_pr_update<<<nblk, kUpdThreads, 0, st>>>(static_cast<const unsigned long long *>(ws.slots), ws.pfirst,
                                                   seg->V, seg->N, rank_in, g->out_degree, scalars_in, damping,
                                                   rank_out, contrib_out, static_cast<double *>(ws.blk));
    CAGRA_LAUNCH_CHECK();
    return launch_reduce4(static_cast<const double *>(ws.blk), nblk, scalars_out, scalars_in, st);
}

cagra_status launch_lp_push(const cagra_segments *seg, const int32_t *labels_in, int32_t *vals, int32_t *labels_out,
                            int32_t *changed_out, void *workspace, hipStream_t st) {
    PushWs ws;
    push_layout(seg, static_cast<char *>(workspace), &ws);
    if (cagra_status s = push_edges<PushMin>(seg, labels_in, vals, ws, st)) return s;
    const int32_t nblk = push_update_blocks(seg->V);
    k_push_lp_update<<<nblk, kUpdThreads, 0, st>>>(static_cast<const int32_t *>(ws.slots), ws.pfirst, seg->V, seg->N,
                                                   labels_in, labels_out, static_cast<int32_t *>(ws.blk));
    CAGRA_LAUNCH_CHECK();
    return launch_reduce_i32(static_cast<const int32_t *>(ws.blk), nblk, changed_out, st);
}

}  // namespace cagra
