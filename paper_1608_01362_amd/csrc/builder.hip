// CSR segmenting preprocessing on the GPU (Section 3.1 of the paper).
//
// The CSC row of a destination v lists its sources in ascending order, so the
// in-edges of v that fall in one segment (source / N) form a contiguous run.
// Every run is one row (s, v) of subgraph s. The builder
//   1. flags run starts and labels every edge with its run and destination
//      (two device-wide scans),
//   2. stable-sorts the runs by segment id (the runs arrive in (v, s) order;
//      segment-major order with v ascending inside each segment is the paper's
//      "sortByDestination" per subgraph), carrying each run's destination and
//      length, and stable-sorts the edges by the segment of their source,
//      carrying the finished edge word (local index + row-start flag): both
//      with the stable digit passes of segsort.hip, whose tile-local ranking in
//      LDS keeps the writes coalesced where a direct scatter of runs and edges
//      writes a few bytes per cache line,
//   3. writes the rows and their offsets from the sorted runs,
//   4. builds the merge block index (Section 3.3) and the gather tile table.
// Everything is integer work; the result is unique and bit-identical run to run.
#include <limits.h>

#include <vector>

#include "common.h"
#include "radix.h"

namespace cagra {

// ------------------------------------------------------------------ scan

constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;  // 4096

struct ScanAdd {
    static __device__ __forceinline__ int32_t id() { return 0; }
    static __device__ __forceinline__ int32_t op(int32_t a, int32_t b) { return a + b; }
};
struct ScanMax {
    static __device__ __forceinline__ int32_t id() { return INT_MIN; }
    static __device__ __forceinline__ int32_t op(int32_t a, int32_t b) { return a > b ? a : b; }
};

template <class Op>
__device__ int32_t block_reduce_i32(int32_t v, int32_t *lds) {
    for (int d = 32; d >= 1; d >>= 1) v = Op::op(v, __shfl_down(v, d, 64));
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x / 64] = v;
    __syncthreads();
    int32_t r = Op::id();
    if (threadIdx.x == 0)
        for (int i = 0; i < kScanThreads / 64; ++i) r = Op::op(r, lds[i]);
    return r;
}

template <class Op>
__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const int32_t *__restrict__ in, int64_t n,
                                                              int32_t *__restrict__ sums) {
    __shared__ int32_t lds[kScanThreads / 64];
    int64_t base = (int64_t)blockIdx.x * kScanTile;
    // all loads issued before any is used (lanes past the end read the tile's first item)
    int32_t v[kScanItems];
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        int64_t j = base + i * kScanThreads + threadIdx.x;
        v[i] = in[j < n ? j : base];
    }
    int32_t acc = Op::id();
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        int64_t j = base + i * kScanThreads + threadIdx.x;
        acc = Op::op(acc, j < n ? v[i] : Op::id());
    }
    int32_t tot = block_reduce_i32<Op>(acc, lds);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

__device__ __forceinline__ int pad_idx(int p) { return p + (p >> 5); }

// Scans one tile of 4096 items; `offsets` (exclusive prefix of earlier tiles)
// may be null for a single tile. Safe in place (in == out).
template <class Op>
__global__ __launch_bounds__(kScanThreads) void k_scan_apply(const int32_t *in, int32_t *out, int64_t n,
                                                             const int32_t *__restrict__ offsets, int inclusive) {
    __shared__ int32_t tile[kScanTile + kScanTile / 32];
    __shared__ int32_t wsum[kScanThreads / 64];
    int64_t base = (int64_t)blockIdx.x * kScanTile;
    {
        // all loads issued before any is stored (lanes past the end read the tile's first item)
        int32_t v[kScanItems];
#pragma unroll
        for (int i = 0; i < kScanItems; ++i) {
            int64_t j = base + i * kScanThreads + threadIdx.x;
            v[i] = in[j < n ? j : base];
        }
#pragma unroll
        for (int i = 0; i < kScanItems; ++i) {
            int p = i * kScanThreads + threadIdx.x;
            tile[pad_idx(p)] = base + p < n ? v[i] : Op::id();
        }
    }
    __syncthreads();
    int32_t vals[kScanItems];
    int32_t run = Op::id();
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        vals[i] = tile[pad_idx(threadIdx.x * kScanItems + i)];
        run = Op::op(run, vals[i]);
    }
    // exclusive scan of per-thread totals
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int32_t incl = run;
    for (int d = 1; d < 64; d <<= 1) {
        int32_t o = __shfl_up(incl, d, 64);
        if (lane >= d) incl = Op::op(o, incl);
    }
    if (lane == 63) wsum[w] = incl;
    int32_t excl = __shfl_up(incl, 1, 64);
    if (lane == 0) excl = Op::id();
    __syncthreads();
    int32_t prefix = offsets ? offsets[blockIdx.x] : Op::id();
    for (int i = 0; i < w; ++i) prefix = Op::op(prefix, wsum[i]);
    prefix = Op::op(prefix, excl);
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        int32_t nxt = Op::op(prefix, vals[i]);
        tile[pad_idx(threadIdx.x * kScanItems + i)] = inclusive ? nxt : prefix;
        prefix = nxt;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        int p = i * kScanThreads + threadIdx.x;
        int64_t j = base + p;
        if (j < n) out[j] = tile[pad_idx(p)];
    }
}

// Workspace bytes the scan temporaries of one scan of n items take (same
// arena rules as scan_i32 below).
static size_t scan_ws_bytes(int64_t n) {
    ArenaSize a;
    while (n > kScanTile) {
        n = ceil_div(n, kScanTile);
        a.take<int32_t>(n + 64);
    }
    return a.used + 256;
}

template <class Op>
static cagra_status scan_i32_rec(const int32_t *in, int32_t *out, int64_t n, bool inclusive, Arena &ar,
                                 hipStream_t st) {
    if (n <= 0) return CAGRA_OK;
    int64_t nblk = ceil_div(n, kScanTile);
    if (nblk == 1) {
        k_scan_apply<Op><<<1, kScanThreads, 0, st>>>(in, out, n, nullptr, inclusive ? 1 : 0);
        CAGRA_LAUNCH_CHECK();
        return CAGRA_OK;
    }
    int32_t *sums = ar.take<int32_t>(nblk + 64);
    if (!sums) return fail(CAGRA_E_BUFFER, "builder workspace too small (scan temporaries)");
    k_scan_reduce<Op><<<(unsigned)nblk, kScanThreads, 0, st>>>(in, n, sums);
    CAGRA_LAUNCH_CHECK();
    cagra_status s = scan_i32_rec<Op>(sums, sums, nblk, false, ar, st);
    if (s != CAGRA_OK) return s;
    k_scan_apply<Op><<<(unsigned)nblk, kScanThreads, 0, st>>>(in, out, n, sums, inclusive ? 1 : 0);
    CAGRA_LAUNCH_CHECK();
    return CAGRA_OK;
}

// Temporaries are released after the scan: later work on the same stream may
// reuse them, as it runs only after the scan's kernels.
template <class Op>
static cagra_status scan_i32(const int32_t *in, int32_t *out, int64_t n, bool inclusive, Arena &ar, hipStream_t st) {
    size_t mark = ar.used;
    cagra_status s = scan_i32_rec<Op>(in, out, n, inclusive, ar, st);
    ar.used = mark;
    return s;
}

size_t scan_add_ws_bytes(int64_t n) { return scan_ws_bytes(n); }

// Exclusive prefix sum of n int32 values (in place allowed), temporaries in ws.
cagra_status scan_add_exclusive(const int32_t *in, int32_t *out, int64_t n, void *ws, size_t ws_bytes,
                                hipStream_t st) {
    Arena ar{(char *)ws, ws_bytes, 0};
    return scan_i32<ScanAdd>(in, out, n, false, ar, st);
}

// ------------------------------------------------------------------ builder kernels

static inline unsigned grid_for(int64_t n, int nt) {
    int64_t g = ceil_div(n, nt);
    return (unsigned)(g < 1 ? 1 : g);
}

__global__ void k_fill_i32(int32_t *p, int64_t n, int32_t v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// mark[off[v]] = v + 1 for every non-empty row (mark pre-filled with 0)
__global__ void k_mark_rows(const int32_t *__restrict__ off, int32_t V, int32_t *__restrict__ mark) {
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v < V) {
        int32_t a = off[v], b = off[v + 1];
        if (b > a) mark[a] = (int32_t)v + 1;
    }
}

// Edges per thread in the edge passes below. Each thread loads its edges (and
// their predecessors) at indices clamped into [0, E) before it uses any of
// them, so the loads are in flight together instead of one dependent round
// trip per edge; threads past E drop their results.
constexpr int kBItems = 8;
constexpr int kBThreads = 256;

__device__ __forceinline__ int64_t clamp_edge(int64_t e, int64_t E) { return e < E ? e : E - 1; }

// Edge e starts a run (a subgraph row) when it is the first edge, the first
// in-edge of its destination (mark != 0), or its source lies in another
// segment than its predecessor's.
__device__ __forceinline__ bool run_start(int64_t e, int32_t m, int32_t u, int32_t u_prev, int32_t N) {
    return e == 0 || m != 0 || (u / N) != (u_prev / N);
}

// Query pass: per-segment edge counts and the number of runs (rows).
__global__ __launch_bounds__(kBThreads) void k_count(const int32_t *__restrict__ src,
                                                     const int32_t *__restrict__ mark, int64_t E, int32_t N,
                                                     int32_t k, int use_lds, int32_t *__restrict__ seg_edges,
                                                     unsigned long long *runs) {
    extern __shared__ int32_t hist[];
    if (use_lds) {
        for (int s = threadIdx.x; s < k; s += blockDim.x) hist[s] = 0;
        __syncthreads();
    }
    unsigned long long nr = 0;
    const int64_t stride = (int64_t)gridDim.x * kBThreads * kBItems;
    for (int64_t e0 = (int64_t)blockIdx.x * kBThreads * kBItems + threadIdx.x; e0 < E; e0 += stride) {
        int32_t m[kBItems], u[kBItems], up[kBItems];
#pragma unroll
        for (int j = 0; j < kBItems; ++j) {
            const int64_t ec = clamp_edge(e0 + j * kBThreads, E);
            m[j] = mark[ec];
            u[j] = src[ec];
            up[j] = src[ec > 0 ? ec - 1 : 0];
        }
#pragma unroll
        for (int j = 0; j < kBItems; ++j) {
            const int64_t e = e0 + j * kBThreads;
            if (e >= E) break;
            const int32_t s = u[j] / N;
            if (use_lds) atomicAdd(&hist[s], 1);
            else atomicAdd(&seg_edges[s], 1);
            nr += run_start(e, m[j], u[j], up[j], N) ? 1 : 0;
        }
    }
    for (int d = 32; d >= 1; d >>= 1) nr += __shfl_down(nr, d, 64);
    if ((threadIdx.x & 63) == 0 && nr) atomicAdd(runs, nr);
    if (use_lds) {
        __syncthreads();
        for (int s = threadIdx.x; s < k; s += blockDim.x)
            if (hist[s]) atomicAdd(&seg_edges[s], hist[s]);
    }
}

__global__ __launch_bounds__(kBThreads) void k_flags(const int32_t *__restrict__ src,
                                                     const int32_t *__restrict__ mark, int64_t E, int32_t N,
                                                     int32_t *__restrict__ flag) {
    const int64_t e0 = (int64_t)blockIdx.x * kBThreads * kBItems + threadIdx.x;
    int32_t m[kBItems], u[kBItems], up[kBItems];
#pragma unroll
    for (int j = 0; j < kBItems; ++j) {
        const int64_t ec = clamp_edge(e0 + j * kBThreads, E);
        m[j] = mark[ec];
        u[j] = src[ec];
        up[j] = src[ec > 0 ? ec - 1 : 0];
    }
#pragma unroll
    for (int j = 0; j < kBItems; ++j) {
        const int64_t e = e0 + j * kBThreads;
        if (e < E) flag[e] = run_start(e, m[j], u[j], up[j], N) ? 1 : 0;
    }
}

// runincl[e] = 1 + run index of edge e; dstp1[e] = 1 + destination of edge e.
__global__ __launch_bounds__(kBThreads) void k_runs(const int32_t *__restrict__ src,
                                                    const int32_t *__restrict__ dstp1,
                                                    const int32_t *__restrict__ runincl, int64_t E, int32_t N,
                                                    int32_t *__restrict__ run_first, int32_t *__restrict__ run_seg,
                                                    int32_t *__restrict__ run_dst) {
    const int64_t e0 = (int64_t)blockIdx.x * kBThreads * kBItems + threadIdx.x;
    int32_t ri[kBItems], rp[kBItems], u[kBItems], d[kBItems];
#pragma unroll
    for (int j = 0; j < kBItems; ++j) {
        const int64_t ec = clamp_edge(e0 + j * kBThreads, E);
        ri[j] = runincl[ec];
        rp[j] = runincl[ec > 0 ? ec - 1 : 0];
        u[j] = src[ec];
        d[j] = dstp1[ec];
    }
#pragma unroll
    for (int j = 0; j < kBItems; ++j) {
        const int64_t e = e0 + j * kBThreads;
        if (e >= E) break;
        if (e == 0 || rp[j] != ri[j]) {
            const int32_t r = ri[j] - 1;
            run_first[r] = (int32_t)e;
            run_seg[r] = u[j] / N;
            run_dst[r] = d[j] - 1;
        }
        if (e == E - 1) run_first[ri[j]] = (int32_t)E;
    }
}

// Sort inputs of the runs: key = segment, value = destination << 32 | length.
__global__ void k_run_kv(const int32_t *__restrict__ run_first, const int32_t *__restrict__ run_seg,
                         const int32_t *__restrict__ run_dst, int64_t Q, uint16_t *__restrict__ key,
                         unsigned long long *__restrict__ val) {
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= Q) return;
    key[r] = (uint16_t)run_seg[r];
    val[r] = ((unsigned long long)(uint32_t)run_dst[r] << 32) | (uint32_t)(run_first[r + 1] - run_first[r]);
}

// Sort inputs of the edges: key = segment of the source, value = the edge word
// (local source index, row-start flag on the first edge of each run).
template <typename W>
__global__ __launch_bounds__(kBThreads) void k_edge_kv(const int32_t *__restrict__ src,
                                                       const int32_t *__restrict__ runincl, int64_t E, int32_t N,
                                                       uint16_t *__restrict__ key, W *__restrict__ val) {
    const int64_t e0 = (int64_t)blockIdx.x * kBThreads * kBItems + threadIdx.x;
    int32_t u[kBItems], ri[kBItems], rp[kBItems];
#pragma unroll
    for (int j = 0; j < kBItems; ++j) {
        const int64_t ec = clamp_edge(e0 + j * kBThreads, E);
        u[j] = src[ec];
        ri[j] = runincl[ec];
        rp[j] = runincl[ec > 0 ? ec - 1 : 0];
    }
#pragma unroll
    for (int j = 0; j < kBItems; ++j) {
        const int64_t e = e0 + j * kBThreads;
        if (e >= E) break;
        const int32_t s = u[j] / N;
        const uint32_t local = (uint32_t)(u[j] - s * N);
        const bool start = e == 0 || rp[j] != ri[j];
        key[e] = (uint16_t)s;
        val[e] = (W)(start ? (local | EdgeWord<W>::kFlag) : local);
    }
}

// Rows from the sorted runs; row_len[Q] = 0 closes the offsets' scan.
__global__ void k_rows_sorted(const unsigned long long *__restrict__ val, int64_t Q, int32_t B,
                              int32_t *__restrict__ row_dst, uint16_t *__restrict__ row_dst_lo,
                              int32_t *__restrict__ row_len) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < Q) {
        const unsigned long long x = val[p];
        const int32_t d = (int32_t)(x >> 32);
        row_dst[p] = d;
        row_dst_lo[p] = (uint16_t)(d % B);
        row_len[p] = (int32_t)(uint32_t)x;
    }
    if (p == Q) row_len[Q] = 0;
}

// seg_row_begin[s] = first sorted run of segment s or later.
__global__ void k_seg_begin_sorted(const uint16_t *__restrict__ key, int64_t Q, int32_t k,
                                   int32_t *__restrict__ seg_row_begin) {
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s > k) return;
    int64_t lo = 0, hi = Q;
    while (lo < hi) {
        const int64_t mid = lo + ((hi - lo) >> 1);
        if ((int64_t)key[mid] < s) lo = mid + 1;
        else hi = mid;
    }
    seg_row_begin[s] = (int32_t)lo;
}

// Merge work items (see block_items in cagra.h): a block whose entries exceed
// four times the mean per block is cut into ceil(P_b / T) equal parts.
static int64_t merge_split_entries(int64_t Q, int32_t nb) {
    const int64_t mean = nb > 0 ? ceil_div(Q, nb) : 1;
    return mean > 0 ? 4 * mean : 4;
}

__global__ __launch_bounds__(64) void k_block_items(const int32_t *__restrict__ block_ptr, int32_t k, int32_t nb,
                                                    int64_t T, int32_t *__restrict__ items) {
    const int64_t b = blockIdx.x;
    int64_t P = 0;
    for (int32_t s = threadIdx.x; s < k; s += 64) P += block_ptr[(b + 1) * k + s] - block_ptr[b * k + s];
    for (int d = 32; d >= 1; d >>= 1) P += __shfl_down(P, d, 64);
    if (threadIdx.x == 0) {
        items[b] = P > T ? (int32_t)ceil_div(P, T) : 1;
        if (b == nb - 1) items[nb] = 0;
    }
}

// First index in [lo, hi) with a[i] >= x (hi if none).
__device__ __forceinline__ int32_t lower_bound_i32(const int32_t *a, int32_t lo, int32_t hi, int64_t x) {
    while (lo < hi) {
        int32_t mid = lo + ((hi - lo) >> 1);
        if ((int64_t)a[mid] < x) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

__global__ void k_block_ptr(const int32_t *__restrict__ row_dst, const int32_t *__restrict__ seg_row_begin,
                            int32_t k, int32_t nb, int32_t B, int32_t *__restrict__ block_ptr) {
    int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= (int64_t)(nb + 1) * k) return;
    int64_t b = id / k;
    int32_t s = (int32_t)(id - b * k);
    block_ptr[id] = lower_bound_i32(row_dst, seg_row_begin[s], seg_row_begin[s + 1], b * (int64_t)B);
}

__global__ void k_tile_count(const int32_t *__restrict__ row_ptr, const int32_t *__restrict__ seg_row_begin,
                             int32_t k, int32_t T, int32_t *__restrict__ tcount) {
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s < k) {
        int64_t es = row_ptr[seg_row_begin[s]], ee = row_ptr[seg_row_begin[s + 1]];
        tcount[s] = (int32_t)ceil_div(ee - es, T);
    } else if (s == k) {
        tcount[k] = 0;
    }
}

__global__ void k_tiles(const int32_t *__restrict__ row_ptr, const int32_t *__restrict__ seg_row_begin,
                        const int32_t *__restrict__ tile_base, int32_t k, int32_t T, int32_t ntiles, int64_t E,
                        int32_t *__restrict__ tile_edge, int32_t *__restrict__ tile_seg) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t > ntiles) return;
    if (t == ntiles) {
        tile_edge[ntiles] = (int32_t)E;
        return;
    }
    // segment s with tile_base[s] <= t < tile_base[s+1]
    int32_t lo = 0, hi = k;  // find last s with tile_base[s] <= t
    while (hi - lo > 1) {
        int32_t mid = (lo + hi) >> 1;
        if (tile_base[mid] <= t) lo = mid;
        else hi = mid;
    }
    int32_t s = lo;
    while (s + 1 < k && tile_base[s + 1] <= t) ++s;  // skip segments without tiles
    int64_t j = t - tile_base[s];
    int32_t r0 = seg_row_begin[s], r1 = seg_row_begin[s + 1];
    int64_t nominal = (int64_t)row_ptr[r0] + j * T;
    int32_t r = lower_bound_i32(row_ptr, r0, r1, nominal);
    tile_edge[t] = row_ptr[r];  // row_ptr[r1] is the end of the segment
    tile_seg[t] = s;
}

__global__ void k_spans(const int32_t *__restrict__ row_ptr, const int32_t *__restrict__ seg_row_begin,
                        const int32_t *__restrict__ tile_edge, const int32_t *__restrict__ tile_seg, int32_t ntiles,
                        int32_t *__restrict__ span_row) {
    int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= (int64_t)ntiles * CAGRA_TILE_WAVES) return;
    int64_t t = id / CAGRA_TILE_WAVES;
    int32_t w = (int32_t)(id - t * CAGRA_TILE_WAVES);
    int64_t lo = tile_edge[t], hi = tile_edge[t + 1];
    int64_t sl = ceil_div(hi - lo, CAGRA_TILE_WAVES);
    int64_t b = lo + w * sl;
    if (b > hi) b = hi;
    int32_t s = tile_seg[t];
    span_row[id] = lower_bound_i32(row_ptr, seg_row_begin[s], seg_row_begin[s + 1], b);
}

// ------------------------------------------------------------------ host orchestration

static int nbits_for(int32_t k) {
    int b = 1;
    while ((1LL << b) < k) ++b;
    return b;
}

size_t query_workspace_bytes(int32_t V, int64_t E, int32_t N) {
    int64_t k = ceil_div(V, N);
    ArenaSize a;
    a.take<int32_t>(E);                  // mark
    a.take<int32_t>(k);                  // per-segment edges
    a.take<unsigned long long>(1);       // run count
    return a.used + 256;
}

// Temporary storage of the two stable sorts by segment (sizes only).
struct SortTemps {
    size_t rows = 0, edges = 0;
};

static cagra_status sort_temps(int64_t E, int64_t Q, int32_t k, bool w16, SortTemps &t) {
    const int bits = nbits_for(k);
    t.rows = seg_sort_ws_bytes(Q, bits, (int)sizeof(unsigned long long));
    t.edges = seg_sort_ws_bytes(E, bits, w16 ? 2 : 4);
    return CAGRA_OK;
}

// Layout of the build workspace (mirrors build_segments below). Arrays that
// are dead by the time a later one is written share its memory:
//   mark (dstp1)       -> edge keys and, for 16-bit words, the unsorted edge words
//   flag (runincl)     -> sorted edge keys
//   run_first          -> sorted run keys
//   run_seg + run_dst  -> sorted run values
static size_t build_layout(int64_t E, int64_t Q, int32_t k, int32_t nb, int wbytes, const SortTemps &t) {
    ArenaSize a;
    a.take<char>(4 * E + 512);            // mark / dstp1; then edge keys (+ 16-bit edge words)
    a.take<int32_t>(E);                   // flags / runincl; then sorted edge keys
    a.take<int32_t>(Q + 1);               // run_first; then sorted run keys
    a.take<int32_t>(2 * Q);               // run_seg, run_dst; then sorted run values
    a.take<uint16_t>(Q);                  // run keys
    a.take<unsigned long long>(Q);        // run values
    if (wbytes == 4) a.take<uint32_t>(E); // 32-bit edge words before sorting
    a.take<int32_t>(k + 1);               // tile counts
    a.take<char>((int64_t)(t.rows > t.edges ? t.rows : t.edges));  // sort temporaries
    int64_t mx = E;
    if (Q + 1 > mx) mx = Q + 1;
    if ((int64_t)nb + 1 > mx) mx = (int64_t)nb + 1;
    if ((int64_t)k + 1 > mx) mx = (int64_t)k + 1;
    return a.used + scan_ws_bytes(mx) + 256;
}

static cagra_status allow_big_lds_impl();
static cagra_status allow_big_lds() { return allow_big_lds_impl(); }

cagra_status query_segments(const cagra_graph *g, cagra_segments *seg, void *ws, size_t ws_bytes, hipStream_t st) {
    const int32_t V = g->V, N = seg->N;
    const int64_t E = g->E;
    const int32_t k = (int32_t)ceil_div(V, N);
    Arena ar{(char *)ws, ws_bytes, 0};
    int32_t *mark = ar.take<int32_t>(E);
    int32_t *seg_edges = ar.take<int32_t>(k);
    unsigned long long *runs = ar.take<unsigned long long>(1);
    if (!mark || !seg_edges || !runs) return fail(CAGRA_E_BUFFER, "query workspace smaller than %zu bytes",
                                                  query_workspace_bytes(V, E, N));
    int64_t Q = 0;
    std::vector<int32_t> host_edges(k, 0);
    if (E > 0) {
        if (cagra_status a = allow_big_lds()) return a;
        k_fill_i32<<<grid_for(E, 256), 256, 0, st>>>(mark, E, 0);
        CAGRA_LAUNCH_CHECK();
        k_fill_i32<<<grid_for(k, 256), 256, 0, st>>>(seg_edges, k, 0);
        CAGRA_LAUNCH_CHECK();
        CAGRA_HIP_CHECK(hipMemsetAsync(runs, 0, sizeof(unsigned long long), st));
        k_mark_rows<<<grid_for(V, 256), 256, 0, st>>>(g->in_offsets, V, mark);
        CAGRA_LAUNCH_CHECK();
        int use_lds = k <= 16384 ? 1 : 0;
        unsigned grid = grid_for(E, kBThreads * kBItems * 8);
        if (grid > 4096) grid = 4096;
        k_count<<<grid, kBThreads, use_lds ? k * sizeof(int32_t) : 0, st>>>(g->in_sources, mark, E, N, k, use_lds,
                                                                      seg_edges, runs);
        CAGRA_LAUNCH_CHECK();
        unsigned long long hr = 0;
        CAGRA_HIP_CHECK(hipMemcpyAsync(&hr, runs, sizeof(hr), hipMemcpyDeviceToHost, st));
        CAGRA_HIP_CHECK(hipMemcpyAsync(host_edges.data(), seg_edges, (size_t)k * sizeof(int32_t),
                                       hipMemcpyDeviceToHost, st));
        CAGRA_HIP_CHECK(hipStreamSynchronize(st));
        Q = (int64_t)hr;
    }
    int64_t ntiles = 0;
    for (int32_t s = 0; s < k; ++s) ntiles += ceil_div(host_edges[s], seg->tile_edges);
    if (ntiles * CAGRA_TILE_WAVES > INT32_MAX) return fail(CAGRA_E_OVERFLOW, "too many gather tiles");
    seg->V = V;
    seg->E = E;
    seg->k = k;
    seg->nb = (int32_t)ceil_div(V, seg->B);
    seg->Q = Q;
    seg->ntiles = (int32_t)ntiles;
    const int64_t items = (int64_t)seg->nb + ceil_div(Q, merge_split_entries(Q, seg->nb)) + 1;
    if (items > INT32_MAX) return fail(CAGRA_E_OVERFLOW, "too many merge work items");
    seg->max_items = (int32_t)items;
    SortTemps t;
    if (cagra_status e = sort_temps(E, Q, k, edge16(N), t)) return e;
    seg->build_workspace_bytes = build_layout(E, Q, k, seg->nb, edge16(N) ? 2 : 4, t);
    return CAGRA_OK;
}

static cagra_status allow_big_lds_impl() {
    if (cagra_status a_ = ensure_dynamic_lds((const void *)k_count)) return a_;
    return CAGRA_OK;
}

// 5. merge work items per block (needs block_ptr)
static cagra_status build_block_items(cagra_segments *seg, Arena &ar, hipStream_t st) {
    k_block_items<<<(unsigned)seg->nb, 64, 0, st>>>(seg->block_ptr, seg->k, seg->nb,
                                                     merge_split_entries(seg->Q, seg->nb), seg->block_items);
    CAGRA_LAUNCH_CHECK();
    return scan_i32<ScanAdd>(seg->block_items, seg->block_items, (int64_t)seg->nb + 1, false, ar, st);
}

cagra_status build_segments(const cagra_graph *g, cagra_segments *seg, void *ws, size_t ws_bytes, hipStream_t st) {
    if (cagra_status a = allow_big_lds()) return a;
    const int32_t V = g->V, N = seg->N, B = seg->B, T = seg->tile_edges, k = seg->k, nb = seg->nb;
    const int64_t E = g->E, Q = seg->Q;
    const int32_t ntiles = seg->ntiles;
    const bool w16 = edge16(N);
    SortTemps tmp;
    if (cagra_status e = sort_temps(E, Q, k, w16, tmp)) return e;
    Arena ar{(char *)ws, ws_bytes, 0};
    char *mreg = ar.take<char>(4 * E + 512);
    int32_t *flag = ar.take<int32_t>(E);
    int32_t *run_first = ar.take<int32_t>(Q + 1);
    int32_t *run_sd = ar.take<int32_t>(2 * Q);
    uint16_t *rkey = ar.take<uint16_t>(Q);
    unsigned long long *rval = ar.take<unsigned long long>(Q);
    char *eval32 = w16 ? nullptr : ar.take<char>(4 * E);
    int32_t *tcount = ar.take<int32_t>(k + 1);
    const size_t tmp_bytes = tmp.rows > tmp.edges ? tmp.rows : tmp.edges;
    char *stmp = ar.take<char>((int64_t)tmp_bytes);
    if (!mreg || !flag || !run_first || !run_sd || !rkey || !rval || (!w16 && !eval32) || !tcount || !stmp)
        return fail(CAGRA_E_BUFFER, "build workspace smaller than %zu bytes", seg->build_workspace_bytes);
    int32_t *mark = reinterpret_cast<int32_t *>(mreg);
    int32_t *run_seg = run_sd, *run_dst = run_sd + Q;
    // reuses of dead arrays (see build_layout)
    uint16_t *ekey = reinterpret_cast<uint16_t *>(mreg);
    char *eval = w16 ? mreg + align_up((size_t)E * 2, 256) : eval32;
    uint16_t *ekey_s = reinterpret_cast<uint16_t *>(flag);
    uint16_t *rkey_s = reinterpret_cast<uint16_t *>(run_first);
    unsigned long long *rval_s = reinterpret_cast<unsigned long long *>(run_sd);
    cagra_status s;
    if (E == 0) {
        k_fill_i32<<<grid_for(k + 1, 256), 256, 0, st>>>(seg->seg_row_begin, k + 1, 0);
        CAGRA_LAUNCH_CHECK();
        k_fill_i32<<<1, 64, 0, st>>>(seg->row_ptr, 1, 0);
        CAGRA_LAUNCH_CHECK();
        k_fill_i32<<<grid_for((int64_t)(nb + 1) * k, 256), 256, 0, st>>>(seg->block_ptr, (int64_t)(nb + 1) * k, 0);
        CAGRA_LAUNCH_CHECK();
        k_fill_i32<<<1, 64, 0, st>>>(seg->tile_edge, 1, 0);
        CAGRA_LAUNCH_CHECK();
        return build_block_items(seg, ar, st);
    }
    // 1. run starts, destinations, run ids
    k_fill_i32<<<grid_for(E, 256), 256, 0, st>>>(mark, E, 0);
    CAGRA_LAUNCH_CHECK();
    k_mark_rows<<<grid_for(V, 256), 256, 0, st>>>(g->in_offsets, V, mark);
    CAGRA_LAUNCH_CHECK();
    k_flags<<<grid_for(E, kBThreads * kBItems), kBThreads, 0, st>>>(g->in_sources, mark, E, N, flag);
    CAGRA_LAUNCH_CHECK();
    if ((s = scan_i32<ScanMax>(mark, mark, E, true, ar, st)) != CAGRA_OK) return s;
    if ((s = scan_i32<ScanAdd>(flag, flag, E, true, ar, st)) != CAGRA_OK) return s;
    k_runs<<<grid_for(E, kBThreads * kBItems), kBThreads, 0, st>>>(g->in_sources, mark, flag, E, N, run_first,
                                                                   run_seg, run_dst);
    CAGRA_LAUNCH_CHECK();
    // 2. stable radix sorts by segment: runs (with destination and length) and edges (with their words)
    const int bits = nbits_for(k);
    k_run_kv<<<grid_for(Q, 256), 256, 0, st>>>(run_first, run_seg, run_dst, Q, rkey, rval);
    CAGRA_LAUNCH_CHECK();
    if ((s = seg_sort_pairs<unsigned long long>(rkey, rval, rkey_s, rval_s, Q, bits, stmp, tmp_bytes, st)) !=
        CAGRA_OK)
        return s;
    if (w16) {
        k_edge_kv<uint16_t><<<grid_for(E, kBThreads * kBItems), kBThreads, 0, st>>>(g->in_sources, flag, E, N, ekey,
                                                                                    (uint16_t *)eval);
        CAGRA_LAUNCH_CHECK();
        if ((s = seg_sort_pairs<uint16_t>(ekey, (const uint16_t *)eval, ekey_s, (uint16_t *)seg->edge_src, E, bits,
                                          stmp, tmp_bytes, st)) != CAGRA_OK)
            return s;
    } else {
        k_edge_kv<uint32_t><<<grid_for(E, kBThreads * kBItems), kBThreads, 0, st>>>(g->in_sources, flag, E, N, ekey,
                                                                                    (uint32_t *)eval);
        CAGRA_LAUNCH_CHECK();
        if ((s = seg_sort_pairs<uint32_t>(ekey, (const uint32_t *)eval, ekey_s, (uint32_t *)seg->edge_src, E, bits,
                                          stmp, tmp_bytes, st)) != CAGRA_OK)
            return s;
    }
    k_seg_begin_sorted<<<grid_for(k + 1, 256), 256, 0, st>>>(rkey_s, Q, k, seg->seg_row_begin);
    CAGRA_LAUNCH_CHECK();
    // 3. rows and their edge offsets
    k_rows_sorted<<<grid_for(Q + 1, 256), 256, 0, st>>>(rval_s, Q, B, seg->row_dst, seg->row_dst_lo, seg->row_ptr);
    CAGRA_LAUNCH_CHECK();
    if ((s = scan_i32<ScanAdd>(seg->row_ptr, seg->row_ptr, Q + 1, false, ar, st)) != CAGRA_OK) return s;
    // 4. merge block index and gather tiles
    k_block_ptr<<<grid_for((int64_t)(nb + 1) * k, 256), 256, 0, st>>>(seg->row_dst, seg->seg_row_begin, k, nb, B,
                                                                       seg->block_ptr);
    CAGRA_LAUNCH_CHECK();
    k_tile_count<<<grid_for(k + 1, 256), 256, 0, st>>>(seg->row_ptr, seg->seg_row_begin, k, T, tcount);
    CAGRA_LAUNCH_CHECK();
    if ((s = scan_i32<ScanAdd>(tcount, tcount, k + 1, false, ar, st)) != CAGRA_OK) return s;
    k_tiles<<<grid_for(ntiles + 1, 256), 256, 0, st>>>(seg->row_ptr, seg->seg_row_begin, tcount, k, T, ntiles, E,
                                                       seg->tile_edge, seg->tile_seg);
    CAGRA_LAUNCH_CHECK();
    if (ntiles > 0) {
        k_spans<<<grid_for((int64_t)ntiles * CAGRA_TILE_WAVES, 256), 256, 0, st>>>(
            seg->row_ptr, seg->seg_row_begin, seg->tile_edge, seg->tile_seg, ntiles, seg->tile_span_row);
        CAGRA_LAUNCH_CHECK();
    }
    return build_block_items(seg, ar, st);
}

}  // namespace cagra
