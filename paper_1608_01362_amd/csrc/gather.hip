// Segment processing (Section 3.2): one pass over each subgraph's edges,
// combining the values of the sources (all inside one segment) per
// destination row and writing one buffer value per row, sequentially.
//
// Work unit = tile: a row-aligned range of one subgraph's edges. The 16 waves
// of a workgroup share the segment's values, staged once into LDS (up to
// 128 KB: 32,768 FP32 or 65,536 BF16 values); larger segments are read through
// the cache hierarchy instead (L2- or Infinity-Cache-sized segments). Each wave
// streams an equal share of the tile's edge array with 16-byte non-temporal
// loads, three chunks ahead. Edge words are 16-bit for segments of at most
// 32,768 vertices (15-bit local index) and 32-bit otherwise; the row-start
// flag is the word's top bit, so the per-row
// combination is a segmented scan across the wave (shuffles), and rows that
// cross from one wave's share into the next are completed after a barrier in
// wave order. No atomics; the combination order is fixed by the data layout,
// so results are bit-identical run to run.
#include "common.h"
#include "wave.h"

namespace cagra {

constexpr int kGatherWaves = CAGRA_TILE_WAVES;  // 16 waves, 1024 threads
constexpr int kGatherThreads = kGatherWaves * kWave;
constexpr int kEPT = 8;                         // edges per lane per chunk
constexpr int kChunk = kWave * kEPT;            // edges per wave per chunk
// Per-wave LDS area where a chunk's finished rows (at most kChunk) are
// collected, so that they leave as contiguous 256-byte wave stores.
constexpr int kStageRows = kChunk;
constexpr size_t kStageBytes = (size_t)kGatherWaves * kStageRows * 4;

typedef int32_t v4i __attribute__((ext_vector_type(4)));

// Source value fetch: from the staged LDS copy, or from global memory.
template <typename VT, bool STAGED>
struct Fetch;
template <>
struct Fetch<float, true> {
    using T = float;
    static __device__ __forceinline__ float get(const float *lds, const float *, int32_t i) { return lds[i]; }
};
template <>
struct Fetch<float, false> {
    using T = float;
    static __device__ __forceinline__ float get(const float *, const float *g, int32_t i) { return g[i]; }
};
template <>
struct Fetch<uint16_t, true> {
    using T = float;
    static __device__ __forceinline__ float get(const uint16_t *lds, const uint16_t *, int32_t i) {
        return bf16_to_f32(lds[i]);
    }
};
template <>
struct Fetch<uint16_t, false> {
    using T = float;
    static __device__ __forceinline__ float get(const uint16_t *, const uint16_t *g, int32_t i) {
        return bf16_to_f32(g[i]);
    }
};
template <>
struct Fetch<int32_t, true> {
    using T = int32_t;
    static __device__ __forceinline__ int32_t get(const int32_t *lds, const int32_t *, int32_t i) { return lds[i]; }
};
template <>
struct Fetch<int32_t, false> {
    using T = int32_t;
    static __device__ __forceinline__ int32_t get(const int32_t *, const int32_t *g, int32_t i) { return g[i]; }
};

template <typename T>
struct WaveFix {
    T head;        // combination of the edges before the wave's first row start
    T last;        // value of the wave's last open row
    int32_t row;   // that row's index
    int32_t has;   // the wave saw at least one row start
};

template <typename VT>
__device__ __forceinline__ void stage_segment(const VT *__restrict__ g, int32_t n, VT *lds) {
    // 16-byte copies when the segment start is 16-byte aligned, element copies otherwise.
    const int per = 16 / sizeof(VT);
    if ((reinterpret_cast<uintptr_t>(g) & 15) == 0) {
        int nv = n / per;
        const v4i *gv = reinterpret_cast<const v4i *>(g);
        v4i *lv = reinterpret_cast<v4i *>(lds);
        for (int i = threadIdx.x; i < nv; i += blockDim.x) lv[i] = gv[i];
        for (int i = nv * per + threadIdx.x; i < n; i += blockDim.x) lds[i] = g[i];
    } else {
        for (int i = threadIdx.x; i < n; i += blockDim.x) lds[i] = g[i];
    }
}

// One step of the segmented scan (flag f, value v): a lane keeps its value if
// it holds a row start, else prepends the value of the lanes before it.
template <class Op, int CTRL, int ROWMASK>
__device__ __forceinline__ void seg_step(int32_t &f, typename Op::T &v) {
    using T = typename Op::T;
    const T pv = dpp_t<CTRL, ROWMASK>(Op::identity(), v);
    const int32_t pf = dpp_i<CTRL, ROWMASK>(0, f);
    v = f ? v : Op::apply(pv, v);
    f |= pf;
}

template <class Op>
__device__ __forceinline__ void wave_seg_scan(int32_t &f, typename Op::T &v) {
    seg_step<Op, kDppRowShr1, 0xf>(f, v);
    seg_step<Op, kDppRowShr2, 0xf>(f, v);
    seg_step<Op, kDppRowShr4, 0xf>(f, v);
    seg_step<Op, kDppRowShr8, 0xf>(f, v);
    seg_step<Op, kDppRowBcast15, 0xa>(f, v);
    seg_step<Op, kDppRowBcast31, 0xc>(f, v);
}

__device__ __forceinline__ int32_t readlane_t(int32_t x, int l) { return __builtin_amdgcn_readlane(x, l); }
__device__ __forceinline__ float readlane_t(float x, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
}

// Per-wave state carried from chunk to chunk.
template <typename T>
struct SpanState {
    T carry;        // value of the row open at the current chunk start
    T head;         // value of the row that began before the wave's share
    int32_t nflags; // row starts seen in earlier chunks
};

// 16-byte loads per lane per chunk for edge words of type W.
template <typename W>
constexpr int kLoads = kEPT * (int)sizeof(W) / 16;

// Processes one chunk of kChunk edges (this lane: kEPT consecutive edges).
// rel0 is the chunk's first edge relative to the wave's share [0, len) (it is
// negative for a first chunk that starts before the share); FULL chunks lie
// entirely inside the share and skip the per-edge bounds tests. Rows finished
// in the chunk are exactly chunk_nf consecutive rows starting at row0 + nflags
// - 1; they are collected in `stage` and written with coalesced stores.
template <class Op, typename VT, bool STAGED, typename W, bool FULL>
__device__ __forceinline__ void process_chunk(const v4i (&wv)[kLoads<W>], int32_t rel0, int32_t len,
                                              const VT *seg_vals, const VT *gvals, typename Op::T *stage,
                                              __amdgpu_buffer_rsrc_t out, SpanState<typename Op::T> &S) {
    using T = typename Op::T;
    using F = Fetch<VT, STAGED>;
    const int lane = __lane_id();
    const int32_t rel = rel0 + lane * kEPT;
    uint32_t w[kEPT];
    if constexpr (sizeof(W) == 4) {
#pragma unroll
        for (int j = 0; j < kLoads<W>; ++j)
#pragma unroll
            for (int c = 0; c < 4; ++c) w[4 * j + c] = (uint32_t)wv[j][c];
    } else {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            w[2 * c] = (uint32_t)wv[0][c] & 0xffffu;
            w[2 * c + 1] = (uint32_t)wv[0][c] >> 16;
        }
    }
    bool fl[kEPT];  // row starts
    T v[kEPT];
#pragma unroll
    for (int i = 0; i < kEPT; ++i) {
        if constexpr (FULL) {
            fl[i] = (w[i] & EdgeWord<W>::kFlag) != 0u;
            v[i] = F::get(seg_vals, gvals, (int32_t)(w[i] & EdgeWord<W>::kIndex));
        } else {
            const bool valid = (uint32_t)(rel + i) < (uint32_t)len;
            fl[i] = valid && (w[i] & EdgeWord<W>::kFlag) != 0u;
            // words outside the share may belong to another segment: read index 0 instead
            const T x = F::get(seg_vals, gvals, valid ? (int32_t)(w[i] & EdgeWord<W>::kIndex) : 0);
            v[i] = valid ? x : Op::identity();
        }
    }
    int32_t nf = 0;
#pragma unroll
    for (int i = 0; i < kEPT; ++i) nf += fl[i] ? 1 : 0;
    const int32_t incl_nf = wave_incl_sum(nf);
    const int32_t excl_nf = incl_nf - nf;
    const int32_t chunk_nf = __builtin_amdgcn_readlane(incl_nf, 63);

    // lane-local pass: at every row start the running value is written to the
    // lane's next stage slot. The first one is the part of a row that began
    // before the lane (completed below with the incoming value); every later
    // one closes a row that lies entirely inside the lane.
    T run = Op::identity();
    T *slot = stage + excl_nf;
#pragma unroll
    for (int i = 0; i < kEPT; ++i) {
        if (fl[i]) *slot = run;
        slot += fl[i] ? 1 : 0;
        run = fl[i] ? v[i] : Op::apply(run, v[i]);
    }
    // segmented inclusive scan of (has row start, tail value) over the wave
    T sv = run;
    int32_t sf = nf > 0;
    wave_seg_scan<Op>(sf, sv);
    const T ex_v = dpp_t<kDppWaveShr1, 0xf>(Op::identity(), sv);
    const int32_t ex_f = dpp_i<kDppWaveShr1, 0xf>(0, sf);
    const T incoming = ex_f ? ex_v : Op::apply(S.carry, ex_v);
    if (nf > 0) stage[excl_nf] = Op::apply(incoming, stage[excl_nf]);
    __builtin_amdgcn_wave_barrier();
    // stage[0] is the row that began before this wave's share when the wave
    // had not seen a row start yet: that one is completed across waves later
    const bool head_here = S.nflags == 0 && chunk_nf > 0;
    const int32_t rbase = S.nflags - 1;  // staged index 0 <-> row row0 + rbase
#pragma unroll
    for (int r = 0; r < kEPT; ++r) {
        if (r * kWave >= chunk_nf) break;  // uniform: chunk_nf is wave-wide
        const int32_t i = r * kWave + lane;
        const T val = stage[i];
        const bool ok = i < chunk_nf && !(head_here && i == 0);
        const uint32_t off = ok ? (uint32_t)(rbase + i) * (uint32_t)sizeof(T) : kOutOfRange;
        __builtin_amdgcn_raw_buffer_store_b32(*reinterpret_cast<const int32_t *>(&val), out, off, 0, 0);
    }
    if (head_here) S.head = stage[0];
    __builtin_amdgcn_wave_barrier();
    const T in63 = readlane_t(sv, 63);
    const int32_t f63 = __builtin_amdgcn_readlane(sf, 63);
    S.carry = f63 ? in63 : Op::apply(S.carry, in63);
    S.nflags += chunk_nf;
}

template <typename W>
__device__ __forceinline__ void load_chunk(v4i (&r)[kLoads<W>], __amdgpu_buffer_rsrc_t ein, uint32_t off) {
#pragma unroll
    for (int j = 0; j < kLoads<W>; ++j) r[j] = __builtin_amdgcn_raw_buffer_load_b128(ein, off + 16 * j, 0, kNonTemporal);
}

// Chunks of edge words each wave keeps in flight (all but one ahead of the one
// processed). The LDS-staged gather with 16-bit words over long tiles keeps
// kStagesDeep: its shares are dozens of chunks long and it runs one workgroup
// per CU whatever its registers. Short tiles (the multi-graph runs, small
// graphs) and the other forms keep kStagesDefault: there a deeper prologue
// mostly loads past the share, or two workgroups per CU must fit in registers.
constexpr int kStagesDeep = 8;
constexpr int kStagesDefault = 4;
constexpr int32_t kDeepTileEdges = 131072;  // tiles at least this long take kStagesDeep

template <class Op, typename VT, bool STAGED, typename W, int DEPTH>
__device__ __forceinline__ void gather_tile(const W *__restrict__ edge_src, int64_t Q,
                                            const int32_t *__restrict__ tile_edge,
                                            const int32_t *__restrict__ tile_seg,
                                            const int32_t *__restrict__ span_row, const VT *__restrict__ values,
                                            int32_t V, int32_t N, int t, typename Op::T *__restrict__ partial,
                                            unsigned char *smem, const uint32_t *__restrict__ seg_active) {
    using T = typename Op::T;
    VT *seg_vals = reinterpret_cast<VT *>(smem + kStageBytes);
    const int64_t e0 = tile_edge[t], e1 = tile_edge[t + 1];
    if (e0 >= e1) return;  // empty tile (uniform over the workgroup)
    const int32_t s = tile_seg[t];
    // an inactive segment (no source in the frontier) contributes nothing: its
    // rows are skipped here and by the merge
    if (seg_active && !((seg_active[s >> 5] >> (s & 31)) & 1u)) return;
    const int64_t vbase = (int64_t)s * N;
    const VT *gvals = values + vbase;
    if (STAGED) {
        int64_t n = (int64_t)V - vbase;
        if (n > N) n = N;
        stage_segment<VT>(gvals, (int32_t)n, seg_vals);
        __syncthreads();
    }

    // wave index as a scalar, so that everything derived from it stays in SGPRs
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int64_t sl = (e1 - e0 + kGatherWaves - 1) / kGatherWaves;
    int64_t w0 = e0 + w * sl;
    if (w0 > e1) w0 = e1;
    int64_t w1 = w0 + sl;
    if (w1 > e1) w1 = e1;
    const int32_t row0 = span_row[(int64_t)t * kGatherWaves + w];

    // Buffer descriptors: loads past the share read zero, and stores to rows
    // outside [row0, Q) are dropped, so the loop needs no bounds branches.
    // ebase: the share's start rounded down to a 16-byte boundary; the range
    // is rounded up to whole dwords so the share's last word is never cut off
    constexpr int kWB = (int)sizeof(W);
    const int64_t ebase = w0 & ~(int64_t)(16 / kWB - 1);
    const __amdgpu_buffer_rsrc_t ein = __builtin_amdgcn_make_buffer_rsrc(
        (void *)(edge_src + ebase), 0, (int32_t)align_up((size_t)(w1 - ebase) * kWB, 4), kBufFlags);
    int64_t rows_left = Q - row0;
    if (rows_left > (1 << 28)) rows_left = 1 << 28;
    if (rows_left < 0) rows_left = 0;
    const __amdgpu_buffer_rsrc_t out = __builtin_amdgcn_make_buffer_rsrc(
        (void *)(partial + row0), 0, (int32_t)(rows_left * (int64_t)sizeof(T)), kBufFlags);

    SpanState<T> S{Op::identity(), Op::identity(), 0};
    T *stage = reinterpret_cast<T *>(smem) + (size_t)w * kStageRows;
    const int64_t len = w1 - ebase;
    const int32_t share = (int32_t)(w1 - w0);
    const uint32_t lane_off = (uint32_t)(lane * kEPT * kWB);
    constexpr int kSt = DEPTH;
    v4i R[kSt][kLoads<W>];
#pragma unroll
    for (int c = 0; c < kSt - 1; ++c) load_chunk<W>(R[c], ein, (uint32_t)(c * kChunk * kWB) + lane_off);
    for (int64_t cc = 0; cc < len; cc += kSt * kChunk) {
#pragma unroll
        for (int c = 0; c < kSt; ++c) {
            if (cc + c * kChunk >= len) break;  // uniform: len and cc are wave-wide
            load_chunk<W>(R[(c + kSt - 1) % kSt], ein,
                          (uint32_t)((cc + (c + kSt - 1) * kChunk) * kWB) + lane_off);
            const int32_t rel0 = (int32_t)(ebase + cc + c * kChunk - w0);
            if (rel0 >= 0 && rel0 + kChunk <= share)
                process_chunk<Op, VT, STAGED, W, true>(R[c], rel0, share, seg_vals, gvals, stage, out, S);
            else
                process_chunk<Op, VT, STAGED, W, false>(R[c], rel0, share, seg_vals, gvals, stage, out, S);
        }
    }

    // complete rows that continue into later waves' shares, in wave order
    __syncthreads();  // all waves are done with the staged values
    WaveFix<T> *fix = reinterpret_cast<WaveFix<T> *>(smem);
    if (lane == 0) {
        WaveFix<T> f;
        f.has = S.nflags > 0;
        f.head = f.has ? S.head : S.carry;
        f.last = S.carry;
        f.row = row0 + S.nflags - 1;
        fix[w] = f;
    }
    __syncthreads();
    if (threadIdx.x < kGatherWaves) {
        const int ww = threadIdx.x;
        if (fix[ww].has) {
            T tot = fix[ww].last;
            for (int x = ww + 1; x < kGatherWaves; ++x) {
                tot = Op::apply(tot, fix[x].head);
                if (fix[x].has) break;
            }
            partial[fix[ww].row] = tot;
        }
    }
}

template <class Op, typename VT, bool STAGED, typename W, int DEPTH>
__global__ __launch_bounds__(kGatherThreads) void k_gather(
    const W *__restrict__ edge_src, int64_t E, int64_t Q, const int32_t *__restrict__ tile_edge,
    const int32_t *__restrict__ tile_seg, const int32_t *__restrict__ span_row, const VT *__restrict__ values,
    int32_t V, int32_t N, int32_t ntiles, typename Op::T *__restrict__ partial,
    const uint32_t *__restrict__ seg_active) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    (void)E;
    gather_tile<Op, VT, STAGED, W, DEPTH>(edge_src, Q, tile_edge, tile_seg, span_row, values, V, N,
                                          xcd_remap(blockIdx.x, ntiles), partial, smem, seg_active);
}

// Persistent form over many graphs: workgroups stride over a global tile list.
__global__ __launch_bounds__(kGatherThreads) void k_multi_gather(const MultiDesc *__restrict__ desc,
                                                                 const int32_t *__restrict__ tile_graph,
                                                                 int64_t total_tiles, int parity) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    for (int64_t gt = blockIdx.x; gt < total_tiles; gt += gridDim.x) {
        __syncthreads();  // LDS reuse across tiles
        const int gi = tile_graph[gt];
        const MultiDesc &d = desc[gi];
        gather_tile<OpSum, float, true, uint16_t, kStagesDefault>(static_cast<const uint16_t *>(d.edge_src), d.Q, d.tile_edge, d.tile_seg, d.tile_span_row,
                                        d.contrib[parity], d.V, d.N, (int)(gt - d.tile_base), d.partial, smem,
                                        nullptr);
    }
}

cagra_status launch_multi_gather(const MultiDesc *desc, const int32_t *tile_graph, int64_t total_tiles, int parity,
                                 int grid, hipStream_t st) {
    if (cagra_status a_ = ensure_dynamic_lds((const void *)k_multi_gather)) return a_;
    if (total_tiles == 0) return CAGRA_OK;
    k_multi_gather<<<grid, kGatherThreads, kStageBytes + CAGRA_STAGE_BYTES, st>>>(desc, tile_graph, total_tiles,
                                                                                   parity);
    CAGRA_LAUNCH_CHECK();
    return CAGRA_OK;
}

template <class Op, typename VT, bool STAGED, typename W>
static cagra_status launch_gather_w(const cagra_segments *seg, const VT *values, typename Op::T *partial,
                                    const uint32_t *seg_active, hipStream_t st) {
    if (seg->ntiles == 0) return CAGRA_OK;
    auto kern = k_gather<Op, VT, STAGED, W, kStagesDefault>;
    if constexpr (STAGED && sizeof(W) == 2)
        if (seg->tile_edges >= kDeepTileEdges) kern = k_gather<Op, VT, STAGED, W, kStagesDeep>;
    const size_t lds = kStageBytes + (STAGED ? (size_t)seg->N * sizeof(VT) : 0);
    if (cagra_status a_ = ensure_dynamic_lds((const void *)kern)) return a_;
    kern<<<seg->ntiles, kGatherThreads, lds, st>>>(static_cast<const W *>(seg->edge_src), seg->E, seg->Q,
                                                  seg->tile_edge, seg->tile_seg, seg->tile_span_row, values, seg->V,
                                                  seg->N, seg->ntiles, partial, seg_active);
    CAGRA_LAUNCH_CHECK();
    return CAGRA_OK;
}

// Staged segments of at most CAGRA_EDGE16_MAX_N vertices use 16-bit edge
// words; larger staged ones (BF16 values) and all unstaged ones use 32-bit words.
template <class Op, typename VT, bool STAGED>
static cagra_status launch_gather_t(const cagra_segments *seg, const VT *values, typename Op::T *partial,
                                    const uint32_t *seg_active, hipStream_t st) {
    if constexpr (STAGED) {
        if (edge16(seg->N)) return launch_gather_w<Op, VT, true, uint16_t>(seg, values, partial, seg_active, st);
        if constexpr (sizeof(VT) == 2)
            return launch_gather_w<Op, VT, true, uint32_t>(seg, values, partial, seg_active, st);
        return fail(CAGRA_E_INVALID, "internal: staged segment of %d vertices with 32-bit edge words", seg->N);
    } else {
        if (edge16(seg->N)) return fail(CAGRA_E_INVALID, "internal: unstaged segment of %d vertices", seg->N);
        return launch_gather_w<Op, VT, false, uint32_t>(seg, values, partial, seg_active, st);
    }
}

bool gather_staged(int32_t N, int32_t value_type) {
    size_t bytes = value_type == CAGRA_BF16 ? 2 : 4;
    static_assert(kStageBytes + CAGRA_STAGE_BYTES <= CAGRA_LDS_BYTES, "LDS budget");
    return (size_t)N * bytes <= CAGRA_STAGE_BYTES;
}

cagra_status launch_gather_active(const cagra_segments *seg, int32_t op, int32_t value_type, const void *values,
                                  void *partial, const uint32_t *seg_active, hipStream_t st) {
    const bool staged = gather_staged(seg->N, value_type);
    if (op == CAGRA_SUM_F32 && value_type == CAGRA_F32) {
        return staged ? launch_gather_t<OpSum, float, true>(seg, (const float *)values, (float *)partial, seg_active, st)
                      : launch_gather_t<OpSum, float, false>(seg, (const float *)values, (float *)partial, seg_active, st);
    }
    if (op == CAGRA_SUM_F32 && value_type == CAGRA_BF16) {
        return staged ? launch_gather_t<OpSum, uint16_t, true>(seg, (const uint16_t *)values, (float *)partial, seg_active, st)
                      : launch_gather_t<OpSum, uint16_t, false>(seg, (const uint16_t *)values, (float *)partial, seg_active, st);
    }
    if (op == CAGRA_MIN_I32 && value_type == CAGRA_I32) {
        return staged ? launch_gather_t<OpMin, int32_t, true>(seg, (const int32_t *)values, (int32_t *)partial, seg_active, st)
                      : launch_gather_t<OpMin, int32_t, false>(seg, (const int32_t *)values, (int32_t *)partial, seg_active, st);
    }
    return fail(CAGRA_E_INVALID, "unsupported gather op %d / value type %d", op, value_type);
}

cagra_status launch_gather(const cagra_segments *seg, int32_t op, int32_t value_type, const void *values,
                           void *partial, hipStream_t st) {
    return launch_gather_active(seg, op, value_type, values, partial, nullptr, st);
}

}  // namespace cagra
