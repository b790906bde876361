// Segment processing (Section 3.2): one pass over each subgraph's edges,
// combining the values of the sources (all inside one segment) per
// destination row and writing one buffer value per row, sequentially.
//
// Work unit = tile: a row-aligned range of one subgraph's edges. The 16 waves
// of a workgroup share the segment's values, staged once into LDS (up to
// 160 KB: 40,960 FP32 or 81,920 BF16 values); larger segments are read through
// the cache hierarchy instead (L2- or Infinity-Cache-sized segments). Each wave
// streams an equal share of the tile's edge array with 16-byte non-temporal
// loads. Row boundaries are bit 31 of the edge word, so the per-row
// combination is a segmented scan across the wave (shuffles), and rows that
// cross from one wave's share into the next are completed after a barrier in
// wave order. No atomics; the combination order is fixed by the data layout,
// so results are bit-identical run to run.
#include "common.h"

namespace cagra {

constexpr int kGatherWaves = CAGRA_TILE_WAVES;  // 16 waves, 1024 threads
constexpr int kGatherThreads = kGatherWaves * kWave;
constexpr int kEPT = 16;                        // edges per lane per chunk
constexpr int kChunk = kWave * kEPT;            // edges per wave per chunk

typedef int32_t v4i __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void load_edges(const int32_t *__restrict__ p, int64_t idx, int64_t E,
                                           int32_t (&w)[kEPT]) {
    if (idx + kEPT <= E) {
#pragma unroll
        for (int j = 0; j < kEPT / 4; ++j) {
            v4i v = __builtin_nontemporal_load(reinterpret_cast<const v4i *>(p + idx) + j);
            w[4 * j + 0] = v.x;
            w[4 * j + 1] = v.y;
            w[4 * j + 2] = v.z;
            w[4 * j + 3] = v.w;
        }
    } else {
#pragma unroll
        for (int i = 0; i < kEPT; ++i) w[i] = (idx + i < E) ? p[idx + i] : 0;
    }
}

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

template <class Op, typename VT, bool STAGED>
__global__ __launch_bounds__(kGatherThreads) void k_gather(
    const int32_t *__restrict__ edge_src, int64_t E, const int32_t *__restrict__ tile_edge,
    const int32_t *__restrict__ tile_seg, const int32_t *__restrict__ span_row, const VT *__restrict__ values,
    int32_t V, int32_t N, int32_t ntiles, typename Op::T *__restrict__ partial) {
    using T = typename Op::T;
    using F = Fetch<VT, STAGED>;
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    VT *seg_vals = reinterpret_cast<VT *>(smem);

    const int t = xcd_remap(blockIdx.x, ntiles);
    const int64_t e0 = tile_edge[t], e1 = tile_edge[t + 1];
    if (e0 >= e1) return;  // empty tile (uniform over the workgroup)
    const int32_t s = tile_seg[t];
    const int64_t vbase = (int64_t)s * N;
    const VT *gvals = values + vbase;
    if (STAGED) {
        int64_t n = (int64_t)V - vbase;
        if (n > N) n = N;
        stage_segment<VT>(gvals, (int32_t)n, seg_vals);
        __syncthreads();
    }

    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t sl = (e1 - e0 + kGatherWaves - 1) / kGatherWaves;
    int64_t w0 = e0 + w * sl;
    if (w0 > e1) w0 = e1;
    int64_t w1 = w0 + sl;
    if (w1 > e1) w1 = e1;
    const int32_t row0 = span_row[(int64_t)t * kGatherWaves + w];

    T carry = Op::identity();  // value of the row open at the current chunk start
    T head = Op::identity();
    int32_t nflags = 0;        // row starts seen by this wave in earlier chunks
    const uint64_t lt = lanemask_lt();

    int64_t c = w0 & ~(int64_t)3;
    int32_t cur[kEPT], nxt[kEPT];
    if (c < w1) load_edges(edge_src, c + lane * kEPT, E, cur);
    for (; c < w1; c += kChunk) {
        const int64_t cn = c + kChunk;
        if (cn < w1) load_edges(edge_src, cn + lane * kEPT, E, nxt);
        const int64_t idx = c + lane * kEPT;
        uint32_t fmask = 0;
        T v[kEPT];
#pragma unroll
        for (int i = 0; i < kEPT; ++i) {
            const bool valid = (idx + i >= w0) && (idx + i < w1);
            const int32_t wd = cur[i];
            fmask |= (valid && wd < 0) ? (1u << i) : 0u;
            v[i] = valid ? F::get(seg_vals, gvals, wd & 0x7fffffff) : Op::identity();
        }
        const int nf = __popc(fmask);
        // exclusive prefix of row starts over lanes, and the chunk total
        int32_t incl_nf = nf;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            int32_t o = __shfl_up(incl_nf, d, 64);
            if (lane >= d) incl_nf += o;
        }
        const int32_t excl_nf = incl_nf - nf;
        const int32_t chunk_nf = __shfl(incl_nf, 63, 64);
        const int32_t rb = row0 + nflags + excl_nf;  // row started by this lane's first flag

        // lane-local: rows that start and end inside the lane are written here
        T run = Op::identity(), headpart = Op::identity();
        int j = 0;
#pragma unroll
        for (int i = 0; i < kEPT; ++i) {
            if ((fmask >> i) & 1u) {
                if (j == 0) headpart = run;
                else partial[rb + j - 1] = run;
                ++j;
                run = Op::identity();
            }
            run = Op::apply(run, v[i]);
        }
        // segmented inclusive scan of (has_flag, tail value) across lanes
        T sv = run;
        int sf = nf > 0;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            T ov = __shfl_up(sv, d, 64);
            int of = __shfl_up(sf, d, 64);
            if (lane >= d) {
                if (!sf) sv = Op::apply(ov, sv);
                sf |= of;
            }
        }
        T ex_v = __shfl_up(sv, 1, 64);
        int ex_f = __shfl_up(sf, 1, 64);
        if (lane == 0) {
            ex_v = Op::identity();
            ex_f = 0;
        }
        const T incoming = ex_f ? ex_v : Op::apply(carry, ex_v);
        const T closed = Op::apply(incoming, headpart);
        const bool first_of_wave = nf > 0 && nflags + excl_nf == 0;
        if (nf > 0 && !first_of_wave) partial[rb - 1] = closed;
        // the row that began before this wave's share ends at the wave's first
        // row start; that lane's value is broadcast for the cross-wave fix-up
        const uint64_t hm = __ballot(first_of_wave);
        if (hm) head = __shfl(closed, __ffsll((unsigned long long)hm) - 1, 64);
        const T in63 = __shfl(sv, 63, 64);
        const int f63 = __shfl(sf, 63, 64);
        carry = f63 ? in63 : Op::apply(carry, in63);
        nflags += chunk_nf;
#pragma unroll
        for (int i = 0; i < kEPT; ++i) cur[i] = nxt[i];
    }
    (void)lt;

    // complete rows that continue into later waves' shares, in wave order
    __syncthreads();  // all waves are done with the staged values
    WaveFix<T> *fix = reinterpret_cast<WaveFix<T> *>(smem);
    if (lane == 0) {
        WaveFix<T> f;
        f.has = nflags > 0;
        f.head = f.has ? head : carry;
        f.last = carry;
        f.row = row0 + nflags - 1;
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

template <class Op, typename VT, bool STAGED>
static cagra_status launch_gather_t(const cagra_segments *seg, const VT *values, typename Op::T *partial,
                                    hipStream_t st) {
    if (seg->ntiles == 0) return CAGRA_OK;
    auto kern = k_gather<Op, VT, STAGED>;
    size_t lds = STAGED ? (size_t)seg->N * sizeof(VT) : 0;
    if (lds < kGatherWaves * sizeof(WaveFix<typename Op::T>)) lds = kGatherWaves * sizeof(WaveFix<typename Op::T>);
    static bool attr_set = false;
    if (!attr_set) {
        if (cagra_status a_ = allow_dynamic_lds((const void *)kern)) return a_;
        attr_set = true;
    }
    kern<<<seg->ntiles, kGatherThreads, lds, st>>>(seg->edge_src, seg->E, seg->tile_edge, seg->tile_seg,
                                                  seg->tile_span_row, values, seg->V, seg->N, seg->ntiles, partial);
    CAGRA_LAUNCH_CHECK();
    return CAGRA_OK;
}

bool gather_staged(int32_t N, int32_t value_type) {
    size_t bytes = value_type == CAGRA_BF16 ? 2 : 4;
    return (size_t)N * bytes <= CAGRA_LDS_BYTES;
}

cagra_status launch_gather(const cagra_segments *seg, int32_t op, int32_t value_type, const void *values,
                           void *partial, hipStream_t st) {
    const bool staged = gather_staged(seg->N, value_type);
    if (op == CAGRA_SUM_F32 && value_type == CAGRA_F32) {
        return staged ? launch_gather_t<OpSum, float, true>(seg, (const float *)values, (float *)partial, st)
                      : launch_gather_t<OpSum, float, false>(seg, (const float *)values, (float *)partial, st);
    }
    if (op == CAGRA_SUM_F32 && value_type == CAGRA_BF16) {
        return staged ? launch_gather_t<OpSum, uint16_t, true>(seg, (const uint16_t *)values, (float *)partial, st)
                      : launch_gather_t<OpSum, uint16_t, false>(seg, (const uint16_t *)values, (float *)partial, st);
    }
    if (op == CAGRA_MIN_I32 && value_type == CAGRA_I32) {
        return staged ? launch_gather_t<OpMin, int32_t, true>(seg, (const int32_t *)values, (int32_t *)partial, st)
                      : launch_gather_t<OpMin, int32_t, false>(seg, (const int32_t *)values, (int32_t *)partial, st);
    }
    return fail(CAGRA_E_INVALID, "unsupported gather op %d / value type %d", op, value_type);
}

}  // namespace cagra
