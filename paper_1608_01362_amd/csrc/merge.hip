// Cache-aware merge (Section 3.3) and the per-vertex update that follows it
// (Section 4, VertexMap of the PageRank program).
//
// Destinations are cut into blocks of B vertices whose accumulators live in
// LDS. For block b, subgraph s contributes the buffer entries
// [block_ptr[b*k+s], block_ptr[(b+1)*k+s]); every read of the buffers and of
// row_dst is sequential, and every random update hits LDS.
//
// Two schedules:
//  * k_merge_ordered: the paper's order exactly -- subgraphs in ascending
//    order, one wave per block, lanes over the entries of one subgraph's range
//    (distinct destinations, so no conflicts). Used by cagra_merge for float
//    sums (plain or Neumaier-compensated) and int minimum.
//  * k_merge_pr / k_merge_lp: all 16 waves of the workgroup stream the block's
//    entries at once (flattened over subgraphs), updating shared LDS
//    accumulators with atomics whose result does not depend on their order:
//    int32 minimum for labels, and for PageRank an int64 fixed-point sum
//    (each FP32 buffer value scaled by 2^56 and truncated), which adds the buffer
//    values exactly. The epilogue then applies the vertex update.
#include <math.h>

#include "blockwalk.h"
#include "common.h"

namespace cagra {

// Dynamic LDS of the fused merges; kFusedStaticLds covers their static arrays.
constexpr size_t kFusedStaticLds = 256;
size_t merge_fused_lds_bytes(int32_t B, int32_t k, int acc_bytes) {
    return align_up((size_t)B * acc_bytes, 16) + (size_t)(2 * (int64_t)k + 2) * sizeof(int32_t) + 64;
}
size_t merge_fused_lds_total(int32_t B, int32_t k, int acc_bytes) {
    return merge_fused_lds_bytes(B, k, acc_bytes) + kFusedStaticLds;
}

// ---------------------------------------------------------------- ordered (paper) merge

// One wave per block, subgraphs strictly in ascending order. The block's range
// bounds are staged in LDS first (when they fit), and the entries of the next
// kOrdDepth - 1 non-empty subgraphs (up to kOrdBatch per range) are in flight
// while the current one is applied, so the wave does not wait on memory once
// per subgraph.
// Entries of one subgraph have distinct destinations, so the lanes of a batch
// never collide; the order across subgraphs is the program order of the wave.
constexpr int kOrdLoads = 4;                    // entries per lane per batch
constexpr int kOrdBatch = kOrdLoads * kWave;    // entries of a range loaded ahead
constexpr int kOrdDepth = 6;                    // ranges in flight (8 loads each)

template <typename T>
struct OrdBatch {
    T x[kOrdLoads];
    int32_t d[kOrdLoads];  // entries past the range hold the range's first entry again
};

template <class Op, bool COMP>
__device__ __forceinline__ void ord_apply(typename Op::T *acc, typename Op::T *cmp, int32_t d,
                                          typename Op::T x) {
    if (COMP) {
        // Neumaier (1974) compensated summation
        float sacc = acc[d];
        float tsum = sacc + x;
        if (fabsf(sacc) >= fabsf(x)) cmp[d] += (sacc - tsum) + x;
        else cmp[d] += (x - tsum) + sacc;
        acc[d] = tsum;
    } else {
        acc[d] = Op::apply(acc[d], x);
    }
}

// Applies the entries of one loaded batch (lane entries lo + j * 64 + lane
// below hi). A range's entries have distinct destinations, so every
// accumulator of the batch is read before any is written: one LDS round trip
// per batch instead of one per entry (R-MAT 25 FP32 sum: 1.80 -> 1.70 ms).
// Entries past the range read the destination of the range's first entry and
// write nothing.
template <class Op, bool COMP>
__device__ __forceinline__ void ord_apply_batch(typename Op::T *acc, typename Op::T *cmp,
                                                const OrdBatch<typename Op::T> &q, int32_t lo, int32_t hi,
                                                int lane) {
    using T = typename Op::T;
    T a[kOrdLoads], cm[kOrdLoads];
#pragma unroll
    for (int j = 0; j < kOrdLoads; ++j) {
        a[j] = acc[q.d[j]];
        if (COMP) cm[j] = cmp[q.d[j]];
    }
#pragma unroll
    for (int j = 0; j < kOrdLoads; ++j) {
        if (lo + j * kWave + lane >= hi) continue;
        const T x = q.x[j];
        if (COMP) {
            // the Neumaier step of ord_apply on the values read above
            const float sacc = a[j];
            const float tsum = sacc + x;
            if (fabsf(sacc) >= fabsf(x)) cmp[q.d[j]] = cm[j] + ((sacc - tsum) + x);
            else cmp[q.d[j]] = cm[j] + ((x - tsum) + sacc);
            acc[q.d[j]] = tsum;
        } else {
            acc[q.d[j]] = Op::apply(a[j], x);
        }
    }
}

template <class Op, bool COMP, bool STAGED>
__global__ __launch_bounds__(64) void k_merge_ordered(const uint16_t *__restrict__ row_dst_lo,
                                                      const int32_t *__restrict__ block_ptr,
                                                      const typename Op::T *__restrict__ partial, int32_t V,
                                                      int32_t k, int32_t B, int32_t nb,
                                                      typename Op::T *__restrict__ out,
                                                      const uint32_t *__restrict__ seg_active) {
    using T = typename Op::T;
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    T *acc = reinterpret_cast<T *>(smem);
    T *cmp = acc + B;  // Neumaier compensation terms (COMP only)
    int32_t *lo_s = reinterpret_cast<int32_t *>(smem + (size_t)B * sizeof(T) * (COMP ? 2 : 1));
    int32_t *hi_s = lo_s + k;
    const int b = xcd_remap(blockIdx.x, nb);
    const int64_t vb = (int64_t)b * B;
    int32_t nv = (int32_t)((int64_t)V - vb < B ? (int64_t)V - vb : B);
    const int lane = threadIdx.x;
    for (int i = lane; i < nv; i += 64) {
        acc[i] = Op::identity();
        if (COMP) cmp[i] = Op::identity();
    }
    // range of subgraph s in this block; inactive subgraphs (no rows written) are empty
    auto range = [&](int32_t s, int32_t &lo, int32_t &hi) {
        if (STAGED) {
            lo = lo_s[s];
            hi = hi_s[s];
        } else {
            lo = block_ptr[(int64_t)b * k + s];
            hi = block_ptr[(int64_t)(b + 1) * k + s];
            if (seg_active && !((seg_active[s >> 5] >> (s & 31)) & 1u)) hi = lo;
        }
    };
    if (STAGED) {
        for (int32_t s = lane; s < k; s += 64) {
            const int32_t lo = block_ptr[(int64_t)b * k + s], hi = block_ptr[(int64_t)(b + 1) * k + s];
            const bool act = !seg_active || ((seg_active[s >> 5] >> (s & 31)) & 1u);
            lo_s[s] = lo;
            hi_s[s] = act ? hi : lo;
        }
    }
    __builtin_amdgcn_wave_barrier();
    // next subgraph at or after s with entries in this block (k if none); uniform
    auto next = [&](int32_t s, int32_t &lo, int32_t &hi) {
        for (; s < k; ++s) {
            range(s, lo, hi);
            if (hi > lo) break;
        }
        return s;
    };
    // Loads only: nothing here uses their values, so none waits; whether an
    // entry belongs to the range is decided when it is applied.
    auto issue = [&](int32_t lo, int32_t hi, OrdBatch<T> &q) {
#pragma unroll
        for (int j = 0; j < kOrdLoads; ++j) {
            const int32_t i = lo + j * kWave + lane;
            const int32_t ii = i < hi ? i : lo;
            q.x[j] = partial[ii];
            q.d[j] = (int32_t)row_dst_lo[ii];
        }
    };
    // A ring of kOrdDepth non-empty ranges: the loads of the range kOrdDepth - 1
    // places ahead are issued before the current one is applied, and ranges
    // are applied strictly in ascending subgraph order. Every slot issues its
    // loads (past the last range, of a known entry) so that the waits for one
    // slot do not cover the slots behind it.
    int32_t safe_lo = 0, safe_hi = 0;
    int32_t scan = next(0, safe_lo, safe_hi);  // next subgraph to examine
    if (scan < k) {  // uniform: the block has entries; safe_lo indexes one of them
        OrdBatch<T> q[kOrdDepth];
        int32_t qs[kOrdDepth], qlo[kOrdDepth], qhi[kOrdDepth];
        auto fetch = [&](OrdBatch<T> &b, int32_t &bs, int32_t &blo, int32_t &bhi) {
            int32_t l = safe_lo, h = safe_lo;
            scan = next(scan, l, h);
            bs = scan;
            if (scan < k) ++scan;
            else l = h = safe_lo;
            blo = l;
            bhi = h;
            issue(l, h, b);
        };
#pragma unroll
        for (int c = 0; c < kOrdDepth - 1; ++c) fetch(q[c], qs[c], qlo[c], qhi[c]);
        for (bool more = true; more;) {
#pragma unroll
            for (int c = 0; c < kOrdDepth; ++c) {
                constexpr int kLast = kOrdDepth - 1;
                const int nx = (c + kLast) % kOrdDepth;
                fetch(q[nx], qs[nx], qlo[nx], qhi[nx]);
                if (qs[c] >= k) {  // uniform; every later slot is empty too
                    more = false;
                    break;
                }
                ord_apply_batch<Op, COMP>(acc, cmp, q[c], qlo[c], qhi[c], lane);
                // the rest of a long range, still before the next subgraph
                for (int32_t i = qlo[c] + kOrdBatch + lane; i < qhi[c]; i += 64)
                    ord_apply<Op, COMP>(acc, cmp, row_dst_lo[i], partial[i]);
                __builtin_amdgcn_wave_barrier();
            }
        }
    }
    __builtin_amdgcn_wave_barrier();
    for (int i = lane; i < nv; i += 64) out[vb + i] = COMP ? (T)(acc[i] + cmp[i]) : acc[i];
}

// Staged range bounds fit next to the accumulators.
static bool ordered_ranges_staged(int32_t B, int32_t k, bool comp) {
    return (size_t)B * 4 * (comp ? 2 : 1) + (size_t)k * 8 <= CAGRA_LDS_BYTES - 1024;
}

template <class Op, bool COMP, bool STAGED>
static cagra_status launch_ordered_t(const cagra_segments *seg, const void *partial, void *out,
                                     const uint32_t *seg_active, hipStream_t st) {
    using T = typename Op::T;
    auto kern = k_merge_ordered<Op, COMP, STAGED>;
    size_t lds = (size_t)seg->B * sizeof(T) * (COMP ? 2 : 1) + (STAGED ? (size_t)seg->k * 8 : 0);
    if (cagra_status a_ = ensure_dynamic_lds((const void *)kern)) return a_;
    kern<<<seg->nb, 64, lds, st>>>(seg->row_dst_lo, seg->block_ptr, (const T *)partial, seg->V, seg->k, seg->B,
                                   seg->nb, (T *)out, seg_active);
    CAGRA_LAUNCH_CHECK();
    return CAGRA_OK;
}

template <class Op, bool COMP>
static cagra_status launch_ordered(const cagra_segments *seg, const void *partial, void *out,
                                   const uint32_t *seg_active, hipStream_t st) {
    if (ordered_ranges_staged(seg->B, seg->k, COMP))
        return launch_ordered_t<Op, COMP, true>(seg, partial, out, seg_active, st);
    return launch_ordered_t<Op, COMP, false>(seg, partial, out, seg_active, st);
}

size_t merge_ordered_lds_bytes(int32_t B, int32_t op) {
    return (size_t)B * 4 * (op == CAGRA_SUM_F32_COMP ? 2 : 1);
}

cagra_status launch_merge_active(const cagra_segments *seg, int32_t op, const void *partial, void *out,
                                 const uint32_t *seg_active, hipStream_t st) {
    if (seg->nb == 0) return CAGRA_OK;
    switch (op) {
        case CAGRA_SUM_F32: return launch_ordered<OpSum, false>(seg, partial, out, seg_active, st);
        case CAGRA_SUM_F32_COMP: return launch_ordered<OpSum, true>(seg, partial, out, seg_active, st);
        case CAGRA_MIN_I32: return launch_ordered<OpMin, false>(seg, partial, out, seg_active, st);
        default: return fail(CAGRA_E_INVALID, "unknown merge op %d", op);
    }
}

cagra_status launch_merge(const cagra_segments *seg, int32_t op, const void *partial, void *out, hipStream_t st) {
    return launch_merge_active(seg, op, partial, out, nullptr, st);
}

// ---------------------------------------------------------------- fused merges

// round(x * 2^24) as int64 (exact for |x| < 2^38; halves round up in magnitude).
__device__ __forceinline__ unsigned long long fix24(float x) {
    const uint32_t u = __float_as_uint(x);
    const int e = (int)((u >> 23) & 0xffu);
    const uint64_t m = (uint64_t)((u & 0x7fffffu) | (e ? 0x800000u : 0u));
    const int sh = (e ? e : 1) - 126;
    uint64_t r = 0;
    if (sh >= 0) r = m << (sh & 63);
    else if (sh > -26) r = ((m >> (-sh - 1)) + 1) >> 1;
    return (u >> 31) ? (unsigned long long)(-(int64_t)r) : (unsigned long long)r;
}

// Streams block b's buffer entries (the ranges of all subgraphs, flattened).
// Each wave takes a contiguous share and walks it in windows of 64 entries,
// kUnroll windows per pass so that many loads are in flight. With long ranges
// (WIDE = false) the wave steps over each window's range starts together
// (window_index); with short ranges each lane searches forward from the
// previous window's subgraph. apply(d, x) updates the LDS accumulator of
// block offset d. The loads keep the default cache policy: the cache line at
// each end of a (subgraph, block) range is shared with the neighbouring
// block, which is merged at the same time on the same XCD and finds the line
// in L2.
template <typename PT, bool WIDE, class Apply>
__device__ __forceinline__ void stream_block(const uint16_t *__restrict__ dlo, const PT *__restrict__ partial,
                                             const int32_t *ofs, const int32_t *pre, int32_t k, int32_t F0,
                                             int32_t F1, Apply apply) {
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int32_t share = ((((F1 - F0) + 15) / 16) + 63) & ~63;
    const int32_t fa = min(F0 + w * share, F1), fb = min(fa + share, F1);
    if (fa >= fb) return;  // uniform over the wave
    int32_t sw = __builtin_amdgcn_readfirstlane(run_of(pre, k, fa));
    int32_t i_safe = __builtin_amdgcn_readfirstlane(ofs[sw]) + fa;  // an entry of the share, for idle lanes
    for (int32_t f0 = fa; f0 < fb; f0 += kWave * kUnroll) {
        int32_t d[kUnroll];
        PT x[kUnroll];
        int32_t sl = WIDE ? run_of(pre, k, f0) : 0;
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
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
                i_safe = __builtin_amdgcn_readfirstlane(ii);  // lane 0's entry is in the share
                i = valid ? ii : i_safe;
            } else {
                i = i_safe;  // a window past the share: loads of an entry already read, results dropped
            }
            const int32_t dd = (int32_t)dlo[i];
            x[u] = partial[i];
            d[u] = valid ? dd : -1;
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u)
            if (d[u] >= 0) apply(d[u], x[u]);
    }
}

constexpr int kEpiBatch = 8;  // vertices per thread whose loads are in flight together

// PageRank vertex update of block b from its exact sums acc (LDS, int64 fixed
// point); writes the block's FP64 partial sums to blk_out[0..3]: dangling mass,
// L1 residual, mass, and the range flag (1 when the buffer values merged into
// the block -- `am` is this thread's share of their absolute sum -- were
// non-finite or too large for exact fixed-point sums, else 0).
template <bool BF16OUT, int EPI = kEpiBatch>
__device__ __forceinline__ void pr_epilogue(const unsigned long long *acc, int32_t V, int64_t vb, int32_t nv,
                                            const float *__restrict__ rank_in, const int32_t *__restrict__ outdeg,
                                            const double *__restrict__ scalars_in, double damping, int32_t seed,
                                            float *__restrict__ rank_out, void *__restrict__ contrib_out,
                                            double *__restrict__ blk_out, double am, double *red) {
    const double dd = damping;
    // teleport and dangling mass: spread over all vertices, or (personalized,
    // seed >= 0) returned to the seed vertex alone
    const double base = seed < 0 ? (1.0 - dd) / (double)V + dd * scalars_in[0] / (double)V : 0.0;
    const double sbase = (1.0 - dd) + dd * scalars_in[0];
    double dang = 0.0, res = 0.0, mass = 0.0;
    // EPI vertices per thread per pass; sums keep the vertex order. The loads are
    // conditional, so they go out pair by pair: measured faster than issuing all
    // of them at once, which crowds the memory queue that the CU's other
    // workgroup streams its buffer entries through.
    for (int i0 = threadIdx.x; i0 < nv; i0 += kMergeThreads * EPI) {
        float rin[EPI];
        int32_t odv[EPI];
#pragma unroll
        for (int u = 0; u < EPI; ++u) {
            const int i = i0 + u * kMergeThreads;
            rin[u] = i < nv ? rank_in[vb + i] : 0.0f;
            odv[u] = i < nv ? outdeg[vb + i] : 0;
        }
#pragma unroll
        for (int u = 0; u < EPI; ++u) {
            const int i = i0 + u * kMergeThreads;
            if (i >= nv) break;
            const int64_t v = vb + i;
            const double sum = (double)(long long)acc[i] * kFixInv;
            const float r = (float)((v == seed ? sbase : base) + dd * sum);
            rank_out[v] = r;
            const int32_t od = odv[u];
            const float c = od > 0 ? r / (float)od : 0.0f;
            if (BF16OUT) reinterpret_cast<uint16_t *>(contrib_out)[v] = f32_to_bf16(c);
            else reinterpret_cast<float *>(contrib_out)[v] = c;
            if (od == 0) dang += (double)r;
            res += fabs((double)r - (double)rin[u]);
            mass += (double)r;
        }
    }
    double v4[4] = {dang, res, mass, am};
    block_sum4_f64<kMergeThreads>(v4, red);
    if (threadIdx.x == 0) {
        blk_out[0] = v4[0];
        blk_out[1] = v4[1];
        blk_out[2] = v4[2];
        blk_out[3] = range_flag(v4[3]);
    }
}

// Item j of the S items of block b: the block's entries (flattened over
// subgraphs) [P*j/S, P*(j+1)/S). With S == 1 the item is the whole block and
// the vertex update follows at once. Otherwise the item stores its exact int64
// sums in its own slot of the workspace and the absolute sum of its buffer
// values in *item_abs, and k_merge_pr_finish adds the S slots of the block
// (exactly, so the split does not change any result) and applies the update.
template <bool BF16OUT, bool WIDE, int EPI = kEpiBatch>
__device__ __forceinline__ void merge_pr_block(
    const uint16_t *__restrict__ row_dst_lo, const int32_t *__restrict__ block_ptr,
    const float *__restrict__ partial, int32_t V, int32_t k, int32_t B, int b, int32_t j, int32_t S,
    const float *__restrict__ rank_in, const int32_t *__restrict__ outdeg, const double *__restrict__ scalars_in,
    double damping, int32_t seed, float *__restrict__ rank_out, void *__restrict__ contrib_out,
    double *__restrict__ blk_out, unsigned long long *__restrict__ slot, double *__restrict__ item_abs,
    unsigned char *smem) {
    unsigned long long *acc = reinterpret_cast<unsigned long long *>(smem);
    int32_t *ofs = reinterpret_cast<int32_t *>(smem + align_up((size_t)B * 8, 16));
    int32_t *pre = ofs + k;
    __shared__ int32_t tmp[16];
    __shared__ double red[4 * (kMergeThreads / 64)];

    const int64_t vb = (int64_t)b * B;
    const int32_t nv = (int32_t)((int64_t)V - vb < B ? (int64_t)V - vb : B);
    for (int i = threadIdx.x; i < nv; i += kMergeThreads) acc[i] = 0ull;
    const int32_t P = load_block_ranges(block_ptr, b, k, ofs, pre, tmp);
    const int32_t F0 = (int32_t)((int64_t)P * j / S), F1 = (int32_t)((int64_t)P * (j + 1) / S);
    float am = 0.0f;  // this thread's share of the absolute buffer mass (range check)
    stream_block<float, WIDE>(row_dst_lo, partial, ofs, pre, k, F0, F1, [&](int32_t d, float x) {
        atomicAdd(&acc[d], fix56(x));
        am += fabsf(x);
    });
    __syncthreads();
    if (S > 1) {
        for (int i = threadIdx.x; i < nv; i += kMergeThreads) slot[i] = acc[i];
        const double tot = block_sum_f64<kMergeThreads>((double)am, red);
        if (threadIdx.x == 0) *item_abs = tot;
        return;
    }
    pr_epilogue<BF16OUT, EPI>(acc, V, vb, nv, rank_in, outdeg, scalars_in, damping, seed, rank_out, contrib_out,
                              blk_out, (double)am, red);
}

// Slot of item j of a split block b whose first item is items_b: 2*(items_b - b)
// + j. items_b - b counts the extra items of earlier blocks; a split block has
// S >= 2 items and adds S - 1 >= S / 2 extra ones, so the slot ranges of split
// blocks are disjoint and all lie below 2 * (items[nb] - nb).
__device__ __forceinline__ int64_t split_slot(int32_t items_b, int32_t b, int32_t j) {
    return 2 * (int64_t)(items_b - b) + j;
}

constexpr int32_t kItemGroup = 4;  // work items per XCD group (1, 2, 4 and 16 time alike; contiguous is slower)

template <bool BF16OUT, bool WIDE>
__global__ __launch_bounds__(kMergeThreads) void k_merge_pr(
    const uint16_t *__restrict__ row_dst_lo, const int32_t *__restrict__ block_ptr,
    const int32_t *__restrict__ block_items, const float *__restrict__ partial, int32_t V, int32_t k, int32_t B,
    int32_t nb, const float *__restrict__ rank_in, const int32_t *__restrict__ outdeg,
    const double *__restrict__ scalars_in, double damping, int32_t seed, float *__restrict__ rank_out,
    void *__restrict__ contrib_out, double *__restrict__ blk, unsigned long long *__restrict__ slots,
    double *__restrict__ item_abs, int32_t one_item) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    // the grid is the bound max_items; slots past the actual item count exit,
    // and the XCD remap spreads the actual items (not the bound) over the XCDs.
    // one_item (the bound equals nb): every block is one item, known without
    // reading the item table; each block is then merged whole, which is right
    // whatever the table holds
    const int32_t total = one_item ? nb : block_items[nb];
    if (total > (int32_t)gridDim.x) {
        // a bound below the item count (an invalid max_items): the slot
        // workspace may be too small, so nothing is merged and the scalars
        // become NaN (block 0's partial sums feed the reduction)
        if (blockIdx.x == 0 && threadIdx.x < 4) blk[threadIdx.x] = __builtin_nan("");
        return;
    }
    if ((int32_t)blockIdx.x >= total) return;  // uniform over the workgroup
    const ItemPlace ip = place_item(block_items, nb, total, xcd_group_map(blockIdx.x, total, kItemGroup));
    const int32_t b = ip.b, j = ip.j, S = ip.S;
    unsigned long long *slot = S > 1 ? slots + split_slot(block_items[b], b, j) * B : nullptr;
    double *ia = S > 1 ? item_abs + block_items[b] + j : nullptr;
    merge_pr_block<BF16OUT, WIDE>(row_dst_lo, block_ptr, partial, V, k, B, b, j, S, rank_in, outdeg, scalars_in,
                                  damping, seed, rank_out, contrib_out, blk + (int64_t)b * 4, slot, ia, smem);
}

// Sum of the item slots of each split block, written into its first slot.
// kSlotParts workgroups share a block (one part of its vertices each), so the
// heaviest block's slots are read at the rate of several CUs.
constexpr int kSlotParts = 8;
constexpr int kSlotThreads = 256;
__global__ __launch_bounds__(kSlotThreads) void k_slot_sum(const int32_t *__restrict__ block_items, int32_t V,
                                                           int32_t B, int32_t nb, int32_t max_items, int32_t parts,
                                                           unsigned long long *__restrict__ slots) {
    if (block_items[nb] > max_items) return;  // invalid bound: slots not written (see k_merge_pr)
    const int32_t b = blockIdx.x / parts, part = blockIdx.x % parts;
    const int32_t S = block_items[b + 1] - block_items[b];
    if (S <= 1) return;  // merged in one piece
    const int64_t vb = (int64_t)b * B;
    const int32_t nv = (int32_t)((int64_t)V - vb < B ? (int64_t)V - vb : B);
    const int32_t span = (nv + parts - 1) / parts;
    const int32_t lo = part * span, hi = min(lo + span, nv);
    unsigned long long *first = slots + split_slot(block_items[b], b, 0) * B;
    constexpr int kSlotBatch = 8;  // independent loads in flight per thread
    for (int32_t i = lo + threadIdx.x; i < hi; i += kSlotThreads) {
        unsigned long long t = first[i];
        int32_t j = 1;
        for (; j + kSlotBatch <= S; j += kSlotBatch) {
            unsigned long long x[kSlotBatch];
#pragma unroll
            for (int u = 0; u < kSlotBatch; ++u) x[u] = first[(int64_t)(j + u) * B + i];
#pragma unroll
            for (int u = 0; u < kSlotBatch; ++u) t += x[u];
        }
        for (; j < S; ++j) t += first[(int64_t)j * B + i];
        first[i] = t;
    }
}

// Vertex update of the split blocks from the summed first slot.
template <bool BF16OUT>
__global__ __launch_bounds__(kMergeThreads) void k_merge_pr_finish(
    const int32_t *__restrict__ block_items, int32_t V, int32_t B, int32_t nb, const float *__restrict__ rank_in,
    const int32_t *__restrict__ outdeg, const double *__restrict__ scalars_in, double damping, int32_t seed,
    float *__restrict__ rank_out, void *__restrict__ contrib_out, double *__restrict__ blk,
    const unsigned long long *__restrict__ slots, const double *__restrict__ item_abs, int32_t max_items) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    __shared__ double red[4 * (kMergeThreads / 64)];
    const int32_t b = blockIdx.x;
    if (block_items[nb] > max_items) return;  // invalid bound: slots not written (see k_merge_pr)
    if (block_items[b + 1] - block_items[b] <= 1) return;  // merged in one piece
    unsigned long long *acc = reinterpret_cast<unsigned long long *>(smem);
    const int64_t vb = (int64_t)b * B;
    const int32_t nv = (int32_t)((int64_t)V - vb < B ? (int64_t)V - vb : B);
    const unsigned long long *first = slots + split_slot(block_items[b], b, 0) * B;
    for (int i = threadIdx.x; i < nv; i += kMergeThreads) acc[i] = first[i];
    // absolute buffer mass of the block: its items' sums in item order (thread 0)
    double am = 0.0;
    if (threadIdx.x == 0)
        for (int32_t it = block_items[b]; it < block_items[b + 1]; ++it) am += item_abs[it];
    __syncthreads();
    pr_epilogue<BF16OUT>(acc, V, vb, nv, rank_in, outdeg, scalars_in, damping, seed, rank_out, contrib_out,
                         blk + (int64_t)b * 4, am, red);
}

// Order-free merge of float buffer values into float sums (int64 fixed point,
// 2^-24 resolution, |sums| < 2^38): used where the values are not bounded by
// one, e.g. sums of log-degrees.
__global__ __launch_bounds__(kMergeThreads) void k_merge_sum_fixed24(
    const uint16_t *__restrict__ row_dst_lo, const int32_t *__restrict__ block_ptr,
    const float *__restrict__ partial, int32_t V, int32_t k, int32_t B, int32_t nb, float *__restrict__ out) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    unsigned long long *acc = reinterpret_cast<unsigned long long *>(smem);
    int32_t *ofs = reinterpret_cast<int32_t *>(smem + align_up((size_t)B * 8, 16));
    int32_t *pre = ofs + k;
    __shared__ int32_t tmp[16];
    const int b = xcd_remap(blockIdx.x, nb);
    const int64_t vb = (int64_t)b * B;
    const int32_t nv = (int32_t)((int64_t)V - vb < B ? (int64_t)V - vb : B);
    for (int i = threadIdx.x; i < nv; i += kMergeThreads) acc[i] = 0ull;
    const int32_t P = load_block_ranges(block_ptr, b, k, ofs, pre, tmp);
    stream_block<float, false>(row_dst_lo, partial, ofs, pre, k, 0, P,
                               [&](int32_t d, float x) { atomicAdd(&acc[d], fix24(x)); });
    __syncthreads();
    for (int i = threadIdx.x; i < nv; i += kMergeThreads)
        out[vb + i] = (float)((double)(long long)acc[i] * (1.0 / 16777216.0));
}

cagra_status launch_merge_sum_fixed24(const cagra_segments *seg, const float *partial, float *out, hipStream_t st) {
    if (cagra_status a_ = ensure_dynamic_lds((const void *)k_merge_sum_fixed24)) return a_;
    if (merge_fused_lds_total(seg->B, seg->k, 8) > CAGRA_LDS_BYTES)
        return fail(CAGRA_E_CAPACITY, "B=%d with k=%d exceeds the merge kernel's LDS", seg->B, seg->k);
    k_merge_sum_fixed24<<<seg->nb, kMergeThreads, merge_fused_lds_bytes(seg->B, seg->k, 8), st>>>(
        seg->row_dst_lo, seg->block_ptr, partial, seg->V, seg->k, seg->B, seg->nb, out);
    CAGRA_LAUNCH_CHECK();
    return CAGRA_OK;
}

// Persistent form over many graphs: workgroups stride over a global block list.
__global__ __launch_bounds__(kMergeThreads) void k_multi_merge(const MultiDesc *__restrict__ desc,
                                                               const int32_t *__restrict__ block_graph,
                                                               int64_t total_blocks, int parity, double damping,
                                                               double *__restrict__ blk) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    for (int64_t gb = blockIdx.x; gb < total_blocks; gb += gridDim.x) {
        __syncthreads();  // LDS reuse across blocks
        const int gi = block_graph[gb];
        const MultiDesc &d = desc[gi];
        // one vertex per pass in the update keeps this kernel within 64 VGPRs
        // (two workgroups per CU)
        merge_pr_block<false, false, 1>(d.row_dst_lo, d.block_ptr, d.partial, d.V, d.k, d.B,
                                        (int)(gb - d.block_base), 0, 1, d.rank[parity], d.out_degree,
                                        d.scalars[parity], damping, -1, d.rank[1 - parity], d.contrib[1 - parity],
                                        blk + gb * 4, nullptr, nullptr, smem);
    }
}

// Uniform start vectors of many graphs (persistent over the block list).
__global__ __launch_bounds__(256) void k_multi_start(const MultiDesc *__restrict__ desc,
                                                     const int32_t *__restrict__ block_graph, int64_t total_blocks,
                                                     double *__restrict__ blk) {
    __shared__ double red[4];
    for (int64_t gb = blockIdx.x; gb < total_blocks; gb += gridDim.x) {
        const int gi = block_graph[gb];
        const MultiDesc &d = desc[gi];
        const int64_t lo = (gb - d.block_base) * (int64_t)d.B;
        const int64_t hi = lo + d.B < d.V ? lo + d.B : d.V;
        const float r = 1.0f / (float)d.V;
        double dang = 0.0, mass = 0.0;
        for (int64_t v = lo + threadIdx.x; v < hi; v += 256) {
            d.rank[0][v] = r;
            const int32_t od = d.out_degree[v];
            d.contrib[0][v] = od > 0 ? r / (float)od : 0.0f;
            if (od == 0) dang += (double)r;
            mass += (double)r;
        }
        dang = block_sum_f64<256>(dang, red);
        mass = block_sum_f64<256>(mass, red);
        if (threadIdx.x == 0) {
            blk[gb * 4 + 0] = dang;
            blk[gb * 4 + 1] = 0.0;
            blk[gb * 4 + 2] = mass;
            blk[gb * 4 + 3] = 0.0;
        }
    }
}

// Per graph: fixed-order sum of its blocks' partials into scalars[parity]. With
// carry, the range count [3] also adds the previous step's (scalars[1 - parity]).
__global__ __launch_bounds__(256) void k_multi_reduce(const MultiDesc *__restrict__ desc,
                                                      const double *__restrict__ blk, int parity, int carry) {
    __shared__ double red[4];
    const MultiDesc &d = desc[blockIdx.x];
    double a[4] = {0.0, 0.0, 0.0, 0.0};
    for (int32_t j = threadIdx.x; j < d.nb; j += 256)
        for (int c = 0; c < 4; ++c) a[c] += blk[(d.block_base + j) * 4 + c];
    for (int c = 0; c < 4; ++c) {
        double t = block_sum_f64<256>(a[c], red);
        if (threadIdx.x == 0) d.scalars[parity][c] = c == 3 && carry ? t + d.scalars[1 - parity][3] : t;
    }
}

cagra_status launch_multi_start(const MultiDesc *desc, const int32_t *block_graph, int64_t total_blocks,
                                int32_t ngraphs, double *blk, int grid, hipStream_t st) {
    if (total_blocks == 0) return CAGRA_OK;
    k_multi_start<<<grid, 256, 0, st>>>(desc, block_graph, total_blocks, blk);
    CAGRA_LAUNCH_CHECK();
    k_multi_reduce<<<ngraphs, 256, 0, st>>>(desc, blk, 0, 0);
    CAGRA_LAUNCH_CHECK();
    return CAGRA_OK;
}

cagra_status launch_multi_merge(const MultiDesc *desc, const int32_t *block_graph, int64_t total_blocks,
                                int32_t ngraphs, int parity, double damping, double *blk, size_t lds, int grid,
                                hipStream_t st) {
    if (cagra_status a_ = ensure_dynamic_lds((const void *)k_multi_merge)) return a_;
    if (total_blocks == 0) return CAGRA_OK;
    k_multi_merge<<<grid, kMergeThreads, lds, st>>>(desc, block_graph, total_blocks, parity, damping, blk);
    CAGRA_LAUNCH_CHECK();
    k_multi_reduce<<<ngraphs, 256, 0, st>>>(desc, blk, 1 - parity, 1);
    CAGRA_LAUNCH_CHECK();
    return CAGRA_OK;
}

__global__ __launch_bounds__(kMergeThreads) void k_merge_lp(
    const uint16_t *__restrict__ row_dst_lo, const int32_t *__restrict__ block_ptr,
    const int32_t *__restrict__ partial, int32_t V, int32_t k, int32_t B, int32_t nb,
    const int32_t *__restrict__ labels_in, int32_t *__restrict__ labels_out, int32_t *__restrict__ blk_changed) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    int32_t *acc = reinterpret_cast<int32_t *>(smem);
    int32_t *ofs = reinterpret_cast<int32_t *>(smem + align_up((size_t)B * 4, 16));
    int32_t *pre = ofs + k;
    __shared__ int32_t tmp[16];
    __shared__ int32_t cnt[16];

    const int b = xcd_remap(blockIdx.x, nb);
    const int64_t vb = (int64_t)b * B;
    const int32_t nv = (int32_t)((int64_t)V - vb < B ? (int64_t)V - vb : B);
    // kEpiBatch labels per thread and pass (conditional loads, as in the
    // PageRank vertex update) before the accumulators take them
    for (int i0 = threadIdx.x; i0 < nv; i0 += kMergeThreads * kEpiBatch) {
        int32_t l[kEpiBatch];
#pragma unroll
        for (int u = 0; u < kEpiBatch; ++u) {
            const int i = i0 + u * kMergeThreads;
            l[u] = i < nv ? labels_in[vb + i] : 0;
        }
#pragma unroll
        for (int u = 0; u < kEpiBatch; ++u) {
            const int i = i0 + u * kMergeThreads;
            if (i < nv) acc[i] = l[u];
        }
    }
    const int32_t P = load_block_ranges(block_ptr, b, k, ofs, pre, tmp);
    stream_block<int32_t, false>(row_dst_lo, partial, ofs, pre, k, 0, P,
                          [&](int32_t d, int32_t x) { atomicMin(&acc[d], x); });
    __syncthreads();
    int32_t changed = 0;
    for (int i0 = threadIdx.x; i0 < nv; i0 += kMergeThreads * kEpiBatch) {
        int32_t old[kEpiBatch];
#pragma unroll
        for (int u = 0; u < kEpiBatch; ++u) {
            const int i = i0 + u * kMergeThreads;
            old[u] = i < nv ? labels_in[vb + i] : 0;
        }
#pragma unroll
        for (int u = 0; u < kEpiBatch; ++u) {
            const int i = i0 + u * kMergeThreads;
            if (i >= nv) break;
            const int32_t l = acc[i];
            labels_out[vb + i] = l;
            changed += (l != old[u]) ? 1 : 0;
        }
    }
    for (int dd = 32; dd >= 1; dd >>= 1) changed += __shfl_down(changed, dd, 64);
    if ((threadIdx.x & 63) == 0) cnt[threadIdx.x >> 6] = changed;
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t tot = 0;
        for (int i = 0; i < kMergeThreads / 64; ++i) tot += cnt[i];
        blk_changed[b] = tot;
    }
}

// PageRank start vector: contributions, dangling mass and total mass.
constexpr int kInitSpan = 16384;  // vertices per init block

template <bool BF16OUT>
__global__ __launch_bounds__(256) void k_pr_init(const float *__restrict__ rank, const int32_t *__restrict__ outdeg,
                                                 int32_t V, void *__restrict__ contrib_out,
                                                 double *__restrict__ blk) {
    __shared__ double red[4];
    const int64_t lo = (int64_t)blockIdx.x * kInitSpan;
    const int64_t hi = lo + kInitSpan < V ? lo + kInitSpan : V;
    double dang = 0.0, mass = 0.0, bad = 0.0;
    for (int64_t v = lo + threadIdx.x; v < hi; v += 256) {
        const float r = rank[v];
        const int32_t od = outdeg[v];
        const float c = od > 0 ? r / (float)od : 0.0f;
        if (BF16OUT) reinterpret_cast<uint16_t *>(contrib_out)[v] = f32_to_bf16(c);
        else reinterpret_cast<float *>(contrib_out)[v] = c;
        if (od == 0) dang += (double)r;
        mass += (double)r;
        bad += isfinite(r) ? 0.0 : 1.0;
    }
    dang = block_sum_f64<256>(dang, red);
    mass = block_sum_f64<256>(mass, red);
    bad = block_sum_f64<256>(bad, red);
    if (threadIdx.x == 0) {
        blk[(int64_t)blockIdx.x * 4 + 0] = dang;
        blk[(int64_t)blockIdx.x * 4 + 1] = 0.0;
        blk[(int64_t)blockIdx.x * 4 + 2] = mass;
        blk[(int64_t)blockIdx.x * 4 + 3] = bad;
    }
}

// Fixed-order FP64 reduction of n rows of 4 partial sums. With carry non-null,
// out[3] also adds carry[3] (the range count accumulates over iterations).
__global__ __launch_bounds__(256) void k_reduce4(const double *__restrict__ blk, int32_t n,
                                                 double *__restrict__ out, const double *__restrict__ carry) {
    __shared__ double red[4];
    double a[4] = {0.0, 0.0, 0.0, 0.0};
    // four rows per thread and pass, loaded before they are added (same order)
    int32_t j = threadIdx.x;
    for (; j + 3 * 256 < n; j += 4 * 256) {
        double x[4][4];
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int c = 0; c < 4; ++c) x[r][c] = blk[(int64_t)(j + r * 256) * 4 + c];
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int c = 0; c < 4; ++c) a[c] += x[r][c];
    }
    for (; j < n; j += 256)
        for (int c = 0; c < 4; ++c) a[c] += blk[(int64_t)j * 4 + c];
    for (int c = 0; c < 4; ++c) {
        double t = block_sum_f64<256>(a[c], red);
        if (threadIdx.x == 0) out[c] = c == 3 && carry ? t + carry[3] : t;
    }
}

__global__ __launch_bounds__(256) void k_reduce_i32(const int32_t *__restrict__ blk, int32_t n,
                                                    int32_t *__restrict__ out) {
    __shared__ int32_t red[4];
    int32_t a = 0;
    for (int32_t j = threadIdx.x; j < n; j += 256) a += blk[j];
    for (int d = 32; d >= 1; d >>= 1) a += __shfl_down(a, d, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
    __syncthreads();
    if (threadIdx.x == 0) out[0] = red[0] + red[1] + red[2] + red[3];
}

// Fixed-order reductions of per-block partial sums (also used by the push path).
cagra_status launch_reduce4(const double *blk, int32_t n, double *out, const double *carry, hipStream_t st) {
    k_reduce4<<<1, 256, 0, st>>>(blk, n, out, carry);
    CAGRA_LAUNCH_CHECK();
    return CAGRA_OK;
}
cagra_status launch_reduce_i32(const int32_t *blk, int32_t n, int32_t *out, hipStream_t st) {
    k_reduce_i32<<<1, 256, 0, st>>>(blk, n, out);
    CAGRA_LAUNCH_CHECK();
    return CAGRA_OK;
}

int32_t init_blocks(int32_t V) { return (int32_t)ceil_div(V, kInitSpan); }

// Iteration workspace: the FP64 (or int32) per-block partial sums at offset 0,
// then the int64 slots of the work items of split merge blocks.
size_t ws_blk_bytes(int32_t V, int32_t nb) {
    const int64_t n = nb > init_blocks(V) ? nb : init_blocks(V);
    return align_up((size_t)n * 4 * sizeof(double), 256);
}
// One double per merge work item: the absolute buffer mass of a split item.
size_t ws_item_bytes(const cagra_segments *seg) { return align_up((size_t)seg->max_items * sizeof(double), 256); }
size_t ws_slot_bytes(const cagra_segments *seg) {
    return (size_t)2 * (size_t)(seg->max_items - seg->nb) * (size_t)seg->B * sizeof(unsigned long long);
}

cagra_status launch_pr_init(const cagra_graph *g, int32_t contrib_type, const float *rank, void *contrib_out,
                            double *scalars_out, void *ws, hipStream_t st) {
    const int32_t nblk = init_blocks(g->V);
    double *blk = reinterpret_cast<double *>(ws);
    if (contrib_type == CAGRA_BF16) k_pr_init<true><<<nblk, 256, 0, st>>>(rank, g->out_degree, g->V, contrib_out, blk);
    else k_pr_init<false><<<nblk, 256, 0, st>>>(rank, g->out_degree, g->V, contrib_out, blk);
    CAGRA_LAUNCH_CHECK();
    k_reduce4<<<1, 256, 0, st>>>(blk, nblk, scalars_out, nullptr);
    CAGRA_LAUNCH_CHECK();
    return CAGRA_OK;
}

template <bool BF16OUT, bool WIDE>
static cagra_status launch_merge_pr_t(const cagra_graph *g, const cagra_segments *seg, double damping, int32_t seed,
                                      const float *rank_in, const double *scalars_in, const float *partial,
                                      float *rank_out, void *contrib_out, double *scalars_out, void *ws,
                                      hipStream_t st) {
    if (cagra_status a_ = ensure_dynamic_lds((const void *)k_merge_pr<BF16OUT, WIDE>)) return a_;
    if (cagra_status a_ = ensure_dynamic_lds((const void *)k_merge_pr_finish<BF16OUT>)) return a_;
    double *blk = reinterpret_cast<double *>(ws);
    double *item_abs = reinterpret_cast<double *>(reinterpret_cast<char *>(ws) + ws_blk_bytes(seg->V, seg->nb));
    unsigned long long *slots = reinterpret_cast<unsigned long long *>(reinterpret_cast<char *>(ws) +
                                                                       ws_blk_bytes(seg->V, seg->nb) +
                                                                       ws_item_bytes(seg));
    k_merge_pr<BF16OUT, WIDE><<<seg->max_items, kMergeThreads, merge_fused_lds_bytes(seg->B, seg->k, 8), st>>>(
        seg->row_dst_lo, seg->block_ptr, seg->block_items, partial, seg->V, seg->k, seg->B, seg->nb, rank_in,
        g->out_degree, scalars_in, damping, seed, rank_out, contrib_out, blk, slots, item_abs,
        seg->max_items == seg->nb ? 1 : 0);
    CAGRA_LAUNCH_CHECK();
    // max_items is a bound on the item count; when it equals nb (a caller that
    // read block_items[nb] after the build may tighten it so) no block is split
    // and the slot pass has nothing to do
    if (seg->max_items > seg->nb) {
        const int32_t parts = (int64_t)seg->nb * kSlotParts <= INT32_MAX ? kSlotParts : 1;
        k_slot_sum<<<(unsigned)((int64_t)seg->nb * parts), kSlotThreads, 0, st>>>(
            seg->block_items, seg->V, seg->B, seg->nb, seg->max_items, parts, slots);
        CAGRA_LAUNCH_CHECK();
        k_merge_pr_finish<BF16OUT><<<seg->nb, kMergeThreads, (size_t)seg->B * 8, st>>>(
            seg->block_items, seg->V, seg->B, seg->nb, rank_in, g->out_degree, scalars_in, damping, seed, rank_out,
            contrib_out, blk, slots, item_abs, seg->max_items);
        CAGRA_LAUNCH_CHECK();
    }
    k_reduce4<<<1, 256, 0, st>>>(blk, seg->nb, scalars_out, scalars_in);
    CAGRA_LAUNCH_CHECK();
    return CAGRA_OK;
}

cagra_status launch_merge_pr(const cagra_graph *g, const cagra_segments *seg, double damping, int32_t seed,
                             int32_t contrib_type,
                             const float *rank_in, const double *scalars_in, const float *partial, float *rank_out,
                             void *contrib_out, double *scalars_out, void *ws, hipStream_t st) {
    // mean entries per (subgraph, block) range below one 64-entry step: wide walk
    const bool wide = seg->Q < (int64_t)kWave * seg->k * seg->nb;
    if (contrib_type == CAGRA_BF16)
        return wide ? launch_merge_pr_t<true, true>(g, seg, damping, seed, rank_in, scalars_in, partial, rank_out,
                                                    contrib_out, scalars_out, ws, st)
                    : launch_merge_pr_t<true, false>(g, seg, damping, seed, rank_in, scalars_in, partial, rank_out,
                                                     contrib_out, scalars_out, ws, st);
    return wide ? launch_merge_pr_t<false, true>(g, seg, damping, seed, rank_in, scalars_in, partial, rank_out, contrib_out,
                                                 scalars_out, ws, st)
                : launch_merge_pr_t<false, false>(g, seg, damping, seed, rank_in, scalars_in, partial, rank_out,
                                                  contrib_out, scalars_out, ws, st);
}

cagra_status launch_merge_lp(const cagra_segments *seg, const int32_t *labels_in, const int32_t *partial,
                             int32_t *labels_out, int32_t *changed_out, void *ws, hipStream_t st) {
    int32_t *blk = reinterpret_cast<int32_t *>(ws);
    const size_t lds = merge_fused_lds_bytes(seg->B, seg->k, 4);
    if (cagra_status a_ = ensure_dynamic_lds((const void *)k_merge_lp)) return a_;
    k_merge_lp<<<seg->nb, kMergeThreads, lds, st>>>(seg->row_dst_lo, seg->block_ptr, partial, seg->V, seg->k, seg->B,
                                                    seg->nb, labels_in, labels_out, blk);
    CAGRA_LAUNCH_CHECK();
    k_reduce_i32<<<1, 256, 0, st>>>(blk, seg->nb, changed_out);
    CAGRA_LAUNCH_CHECK();
    return CAGRA_OK;
}

}  // namespace cagra
