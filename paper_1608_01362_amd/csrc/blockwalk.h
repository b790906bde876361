// Block-range walk shared by the cache-aware merge and the push expand:
// per-subgraph entry ranges of a vertex block loaded into LDS as an exclusive
// prefix, and the forward search that maps a flattened entry to its subgraph.
// Also the exact int64 fixed-point form of FP32 values that the order-free
// sums accumulate.
#pragma once

#include "common.h"

namespace cagra {

constexpr int kMergeThreads = 1024;
constexpr double kFixInv = 1.0 / 72057594037927936.0;  // 2^-56

// In-place exclusive scan of a[0..n) in LDS by the whole 1024-thread block;
// returns the total (all threads). `tmp` holds 16 ints.
__device__ inline int32_t block_excl_scan_lds(int32_t *a, int32_t n, int32_t *tmp) {
    const int per = (n + kMergeThreads - 1) / kMergeThreads;
    const int lo = threadIdx.x * per;
    int32_t sum = 0;
    for (int i = 0; i < per; ++i)
        if (lo + i < n) sum += a[lo + i];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int32_t incl = sum;
    for (int d = 1; d < 64; d <<= 1) {
        int32_t o = __shfl_up(incl, d, 64);
        if (lane >= d) incl += o;
    }
    if (lane == 63) tmp[w] = incl;
    __syncthreads();
    int32_t pre = incl - sum;
    for (int i = 0; i < w; ++i) pre += tmp[i];
    int32_t total = 0;
    for (int i = 0; i < kMergeThreads / 64; ++i) total += tmp[i];
    for (int i = 0; i < per; ++i)
        if (lo + i < n) {
            int32_t x = a[lo + i];
            a[lo + i] = pre;
            pre += x;
        }
    __syncthreads();
    return total;
}

// Loads the block's range bounds per subgraph into LDS: pre = exclusive prefix
// of the range lengths, ofs[s] = (first entry of subgraph s's range) - pre[s],
// so that flattened entry f of subgraph s is entry ofs[s] + f. Returns the
// block's entry count.
__device__ inline int32_t load_block_ranges(const int32_t *__restrict__ block_ptr, int b, int32_t k, int32_t *ofs,
                                            int32_t *pre, int32_t *tmp) {
    for (int s = threadIdx.x; s < k; s += kMergeThreads) {
        int32_t a = block_ptr[(int64_t)b * k + s], e = block_ptr[(int64_t)(b + 1) * k + s];
        ofs[s] = a;
        pre[s] = e - a;
    }
    __syncthreads();
    int32_t P = block_excl_scan_lds(pre, k, tmp);
    if (threadIdx.x == 0) pre[k] = P;
    for (int s = threadIdx.x; s < k; s += kMergeThreads) ofs[s] -= pre[s];
    __syncthreads();
    return P;
}

// Entry index of flattened entry f = fs + lane in a window of 64 entries that
// starts at fs (wave-uniform); entries up to wend (< pre[k], wave-uniform) are
// in the share. sl, wave-uniform, is moved to the subgraph of fs. The whole
// wave then steps over the range starts inside the window together, each lane
// keeping the offset of the last subgraph that starts at or before its entry,
// so a window costs one compare and one select per lane and range start
// instead of a search per lane.
__device__ __forceinline__ int32_t window_index(const int32_t *ofs, const int32_t *pre, int32_t &sl, int32_t fs,
                                                int32_t wend, int32_t f) {
    int32_t nxt = __builtin_amdgcn_readfirstlane(pre[sl + 1]);
    while (nxt <= fs) {
        ++sl;
        nxt = __builtin_amdgcn_readfirstlane(pre[sl + 1]);
    }
    int32_t o = __builtin_amdgcn_readfirstlane(ofs[sl]);
    int32_t s2 = sl;
    while (nxt <= wend) {
        ++s2;
        const int32_t o2 = __builtin_amdgcn_readfirstlane(ofs[s2]);
        o = f >= nxt ? o2 : o;
        nxt = __builtin_amdgcn_readfirstlane(pre[s2 + 1]);
    }
    return o + f;
}

// Last subgraph s with pre[s] <= f (pre is non-decreasing; empty ranges skipped).
__device__ __forceinline__ int32_t run_of(const int32_t *pre, int32_t k, int32_t f) {
    int32_t lo = 0, hi = k;
    while (hi - lo > 1) {
        const int32_t mid = (lo + hi) >> 1;
        if (pre[mid] <= f) lo = mid;
        else hi = mid;
    }
    return lo;
}

// |x| * 2^56 truncated toward zero, from the float's bits: |x| * 2^56 =
// m * 2^(e - 94) for the 24-bit significand m and biased exponent e, i.e. the
// 64-bit word m << 40 shifted right by 134 - e. The high dword of m << 40 is
// the float's bits shifted left by 8 with the leading one set; shifts of 64
// or more (|x| < 2^-56, zeros, denormals) give 0. Exact for |x| < 64.
__device__ __forceinline__ uint64_t fix56_magnitude(uint32_t u) {
    const uint32_t amt = 134u - ((u >> 23) & 0xffu);
    const uint32_t hi = amt < 64u ? (u << 8) | 0x80000000u : 0u;
    return ((uint64_t)hi << 32) >> (amt & 63u);
}

// trunc(x * 2^56) as a two's-complement int64: sums of these are exact, so
// they do not depend on the order of the additions (error below 2^-56 per term).
__device__ __forceinline__ unsigned long long fix56(float x) {
    const uint32_t u = __float_as_uint(x);
    const uint64_t m = fix56_magnitude(u);
    return (u >> 31) ? (unsigned long long)(-(int64_t)m) : (unsigned long long)m;
}

constexpr int kUnroll = 8;

// Subgraph of flattened entry f, searching forward from sl (pre[sl] <= f,
// pre[k] > f). A 64-entry step advances 64 / (mean range length) subgraphs on
// average: WIDE = false reads the next two starts per LDS round trip (ranges
// of 64 entries or more); WIDE = true tests one start and then reads four per
// round trip (short ranges, e.g. blocks of low in-degree vertices after
// clustering). pre is non-decreasing, so the starts <= f form a prefix.
template <bool WIDE>
__device__ __forceinline__ int32_t advance(const int32_t *pre, int32_t k, int32_t sl, int32_t f) {
    if (!WIDE) {
        for (;;) {
            const int32_t q1 = pre[min(sl + 1, k)], q2 = pre[min(sl + 2, k)];
            const int32_t adv = (q1 <= f) + (q2 <= f);
            sl += adv;
            if (adv < 2) return sl;
        }
    }
    if (pre[min(sl + 1, k)] > f) return sl;
    ++sl;
    for (;;) {
        const int32_t q1 = pre[min(sl + 1, k)], q2 = pre[min(sl + 2, k)];
        const int32_t q3 = pre[min(sl + 3, k)], q4 = pre[min(sl + 4, k)];
        const int32_t adv = (q1 <= f) + (q2 <= f) + (q3 <= f) + (q4 <= f);
        sl += adv;
        if (adv < 4) return sl;
    }
}

// Block of merge work item i: last b with items[b] <= i (items ascending).
__device__ __forceinline__ int32_t block_of_item(const int32_t *__restrict__ items, int32_t nb, int32_t i) {
    int32_t lo = 0, hi = nb;
    while (hi - lo > 1) {
        const int32_t mid = (lo + hi) >> 1;
        if (items[mid] <= i) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Block b of work item it, and the item's index j among the S items of b.
// Every block has at least one item, so a total of nb items means one item per
// block and item it is block it: no search (a chain of dependent global loads)
// before the block's work starts.
struct ItemPlace {
    int32_t b, j, S;
};
__device__ __forceinline__ ItemPlace place_item(const int32_t *__restrict__ items, int32_t nb, int32_t total,
                                                int32_t it) {
    if (total == nb) return {it, 0, 1};
    const int32_t b = block_of_item(items, nb, it);
    return {b, it - items[b], items[b + 1] - items[b]};
}

// Groups of g consecutive work items share an XCD (workgroup id mod 8), and
// the groups cycle over the XCDs: neighbouring blocks still meet in one L2,
// while the heavy blocks at the front (high in-degree destinations after
// clustering) spread over all XCDs. Bijective on [0, n): ids past the last
// whole round of 8 g keep their place.
__device__ __forceinline__ int32_t xcd_group_map(int32_t id, int32_t n, int32_t g) {
    const int32_t round = 8 * g;
    if (id >= n / round * round) return id;
    const int32_t x = id & 7, q = id >> 3;
    return (q / g) * round + x * g + (q % g);
}

}  // namespace cagra
