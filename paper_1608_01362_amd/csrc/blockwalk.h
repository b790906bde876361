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

// Loads the block's range bounds per subgraph into LDS and turns the lengths
// into an exclusive prefix; returns the block's entry count.
__device__ inline int32_t load_block_ranges(const int32_t *__restrict__ block_ptr, int b, int32_t k, int32_t *lo_s,
                                     int32_t *pre, int32_t *tmp) {
    for (int s = threadIdx.x; s < k; s += kMergeThreads) {
        int32_t a = block_ptr[(int64_t)b * k + s], e = block_ptr[(int64_t)(b + 1) * k + s];
        lo_s[s] = a;
        pre[s] = e - a;
    }
    __syncthreads();
    int32_t P = block_excl_scan_lds(pre, k, tmp);
    if (threadIdx.x == 0) pre[k] = P;
    __syncthreads();
    return P;
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

// round(x * 2^56) as a two's-complement int64, computed from the float's bits
// (exact for |x| < 64; halves round up in magnitude).
__device__ __forceinline__ unsigned long long fix56(float x) {
    const uint32_t u = __float_as_uint(x);
    const int e = (int)((u >> 23) & 0xffu);
    const uint64_t m = (uint64_t)((u & 0x7fffffu) | (e ? 0x800000u : 0u));
    const int sh = (e ? e : 1) - 94;
    uint64_t r = 0;
    if (sh >= 0) r = m << (sh & 63);
    else if (sh > -26) r = ((m >> (-sh - 1)) + 1) >> 1;
    return (u >> 31) ? (unsigned long long)(-(int64_t)r) : (unsigned long long)r;
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
