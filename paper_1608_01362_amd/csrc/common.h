// Internal helpers shared by the library's HIP sources (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cagra.h"

namespace cagra {

constexpr int kWave = 64;

// Set the thread-local error text and return the status.
cagra_status fail(cagra_status st, const char *fmt, ...);

#define CAGRA_HIP_CHECK(expr)                                                        \
    do {                                                                             \
        hipError_t _e = (expr);                                                      \
        if (_e != hipSuccess)                                                        \
            return ::cagra::fail(CAGRA_E_HIP, "%s failed: %s", #expr, hipGetErrorString(_e)); \
    } while (0)

#define CAGRA_LAUNCH_CHECK() CAGRA_HIP_CHECK(hipGetLastError())

__host__ __device__ static inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
__host__ __device__ static inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Bump allocator over a caller-provided workspace.
struct Arena {
    char *base;
    size_t cap;
    size_t used;
    template <typename T>
    T *take(int64_t count) {
        size_t off = align_up(used, 256);
        size_t bytes = (size_t)(count > 0 ? count : 1) * sizeof(T);
        if (base == nullptr || off + bytes > cap) return nullptr;
        used = off + bytes;
        return reinterpret_cast<T *>(base + off);
    }
};
// Same layout rules, no memory: returns the bytes needed.
struct ArenaSize {
    size_t used = 0;
    template <typename T>
    void take(int64_t count) {
        size_t off = align_up(used, 256);
        used = off + (size_t)(count > 0 ? count : 1) * sizeof(T);
    }
};

// Lets `fn` use all LDS not taken by its static __shared__ arrays as dynamic LDS.
static inline cagra_status allow_dynamic_lds(const void *fn) {
    hipFuncAttributes attr;
    hipError_t e = hipFuncGetAttributes(&attr, fn);
    if (e != hipSuccess) return fail(CAGRA_E_HIP, "hipFuncGetAttributes failed: %s", hipGetErrorString(e));
    int dyn = CAGRA_LDS_BYTES - (int)attr.sharedSizeBytes;
    e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, dyn);
    if (e != hipSuccess) return fail(CAGRA_E_HIP, "hipFuncSetAttribute(%d) failed: %s", dyn, hipGetErrorString(e));
    return CAGRA_OK;
}

// allow_dynamic_lds for `fn` once per device (thread-safe; later calls on the
// same device return at once). Every launch with more than 64 KB of dynamic
// LDS goes through this.
cagra_status ensure_dynamic_lds(const void *fn);

// Per-graph descriptor of the persistent multi-graph kernels (device memory).
struct MultiDesc {
    const void *edge_src;  // 16-bit edge words (multi-graph runs use N <= CAGRA_EDGE16_MAX_N)
    const int32_t *tile_edge;
    const int32_t *tile_seg;
    const int32_t *tile_span_row;
    const uint16_t *row_dst_lo;
    const int32_t *block_ptr;
    const int32_t *out_degree;
    float *rank[2];
    float *contrib[2];
    double *scalars[2];
    float *partial;
    int64_t Q;
    int64_t tile_base;   // first global tile of this graph
    int64_t block_base;  // first global merge block of this graph
    int32_t V, N, k, B, nb, ntiles;
};

// Edge words of a segmented graph: local source index plus a row-start flag.
// 16-bit words for N <= CAGRA_EDGE16_MAX_N, 32-bit words otherwise.
__host__ __device__ static inline bool edge16(int32_t N) { return N <= CAGRA_EDGE16_MAX_N; }
template <typename W>
struct EdgeWord;
template <>
struct EdgeWord<uint16_t> {
    static constexpr uint32_t kFlag = 0x8000u, kIndex = 0x7fffu;
};
template <>
struct EdgeWord<uint32_t> {
    static constexpr uint32_t kFlag = 0x80000000u, kIndex = 0x7fffffffu;
};

// ---------------------------------------------------------------- device helpers

// Workgroups are dispatched round-robin over the 8 XCDs (id mod 8). Remap so
// that XCD x receives a contiguous range of logical ids: neighbouring tiles
// (same segment) then share one L2. Bijective on [0, n).
__device__ __forceinline__ int xcd_remap(int b, int n) {
    const int nx = 8;
    int x = b % nx, i = b / nx;
    int q = n / nx, r = n % nx;
    return x * q + (x < r ? x : r) + i;
}

__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// Round-to-nearest-even FP32 -> BF16 (NaN kept quiet NaN).
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x40);
    uint32_t lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ uint64_t lanemask_lt() {
    int lane = __lane_id();
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// Combine operators used by gather and merge.
struct OpSum {
    using T = float;
    static __device__ __forceinline__ float identity() { return 0.0f; }
    static __device__ __forceinline__ float apply(float a, float b) { return a + b; }
};
struct OpMin {
    using T = int32_t;
    static __device__ __forceinline__ int32_t identity() { return 0x7fffffff; }
    static __device__ __forceinline__ int32_t apply(int32_t a, int32_t b) { return a < b ? a : b; }
};

// Deterministic FP64 block reduction (fixed shuffle tree, then waves in order).
template <int NT>
__device__ double block_sum_f64(double v, double *lds /* NT/64 entries */) {
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_down(v, d, 64);
    int w = threadIdx.x / 64;
    if ((threadIdx.x & 63) == 0) lds[w] = v;
    __syncthreads();
    double tot = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < NT / 64; ++i) tot += lds[i];
    __syncthreads();
    return tot;  // valid in thread 0
}

// Four FP64 block sums at once, each in the order block_sum_f64 uses (fixed
// shuffle tree, then waves in order); one LDS round trip for all four.
// Results valid in thread 0.
template <int NT>
__device__ void block_sum4_f64(double (&v)[4], double *lds /* 4 * NT/64 entries */) {
#pragma unroll
    for (int c = 0; c < 4; ++c)
        for (int d = 32; d >= 1; d >>= 1) v[c] += __shfl_down(v[c], d, 64);
    const int w = threadIdx.x / 64;
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int c = 0; c < 4; ++c) lds[c * (NT / 64) + w] = v[c];
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            double tot = 0.0;
            for (int i = 0; i < NT / 64; ++i) tot += lds[c * (NT / 64) + i];
            v[c] = tot;
        }
    __syncthreads();
}

// Absolute buffer mass from which the int64 fixed-point sums (2^-56 per unit,
// see fix56) could leave the exact range: a merge block whose buffer values
// have |x| summing to this or more, or holding a non-finite value, is counted
// in the iteration's range scalar instead of being trusted. Every partial sum
// of a block below it stays under 2^62 in fixed point (the int64 limit is
// 2^63), so FP rounding of the check itself cannot hide an overflow.
constexpr double kFixAbsLimit = 64.0;
__device__ __forceinline__ double range_flag(double absmass) { return absmass < kFixAbsLimit ? 0.0 : 1.0; }

}  // namespace cagra
