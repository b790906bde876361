// Stable reorder of (key, value) pairs by an unsigned key: the segment-major
// step of the Section 3.1 preprocessing, where the rows and the edges,
// produced in destination order, are regrouped by the segment of their
// sources while keeping destination order inside a segment (16-bit keys), and
// the vertex order and edge relabelling of the Section 5 clustering (32- and
// 64-bit keys, the latter without values).
//
// Least-significant-digit radix passes over digits of at most 6 bits. One
// pass: every tile of kSortTile pairs counts its digits (k_sort_count), one
// device-wide exclusive scan over the digit-major count matrix gives each
// (digit, tile) its output offset, and k_sort_scatter ranks the tile's pairs
// stably in LDS (wave ballots give each lane its rank among equal digits of
// its wave; per-wave digit counts order the waves) and writes each digit's run
// of the tile contiguously. The passes are stable, so the last one leaves the
// pairs ordered by key and, for equal keys, in input order.
#include <type_traits>

#include "common.h"

namespace cagra {

// Value type of a sort of keys alone.
struct NoValue {};

constexpr int kSortThreads = 256;
constexpr int kSortItems = 16;
constexpr int kSortTile = kSortThreads * kSortItems;  // 4096 pairs per tile
constexpr int kSortWaves = kSortThreads / 64;
constexpr int kMaxDigitBits = 6;
constexpr int kMaxDigits = 1 << kMaxDigitBits;

// declared in builder.hip (device-wide scans)
cagra_status scan_add_exclusive(const int32_t *in, int32_t *out, int64_t n, void *ws, size_t ws_bytes,
                                hipStream_t st);
size_t scan_add_ws_bytes(int64_t n);

static int sort_passes(int bits) { return bits <= 0 ? 0 : (bits + kMaxDigitBits - 1) / kMaxDigitBits; }

// Digit counts of one tile, digit-major: counts[d * ntiles + tile].
template <typename K>
__global__ __launch_bounds__(kSortThreads) void k_sort_count(const K *__restrict__ keys, int64_t n, int shift,
                                                             int dbits, int32_t ntiles, int32_t *__restrict__ counts) {
    __shared__ int32_t h[kMaxDigits];
    const int ndig = 1 << dbits, mask = ndig - 1;
    for (int d = threadIdx.x; d < ndig; d += kSortThreads) h[d] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
#pragma unroll
    for (int j = 0; j < kSortItems; ++j) {
        const int64_t i = base + j * kSortThreads + threadIdx.x;
        if (i < n) atomicAdd(&h[(int)((keys[i] >> shift) & (K)mask)], 1);
    }
    __syncthreads();
    for (int d = threadIdx.x; d < ndig; d += kSortThreads) counts[(int64_t)d * ntiles + blockIdx.x] = h[d];
}

// One stable pass: pair i of the tile (i = j * kSortThreads + thread) goes to
// offsets[digit * ntiles + tile] + (its rank among the tile's pairs with that
// digit, in input order).
template <typename K, typename V>
__global__ __launch_bounds__(kSortThreads) void k_sort_scatter(const K *__restrict__ kin, const V *__restrict__ vin,
                                                               int64_t n, int shift, int dbits, int32_t ntiles,
                                                               const int32_t *__restrict__ offsets,
                                                               K *__restrict__ kout, V *__restrict__ vout) {
    constexpr bool kVals = !std::is_same<V, NoValue>::value;
    using VS = typename std::conditional<kVals, V, char>::type;  // stored value type
    __shared__ K sk[kSortTile];
    __shared__ VS sv[kVals ? kSortTile : 1];
    __shared__ int32_t run[kMaxDigits];                 // next local slot of each digit
    __shared__ int32_t lofs[kMaxDigits];                // first local slot of each digit
    __shared__ int32_t gofs[kMaxDigits];                // output offset of this tile's run of each digit
    __shared__ int32_t wcnt[2][kSortWaves][kMaxDigits];  // per-wave digit counts of a step (two steps alternate)
    const int ndig = 1 << dbits, mask = ndig - 1;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    const int cnt = (int)(n - base < kSortTile ? n - base : kSortTile);

    K key[kSortItems];
    VS val[kSortItems];
    int dig[kSortItems];
#pragma unroll
    for (int j = 0; j < kSortItems; ++j) {
        const int p = j * kSortThreads + tid;
        const bool ok = p < cnt;
        key[j] = ok ? kin[base + p] : (K)0;
        if constexpr (kVals) val[j] = ok ? vin[base + p] : (V)0;
        dig[j] = ok ? (int)((key[j] >> shift) & (K)mask) : ndig;  // ndig: no pair
    }
    for (int d = tid; d < ndig; d += kSortThreads) run[d] = 0;
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kSortItems; ++j)
        if (dig[j] < ndig) atomicAdd(&run[dig[j]], 1);
    __syncthreads();
    if (tid == 0) {
        int32_t s = 0;
        for (int d = 0; d < ndig; ++d) {
            const int32_t c = run[d];
            lofs[d] = s;
            s += c;
        }
    }
    __syncthreads();
    for (int d = tid; d < ndig; d += kSortThreads) {
        run[d] = lofs[d];
        gofs[d] = offsets[(int64_t)d * ntiles + blockIdx.x];
    }
#pragma unroll
    for (int j = 0; j < kSortItems; ++j) {
        const int par = j & 1;
        wcnt[par][w][lane] = 0;  // this wave's row (ndig <= 64 = lanes)
        const int d = dig[j];
        const bool ok = d < ndig;
        // lanes of this wave holding the same digit
        uint64_t peers = __ballot(ok);
        for (int b = 0; b < dbits; ++b) {
            const uint64_t bal = __ballot(ok && ((d >> b) & 1));
            peers &= ((d >> b) & 1) ? bal : ~bal;
        }
        const int lrank = (int)__popcll(peers & lanemask_lt());
        if (ok && lrank == 0) wcnt[par][w][d] = (int32_t)__popcll(peers);
        __syncthreads();
        if (ok) {
            int32_t pos = run[d] + lrank;
            for (int x = 0; x < w; ++x) pos += wcnt[par][x][d];
            sk[pos] = key[j];
            if constexpr (kVals) sv[pos] = val[j];
        }
        __syncthreads();
        if (tid < ndig) {
            int32_t add = 0;
            for (int x = 0; x < kSortWaves; ++x) add += wcnt[par][x][tid];
            run[tid] += add;
        }
        // the next step writes the other wcnt buffer; the one after it waits
        // behind that step's barriers, by which time these reads are done
    }
    __syncthreads();
    for (int p = tid; p < cnt; p += kSortThreads) {
        const K kk = sk[p];
        const int d = (int)((kk >> shift) & (K)mask);
        const int64_t g = (int64_t)gofs[d] + (p - lofs[d]);
        kout[g] = kk;
        if constexpr (kVals) vout[g] = sv[p];
    }
}

size_t sort_ws_bytes(int64_t n, int bits, int key_bytes, int value_bytes) {
    const int passes = sort_passes(bits);
    if (passes == 0 || n <= 0) return 256;
    const int dbits = (bits + passes - 1) / passes;
    const int64_t ntiles = ceil_div(n, kSortTile);
    const int64_t ncounts = ((int64_t)1 << dbits) * ntiles;
    ArenaSize a;
    a.take<char>(n * (int64_t)key_bytes);    // keys between passes
    a.take<char>(n * (int64_t)value_bytes);  // values between passes
    a.take<int32_t>(ncounts);                // digit counts, then offsets
    return a.used + scan_add_ws_bytes(ncounts) + 512;
}

size_t seg_sort_ws_bytes(int64_t n, int bits, int value_bytes) { return sort_ws_bytes(n, bits, 2, value_bytes); }

// Stable sort of n (key, value) pairs by key (keys < 2^bits, bits up to the key
// width); V = NoValue sorts keys alone. keys_in/vals_in are read (not
// modified); keys_out/vals_out receive the sorted pairs and must not alias the
// inputs.
template <typename K, typename V>
cagra_status radix_sort_stable(const K *keys_in, const V *vals_in, K *keys_out, V *vals_out, int64_t n, int bits,
                               void *ws, size_t ws_bytes, hipStream_t st) {
    constexpr bool kVals = !std::is_same<V, NoValue>::value;
    constexpr int kValBytes = kVals ? (int)sizeof(V) : 0;
    if (n <= 0) return CAGRA_OK;
    if (bits < 1) bits = 1;
    if (bits > (int)(8 * sizeof(K))) return fail(CAGRA_E_CAPACITY, "sort keys wider than the key type");
    const int passes = sort_passes(bits);
    const int dbits = (bits + passes - 1) / passes;
    if (ws_bytes < sort_ws_bytes(n, bits, (int)sizeof(K), kValBytes))
        return fail(CAGRA_E_BUFFER, "workspace too small (sort temporaries)");
    const int64_t ntiles64 = ceil_div(n, kSortTile);
    if (ntiles64 * ((int64_t)1 << dbits) > INT32_MAX) return fail(CAGRA_E_OVERFLOW, "sort too large");
    const int32_t ntiles = (int32_t)ntiles64;
    Arena ar{(char *)ws, ws_bytes, 0};
    K *ktmp = reinterpret_cast<K *>(ar.take<char>(n * (int64_t)sizeof(K)));
    V *vtmp = kVals ? reinterpret_cast<V *>(ar.take<char>(n * (int64_t)kValBytes)) : nullptr;
    int32_t *counts = ar.take<int32_t>(((int64_t)1 << dbits) * ntiles);
    char *scan_ws = ar.base + align_up(ar.used, 256);
    const size_t scan_bytes = ws_bytes - align_up(ar.used, 256);
    const K *ks = keys_in;
    const V *vs = vals_in;
    for (int p = 0; p < passes; ++p) {
        // the last pass writes the output; earlier ones alternate between the
        // temporaries and the output
        const bool to_out = ((passes - 1 - p) & 1) == 0;
        K *kd = to_out ? keys_out : ktmp;
        V *vd = to_out ? vals_out : vtmp;
        const int shift = p * dbits;
        k_sort_count<K><<<ntiles, kSortThreads, 0, st>>>(ks, n, shift, dbits, ntiles, counts);
        CAGRA_LAUNCH_CHECK();
        if (cagra_status s = scan_add_exclusive(counts, counts, ((int64_t)1 << dbits) * ntiles, scan_ws, scan_bytes,
                                                st))
            return s;
        k_sort_scatter<K, V><<<ntiles, kSortThreads, 0, st>>>(ks, vs, n, shift, dbits, ntiles, counts, kd, vd);
        CAGRA_LAUNCH_CHECK();
        ks = kd;
        vs = vd;
    }
    return CAGRA_OK;
}

template <typename V>
cagra_status seg_sort_pairs(const uint16_t *keys_in, const V *vals_in, uint16_t *keys_out, V *vals_out, int64_t n,
                            int bits, void *ws, size_t ws_bytes, hipStream_t st) {
    if (bits > 16) return fail(CAGRA_E_CAPACITY, "sort keys wider than 16 bits");
    return radix_sort_stable<uint16_t, V>(keys_in, vals_in, keys_out, vals_out, n, bits, ws, ws_bytes, st);
}

template cagra_status seg_sort_pairs<uint16_t>(const uint16_t *, const uint16_t *, uint16_t *, uint16_t *, int64_t,
                                               int, void *, size_t, hipStream_t);
template cagra_status seg_sort_pairs<uint32_t>(const uint16_t *, const uint32_t *, uint16_t *, uint32_t *, int64_t,
                                               int, void *, size_t, hipStream_t);
template cagra_status seg_sort_pairs<unsigned long long>(const uint16_t *, const unsigned long long *, uint16_t *,
                                                         unsigned long long *, int64_t, int, void *, size_t,
                                                         hipStream_t);
template cagra_status radix_sort_stable<uint32_t, int32_t>(const uint32_t *, const int32_t *, uint32_t *, int32_t *,
                                                           int64_t, int, void *, size_t, hipStream_t);
template cagra_status radix_sort_stable<unsigned long long, NoValue>(const unsigned long long *, const NoValue *,
                                                                     unsigned long long *, NoValue *, int64_t, int,
                                                                     void *, size_t, hipStream_t);

}  // namespace cagra
