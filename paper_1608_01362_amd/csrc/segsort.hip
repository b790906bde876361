// Stable reorder of (key, value) pairs by an unsigned key: the segment-major
// step of the Section 3.1 preprocessing, where the rows and the edges,
// produced in destination order, are regrouped by the segment of their
// sources while keeping destination order inside a segment (16-bit keys), and
// the vertex order and edge relabelling of the Section 5 clustering (32- and
// 64-bit keys, the latter without values).
//
// Least-significant-digit radix passes over digits of at most 8 bits. One
// pass: every tile of kSortTile pairs counts its digits (k_sort_count), one
// device-wide exclusive scan over the digit-major count matrix gives each
// (digit, tile) its output offset, and k_sort_scatter ranks the tile's pairs
// stably in LDS (each wave ranks a contiguous part of the tile on its own
// through ballots or per-digit lane masks; one scan over the digits orders
// the waves) and writes each digit's run of the tile contiguously. The passes
// are stable, so the last one leaves the pairs ordered by key and, for equal
// keys, in input order.
#include <type_traits>

#include "radix.h"

namespace cagra {

constexpr int kSortThreads = 512;
constexpr int kSortItems = 8;
constexpr int kSortTile = kSortThreads * kSortItems;
static_assert(kSortTile == kRadixTile, "a tile is the unit of the published digit counts");
constexpr int kSortWaves = kSortThreads / 64;
constexpr int kMaxDigitBits = 8;
constexpr int kMaxDigits = 1 << kMaxDigitBits;
constexpr int kBallotDigitBits = 5;  // digits this narrow are matched with ballots
static_assert(kMaxDigits <= kSortThreads && kMaxDigits % 64 == 0, "digit tables are one entry per thread");

static int sort_passes(int bits) { return bits <= 0 ? 0 : (bits + kMaxDigitBits - 1) / kMaxDigitBits; }

int sort_digit_bits(int bits) {
    if (bits < 1) bits = 1;
    const int passes = sort_passes(bits);
    return (bits + passes - 1) / passes;
}

// Digit counts of one tile, digit-major: counts[d * ntiles + tile].
template <typename K>
__global__ __launch_bounds__(kSortThreads) void k_sort_count(const K *__restrict__ keys, int64_t n, int shift,
                                                             int dbits, int32_t ntiles, int32_t *__restrict__ counts) {
    __shared__ int32_t h[kMaxDigits];
    const int ndig = 1 << dbits, mask = ndig - 1;
    for (int d = threadIdx.x; d < ndig; d += kSortThreads) h[d] = 0;
    __syncthreads();
    const int tile = blockIdx.x;
    const int64_t base = (int64_t)tile * kSortTile;
    const int lane = threadIdx.x & 63;
    K kk[kSortItems];
#pragma unroll
    for (int j = 0; j < kSortItems; ++j) {
        const int64_t i = base + j * kSortThreads + threadIdx.x;
        kk[j] = keys[i < n ? i : base];  // unconditional: all loads in flight together
    }
#pragma unroll
    for (int j = 0; j < kSortItems; ++j) {
        // lane 0 holds the wave's first pair: if it is past the end, so is the rest
        const bool ok = base + j * kSortThreads + threadIdx.x < n;
        const int d = (int)((kk[j] >> shift) & (K)mask);
        const int d0 = __builtin_amdgcn_readfirstlane(d);
        const uint64_t act = __ballot(ok);
        if (__ballot(ok && d != d0) == 0) {
            // one digit across the wave (the common case in the high passes): one atomic
            if (lane == 0 && act) atomicAdd(&h[d0], (int32_t)__popcll(act));
        } else if (ok) {
            atomicAdd(&h[d], 1);
        }
    }
    __syncthreads();
    for (int d = threadIdx.x; d < ndig; d += kSortThreads) counts[(int64_t)d * ntiles + tile] = h[d];
}

// One stable pass. Wave w holds the tile's pairs [w * kWaveItems, (w + 1) *
// kWaveItems), pair w * kWaveItems + j * 64 + lane in its step j. Each wave
// ranks its pairs among equal digits on its own (the lanes of a step sharing
// its digit give a lane its rank within the step, a per-wave digit count
// carries it across steps), one scan
// over the digits orders the waves, and the pairs are placed in LDS by digit
// and written out so that each digit's run of the tile lands contiguously at
// offsets[digit * ntiles + tile].
// With kLow the pass writes only (int32)(key & low_mask) to low_out.
template <typename K, typename V, bool kLow = false>
__global__ __launch_bounds__(kSortThreads) void k_sort_scatter(const K *__restrict__ kin, const V *__restrict__ vin,
                                                               int64_t n, int shift, int dbits, int32_t ntiles,
                                                               const int32_t *__restrict__ offsets,
                                                               K *__restrict__ kout, V *__restrict__ vout,
                                                               int32_t *__restrict__ low_out, K low_mask) {
    constexpr bool kVals = !std::is_same<V, NoValue>::value;
    using VS = typename std::conditional<kVals, V, char>::type;  // stored value type
    constexpr int kWaveItems = kSortItems * 64;
    // The ranking's lane masks (per wave and digit, cleared again by each
    // digit's first lane) and, after them, the tile's keys in digit order share
    // one LDS area.
    constexpr size_t kKeyBytes = sizeof(K) * kSortTile;
    constexpr size_t kMatchBytes = sizeof(unsigned long long) * kSortWaves * kMaxDigits;
    __shared__ __attribute__((aligned(16))) unsigned char area[kKeyBytes > kMatchBytes ? kKeyBytes : kMatchBytes];
    K *sk = reinterpret_cast<K *>(area);
    unsigned long long *match = reinterpret_cast<unsigned long long *>(area);
    __shared__ VS sv[kVals ? kSortTile : 1];
    // per-wave digit counts; after the scan, the first local slot of each wave's pairs of a digit
    __shared__ int32_t wbase[kSortWaves][kMaxDigits];
    __shared__ int32_t gofs[kMaxDigits];  // output index of a digit's pair = gofs[digit] + local slot
    __shared__ int32_t wsum[kMaxDigits / 64];  // digit totals of each scanning wave
    const int ndig = 1 << dbits, mask = ndig - 1;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    // consecutive tiles run on one XCD: its L2 then holds the offset lines and
    // the run boundaries that neighbouring tiles share
    const int tile = xcd_remap(blockIdx.x, ntiles);
    const int64_t base = (int64_t)tile * kSortTile;
    const int cnt = (int)(n - base < kSortTile ? n - base : kSortTile);

    K key[kSortItems];
    VS val[kSortItems];
    int dig[kSortItems];
    int rank[kSortItems];
    // unconditional loads (lanes past the end read the tile's first pair), all
    // issued before any is used
#pragma unroll
    for (int j = 0; j < kSortItems; ++j) {
        const int p = w * kWaveItems + j * 64 + lane;
        const int64_t i = base + (p < cnt ? p : 0);
        key[j] = kin[i];
        if constexpr (kVals) val[j] = vin[i];
    }
#pragma unroll
    for (int j = 0; j < kSortItems; ++j) {
        const int p = w * kWaveItems + j * 64 + lane;
        dig[j] = p < cnt ? (int)((key[j] >> shift) & (K)mask) : ndig;  // ndig: no pair
    }
    // this tile's output offset of digit tid (threads past the digits read
    // digit 0's), issued after the pairs without a branch: loads complete in
    // order, so the ranking waits for the pairs only
    const int32_t my_off = offsets[(int64_t)(tid < ndig ? tid : 0) * ntiles + tile];
    unsigned long long *wmatch = match + w * kMaxDigits;
    for (int d = lane; d < ndig; d += 64) {
        wbase[w][d] = 0;
        wmatch[d] = 0ull;
    }
    // The lanes of a step holding the same digit (peers) come from one ballot
    // per digit bit for narrow digits, whose cost does not depend on how the
    // digits are spread, and otherwise from an LDS OR of lane bits per digit
    // (fewer instructions, but lanes sharing a digit share an address); a step
    // whose lanes all hold one digit needs neither.
    // Only this wave touches its rows until the barrier, and the LDS carries
    // out one wave's accesses in program order: every lane's OR of a step
    // lands before any lane reads the mask back, and the reads before the
    // first lane of the digit clears it. OR does not depend on the order in
    // which lanes sharing a digit are served.
    const bool by_ballot = dbits <= kBallotDigitBits;
#pragma unroll
    for (int j = 0; j < kSortItems; ++j) {
        const int d = dig[j];
        const bool ok = d < ndig;
        const uint64_t act = __ballot(ok);
        const int d0 = __builtin_amdgcn_readfirstlane(d);  // lane 0 holds the wave's first pair
        const bool one = __ballot(ok && d != d0) == 0;
        uint64_t peers = act;
        if (!one) {
            if (by_ballot) {
                for (int b = 0; b < dbits; ++b) {
                    const uint64_t bal = __ballot(ok && ((d >> b) & 1));
                    peers &= ((d >> b) & 1) ? bal : ~bal;
                }
            } else {
                if (ok) atomicOr(&wmatch[d], 1ull << lane);
                __builtin_amdgcn_wave_barrier();
                peers = ok ? wmatch[d] : 0ull;
            }
        }
        const int lrank = (int)__popcll(peers & lanemask_lt());
        const int32_t before = ok ? wbase[w][d] : 0;
        rank[j] = before + lrank;
        __builtin_amdgcn_wave_barrier();
        if (ok && lrank == 0) {
            wbase[w][d] = before + (int32_t)__popcll(peers);
            if (!one && !by_ballot) wmatch[d] = 0ull;
        }
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    // exclusive scan of the tile's digit counts over the digits, thread d for
    // digit d (the first kMaxDigits / 64 waves; digits >= ndig count 0)
    int32_t tot = 0, incl = 0;
    if (tid < kMaxDigits) {
        if (tid < ndig)
            for (int x = 0; x < kSortWaves; ++x) tot += wbase[x][tid];
        incl = tot;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int32_t t = __shfl_up(incl, o);
            if (lane >= o) incl += t;
        }
        if (lane == 63) wsum[w] = incl;
    }
    __syncthreads();
    if (tid < ndig) {
        int32_t ex = incl - tot;
        for (int x = 0; x < w; ++x) ex += wsum[x];
        gofs[tid] = my_off - ex;
        int32_t run = ex;
        for (int x = 0; x < kSortWaves; ++x) {
            const int32_t c = wbase[x][tid];
            wbase[x][tid] = run;
            run += c;
        }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kSortItems; ++j) {
        if (dig[j] < ndig) {
            const int32_t pos = wbase[w][dig[j]] + rank[j];
            sk[pos] = key[j];
            if constexpr (kVals) sv[pos] = val[j];
        }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kSortItems; ++j) {
        const int p = j * kSortThreads + tid;
        if (p >= cnt) break;
        const K kk = sk[p];
        const int d = (int)((kk >> shift) & (K)mask);
        const int64_t g = (int64_t)gofs[d] + p;
        if constexpr (kLow) {
            low_out[g] = (int32_t)(kk & low_mask);
        } else {
            kout[g] = kk;
            if constexpr (kVals) vout[g] = sv[p];
        }
    }
}

size_t sort_ws_bytes(int64_t n, int bits, int key_bytes, int value_bytes) {
    const int passes = sort_passes(bits);
    if (passes == 0 || n <= 0) return 256;
    const int dbits = sort_digit_bits(bits);
    const int64_t ntiles = ceil_div(n, kSortTile);
    const int64_t ncounts = ((int64_t)1 << dbits) * ntiles;
    ArenaSize a;
    a.take<char>(n * (int64_t)key_bytes);    // keys between passes
    a.take<char>(n * (int64_t)value_bytes);  // values between passes
    a.take<int32_t>(ncounts);                // digit counts, then offsets
    return a.used + scan_add_ws_bytes(ncounts) + 512;
}

size_t seg_sort_ws_bytes(int64_t n, int bits, int value_bytes) { return sort_ws_bytes(n, bits, 2, value_bytes); }

template <typename K, typename V>
cagra_status radix_sort_stable(const K *keys_in, const V *vals_in, K *keys_out, V *vals_out, int64_t n, int bits,
                               void *ws, size_t ws_bytes, hipStream_t st) {
    constexpr bool kVals = !std::is_same<V, NoValue>::value;
    constexpr int kValBytes = kVals ? (int)sizeof(V) : 0;
    if (n <= 0) return CAGRA_OK;
    if (bits < 1) bits = 1;
    if (bits > (int)(8 * sizeof(K))) return fail(CAGRA_E_CAPACITY, "sort keys wider than the key type");
    const int passes = sort_passes(bits);
    const int dbits = sort_digit_bits(bits);
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
        k_sort_scatter<K, V><<<ntiles, kSortThreads, 0, st>>>(ks, vs, n, shift, dbits, ntiles, counts, kd, vd,
                                                              nullptr, (K)0);
        CAGRA_LAUNCH_CHECK();
        ks = kd;
        vs = vd;
    }
    return CAGRA_OK;
}

size_t sort_low32_ws_bytes(int64_t n, int bits) {
    const int passes = sort_passes(bits < 1 ? 1 : bits);
    if (passes == 0 || n <= 0) return 256;
    const int64_t ncounts = ((int64_t)1 << sort_digit_bits(bits)) * ceil_div(n, kSortTile);
    ArenaSize a;
    a.take<int32_t>(ncounts);
    return a.used + scan_add_ws_bytes(ncounts) + 512;
}

cagra_status radix_sort_low32(unsigned long long *keys, unsigned long long *tmp, const int32_t *pass0_counts,
                              int32_t *low_out, int64_t n, int bits, int low_bits, void *ws, size_t ws_bytes,
                              hipStream_t st) {
    using K = unsigned long long;
    if (n <= 0) return CAGRA_OK;
    if (bits < 1) bits = 1;
    if (bits > 64) return fail(CAGRA_E_CAPACITY, "sort keys wider than 64 bits");
    if (low_bits < 1 || low_bits > 31) return fail(CAGRA_E_INVALID, "low_bits must be in [1, 31]");
    const int passes = sort_passes(bits);
    const int dbits = sort_digit_bits(bits);
    if (ws_bytes < sort_low32_ws_bytes(n, bits)) return fail(CAGRA_E_BUFFER, "workspace too small (sort counts)");
    const int64_t ntiles64 = ceil_div(n, kSortTile);
    if (ntiles64 * ((int64_t)1 << dbits) > INT32_MAX) return fail(CAGRA_E_OVERFLOW, "sort too large");
    const int32_t ntiles = (int32_t)ntiles64;
    const int64_t ncounts = ((int64_t)1 << dbits) * ntiles;
    Arena ar{(char *)ws, ws_bytes, 0};
    int32_t *counts = ar.take<int32_t>(ncounts);
    char *scan_ws = ar.base + align_up(ar.used, 256);
    const size_t scan_bytes = ws_bytes - align_up(ar.used, 256);
    const K low_mask = ((K)1 << low_bits) - 1;
    const K *ks = keys;
    for (int p = 0; p < passes; ++p) {
        const bool last = p == passes - 1;
        K *kd = (p & 1) ? keys : tmp;  // keys -> tmp -> keys -> ...
        const int shift = p * dbits;
        const int32_t *cin = counts;
        if (p == 0 && pass0_counts) {
            cin = pass0_counts;
        } else {
            k_sort_count<K><<<ntiles, kSortThreads, 0, st>>>(ks, n, shift, dbits, ntiles, counts);
            CAGRA_LAUNCH_CHECK();
        }
        if (cagra_status s = scan_add_exclusive(cin, counts, ncounts, scan_ws, scan_bytes, st)) return s;
        if (last) {
            k_sort_scatter<K, NoValue, true><<<ntiles, kSortThreads, 0, st>>>(
                ks, nullptr, n, shift, dbits, ntiles, counts, nullptr, nullptr, low_out, low_mask);
        } else {
            k_sort_scatter<K, NoValue><<<ntiles, kSortThreads, 0, st>>>(ks, nullptr, n, shift, dbits, ntiles, counts,
                                                                        kd, nullptr, nullptr, (K)0);
        }
        CAGRA_LAUNCH_CHECK();
        ks = kd;
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
