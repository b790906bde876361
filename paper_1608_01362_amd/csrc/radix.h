// Stable least-significant-digit radix sorts (segsort.hip) and the device-wide
// exclusive scan (builder.hip): the interface shared by the segment builder
// and the clustering step.
#pragma once

#include "common.h"

namespace cagra {

// Value type of a sort of keys alone.
struct NoValue {};

// Pairs per tile. A pass counts the digits of each tile of kRadixTile
// consecutive pairs (tile t = pairs [t * kRadixTile, (t + 1) * kRadixTile)).
constexpr int kRadixTile = 4096;

// Digit width of every pass for keys below 2^bits.
int sort_digit_bits(int bits);

// Temporary bytes for radix_sort_stable.
size_t sort_ws_bytes(int64_t n, int bits, int key_bytes, int value_bytes);

// Stable sort of n (key, value) pairs by key (keys < 2^bits, bits up to the key
// width); V = NoValue sorts keys alone. keys_in/vals_in are read, not modified;
// keys_out/vals_out receive the sorted pairs and must not alias the inputs.
template <typename K, typename V>
cagra_status radix_sort_stable(const K *keys_in, const V *vals_in, K *keys_out, V *vals_out, int64_t n, int bits,
                               void *ws, size_t ws_bytes, hipStream_t st);

// The same for 16-bit keys (segment ids), values of 2, 4 or 8 bytes.
size_t seg_sort_ws_bytes(int64_t n, int bits, int value_bytes);
template <typename V>
cagra_status seg_sort_pairs(const uint16_t *keys_in, const V *vals_in, uint16_t *keys_out, V *vals_out, int64_t n,
                            int bits, void *ws, size_t ws_bytes, hipStream_t st);

// Temporary bytes for radix_sort_low32 (digit counts and the scan; the key
// buffers between passes are the caller's).
size_t sort_low32_ws_bytes(int64_t n, int bits);

// Stable sort of n 64-bit keys (< 2^bits) whose result is only the low
// low_bits bits of each key, in sorted order, as int32 (low_out). The passes
// alternate between keys and tmp (n keys each, both overwritten). If
// pass0_counts is not null it holds the first pass's digit counts, digit-major
// (counts[d * ntiles + t] for tile t of kRadixTile keys, digit width
// sort_digit_bits(bits)), and that counting pass is skipped.
cagra_status radix_sort_low32(unsigned long long *keys, unsigned long long *tmp, const int32_t *pass0_counts,
                              int32_t *low_out, int64_t n, int bits, int low_bits, void *ws, size_t ws_bytes,
                              hipStream_t st);

// Device-wide exclusive sum of n int32 values (in and out may alias).
size_t scan_add_ws_bytes(int64_t n);
cagra_status scan_add_exclusive(const int32_t *in, int32_t *out, int64_t n, void *ws, size_t ws_bytes,
                                hipStream_t st);

}  // namespace cagra
