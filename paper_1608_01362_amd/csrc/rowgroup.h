// Edge groups for gathers of 256-byte vertex records ([V][64] FP32): a wave's
// share of a tile's edges is cut into four contiguous parts, one per 16-lane
// group (one DPP row), and each group walks its part one edge at a time with
// four of the 64 columns per lane, so a record is one 16-byte load per lane.
#pragma once

#include "common.h"

namespace cagra {

constexpr int kGroup = 16;
constexpr int kGroupsPerWave = kWave / kGroup;

// Lane J of each 16-lane group, to every lane of the group (ds_swizzle bit
// mode: lane id bit 4 kept, bits 0-3 set to J, within each 32-lane half).
template <int J>
__device__ __forceinline__ int32_t group_bcast(int32_t v) {
    return __builtin_amdgcn_ds_swizzle(v, 0x10 | (J << 5));
}

// Lane j < 4 of the group, to every lane of the group (j known after unrolling).
__device__ __forceinline__ int32_t group_bcast4(int32_t v, int j) {
    return j == 0 ? group_bcast<0>(v) : j == 1 ? group_bcast<1>(v) : j == 2 ? group_bcast<2>(v) : group_bcast<3>(v);
}

struct GroupPart {
    int64_t a, b;    // the group's part [a, b) of the share
    int64_t len;     // the longest part's length (the same for the wave's four groups)
    int32_t before;  // row starts (flagged edge words) in [w0, a)
};

// Group g's part of the share [w0, w1) of a tile, with the row starts before
// it, counted by the wave (ballots over 64-word chunks up to the last part's
// start). Every lane of the wave must call it.
template <typename W>
__device__ __forceinline__ GroupPart group_part(const W *__restrict__ edge_src, int64_t w0, int64_t w1, int g,
                                                int lane) {
    GroupPart p;
    p.len = (w1 - w0 + kGroupsPerWave - 1) / kGroupsPerWave;
    p.a = w0 + g * p.len;
    if (p.a > w1) p.a = w1;
    p.b = p.a + p.len;
    if (p.b > w1) p.b = w1;
    int64_t a_last = w0 + (kGroupsPerWave - 1) * p.len;
    if (a_last > w1) a_last = w1;
    int32_t c1 = 0, c2 = 0, c3 = 0;
    for (int64_t c0 = w0; c0 < a_last; c0 += kWave) {
        const int64_t e = c0 + lane;
        const bool f = e < a_last && ((uint32_t)edge_src[e < a_last ? e : c0] & EdgeWord<W>::kFlag);
        const uint64_t m = __ballot(f);
        auto below = [&](int64_t n) -> int32_t {  // flags at chunk positions < n
            if (n <= 0) return 0;
            if (n >= 64) return __builtin_popcountll(m);
            return __builtin_popcountll(m & ((1ull << n) - 1ull));
        };
        c1 += below(w0 + p.len - c0);
        c2 += below(w0 + 2 * p.len - c0);
        c3 += below(w0 + 3 * p.len - c0);
    }
    p.before = g == 0 ? 0 : (g == 1 ? c1 : (g == 2 ? c2 : c3));
    return p;
}

// Index of the edge whose word and value lane `sub` of a group loads for the
// window starting at offset o of the part: edge a + o + (sub mod 4), or an
// edge of the part (of the tile when the part is empty) for lanes past it.
__device__ __forceinline__ int64_t group_window_edge(const GroupPart &p, int64_t o, int sub, int64_t e0,
                                                     int64_t e1) {
    const int64_t ej = p.a + o + (sub & 3);
    const int64_t ec = ej < p.b ? ej : (p.a < p.b ? p.a : e0);
    return ec < e1 ? ec : e0;
}

}  // namespace cagra
