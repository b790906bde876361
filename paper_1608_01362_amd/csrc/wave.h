// Wave-level building blocks shared by the edge-streaming kernels: DPP
// shifts and the inclusive wave sum, and raw buffer descriptor constants.
#pragma once

#include "common.h"

namespace cagra {

// ---- wave-level scans with DPP (row shifts within 16 lanes, then row broadcasts)
constexpr int kDppRowShr1 = 0x111, kDppRowShr2 = 0x112, kDppRowShr4 = 0x114, kDppRowShr8 = 0x118;
constexpr int kDppRowBcast15 = 0x142, kDppRowBcast31 = 0x143, kDppWaveShr1 = 0x138;

template <int CTRL, int ROWMASK>
__device__ __forceinline__ int32_t dpp_i(int32_t old, int32_t x) {
    return __builtin_amdgcn_update_dpp(old, x, CTRL, ROWMASK, 0xf, false);
}
template <int CTRL, int ROWMASK>
__device__ __forceinline__ float dpp_f(float old, float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(x), CTRL, ROWMASK, 0xf,
                                                      false));
}
template <int CTRL, int ROWMASK>
__device__ __forceinline__ int32_t dpp_t(int32_t old, int32_t x) { return dpp_i<CTRL, ROWMASK>(old, x); }
template <int CTRL, int ROWMASK>
__device__ __forceinline__ float dpp_t(float old, float x) { return dpp_f<CTRL, ROWMASK>(old, x); }

template <int CTRL, int ROWMASK>
__device__ __forceinline__ void add_step(int32_t &x) { x += dpp_i<CTRL, ROWMASK>(0, x); }

__device__ __forceinline__ int32_t wave_incl_sum(int32_t x) {
    add_step<kDppRowShr1, 0xf>(x);
    add_step<kDppRowShr2, 0xf>(x);
    add_step<kDppRowShr4, 0xf>(x);
    add_step<kDppRowShr8, 0xf>(x);
    add_step<kDppRowBcast15, 0xa>(x);
    add_step<kDppRowBcast31, 0xc>(x);
    return x;
}

constexpr int32_t kBufFlags = 0x00020000;   // raw buffer descriptor word 3 (gfx9)
constexpr int kNonTemporal = 2;             // cache policy: streaming
constexpr uint32_t kOutOfRange = 0x80000000u;

}  // namespace cagra
