// Cross-lane helpers for 64-lane CDNA wavefronts.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bh {

__device__ __forceinline__ uint32_t lane_id() {
    return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

// lanes strictly below / at-or-below this lane
__device__ __forceinline__ uint64_t mask_lt(uint32_t lane) {
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}
__device__ __forceinline__ uint64_t mask_le(uint32_t lane) {
    return ~0ull >> (63 - lane);
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

// popcount of the set bits of m below this lane (v_mbcnt)
__device__ __forceinline__ uint32_t count_below(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ uint32_t shfl(uint32_t v, int src) { return __shfl(v, src, 64); }
__device__ __forceinline__ float shfl(float v, int src) { return __shfl(v, src, 64); }

// inclusive prefix sum over the 64 lanes (all lanes active): a Hillis-Steele
// scan inside each row of 16 lanes with DPP row shifts (lanes whose source is
// outside the row add 0), then the row totals carried by the row broadcasts.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v, uint32_t lane) {
    (void)lane;
    int s = (int)v;
    s += __builtin_amdgcn_update_dpp(0, s, 0x111, 0xf, 0xf, false);  // row_shr:1
    s += __builtin_amdgcn_update_dpp(0, s, 0x112, 0xf, 0xf, false);  // row_shr:2
    s += __builtin_amdgcn_update_dpp(0, s, 0x114, 0xf, 0xf, false);  // row_shr:4
    s += __builtin_amdgcn_update_dpp(0, s, 0x118, 0xf, 0xf, false);  // row_shr:8
    s += __builtin_amdgcn_update_dpp(0, s, 0x142, 0xa, 0xf, false);  // row_bcast:15 -> rows 1, 3
    s += __builtin_amdgcn_update_dpp(0, s, 0x143, 0xc, 0xf, false);  // row_bcast:31 -> rows 2, 3
    return (uint32_t)s;
}

// value of v in lane src (src uniform across the wave)
__device__ __forceinline__ uint32_t read_lane(uint32_t v, uint32_t src) {
    return (uint32_t)__builtin_amdgcn_readlane((int)v, (int)src);
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

__device__ __forceinline__ float wave_min(float v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v = fminf(v, __shfl_xor(v, d, 64));
    return v;
}

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v = fmaxf(v, __shfl_xor(v, d, 64));
    return v;
}

// uniform value from lane 0 held in a scalar register
__device__ __forceinline__ uint32_t uniform(uint32_t v) {
    return __builtin_amdgcn_readfirstlane(v);
}

}  // namespace bh
