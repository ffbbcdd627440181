// Device-side helpers shared by the HIP kernels (not included by host code).
#pragma once

#include <hip/hip_runtime.h>

namespace gem {

// Neighbour lanes of a wavefront through the DPP wavefront shifts of the
// GFX9 family (a modifier of one VALU move, instead of an LDS permute):
// lane l gets x of lane l + 1 (lane_next) or l - 1 (lane_prev); the last,
// resp. first, lane keeps its own value, as __shfl_down / __shfl_up(x, 1)
// do.
__device__ __forceinline__ float lane_next(float x) {
    const int i = __float_as_int(x);
    return __int_as_float(__builtin_amdgcn_update_dpp(i, i, 0x130 /* wave_shl:1 */, 0xf, 0xf, false));
}
__device__ __forceinline__ float lane_prev(float x) {
    const int i = __float_as_int(x);
    return __int_as_float(__builtin_amdgcn_update_dpp(i, i, 0x138 /* wave_shr:1 */, 0xf, 0xf, false));
}

// V consecutive floats (V = 1, 2, 4) as one aligned vector access.
template <int V>
__device__ __forceinline__ void ldv(float (&r)[V], const float *p) {
    if constexpr (V == 4) {
        const float4 t = *reinterpret_cast<const float4 *>(p);
        r[0] = t.x; r[1] = t.y; r[2] = t.z; r[3] = t.w;
    } else if constexpr (V == 2) {
        const float2 t = *reinterpret_cast<const float2 *>(p);
        r[0] = t.x; r[1] = t.y;
    } else {
        r[0] = *p;
    }
}

template <int V>
__device__ __forceinline__ void stv(float *p, const float (&r)[V]) {
    if constexpr (V == 4) {
        *reinterpret_cast<float4 *>(p) = make_float4(r[0], r[1], r[2], r[3]);
    } else if constexpr (V == 2) {
        *reinterpret_cast<float2 *>(p) = make_float2(r[0], r[1]);
    } else {
        *p = r[0];
    }
}

// Blocks stay round-robin over the XCDs in aligned groups of 8, but each
// group is rotated by a hash of its index, so work that recurs at a fixed
// block stride (a multiple of 8) does not fall on the same XCDs; the last
// nb % 8 blocks stay in place.  A bijection of [0, nb).
__device__ __forceinline__ int xcd_scatter(int b, int nb) {
    if (b >= (nb & ~7)) return b;
    const unsigned g = (unsigned)b >> 3;
    const unsigned h = (g * 2654435761u) >> 29;
    return (int)((g << 3) | (((unsigned)b + h) & 7u));
}

// Blocks are handed to the 8 XCDs round-robin; remap so that each XCD works
// on a contiguous range of tiles (neighbouring tiles share halo lines in the
// same L2).
__device__ __forceinline__ int xcd_block(int b, int nb) {
    return (nb % 8 == 0) ? (b % 8) * (nb / 8) + (b / 8) : b;
}

}  // namespace gem
