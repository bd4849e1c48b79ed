// Cross-lane sums inside a wavefront by DPP (no LDS round trip).
#pragma once

#include <hip/hip_runtime.h>

namespace gca {

// DPP move within a row of 16 lanes (64-bit values move as two 32-bit
// halves).  The source lanes must be active.
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v)
{
    const int2 h = __builtin_bit_cast(int2, v);
    return __builtin_bit_cast(double, int2{__builtin_amdgcn_update_dpp(0, h.x, CTRL, 0xF, 0xF, false),
                                           __builtin_amdgcn_update_dpp(0, h.y, CTRL, 0xF, 0xF, false)});
}

// Sum over the N consecutive lanes of each aligned group (N = 1 .. 16); every
// lane of the group receives the sum.  DPP: lane ^ 1, lane ^ 2, mirror in 8,
// mirror in 16 -- each step pairs the two halves of the next larger group.
template <int N, typename T>
__device__ __forceinline__ T group_sum(T v)
{
    if constexpr (N >= 2) v += dpp_mov<0xB1>(v);    // quad_perm [1,0,3,2]
    if constexpr (N >= 4) v += dpp_mov<0x4E>(v);    // quad_perm [2,3,0,1]
    if constexpr (N >= 8) v += dpp_mov<0x141>(v);   // row_half_mirror
    if constexpr (N >= 16) v += dpp_mov<0x140>(v);  // row_mirror
    return v;
}

}  // namespace gca
