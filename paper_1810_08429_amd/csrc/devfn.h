// Device helpers shared by the kernels: reciprocal square roots, cross-lane
// sums inside a wavefront by DPP (no LDS round trip) and an XCD-aware
// workgroup order.
#pragma once

#include <hip/hip_runtime.h>

namespace gca {

template <typename T>
__device__ __forceinline__ T rsq(T x);
template <>
__device__ __forceinline__ float rsq<float>(float x) { return __builtin_amdgcn_rsqf(x); }
// FP64: the hardware estimate refined by one step of the binomial series
// (1 - e)^(-1/2) = 1 + e/2 + 3e^2/8 + ..., e = 1 - x y0^2, which triples the
// number of correct bits; valid for positive finite arguments (no
// special-value handling).
template <>
__device__ __forceinline__ double rsq<double>(double x)
{
    const double y = __builtin_amdgcn_rsq(x);
    const double e = __builtin_fma(-x * y, y, 1.0);
    return __builtin_fma(y * e, __builtin_fma(e, 0.375, 0.5), y);
}

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

// Workgroups are dealt to the 8 XCDs of the chip round-robin by id; this
// bijection of [0, nb) gives each XCD a contiguous range of work items, so
// the neighbouring data that adjacent items read stays in that XCD's L2.
__device__ __forceinline__ int xcd_contiguous(int b, int nb)
{
    const int q = nb / 8, r = nb % 8, x = b % 8;
    return x * q + min(x, r) + b / 8;
}

}  // namespace gca
