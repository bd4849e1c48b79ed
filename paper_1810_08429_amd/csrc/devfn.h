// Device helpers shared by the kernels: reciprocal square roots, cross-lane
// sums inside a wavefront by DPP (no LDS round trip) and the moves between
// its rows of 16 lanes, sums over slot lists, and an XCD-aware workgroup
// order.
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

// Cross-lane moves for the tile reductions: DPP (above) within a row of 16
// lanes, an LDS swizzle for lane ^ 16 and a permute for lane ^ 32 (64-bit
// values move as two 32-bit halves).  Every lane of the wavefront must be
// active.
__device__ __forceinline__ float xor16_mov(float v)
{   // ds_swizzle bit mode within 32 lanes: and 0x1f, or 0, xor 0x10
    return __builtin_bit_cast(float, __builtin_amdgcn_ds_swizzle(__builtin_bit_cast(int, v), 0x401F));
}
__device__ __forceinline__ double xor16_mov(double v)
{
    const int2 h = __builtin_bit_cast(int2, v);
    return __builtin_bit_cast(double, int2{__builtin_amdgcn_ds_swizzle(h.x, 0x401F),
                                           __builtin_amdgcn_ds_swizzle(h.y, 0x401F)});
}
__device__ __forceinline__ float xor32_mov(float v, int addr)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_ds_bpermute(addr, __builtin_bit_cast(int, v)));
}
__device__ __forceinline__ double xor32_mov(double v, int addr)
{
    const int2 h = __builtin_bit_cast(int2, v);
    return __builtin_bit_cast(double, int2{__builtin_amdgcn_ds_bpermute(addr, h.x),
                                           __builtin_amdgcn_ds_bpermute(addr, h.y)});
}

// sum_{q in [b, e)} part[slots[q] * stride + x] on four partial sums (slots
// b + 4k + j on sum j, then (s0 + s1) + (s2 + s3)), so that four loads are in
// flight together; the order is fixed, the result reproducible.
template <typename T>
__device__ __forceinline__ T slot_sum(const T *part, const int64_t *slots, int64_t b, int64_t e, int64_t stride,
                                      int64_t x)
{
    T s0 = 0, s1 = 0, s2 = 0, s3 = 0;
    int64_t q = b;
    for (; q + 3 < e; q += 4) {
        s0 += part[slots[q] * stride + x];
        s1 += part[slots[q + 1] * stride + x];
        s2 += part[slots[q + 2] * stride + x];
        s3 += part[slots[q + 3] * stride + x];
    }
    if (q < e) s0 += part[slots[q] * stride + x];
    if (q + 1 < e) s1 += part[slots[q + 1] * stride + x];
    if (q + 2 < e) s2 += part[slots[q + 2] * stride + x];
    return (s0 + s1) + (s2 + s3);
}

// sum_{k < kt} val[e_k] x[oth[e_k] * stride + n] with e_k = e0 + k ld (a row
// of an ELL table whose entry k lies ld apart): four partners on four
// partial sums, so that their dependent loads (partner, then its x) are in
// flight together; fixed order.
__device__ __forceinline__ double ell_sum(const double *val, const int32_t *oth, const double *x, int64_t e0,
                                          int64_t ld, int kt, int64_t stride, int n)
{
    double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
    int k = 0;
    for (; k + 3 < kt; k += 4) {
        const int64_t e = e0 + (int64_t)k * ld;
        const int64_t o0 = oth[e], o1 = oth[e + ld], o2 = oth[e + 2 * ld], o3 = oth[e + 3 * ld];
        s0 += val[e] * x[o0 * stride + n];
        s1 += val[e + ld] * x[o1 * stride + n];
        s2 += val[e + 2 * ld] * x[o2 * stride + n];
        s3 += val[e + 3 * ld] * x[o3 * stride + n];
    }
    for (; k < kt; ++k) {
        const int64_t e = e0 + (int64_t)k * ld;
        s0 += val[e] * x[(int64_t)oth[e] * stride + n];
    }
    return (s0 + s1) + (s2 + s3);
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
