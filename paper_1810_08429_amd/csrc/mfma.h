// Matrix-core tiles of the batched (16 right-hand sides) products on gfx950.
//
// One v_mfma_{f32,f64}_16x16x4 per call: D (16 x 16) += A (16 x 4) B (4 x 16)
// over a wavefront of 64 lanes.  Lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16], and holds D[row(l, v)][l % 16] in element v of its
// accumulator (v = 0..3): row 4 (l / 16) + v for FP32, row l / 16 + 4 v for
// FP64 (both checked on the device).  Every lane of the wavefront must be
// active.
#pragma once

#include <hip/hip_runtime.h>

#include "gca_internal.h"

namespace gca {

template <typename T>
struct Mfma;

template <>
struct Mfma<float> {
    typedef float acc_t __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};

template <>
struct Mfma<double> {
    typedef double acc_t __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int v) { return (lane >> 4) + 4 * v; }
};

template <typename T>
__device__ __forceinline__ typename Mfma<T>::acc_t mfma_zero()
{
    typename Mfma<T>::acc_t z;
    z[0] = z[1] = z[2] = z[3] = (T)0;
    return z;
}

}  // namespace gca
