// Vector kernels for the conjugate-gradient solve of G~ u = f with FP64
// iterative refinement (gca_solve_refined): fused axpy-type updates and FP64
// dot products reduced in a fixed order (per-workgroup partials, then one
// workgroup), so every iteration is bitwise reproducible.
#include <hip/hip_runtime.h>

#include "gca_internal.h"

namespace gca {

constexpr int DOT_THREADS = 256;
constexpr int DOT_BLOCKS = 1024;

__device__ double block_sum(double v, double *sh)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    if (l == 0) sh[w] = v;
    __syncthreads();
    double s = 0;
    if (threadIdx.x == 0)
        for (int k = 0; k < DOT_THREADS / 64; ++k) s += sh[k];
    return s;
}

// partial[b] = sum over the block's grid-stride share of a[i] * b[i]
__global__ void __launch_bounds__(DOT_THREADS) k_dot_partial(const double *a, const double *b, int64_t n,
                                                             double *partial)
{
    __shared__ double sh[DOT_THREADS / 64];
    double v = 0;
    for (int64_t i = (int64_t)blockIdx.x * DOT_THREADS + threadIdx.x; i < n; i += (int64_t)gridDim.x * DOT_THREADS)
        v += a[i] * b[i];
    double s = block_sum(v, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ void __launch_bounds__(DOT_THREADS) k_dot_final(const double *partial, int np, double factor,
                                                           double *out)
{
    __shared__ double sh[DOT_THREADS / 64];
    double v = 0;
    for (int i = threadIdx.x; i < np; i += DOT_THREADS) v += partial[i];
    double s = block_sum(v, sh);
    if (threadIdx.x == 0) *out = factor * s;
}

hipError_t launch_dot(const double *a, const double *b, int64_t n, double *partial, double *out, hipStream_t s,
                      double factor)
{
    int nb = (int)std::min<int64_t>(DOT_BLOCKS, (n + DOT_THREADS - 1) / DOT_THREADS);
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(k_dot_partial, dim3(nb), dim3(DOT_THREADS), 0, s, a, b, n, partial);
    hipLaunchKernelGGL(k_dot_final, dim3(1), dim3(DOT_THREADS), 0, s, partial, nb, factor, out);
    return hipGetLastError();
}

// y = (scale ? *scale : 1) * x
__global__ void k_scale(const double *scale, const double *x, double *y, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = (scale ? *scale : 1.0) * x[i];
}

hipError_t launch_scale(const double *scale, const double *x, double *y, int64_t n, hipStream_t s)
{
    if (n > 0) hipLaunchKernelGGL(k_scale, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, scale, x, y, n);
    return hipGetLastError();
}

// y = alpha * x + beta * y
__global__ void k_axpby(double alpha, const double *x, double beta, double *y, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = alpha * x[i] + beta * y[i];
}

// CG update: d += alpha p, r -= alpha q
__global__ void k_cg_update(double alpha, const double *p, const double *q, double *d, double *r, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        d[i] += alpha * p[i];
        r[i] -= alpha * q[i];
    }
}

__global__ void k_fill(double *y, double v, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = v;
}

hipError_t launch_fill(double *y, double v, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, y, v, n);
    return hipGetLastError();
}

// out = a - b
__global__ void k_sub(const double *a, const double *b, double *out, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = a[i] - b[i];
}

hipError_t launch_axpby(double alpha, const double *x, double beta, double *y, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_axpby, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, alpha, x, beta, y, n);
    return hipGetLastError();
}

hipError_t launch_cg_update(double alpha, const double *p, const double *q, double *d, double *r, int64_t n,
                            hipStream_t s)
{
    hipLaunchKernelGGL(k_cg_update, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, alpha, p, q, d, r, n);
    return hipGetLastError();
}

hipError_t launch_sub(const double *a, const double *b, double *out, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_sub, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a, b, out, n);
    return hipGetLastError();
}

}  // namespace gca
