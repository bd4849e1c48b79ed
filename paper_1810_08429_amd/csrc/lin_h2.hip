// Product kernels of the nodal-basis GCA-H^2 handle (Sections 2-5 with one
// basis function per vertex, Section 5): the coupling matrices G|t~ x s~ and
// the nearfield blocks are stored at build time as sub-blocks (pivot or leaf
// chunks small enough for the pair-wise assembly); the forward and backward
// transforms are those of the piecewise-constant handle (h2.hip).  FP64.
#include <hip/hip_runtime.h>

#include "gca_internal.h"

namespace gca {
namespace {

// sum over the target's sub-blocks (stored order) that cover row i
__device__ __forceinline__ double sub_rows(const LinApply &a, int64_t b0, int64_t b1, int i, const double *src)
{
    double acc = 0.0;
    for (int64_t b = b0; b < b1; ++b) {
        const int nr = a.sub_meta[3 * b], nc = a.sub_meta[3 * b + 1], row0 = a.sub_meta[3 * b + 2];
        if (i < row0 || i >= row0 + nr) continue;
        const double *G = a.G + a.goff[b] + (int64_t)(i - row0) * nc;
        const double *x = src + a.srcoff[b];
        for (int j = 0; j < nc; ++j) acc += G[j] * x[j];
    }
    return acc;
}

// one workgroup per cluster, thread per pivot: yh_t = sum_s G|t~ x s~ xh_s
__global__ void __launch_bounds__(128) k_lin_far_apply(LinApply a, const int32_t *rank, const int64_t *piv_off,
                                                       const double *xh, double *yh)
{
    const int g = blockIdx.x;
    const int t = a.tgt[g];
    const int r = rank[t];
    for (int i = threadIdx.x; i < r; i += blockDim.x)
        yh[piv_off[t] + i] = sub_rows(a, a.sub_ptr[g], a.sub_ptr[g + 1], i, xh);
}

// one workgroup per leaf, thread per row: y = V_t yh_t + the nearfield blocks,
// written in the original vertex order
__global__ void __launch_bounds__(64) k_lin_gather(LinApply a, const int32_t *node, const int32_t *rank,
                                                   const int64_t *piv_off, const int64_t *v_off, const double *Vt,
                                                   const int32_t *perm, const double *xp, const double *yh,
                                                   double *y)
{
    const int g = blockIdx.x;
    const int t = a.tgt[g];
    const int b = node[5 * t], nr = node[5 * t + 1] - b, r = rank[t];
    const double *Vc = Vt + v_off[t];
    const double *yc = yh + piv_off[t];
    for (int i = threadIdx.x; i < nr; i += blockDim.x) {
        double acc = 0.0;
        for (int k = 0; k < r; ++k) acc += Vc[(int64_t)k * nr + i] * yc[k];
        acc += sub_rows(a, a.sub_ptr[g], a.sub_ptr[g + 1], i, xp);
        y[perm[b + i]] = acc;
    }
}

__global__ void k_lin_compact(const double *in, int64_t ld, const int32_t *meta, const int64_t *goff, double *out)
{
    const int b = blockIdx.x;
    const int n = meta[3 * b] * meta[3 * b + 1];
    for (int e = threadIdx.x; e < n; e += blockDim.x) out[goff[b] + e] = in[(int64_t)b * ld + e];
}

}  // namespace

hipError_t launch_lin_far_apply(const gca_h2_s *h, const LinApply &a, const double *xh, double *yh, hipStream_t s)
{
    if (a.ntarget == 0) return hipSuccess;
    hipLaunchKernelGGL(k_lin_far_apply, dim3(a.ntarget), dim3(128), 0, s, a, h->d_rank, h->d_piv_off, xh, yh);
    return hipGetLastError();
}

hipError_t launch_lin_gather(const gca_h2_s *h, const LinApply &a, const double *xp, const double *yh, double *y,
                             hipStream_t s)
{
    if (a.ntarget == 0) return hipSuccess;
    hipLaunchKernelGGL(k_lin_gather, dim3(a.ntarget), dim3(64), 0, s, a, h->d_node, h->d_rank, h->d_piv_off,
                       h->d_v_off, h->d_Vt, h->d_perm, xp, yh, y);
    return hipGetLastError();
}

hipError_t launch_lin_compact(const double *in, int64_t ld, int32_t nb, const int32_t *meta, const int64_t *goff,
                              double *out, hipStream_t s)
{
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL(k_lin_compact, dim3(nb), dim3(256), 0, s, in, ld, meta, goff, out);
    return hipGetLastError();
}

}  // namespace gca
