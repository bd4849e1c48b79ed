// Product kernels of the nodal-basis GCA-H^2 handle (Sections 2-5 with one
// basis function per vertex, Section 5): the coupling matrices G|t~ x s~ and
// the nearfield blocks are stored whole at build time (column-major) and
// applied in column pieces, one wavefront each, whose partial row sums are
// added per target; the forward and backward transforms are those of the
// piecewise-constant handle (h2.hip).  FP64.
#include <hip/hip_runtime.h>

#include "gca_internal.h"

namespace gca {
namespace {

constexpr int AW = 4;          // wavefronts per workgroup: one piece each

// Row sums of one column piece of a stored block per wavefront: entries
// column-major (G[j nr + i]: a column is one coalesced load per 64 rows);
// blocks of up to 32 rows let the two half-wavefronts take the even and the
// odd columns; four columns per lane in flight.
__global__ void __launch_bounds__(64 * AW) k_lin_sub(LinApply a, const double *src)
{
    const int64_t b = (int64_t)blockIdx.x * AW + (threadIdx.x >> 6);
    if (b >= a.nsub) return;
    const int lane = threadIdx.x & 63;
    const int nr = a.sub_meta[3 * b], nc = a.sub_meta[3 * b + 1];
    const double *G = a.G + a.goff[b];
    const double *x = src + a.srcoff[b];
    double *out = a.part + a.poff[b];
    const int hs = nr <= 32 ? 2 : 1;
    const int rp = 64 / hs;
    const int h = hs == 2 ? (lane >> 5) : 0, rl = lane & (rp - 1);
    for (int r0 = 0; r0 < nr; r0 += rp) {
        const int r = r0 + rl;
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
        if (r < nr) {
            int j = h;
            for (; j + 3 * hs < nc; j += 4 * hs) {
                a0 += G[(int64_t)j * nr + r] * x[j];
                a1 += G[(int64_t)(j + hs) * nr + r] * x[j + hs];
                a2 += G[(int64_t)(j + 2 * hs) * nr + r] * x[j + 2 * hs];
                a3 += G[(int64_t)(j + 3 * hs) * nr + r] * x[j + 3 * hs];
            }
            for (; j < nc; j += hs) a0 += G[(int64_t)j * nr + r] * x[j];
        }
        double v = (a0 + a1) + (a2 + a3);
        if (hs == 2) v += __shfl_xor(v, 32);
        if (r < nr && h == 0) out[r] = v;
    }
}

// One workgroup per target, thread per row: the partial sums of the target's
// sub-blocks that cover the row, in stored order.  FAR: yh_t = the sum; else
// y|t = V_t yh_t + the sum, written in the original vertex order.
template <bool FAR>
__global__ void __launch_bounds__(128) k_lin_reduce(LinApply a, const int32_t *node, const int32_t *rank,
                                                    const int64_t *piv_off, const int64_t *v_off, const double *Vt,
                                                    const int32_t *perm, double *yh, double *y)
{
    const int g = blockIdx.x;
    const int t = a.tgt[g];
    const int b0 = node[5 * t];
    const int nrow = FAR ? rank[t] : node[5 * t + 1] - b0;
    const int64_t s0 = a.sub_ptr[g], s1 = a.sub_ptr[g + 1];
    for (int i = threadIdx.x; i < nrow; i += blockDim.x) {
        double acc = 0.0;
        for (int64_t b = s0; b < s1; ++b) {
            const int nr = a.sub_meta[3 * b], row0 = a.sub_meta[3 * b + 2];
            if (i >= row0 && i < row0 + nr) acc += a.part[a.poff[b] + i - row0];
        }
        if (FAR) {
            yh[piv_off[t] + i] = acc;
        } else {
            const double *Vc = Vt + v_off[t];
            const double *yc = yh + piv_off[t];
            double v = 0.0;
            for (int k = 0; k < rank[t]; ++k) v += Vc[(int64_t)k * nrow + i] * yc[k];
            y[perm[b0 + i]] = v + acc;
        }
    }
}

// sub-block b of a batch (row-major nr x nc at in + b ld) into the store:
// column-major with leading dimension ldo at out + dst[b] (meta: nr, nc, ldo)
__global__ void k_lin_compact(const double *in, int64_t ld, const int32_t *meta, const int64_t *dst, double *out)
{
    const int b = blockIdx.x;
    const int nr = meta[3 * b], nc = meta[3 * b + 1], ldo = meta[3 * b + 2];
    for (int e = threadIdx.x; e < nr * nc; e += blockDim.x) {
        const int i = e / nc, j = e - i * nc;
        out[dst[b] + (int64_t)j * ldo + i] = in[(int64_t)b * ld + e];
    }
}

}  // namespace

hipError_t launch_lin_sub(const LinApply &a, const double *src, hipStream_t s)
{
    if (a.nsub == 0) return hipSuccess;
    hipLaunchKernelGGL(k_lin_sub, dim3((unsigned)((a.nsub + AW - 1) / AW)), dim3(64 * AW), 0, s, a, src);
    return hipGetLastError();
}

hipError_t launch_lin_reduce(const gca_h2_s *h, const LinApply &a, bool far, double *yh, double *y, hipStream_t s)
{
    if (a.ntarget == 0) return hipSuccess;
    if (far)
        hipLaunchKernelGGL(k_lin_reduce<true>, dim3(a.ntarget), dim3(128), 0, s, a, h->d_node, h->d_rank,
                           h->d_piv_off, h->d_v_off, h->d_Vt, h->d_perm, yh, y);
    else
        hipLaunchKernelGGL(k_lin_reduce<false>, dim3(a.ntarget), dim3(128), 0, s, a, h->d_node, h->d_rank,
                           h->d_piv_off, h->d_v_off, h->d_Vt, h->d_perm, yh, y);
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
