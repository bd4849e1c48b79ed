// The H^2 product for NB = 16 right-hand sides at once (h2_matvec with
// nrhs > 1): the four phases of Section 4's representation with every basis
// and transfer product a small dense GEMM on the matrix cores (mfma.h).
// Vectors, pivot vectors and partial slots hold the NB values of a row
// contiguously (row-major n x NB), so a 16 x 16 tile of a product reads its
// B operand as four rows of 16 consecutive values.  Transfers are level-wise
// launches with one wavefront per cluster; every sum has a fixed order.
#include <hip/hip_runtime.h>

#include "gca_internal.h"
#include "devfn.h"
#include "mfma.h"

namespace gca {

// xb[pos][k] = x[k * ld + perm[pos]] for k < nrhs, 0 for the padding columns;
// xb64 (if not null) the same in FP64 (the touching values are FP64).  A
// workgroup takes 64 consecutive original ids o: every column's 64 values
// are read coalesced and transposed in LDS, then the NB values of each row
// are written contiguously at position iperm[o] (four per thread).
template <typename T>
__device__ __forceinline__ void store4(T *dst, const double *v);
template <>
__device__ __forceinline__ void store4<float>(float *dst, const double *v)
{
    *reinterpret_cast<float4 *>(dst) = float4{(float)v[0], (float)v[1], (float)v[2], (float)v[3]};
}
template <>
__device__ __forceinline__ void store4<double>(double *dst, const double *v)
{
    reinterpret_cast<double2 *>(dst)[0] = double2{v[0], v[1]};
    reinterpret_cast<double2 *>(dst)[1] = double2{v[2], v[3]};
}

template <typename Tin, typename T>
__global__ void __launch_bounds__(256) k_permute_in_nb(const Tin *x, int64_t ld, int nrhs, const int32_t *iperm,
                                                       int64_t n, T *xb, double *xb64)
{
    __shared__ double tile[64][NB + 1];
    const int64_t o0 = (int64_t)blockIdx.x * 64;
    const int t = threadIdx.x, oo = t & 63;
    for (int k = t >> 6; k < NB; k += 4) {
        const int64_t o = o0 + oo;
        tile[oo][k] = (k < nrhs && o < n) ? (double)x[k * ld + o] : 0.0;
    }
    __syncthreads();
    const int r = t >> 2, kq = (t & 3) * 4;
    const int64_t o = o0 + r;
    if (o >= n) return;
    const int64_t pos = iperm[o];
    const double v[4] = {tile[r][kq], tile[r][kq + 1], tile[r][kq + 2], tile[r][kq + 3]};
    store4<T>(xb + pos * NB + kq, v);
    if (xb64) store4<double>(xb64 + pos * NB + kq, v);
}

template <typename T>
hipError_t launch_permute_in_nb(const void *x, bool xf32, int64_t ld, int nrhs, const int32_t *iperm, int64_t n,
                                T *xb, double *xb64, hipStream_t s)
{
    const dim3 grid((unsigned)((n + 63) / 64)), blk(256);
    if (xf32)
        hipLaunchKernelGGL((k_permute_in_nb<float, T>), grid, blk, 0, s, (const float *)x, ld, nrhs, iperm, n, xb,
                           xb64);
    else
        hipLaunchKernelGGL((k_permute_in_nb<double, T>), grid, blk, 0, s, (const double *)x, ld, nrhs, iperm, n,
                           xb, xb64);
    return hipGetLastError();
}

// Forward transform of one level, one wavefront per cluster:
//   leaf   xh_t = V_t^T x|t^      (V_t row-major |t^| x r, the K dimension its rows)
//   parent xh_t = sum_sons E_s^T xh_s  (E_s row-major r_s x r)
// as 16 x 16 tiles over (basis column, right-hand side).
template <typename T>
__global__ void __launch_bounds__(64) k_forward_nb(const int32_t *clusters, const int32_t *node, const int32_t *rank,
                                                   const int64_t *piv_off, const int64_t *v_off, const int64_t *e_off,
                                                   const T *V, const T *E, const T *xb, T *xhb)
{
    const int c = clusters[blockIdx.x];
    const int r = rank[c];
    const int s0 = node[5 * c + 2], s1 = node[5 * c + 3];
    const int lane = threadIdx.x, n = lane & 15, kq = lane >> 4;
    T *out = xhb + piv_off[c] * NB;
    for (int k0 = 0; k0 < r; k0 += 16) {
        const int k = k0 + (lane & 15);
        typename Mfma<T>::acc_t acc = mfma_zero<T>();
        auto run = [&](const T *M, int rows, const T *X) {
            for (int i0 = 0; i0 < rows; i0 += 4) {
                const int i = i0 + kq;
                const T a = (i < rows && k < r) ? M[(int64_t)i * r + k] : (T)0;
                const T b = i < rows ? X[(int64_t)i * NB + n] : (T)0;
                acc = Mfma<T>::mma(a, b, acc);
            }
        };
        if (s0 < 0) {
            const int b = node[5 * c], nr = node[5 * c + 1] - b;
            run(V + v_off[c], nr, xb + (int64_t)b * NB);
        } else {
            run(E + e_off[s0], rank[s0], xhb + piv_off[s0] * NB);
            run(E + e_off[s1], rank[s1], xhb + piv_off[s1] * NB);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int kk = k0 + Mfma<T>::row(lane, v);
            if (kk < r) out[(int64_t)kk * NB + n] = acc[v];
        }
    }
}

template <typename T>
hipError_t launch_forward_nb(gca_h2_s *h, const T *xb, T *xhb, hipStream_t s)
{
    const bool f32 = std::is_same<T, float>::value;
    const T *V = f32 ? (const T *)h->d_Vf : (const T *)h->d_V;
    const T *E = f32 ? (const T *)h->d_Ef : (const T *)h->d_E;
    for (int l = (int)h->level_clusters.size() - 1; l >= 0; --l) {
        const int nc = (int)h->level_clusters[l].size();
        if (!nc) continue;
        hipLaunchKernelGGL(k_forward_nb<T>, dim3(nc), dim3(64), 0, s, h->d_level_clusters[l], h->d_node, h->d_rank,
                           h->d_piv_off, h->d_v_off, h->d_e_off, V, E, xb, xhb);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// yh_c = sum over the cluster's coupling partial slots (fixed order), NB wide
template <typename T>
__global__ void k_coupling_reduce_nb(const int32_t *rank, const int64_t *piv_off, const int64_t *slot_ptr,
                                     const int64_t *slots, const T *part, T *yhb)
{
    const int c = blockIdx.x;
    const int m = rank[c] * NB;
    const int64_t b = slot_ptr[c], e = slot_ptr[c + 1];
    for (int x = threadIdx.x; x < m; x += blockDim.x) yhb[piv_off[c] * NB + x] = slot_sum(part, slots, b, e, NB, x);
}

template <typename T>
hipError_t launch_coupling_reduce_nb(gca_h2_s *h, const T *cpart, T *yhb, hipStream_t s)
{
    hipLaunchKernelGGL(k_coupling_reduce_nb<T>, dim3((unsigned)h->nc), dim3(256), 0, s, h->d_rank, h->d_piv_off,
                       h->d_gslot_ptr, h->d_gslot, cpart, yhb);
    return hipGetLastError();
}

// Backward transform of one level below the root, one wavefront per
// cluster: yh_c += E_c yh_parent (Et column-major: Et[k * r_c + j]).
template <typename T>
__global__ void __launch_bounds__(64) k_backward_nb(const int32_t *clusters, const int32_t *node, const int32_t *rank,
                                                    const int64_t *piv_off, const int64_t *e_off, const T *Et,
                                                    T *yhb)
{
    const int c = clusters[blockIdx.x];
    const int par = node[5 * c + 4];
    const int rc = rank[c], rp = rank[par];
    const T *M = Et + e_off[c];
    const T *Yp = yhb + piv_off[par] * NB;
    T *Yc = yhb + piv_off[c] * NB;
    const int lane = threadIdx.x, n = lane & 15, kq = lane >> 4;
    for (int j0 = 0; j0 < rc; j0 += 16) {
        const int j = j0 + (lane & 15);
        typename Mfma<T>::acc_t acc = mfma_zero<T>();
        for (int k0 = 0; k0 < rp; k0 += 4) {
            const int k = k0 + kq;
            const T a = (j < rc && k < rp) ? M[(int64_t)k * rc + j] : (T)0;
            const T b = k < rp ? Yp[(int64_t)k * NB + n] : (T)0;
            acc = Mfma<T>::mma(a, b, acc);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int jj = j0 + Mfma<T>::row(lane, v);
            if (jj < rc) Yc[(int64_t)jj * NB + n] += acc[v];
        }
    }
}

template <typename T>
hipError_t launch_backward_nb(gca_h2_s *h, T *yhb, hipStream_t s)
{
    const T *Et = std::is_same<T, float>::value ? (const T *)h->d_Etf : (const T *)h->d_Et;
    for (int l = 1; l < (int)h->level_clusters.size(); ++l) {
        const int nc = (int)h->level_clusters[l].size();
        if (!nc) continue;
        hipLaunchKernelGGL(k_backward_nb<T>, dim3(nc), dim3(64), 0, s, h->d_level_clusters[l], h->d_node, h->d_rank,
                           h->d_piv_off, h->d_e_off, Et, yhb);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Gather per leaf (one wavefront): y|t^ = V_t yh_t on the matrix cores (Vt
// column-major: Vt[k * |t^| + i]), plus the nearfield partials, the
// near-regular list values and the touching values (FP64, against the FP64
// copy of x), written to column k < nrhs of y in the original order.
template <typename T, typename Tout>
__global__ void __launch_bounds__(64) k_gather_nb(const int32_t *leaves, const int32_t *node, const int32_t *rank,
                                                  const int64_t *piv_off, const int64_t *v_off, const T *Vt,
                                                  const T *yhb, const int64_t *nslot_ptr, const int64_t *nslot,
                                                  const T *npart, const int64_t *tell_off, const int32_t *tell_k,
                                                  const int32_t *tother, const double *tval, const int64_t *nptr,
                                                  const int32_t *nother, const T *nval, const T *xb,
                                                  const double *xb64, const int32_t *perm, Tout *y, int64_t ld,
                                                  int nrhs)
{
    const int li = xcd_contiguous(blockIdx.x, gridDim.x);  // XCD-local neighbours
    const int c = leaves[li];
    const int b = node[5 * c], nr = node[5 * c + 1] - b;
    const int r = rank[c];
    const T *M = Vt + v_off[c];
    const T *Y = yhb + piv_off[c] * NB;
    const int lane = threadIdx.x, n = lane & 15, kq = lane >> 4;
    for (int i0 = 0; i0 < nr; i0 += 16) {
        const int i = i0 + (lane & 15);
        typename Mfma<T>::acc_t acc = mfma_zero<T>();
        for (int k0 = 0; k0 < r; k0 += 4) {
            const int k = k0 + kq;
            const T a = (i < nr && k < r) ? M[(int64_t)k * nr + i] : (T)0;
            const T bb = k < r ? Y[(int64_t)k * NB + n] : (T)0;
            acc = Mfma<T>::mma(a, bb, acc);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int ii = i0 + Mfma<T>::row(lane, v);
            if (ii >= nr) continue;
            T sum = acc[v] + slot_sum(npart, nslot, nslot_ptr[li], nslot_ptr[li + 1], NB, (int64_t)ii * NB + n);
            const int pos = b + ii;
            for (int64_t q = nptr[pos]; q < nptr[pos + 1]; ++q) sum += nval[q] * xb[(int64_t)nother[q] * NB + n];
            const double s64 = ell_sum(tval, tother, xb64, tell_off[li] + ii, nr, tell_k[li], NB, n);
            if (n < nrhs) y[(int64_t)n * ld + perm[pos]] = (Tout)((double)sum + s64);
        }
    }
}

template <typename T>
hipError_t launch_gather_nb(gca_h2_s *h, const T *xb, const double *xb64, const T *yhb, const T *npart,
                            const T *nval, void *y, bool yf32, int64_t ld, int nrhs, hipStream_t s)
{
    const T *Vt = std::is_same<T, float>::value ? (const T *)h->d_Vtf : (const T *)h->d_Vt;
    const dim3 grid((unsigned)h->leaves.size()), blk(64);
#define GATHER(TO)                                                                                              \
    hipLaunchKernelGGL((k_gather_nb<T, TO>), grid, blk, 0, s, h->d_leaves, h->d_node, h->d_rank, h->d_piv_off,  \
                       h->d_v_off, Vt, yhb, h->d_gnslot_ptr, h->d_gnslot, npart, h->d_tell_off, h->d_tell_k,     \
                       h->d_tell_other, h->d_tval, h->d_nptr, h->d_nother, nval, xb, xb64, h->d_perm, (TO *)y,   \
                       ld, nrhs)
    if (yf32)
        GATHER(float);
    else
        GATHER(double);
#undef GATHER
    return hipGetLastError();
}

#define INST(T)                                                                                                  \
    template hipError_t launch_permute_in_nb<T>(const void *, bool, int64_t, int, const int32_t *, int64_t, T *,  \
                                                double *, hipStream_t);                                          \
    template hipError_t launch_forward_nb<T>(gca_h2_s *, const T *, T *, hipStream_t);                           \
    template hipError_t launch_coupling_reduce_nb<T>(gca_h2_s *, const T *, T *, hipStream_t);                   \
    template hipError_t launch_backward_nb<T>(gca_h2_s *, T *, hipStream_t);                                     \
    template hipError_t launch_gather_nb<T>(gca_h2_s *, const T *, const double *, const T *, const T *,         \
                                            const T *, void *, bool, int64_t, int, hipStream_t);
INST(float)
INST(double)
#undef INST

}  // namespace gca
