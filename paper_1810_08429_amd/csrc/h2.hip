// The four phases of the H^2 matrix-vector product (Section 4's
// representation G|t^ x s^ ~ V_t G|t~ x s~ V_s^* with nested bases
// V_t = [V_t1 E_t1; V_t2 E_t2]):
//   forward : xh_t = V_t^T x|t^ at leaves, xh_t = sum_sons E_t'^T xh_t' above;
//   coupling: yh_t = sum_s G|t~ x s~ xh_s (entries recomputed, quad.hip);
//   backward: yh_t' += E_t' yh_t downwards, y|t^ += V_t yh_t at the leaves;
//   nearfield: y|t^ += G|t^ x s^ x|s^ (quad.hip) plus the per-case pair lists.
// Transfers are level-wise launches, one workgroup per cluster; all sums are
// in a fixed order (no atomics), so results are bitwise reproducible.
#include <hip/hip_runtime.h>

#include "gca_internal.h"
#include "devfn.h"

namespace gca {

template <typename Tin, typename T>
__global__ void k_permute_in(const Tin *x, const int32_t *perm, int64_t n, T *xp, double *xp64)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double v = (double)x[perm[i]];
    xp[i] = (T)v;
    if (xp64) xp64[i] = v;
}

template <typename T>
hipError_t launch_permute_in(const void *x, bool xf32, const int32_t *perm, int64_t n, T *xp, double *xp64,
                             hipStream_t s)
{
    const dim3 grid((unsigned)((n + 255) / 256)), blk(256);
    if (xf32)
        hipLaunchKernelGGL((k_permute_in<float, T>), grid, blk, 0, s, (const float *)x, perm, n, xp, xp64);
    else
        hipLaunchKernelGGL((k_permute_in<double, T>), grid, blk, 0, s, (const double *)x, perm, n, xp, xp64);
    return hipGetLastError();
}
template hipError_t launch_permute_in<float>(const void *, bool, const int32_t *, int64_t, float *, double *,
                                             hipStream_t);
template hipError_t launch_permute_in<double>(const void *, bool, const int32_t *, int64_t, double *, double *,
                                              hipStream_t);

// sum_i M[i * ld + k] v[i] for i < m: rows are fetched sixteen at a time into
// registers before they are used, so their loads are in flight together
// (v is read at the same address by the whole wavefront); four partial sums
template <typename T>
__device__ __forceinline__ T col_dot(const T *M, int64_t ld, int m, const T *v, int k)
{
    constexpr int U = 16;
    T acc[4] = {0, 0, 0, 0};
    for (int i0 = 0; i0 < m; i0 += U) {
        T mv[U], vv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = i0 + u;
            mv[u] = i < m ? M[(int64_t)i * ld + k] : (T)0;
            vv[u] = i < m ? v[i] : (T)0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) acc[u & 3] += mv[u] * vv[u];
    }
    return (acc[0] + acc[1]) + (acc[2] + acc[3]);
}

// sum_{i0 <= i < i1} M[i * ld + k] v[i]: col_dot over a row range
template <typename T>
__device__ __forceinline__ T col_dot_range(const T *M, int64_t ld, int i0, int i1, const T *v, int k)
{
    return col_dot(M + (int64_t)i0 * ld, ld, i1 - i0, v + i0, k);
}

// forward transform for the clusters of one level (one wavefront per
// cluster).  Leaf: V row-major |t^| x r.  Parent: E_son row-major
// r_son x r.  With r <= 32 the two half-wavefronts take the two halves of
// the rows of the same column k and add their sums across lane ^ 32 (twice
// the active lanes, half the dependent loads); else a lane per column.
template <typename T>
__global__ void __launch_bounds__(64) k_forward(const int32_t *clusters, const int32_t *node, const int32_t *rank,
                                                const int64_t *piv_off, const int64_t *v_off, const int64_t *e_off,
                                                const T *V, const T *E, const T *xp, T *xh)
{
    const int c = clusters[blockIdx.x];
    const int r = rank[c];
    const int s0 = node[5 * c + 2], s1 = node[5 * c + 3];
    const int lane = threadIdx.x;
    T *out = xh + piv_off[c];
    if (r <= 32) {
        const int k = lane & 31, h = lane >> 5;
        T acc = 0;
        if (k < r) {
            if (s0 < 0) {
                const int b = node[5 * c], nr = node[5 * c + 1] - b, m = (nr + 1) >> 1;
                acc = col_dot_range(V + v_off[c], r, h ? m : 0, h ? nr : m, xp + b, k);
            } else {
                const int r0 = rank[s0], r1 = rank[s1];
                // half 0: son 0, half 1: son 1
                acc = h ? col_dot(E + e_off[s1], r, r1, xh + piv_off[s1], k)
                        : col_dot(E + e_off[s0], r, r0, xh + piv_off[s0], k);
            }
        }
        acc += __shfl_xor(acc, 32, 64);
        if (h == 0 && k < r) out[k] = acc;
        return;
    }
    if (s0 < 0) {
        const int b = node[5 * c], nr = node[5 * c + 1] - b;
        const T *Vc = V + v_off[c];
        for (int k = lane; k < r; k += 64) out[k] = col_dot(Vc, r, nr, xp + b, k);
    } else {
        const int r0 = rank[s0], r1 = rank[s1];
        const T *E0 = E + e_off[s0], *E1 = E + e_off[s1];
        const T *x0 = xh + piv_off[s0], *x1 = xh + piv_off[s1];
        for (int k = lane; k < r; k += 64) out[k] = col_dot(E0, r, r0, x0, k) + col_dot(E1, r, r1, x1, k);
    }
}

// The levels with few clusters (the upper tree, where ranks are largest):
// a workgroup of four wavefronts per cluster, each wavefront a quarter of the
// rows (leaf: the rows of V; parent: the rows of E_son0 then E_son1), lanes
// over the basis columns, the quarters added in LDS in a fixed order.
constexpr int WIDE_LEVEL = 1024;   // clusters of a level below which it runs wide
constexpr int WIDE_MINR = 64;      // ... when some rank exceeds a wavefront (measured: slower below)
constexpr int WIDE_MAXR = 512;     // ranks (at most the 2k <= 512 Green columns)

template <typename T>
__global__ void __launch_bounds__(256) k_forward_wide(const int32_t *clusters, const int32_t *node,
                                                      const int32_t *rank, const int64_t *piv_off,
                                                      const int64_t *v_off, const int64_t *e_off, const T *V,
                                                      const T *E, const T *xp, T *xh)
{
    __shared__ T part[4][WIDE_MAXR];
    const int c = clusters[blockIdx.x];
    const int r = rank[c];
    const int s0 = node[5 * c + 2], s1 = node[5 * c + 3];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const bool leaf = s0 < 0;
    const int b = node[5 * c];
    const int r0 = leaf ? node[5 * c + 1] - b : rank[s0];
    const int nrow = leaf ? r0 : r0 + rank[s1];
    const int i0 = (w * nrow) / 4, i1 = ((w + 1) * nrow) / 4;
    for (int k = lane; k < r; k += 64) {
        T acc = 0;
        if (leaf) {
            acc = col_dot_range(V + v_off[c], r, i0, i1, xp + b, k);
        } else {
            // rows [i0, i1) of E_son0 (i < r0) and E_son1 (i >= r0)
            const int a0 = min(i0, r0), a1 = min(i1, r0);
            if (a1 > a0) acc += col_dot_range(E + e_off[s0], r, a0, a1, xh + piv_off[s0], k);
            const int b0 = max(i0, r0) - r0, b1 = max(i1, r0) - r0;
            if (b1 > b0) acc += col_dot_range(E + e_off[s1], r, b0, b1, xh + piv_off[s1], k);
        }
        part[w][k] = acc;
    }
    __syncthreads();
    T *out = xh + piv_off[c];
    for (int k = threadIdx.x; k < r; k += 256) out[k] = (part[0][k] + part[1][k]) + (part[2][k] + part[3][k]);
}

// yh_c += E_c yh_parent for the clusters of a level with few clusters: the
// parent's rows in quarters over the four wavefronts, lanes over the columns
template <typename T>
__global__ void __launch_bounds__(256) k_backward_wide(const int32_t *clusters, const int32_t *node,
                                                       const int32_t *rank, const int64_t *piv_off,
                                                       const int64_t *e_off, const T *Et, T *yh)
{
    __shared__ T part[4][WIDE_MAXR];
    const int c = clusters[blockIdx.x];
    const int par = node[5 * c + 4];
    const int rc = rank[c], rp = rank[par];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int i0 = (w * rp) / 4, i1 = ((w + 1) * rp) / 4;
    const T *Ec = Et + e_off[c];
    const T *yp = yh + piv_off[par];
    for (int j = lane; j < rc; j += 64) part[w][j] = col_dot_range(Ec, rc, i0, i1, yp, j);
    __syncthreads();
    T *yc = yh + piv_off[c];
    for (int j = threadIdx.x; j < rc; j += 256) yc[j] += (part[0][j] + part[1][j]) + (part[2][j] + part[3][j]);
}

template <typename T>
hipError_t launch_forward(gca_h2_s *h, const T *xp, T *xh, hipStream_t s)
{
    const T *V = std::is_same<T, float>::value ? (const T *)h->d_Vf : (const T *)h->d_V;
    const T *E = std::is_same<T, float>::value ? (const T *)h->d_Ef : (const T *)h->d_E;
    for (int l = (int)h->level_clusters.size() - 1; l >= 0; --l) {
        int nc = (int)h->level_clusters[l].size();
        if (!nc) continue;
        if (nc < WIDE_LEVEL && h->max_rank > WIDE_MINR && h->max_rank <= WIDE_MAXR)
            hipLaunchKernelGGL(k_forward_wide<T>, dim3(nc), dim3(256), 0, s, h->d_level_clusters[l], h->d_node,
                               h->d_rank, h->d_piv_off, h->d_v_off, h->d_e_off, V, E, xp, xh);
        else
            hipLaunchKernelGGL(k_forward<T>, dim3(nc), dim3(64), 0, s, h->d_level_clusters[l], h->d_node,
                               h->d_rank, h->d_piv_off, h->d_v_off, h->d_e_off, V, E, xp, xh);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}
template hipError_t launch_forward<float>(gca_h2_s *, const float *, float *, hipStream_t);
template hipError_t launch_forward<double>(gca_h2_s *, const double *, double *, hipStream_t);

// yh_c = sum over the cluster's partial slots (fixed order)
template <typename T>
__global__ void k_coupling_reduce(const int32_t *rank, const int64_t *piv_off, const int64_t *slot_ptr,
                                  const int64_t *slots, const T *part, T *yh)
{
    const int c = blockIdx.x;
    const int r = rank[c];
    const int64_t b = slot_ptr[c], e = slot_ptr[c + 1];
    for (int k = threadIdx.x; k < r; k += blockDim.x) yh[piv_off[c] + k] = slot_sum(part, slots, b, e, 1, k);
}

template <typename T>
hipError_t launch_coupling_reduce(gca_h2_s *h, const int64_t *slot_ptr, const int64_t *slots, const T *cpart,
                                  T *yh, hipStream_t s)
{
    hipLaunchKernelGGL(k_coupling_reduce<T>, dim3((unsigned)h->nc), dim3(128), 0, s, h->d_rank, h->d_piv_off,
                       slot_ptr, slots, cpart, yh);
    return hipGetLastError();
}
template hipError_t launch_coupling_reduce<float>(gca_h2_s *, const int64_t *, const int64_t *, const float *,
                                                  float *, hipStream_t);
template hipError_t launch_coupling_reduce<double>(gca_h2_s *, const int64_t *, const int64_t *, const double *,
                                                   double *, hipStream_t);

// backward transform for the clusters of one level below the root:
// yh_c += E_c yh_parent (E_c column-major: Et[k * r_c + j]); one wavefront
// per cluster, lane per basis column j (with r_c <= 32 the two
// half-wavefronts split the parent's rows and add across lane ^ 32)
template <typename T>
__global__ void __launch_bounds__(64) k_backward(const int32_t *clusters, const int32_t *node, const int32_t *rank,
                                                 const int64_t *piv_off, const int64_t *e_off, const T *Et, T *yh)
{
    const int c = clusters[blockIdx.x];
    const int par = node[5 * c + 4];
    const int rc = rank[c], rp = rank[par];
    const T *Ec = Et + e_off[c];
    const T *yp = yh + piv_off[par];
    T *yc = yh + piv_off[c];
    const int lane = threadIdx.x;
    if (rc <= 32) {
        const int j = lane & 31, h = lane >> 5, m = (rp + 1) >> 1;
        T acc = 0;
        if (j < rc) acc = col_dot_range(Ec, rc, h ? m : 0, h ? rp : m, yp, j);
        acc += __shfl_xor(acc, 32, 64);
        if (h == 0 && j < rc) yc[j] += acc;
        return;
    }
    for (int j = lane; j < rc; j += 64) yc[j] += col_dot(Ec, rc, rp, yp, j);
}

template <typename T>
hipError_t launch_backward(gca_h2_s *h, T *yh, hipStream_t s)
{
    const T *Et = std::is_same<T, float>::value ? (const T *)h->d_Etf : (const T *)h->d_Et;
    for (int l = 1; l < (int)h->level_clusters.size(); ++l) {
        int nc = (int)h->level_clusters[l].size();
        if (!nc) continue;
        if (nc < WIDE_LEVEL && h->max_rank > WIDE_MINR && h->max_rank <= WIDE_MAXR)
            hipLaunchKernelGGL(k_backward_wide<T>, dim3(nc), dim3(256), 0, s, h->d_level_clusters[l], h->d_node,
                               h->d_rank, h->d_piv_off, h->d_e_off, Et, yh);
        else
            hipLaunchKernelGGL(k_backward<T>, dim3(nc), dim3(64), 0, s, h->d_level_clusters[l], h->d_node,
                               h->d_rank, h->d_piv_off, h->d_e_off, Et, yh);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}
template hipError_t launch_backward<float>(gca_h2_s *, float *, hipStream_t);
template hipError_t launch_backward<double>(gca_h2_s *, double *, hipStream_t);

// Per leaf, thread per row: y|t^ = V_t yh_t + near partials + pair lists;
// written back in the original triangle order.  The touching values (FP64)
// are stored per leaf in ELL form (partner k of row i at k * nr + i, so the
// rows of a leaf read consecutive addresses), the near-regular values (T) in
// a row CSR aligned with their column indices.
// Leaves are taken in XCD-contiguous order, so the neighbouring positions a
// leaf's touching pairs read stay in one XCD's L2.

template <typename T, typename Tout>
__global__ void __launch_bounds__(64) k_gather(const int32_t *leaves, const int32_t *node, const int32_t *rank,
                                               const int64_t *piv_off, const int64_t *v_off, const T *Vt,
                                               const T *yh, const int64_t *nslot_ptr, const int64_t *nslot,
                                               const T *npart, const int64_t *tell_off, const int32_t *tell_k,
                                               const int32_t *tother, const double *tval, const int64_t *nptr,
                                               const int32_t *nother,
                                               const T *nval, const T *xp, const double *xp64,
                                               const int32_t *perm, Tout *y)
{
    const int li = xcd_contiguous(blockIdx.x, gridDim.x);
    const int c = leaves[li];
    const int b = node[5 * c], nr = node[5 * c + 1] - b;
    const int r = rank[c];
    const T *Vc = Vt + v_off[c];
    const T *yc = yh + piv_off[c];
    for (int i = threadIdx.x; i < nr; i += blockDim.x) {
        T acc = col_dot(Vc, nr, r, yc, i) + slot_sum(npart, nslot, nslot_ptr[li], nslot_ptr[li + 1], 1, i);
        const int pos = b + i;
        for (int64_t q = nptr[pos]; q < nptr[pos + 1]; ++q) acc += nval[q] * xp[nother[q]];
        const double acc64 = ell_sum(tval, tother, xp64, tell_off[li] + i, nr, tell_k[li], 1, 0);
        y[perm[pos]] = (Tout)((double)acc + acc64);
    }
}

// thread per position: its k-th touching partner (or itself as padding) at
// ELL entry tell_off[li] + k nr + i, and the CSR -> ELL map of its entries
__global__ void k_touching_ell(int64_t n, const int32_t *pos_li, const int32_t *leaves, const int32_t *node,
                               const int64_t *tell_off, const int32_t *tell_k, const int64_t *tptr,
                               const int32_t *tother, int32_t *ell_other, int32_t *qmap)
{
    const int64_t pos = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (pos >= n) return;
    const int li = pos_li[pos];
    const int c = leaves[li];
    const int b = node[5 * c], nr = node[5 * c + 1] - b;
    const int64_t q0 = tptr[pos], cnt = tptr[pos + 1] - q0;
    const int64_t base = tell_off[li] + (pos - b);
    for (int k = 0; k < tell_k[li]; ++k) {
        const int64_t e = base + (int64_t)k * nr;
        if (k < cnt) {
            ell_other[e] = tother[q0 + k];
            qmap[q0 + k] = (int32_t)e;
        } else {
            ell_other[e] = (int32_t)pos;
        }
    }
}

// thread per touching pair: the ELL slots of its two rows (-1: identical pair)
__global__ void k_touching_slots(int64_t np, const int32_t *slot_a, const int32_t *slot_b, const int32_t *qmap,
                                 int32_t *tslot_a, int32_t *tslot_b)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    tslot_a[p] = qmap[slot_a[p]];
    tslot_b[p] = slot_b[p] >= 0 ? qmap[slot_b[p]] : -1;
}

hipError_t launch_touching_ell(gca_h2_s *h, const int32_t *pos_li, int32_t *qmap, int64_t ntouch, hipStream_t s)
{
    if (h->n > 0)
        hipLaunchKernelGGL(k_touching_ell, dim3((unsigned)((h->n + 255) / 256)), dim3(256), 0, s, h->n, pos_li,
                           h->d_leaves, h->d_node, h->d_tell_off, h->d_tell_k, h->d_tptr, h->d_tother,
                           h->d_tell_other, qmap);
    if (ntouch > 0)
        hipLaunchKernelGGL(k_touching_slots, dim3((unsigned)((ntouch + 255) / 256)), dim3(256), 0, s, ntouch,
                           h->d_slot_a, h->d_slot_b, qmap, h->d_tslot_a, h->d_tslot_b);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_gather(gca_h2_s *h, const T *xp, const double *xp64, const T *yh, const T *npart,
                         const T *nval, void *y, bool yf32, hipStream_t s)
{
    const T *Vt = std::is_same<T, float>::value ? (const T *)h->d_Vtf : (const T *)h->d_Vt;
    const dim3 grid((unsigned)h->leaves.size()), blk(64);
#define GATHER(TO)                                                                                               \
    hipLaunchKernelGGL((k_gather<T, TO>), grid, blk, 0, s, h->d_leaves, h->d_node, h->d_rank, h->d_piv_off,      \
                       h->d_v_off, Vt, yh, h->d_gnslot_ptr, h->d_gnslot, npart, h->d_tell_off, h->d_tell_k,       \
                       h->d_tell_other, h->d_tval, h->d_nptr, h->d_nother, nval, xp, xp64, h->d_perm, (TO *)y)
    if (yf32)
        GATHER(float);
    else
        GATHER(double);
#undef GATHER
    return hipGetLastError();
}
template hipError_t launch_gather<float>(gca_h2_s *, const float *, const double *, const float *, const float *,
                                         const float *, void *, bool, hipStream_t);
template hipError_t launch_gather<double>(gca_h2_s *, const double *, const double *, const double *,
                                          const double *, const double *, void *, bool, hipStream_t);

}  // namespace gca
