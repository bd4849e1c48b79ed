// Frozen-structure basis kernels (gca_update_geometry, h2_bilinear_grad).
//
// With the cluster tree, the block partition, the boxes omega, the Green
// points and the pivot rows I and columns J of every cluster held fixed, the
// interpolation matrix of a cluster is the smooth function of the vertex
// coordinates
//     V^ = A^[:, J] C^{-1},   C = A^[I, J]
// (Section 3's V_tau A|tau~ = A on the pivot rows; Section 4's A^ for parents),
// where A^ holds the Green factor of Section 2 at the cluster's rows (leaf:
// its triangles; parent: its sons' pivots).  These kernels evaluate A^ at the
// pivot columns, factor C per cluster (one workgroup, partial pivoting, FP64),
// and solve for V^ (refresh) or for the adjoint  Z = V^bar C^{-T}.
#include <hip/hip_runtime.h>

#include "gca_internal.h"
#include "devfn.h"
#include "mfma.h"

namespace gca {

#define INV4PI_A 0.07957747154594766788

struct GLRuleA {
    double x[32], w[32];
};

// Green point nu of cluster c (same construction as the factor kernel).
__device__ inline void green_point(const double *bx, int m, int nu, const GLRuleA &g, double eta, double omega_scale,
                                   double z[3], double n[3], double &w, double &diam)
{
    diam = bx[6];
    const double delta = omega_scale * diam / eta;
    double L[3], H[3];
    for (int d = 0; d < 3; ++d) {
        L[d] = bx[d] - delta;
        H[d] = bx[3 + d] + delta;
    }
    const int f = nu / (m * m), ij = nu - f * m * m, i = ij / m, j = ij - i * m;
    const int ax = f >> 1;
    const int b1 = ax == 0 ? 1 : 0, b2 = ax == 2 ? 1 : 2;
    n[0] = n[1] = n[2] = 0;
    z[ax] = (f & 1) ? H[ax] : L[ax];
    z[b1] = L[b1] + g.x[i] * (H[b1] - L[b1]);
    z[b2] = L[b2] + g.x[j] * (H[b2] - L[b2]);
    n[ax] = (f & 1) ? 1.0 : -1.0;
    w = g.w[i] * g.w[j] * (H[b1] - L[b1]) * (H[b2] - L[b2]);
}

struct ClusterArgs {
    const int32_t *clusters;   // batch -> cluster id
    const double *box;         // nc x 8
    const int32_t *rank;
    const int64_t *piv_off;    // per cluster, into pivrow / pivcol
    const int32_t *pivrow, *pivcol;
    const int64_t *arow_off;   // per cluster, into arows
    const int32_t *arows;      // positions
    const int64_t *aj_off;     // per batch entry: offset of m x r blocks
    const int64_t *c_off;      // per batch entry: offset of r x r blocks
    int m_green;
    double eta, omega_scale;
};

// A^[:, J] for every cluster of the batch (workgroup per cluster).
template <int PA>
__global__ void __launch_bounds__(256) k_eval_AJ(ClusterArgs ca, const double *qA, GLRuleA g, double *AJ)
{
    const int b = blockIdx.x;
    const int c = ca.clusters[b];
    const int r = ca.rank[c];
    const int64_t ro = ca.arow_off[c];
    const int m = (int)(ca.arow_off[c + 1] - ro);
    const int k = 6 * ca.m_green * ca.m_green;
    const double *bx = ca.box + 8 * (size_t)c;
    double *out = AJ + ca.aj_off[b];
    for (int e = threadIdx.x; e < m * r; e += blockDim.x) {
        const int i = e / r, l = e - i * r;
        const int col = ca.pivcol[ca.piv_off[c] + l];
        const int nu = col < k ? col : col - k;
        double z[3], n[3], w, diam;
        green_point(bx, ca.m_green, nu, g, ca.eta, ca.omega_scale, z, n, w, diam);
        const double *pts = qA + (size_t)ca.arows[ro + i] * PA * 4;
        double sg = 0, sd = 0;
#pragma unroll
        for (int p = 0; p < PA; ++p) {
            double dx = pts[4 * p] - z[0], dy = pts[4 * p + 1] - z[1], dz = pts[4 * p + 2] - z[2];
            double ri = rsqrt(dx * dx + dy * dy + dz * dz);
            double wq = pts[4 * p + 3];
            sg += wq * ri;
            sd += wq * (n[0] * dx + n[1] * dy + n[2] * dz) * ri * ri * ri;
        }
        const double sw = sqrt(w);
        out[(int64_t)i * r + l] = col < k ? sw * sg * INV4PI_A : -diam * sw * sd * INV4PI_A;
    }
}

// LU with partial pivoting of C = A^[I, :] (r x r) per cluster, in place in
// LU + c_off[b]; perm[c_off-base + k] = original row of pivot k.
__global__ void __launch_bounds__(256) k_lu(ClusterArgs ca, const double *AJ, double *LU, int32_t *perm,
                                            const int64_t *perm_off)
{
    __shared__ double sv[256];
    __shared__ int si[256];
    __shared__ int prow;
    const int b = blockIdx.x, tid = threadIdx.x;
    const int c = ca.clusters[b];
    const int r = ca.rank[c];
    double *A = LU + ca.c_off[b];
    int32_t *pm = perm + perm_off[b];
    const double *src = AJ + ca.aj_off[b];
    const int32_t *I = ca.pivrow + ca.piv_off[c];
    for (int e = tid; e < r * r; e += blockDim.x) {
        const int i = e / r, j = e - i * r;
        A[e] = src[(int64_t)I[i] * r + j];
    }
    for (int i = tid; i < r; i += blockDim.x) pm[i] = i;
    __syncthreads();
    for (int kk = 0; kk < r; ++kk) {
        // pivot search in column kk (largest magnitude, smallest row on ties)
        double best = -1.0;
        int bi = kk;
        for (int i = kk + tid; i < r; i += blockDim.x) {
            double v = fabs(A[(int64_t)i * r + kk]);
            if (v > best) {
                best = v;
                bi = i;
            }
        }
        sv[tid] = best;
        si[tid] = bi;
        __syncthreads();
        if (tid == 0) {
            double bv = -1.0;
            int bb = kk;
            for (int t = 0; t < (int)blockDim.x; ++t)
                if (sv[t] > bv || (sv[t] == bv && si[t] < bb)) {
                    bv = sv[t];
                    bb = si[t];
                }
            prow = bb;
        }
        __syncthreads();
        const int pr = prow;
        if (pr != kk) {
            for (int j = tid; j < r; j += blockDim.x) {
                double t = A[(int64_t)kk * r + j];
                A[(int64_t)kk * r + j] = A[(int64_t)pr * r + j];
                A[(int64_t)pr * r + j] = t;
            }
            if (tid == 0) {
                int t = pm[kk];
                pm[kk] = pm[pr];
                pm[pr] = t;
            }
        }
        __syncthreads();
        const double piv = A[(int64_t)kk * r + kk];
        for (int i = kk + 1 + tid; i < r; i += blockDim.x) A[(int64_t)i * r + kk] /= piv;
        __syncthreads();
        const int rem = r - kk - 1;
        for (int e = tid; e < rem * rem; e += blockDim.x) {
            const int i = kk + 1 + e / rem, j = kk + 1 + e % rem;
            A[(int64_t)i * r + j] -= A[(int64_t)i * r + kk] * A[(int64_t)kk * r + j];
        }
        __syncthreads();
    }
}

// Row solves v C = a with P C = L U (P: perm, L unit lower, U upper, both in
// LU): the rows of V^ from those of A^[:, J], and the rows of C^{-1} from
// those of the identity.  Rows of `in` and `out`: m x r row-major at
// aj_off[b]; `tmp` the same size.
__global__ void __launch_bounds__(256) k_row_solve(ClusterArgs ca, const double *LU, const int32_t *perm,
                                                   const int64_t *perm_off, const double *in, double *out,
                                                   double *tmp)
{
    const int b = blockIdx.x;
    const int c = ca.clusters[b];
    const int r = ca.rank[c];
    const int m = (int)(ca.arow_off[c + 1] - ca.arow_off[c]);
    const double *A = LU + ca.c_off[b];
    const int32_t *pm = perm + perm_off[b];
    for (int i = threadIdx.x; i < m; i += blockDim.x) {
        const double *a = in + ca.aj_off[b] + (int64_t)i * r;
        double *t = tmp + ca.aj_off[b] + (int64_t)i * r;
        double *v = out + ca.aj_off[b] + (int64_t)i * r;
        // v P^T L U = a: t U = a (forward over columns), w L = t (backward), v = w P
        for (int j = 0; j < r; ++j) {
            double s = a[j];
            for (int q = 0; q < j; ++q) s -= t[q] * A[(int64_t)q * r + j];
            t[j] = s / A[(int64_t)j * r + j];
        }
        for (int j = r - 1; j >= 0; --j) {
            double s = t[j];
            for (int q = j + 1; q < r; ++q) s -= t[q] * A[(int64_t)q * r + j];
            t[j] = s;   // w_j (unit diagonal of L)
        }
        for (int j = 0; j < r; ++j) v[pm[j]] = t[j];
    }
}

// The same factorisation and row solves with C staged in LDS, for ranks up
// to FZ_MAXR: k_lu_lds factors in LDS (one workgroup per cluster); in
// k_row_solve_lds eight threads share a row and hold its entries q = t + 8 s
// in registers, the sums over q are split over the eight and combined by
// shuffles.  Same operations as k_lu / k_row_solve, different summation order.
constexpr int FZ_MAXR = 64;

__global__ void __launch_bounds__(256) k_lu_lds(ClusterArgs ca, const double *AJ, double *LU, int32_t *perm,
                                                const int64_t *perm_off)
{
    __shared__ double A[FZ_MAXR * FZ_MAXR];
    __shared__ double sv[256];
    __shared__ int si[256];
    __shared__ int pmv[FZ_MAXR];
    const int b = blockIdx.x, tid = threadIdx.x;
    const int c = ca.clusters[b];
    const int r = ca.rank[c];
    const double *src = AJ + ca.aj_off[b];
    const int32_t *I = ca.pivrow + ca.piv_off[c];
    for (int e = tid; e < r * r; e += blockDim.x) {
        const int i = e / r, j = e - i * r;
        A[e] = src[(int64_t)I[i] * r + j];
    }
    for (int i = tid; i < r; i += blockDim.x) pmv[i] = i;
    __syncthreads();
    for (int kk = 0; kk < r; ++kk) {
        double best = -1.0;
        int bi = kk;
        for (int i = kk + tid; i < r; i += blockDim.x) {
            const double v = fabs(A[i * r + kk]);
            if (v > best) {
                best = v;
                bi = i;
            }
        }
        // wavefront argmax (ties: smallest row), then across the 4 wavefronts
        for (int off = 32; off > 0; off >>= 1) {
            const double ov = __shfl_xor(best, off, 64);
            const int oi = __shfl_xor(bi, off, 64);
            if (ov > best || (ov == best && oi < bi)) {
                best = ov;
                bi = oi;
            }
        }
        if ((tid & 63) == 0) {
            sv[tid >> 6] = best;
            si[tid >> 6] = bi;
        }
        __syncthreads();
        double bv = -1.0;
        int pr = kk;
        for (int w = 0; w < (int)blockDim.x / 64; ++w)
            if (sv[w] > bv || (sv[w] == bv && si[w] < pr)) {
                bv = sv[w];
                pr = si[w];
            }
        if (pr != kk) {
            for (int j = tid; j < r; j += blockDim.x) {
                const double t = A[kk * r + j];
                A[kk * r + j] = A[pr * r + j];
                A[pr * r + j] = t;
            }
            if (tid == 0) {
                const int t = pmv[kk];
                pmv[kk] = pmv[pr];
                pmv[pr] = t;
            }
        }
        __syncthreads();
        const double piv = A[kk * r + kk];
        for (int i = kk + 1 + tid; i < r; i += blockDim.x) A[i * r + kk] /= piv;
        __syncthreads();
        const int rem = r - kk - 1;
        for (int e = tid; e < rem * rem; e += blockDim.x) {
            const int i = kk + 1 + e / rem, j = kk + 1 + e % rem;
            A[i * r + j] -= A[i * r + kk] * A[kk * r + j];
        }
        __syncthreads();
    }
    double *out = LU + ca.c_off[b];
    for (int e = tid; e < r * r; e += blockDim.x) out[e] = A[e];
    int32_t *pm = perm + perm_off[b];
    for (int i = tid; i < r; i += blockDim.x) pm[i] = pmv[i];
}

__global__ void __launch_bounds__(256) k_row_solve_lds(ClusterArgs ca, const double *LU, const int32_t *perm,
                                                       const int64_t *perm_off, const double *in, double *out)
{
    constexpr int NS = FZ_MAXR / 8;
    __shared__ double A[FZ_MAXR * FZ_MAXR];
    __shared__ int pmv[FZ_MAXR];
    const int b = blockIdx.x, tid = threadIdx.x;
    const int c = ca.clusters[b];
    const int r = ca.rank[c];
    const int m = (int)(ca.arow_off[c + 1] - ca.arow_off[c]);
    const double *LUb = LU + ca.c_off[b];
    for (int e = tid; e < r * r; e += blockDim.x) A[e] = LUb[e];
    for (int i = tid; i < r; i += blockDim.x) pmv[i] = perm[perm_off[b] + i];
    __syncthreads();
    const int t8 = tid & 7;
    for (int i = tid >> 3; i < m; i += blockDim.x / 8) {
        const double *a = in + ca.aj_off[b] + (int64_t)i * r;
        double *v = out + ca.aj_off[b] + (int64_t)i * r;
        double t[NS], av[NS];
        // the right-hand side entries this thread consumes, fetched up front
#pragma unroll
        for (int sl = 0; sl < NS; ++sl) {
            const int q = t8 + 8 * sl;
            av[sl] = q < r ? a[q] : 0.0;
        }
        // v P^T L U = a: t U = a (forward over columns), w L = t (backward), v = w P
#pragma unroll
        for (int sl = 0; sl < NS; ++sl) t[sl] = 0.0;
        for (int j = 0; j < r; ++j) {
            double acc = 0.0;
#pragma unroll
            for (int sl = 0; sl < NS; ++sl) {
                const int q = t8 + 8 * sl;
                if (q < j) acc += t[sl] * A[q * r + j];
            }
            acc = group_sum<8>(acc);   // the row's eight lanes, DPP
            if (t8 == (j & 7)) {
#pragma unroll
                for (int sl = 0; sl < NS; ++sl)
                    if (sl == (j >> 3)) t[sl] = (av[sl] - acc) / A[j * r + j];
            }
        }
        for (int j = r - 1; j >= 0; --j) {
            double acc = 0.0;
#pragma unroll
            for (int sl = 0; sl < NS; ++sl) {
                const int q = t8 + 8 * sl;
                if (q > j && q < r) acc += t[sl] * A[q * r + j];
            }
            acc = group_sum<8>(acc);   // the row's eight lanes, DPP
            if (t8 == (j & 7)) {
#pragma unroll
                for (int sl = 0; sl < NS; ++sl)
                    if (sl == (j >> 3)) t[sl] -= acc;
            }
        }
#pragma unroll
        for (int sl = 0; sl < NS; ++sl) {
            const int q = t8 + 8 * sl;
            if (q < r) v[pmv[q]] = t[sl];
        }
    }
}

// identity r x r blocks at aj_off[b] (the right-hand sides of C^{-1})
__global__ void k_eye(ClusterArgs ca, double *out)
{
    const int b = blockIdx.x;
    const int r = ca.rank[ca.clusters[b]];
    double *o = out + ca.aj_off[b];
    for (int e = threadIdx.x; e < r * r; e += blockDim.x) o[e] = (e / r == e % r) ? 1.0 : 0.0;
}

// Z = Vbar C^{-T} per cluster (row i of Z solves C z = Vbar[i, :]^T) as a
// product with the stored C^{-1}: 16 x 16 tiles over (row of Vbar, column of
// Z) on the matrix cores (v_mfma_f64_16x16x4, mfma.h), the sum over the r
// columns of Vbar in steps of four; the four wavefronts take every fourth
// tile.
__global__ void __launch_bounds__(256) k_cinv_apply(ClusterArgs ca, const double *Cinv, const double *Vbar,
                                                    double *Z)
{
    const int b = blockIdx.x;
    const int c = ca.clusters[b];
    const int r = ca.rank[c];
    const int m = (int)(ca.arow_off[c + 1] - ca.arow_off[c]);
    const double *Ci = Cinv + ca.c_off[b];
    const double *Vb = Vbar + ca.aj_off[b];
    double *Zb = Z + ca.aj_off[b];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63, q = lane & 15, kq = lane >> 4;
    const int ntc = (r + 15) >> 4, nt = ((m + 15) >> 4) * ntc;
    for (int tile = wv; tile < nt; tile += 4) {
        const int i0 = (tile / ntc) * 16, l0 = (tile % ntc) * 16;
        const int i = i0 + q, l = l0 + q;
        Mfma<double>::acc_t acc = mfma_zero<double>();
        for (int k0 = 0; k0 < r; k0 += 16) {
            // the operands of four steps loaded before their products
            double a[4], bb[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int k = k0 + 4 * u + kq;
                a[u] = (i < m && k < r) ? Vb[(int64_t)i * r + k] : 0.0;
                bb[u] = (l < r && k < r) ? Ci[(int64_t)l * r + k] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) acc = Mfma<double>::mma(a[u], bb[u], acc);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int ii = i0 + Mfma<double>::row(lane, v);
            if (ii < m && l < r) Zb[(int64_t)ii * r + l] = acc[v];
        }
    }
}

// rows I of V^ are the unit vectors (interpolation property)
__global__ void k_unit_rows(ClusterArgs ca, double *V)
{
    const int b = blockIdx.x;
    const int c = ca.clusters[b];
    const int r = ca.rank[c];
    const int32_t *I = ca.pivrow + ca.piv_off[c];
    double *Vb = V + ca.aj_off[b];
    for (int e = threadIdx.x; e < r * r; e += blockDim.x) {
        const int k = e / r, j = e - k * r;
        Vb[(int64_t)I[k] * r + j] = (j == k) ? 1.0 : 0.0;
    }
}

static GLRuleA make_rule(const double *x, const double *w, int m)
{
    GLRuleA g{};
    for (int i = 0; i < m; ++i) {
        g.x[i] = x[i];
        g.w[i] = w[i];
    }
    return g;
}

static ClusterArgs cluster_args(gca_h2_s *h)
{
    ClusterArgs ca{};
    ca.clusters = h->fz.d_batch;
    ca.box = h->d_box;
    ca.rank = h->d_rank;
    ca.piv_off = h->d_piv_off;
    ca.pivrow = h->fz.d_pivrow;
    ca.pivcol = h->fz.d_pivcol;
    ca.arow_off = h->fz.d_arow_off;
    ca.arows = h->fz.d_arows;
    ca.aj_off = h->fz.d_aj_off;
    ca.c_off = h->fz.d_c_off;
    ca.m_green = h->prm.green_m;
    ca.eta = h->prm.eta;
    ca.omega_scale = h->prm.omega_scale;
    return ca;
}

// A^[:, J], LU of A^[I, J] and V^ = A^[:, J] A^[I, J]^{-1} for every cluster,
// with the current triangle quadrature points.
hipError_t launch_frozen_basis(gca_h2_s *h, hipStream_t s)
{
    const int nc = (int)h->nc;
    ClusterArgs ca = cluster_args(h);
    GLRuleA g = make_rule(h->gl_x, h->gl_w, h->prm.green_m);
    const int PA = h->prm.q_A * h->prm.q_A;
    switch (PA) {
#define CASE(PP)                                                                                  \
    case PP:                                                                                      \
        hipLaunchKernelGGL((k_eval_AJ<PP>), dim3(nc), dim3(256), 0, s, ca, h->d_qA, g, h->fz.d_AJ); \
        break;
        CASE(1) CASE(4) CASE(9) CASE(16) CASE(25) CASE(36)
#undef CASE
    default:
        return hipErrorInvalidValue;
    }
    // C^{-1} from the identity's rows (Z serves as their buffer: r x r
    // blocks at c_off, as many rows as the rank)
    ClusterArgs ci = ca;
    ci.arow_off = h->fz.d_roff;
    ci.aj_off = h->fz.d_c_off;
    hipLaunchKernelGGL(k_eye, dim3(nc), dim3(256), 0, s, ci, h->fz.d_Z);
    if (h->max_rank <= FZ_MAXR) {
        hipLaunchKernelGGL(k_lu_lds, dim3(nc), dim3(256), 0, s, ca, h->fz.d_AJ, h->fz.d_LU, h->fz.d_perm,
                           h->d_piv_off);
        hipLaunchKernelGGL(k_row_solve_lds, dim3(nc), dim3(256), 0, s, ca, h->fz.d_LU, h->fz.d_perm, h->d_piv_off,
                           h->fz.d_AJ, h->fz.d_Vh);
        hipLaunchKernelGGL(k_row_solve_lds, dim3(nc), dim3(256), 0, s, ci, h->fz.d_LU, h->fz.d_perm, h->d_piv_off,
                           h->fz.d_Z, h->fz.d_Cinv);
    } else {
        hipLaunchKernelGGL(k_lu, dim3(nc), dim3(256), 0, s, ca, h->fz.d_AJ, h->fz.d_LU, h->fz.d_perm, h->d_piv_off);
        hipLaunchKernelGGL(k_row_solve, dim3(nc), dim3(256), 0, s, ca, h->fz.d_LU, h->fz.d_perm, h->d_piv_off,
                           h->fz.d_AJ, h->fz.d_Vh, h->fz.d_tmp);
        hipLaunchKernelGGL(k_row_solve, dim3(nc), dim3(256), 0, s, ci, h->fz.d_LU, h->fz.d_perm, h->d_piv_off,
                           h->fz.d_Z, h->fz.d_Cinv, h->fz.d_tmp);
    }
    hipLaunchKernelGGL(k_unit_rows, dim3(nc), dim3(256), 0, s, ca, h->fz.d_Vh);
    return hipGetLastError();
}

// Z = Vbar C^{-T} per cluster (Vbar in fz.d_Vbar, result in fz.d_Z)
hipError_t launch_frozen_adjoint_solve(gca_h2_s *h, hipStream_t s)
{
    ClusterArgs ca = cluster_args(h);
    hipLaunchKernelGGL(k_cinv_apply, dim3((unsigned)h->nc), dim3(256), 0, s, ca, h->fz.d_Cinv, h->fz.d_Vbar,
                       h->fz.d_Z);
    return hipGetLastError();
}

}  // namespace gca
