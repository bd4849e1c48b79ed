// Construction of the nested cluster basis on gfx950 (Sections 2-4):
//   - per-triangle quadrature points of the collapsed Gauss rule;
//   - the Green factor A of Section 2 for the rows of one tree level
//       a_{i nu}    =  sqrt(w_nu) int g(x, z_nu) phi_i(x) dx
//       a_{i nu+k}  = -d_tau sqrt(w_nu) int dg/dn_z(x, z_nu) phi_i(x) dx,
//     with Green points z_nu: an m x m Gauss rule on each face of the box
//     omega = [lo - delta, hi + delta], delta = omega_scale * diam / eta,
//     outward normals;
//   - cross approximation with full pivoting in FP64 (Section 3), one
//     workgroup per cluster, producing the pivot rows tau~ and the
//     interpolation matrix V with V A|tau~ ~ A;
//   - copies of the results into the final leaf-basis / transfer layouts.
#include <hip/hip_runtime.h>

#include "gca_internal.h"
#include "devfn.h"

namespace gca {

#define INV4PI_D 0.07957747154594766788

struct GLRule {
    double x[32], w[32];
};

// ---------------------------------------------------------- triangle rule --
// point p of the rule: chi(s) = P0 + s1 (P1 - P0) + s2 (P2 - P1), weight
// w_p |(P1 - P0) x (P2 - P1)|; thread per (triangle, point).
__global__ void k_tri_points(const double *xyz, const int32_t *tv, int64_t n, TriRule r, double *out)
{
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int P = r.np;
    if (e >= n * P) return;
    int64_t t = e / P;
    int p = (int)(e - t * P);
    const int32_t *v = tv + 3 * t;
    double P0[3], P1[3], P2[3];
    for (int d = 0; d < 3; ++d) {
        P0[d] = xyz[3 * (size_t)v[0] + d];
        P1[d] = xyz[3 * (size_t)v[1] + d];
        P2[d] = xyz[3 * (size_t)v[2] + d];
    }
    double e1[3], e2[3];
    for (int d = 0; d < 3; ++d) {
        e1[d] = P1[d] - P0[d];
        e2[d] = P2[d] - P1[d];
    }
    double cx = e1[1] * e2[2] - e1[2] * e2[1], cy = e1[2] * e2[0] - e1[0] * e2[2], cz = e1[0] * e2[1] - e1[1] * e2[0];
    double J = sqrt(cx * cx + cy * cy + cz * cz);
    const double s1 = r.s1[p], s2 = r.s2[p];
    double *o = out + 4 * e;
    for (int d = 0; d < 3; ++d) o[d] = P0[d] + s1 * e1[d] + s2 * e2[d];
    o[3] = r.w[p] * J;
}

hipError_t launch_tri_points(const double *xyz, const int32_t *tv, int64_t n, const TriRule &rule, double *out,
                             hipStream_t s)
{
    if (rule.np < 1 || rule.np > 64) return hipErrorInvalidValue;
    int64_t tot = n * rule.np;
    dim3 grid((unsigned)((tot + 255) / 256)), blk(256);
    hipLaunchKernelGGL(k_tri_points, grid, blk, 0, s, xyz, tv, n, rule, out);
    return hipGetLastError();
}

// ------------------------------------------------------------ Green factor --
// thread per (row r, Green point nu); row r has triangle row_tri[r] (position)
// and cluster row_cl[r]; its 2k values go to A + row_out[r].
template <int PA>
__global__ void __launch_bounds__(256) k_green_A(const double *qA, const double *box, const int32_t *row_tri,
                                                 const int32_t *row_cl, const int64_t *row_out, int64_t nrows,
                                                 int m, GLRule g, double eta, double omega_scale, double *A)
{
    const int k = 6 * m * m;
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nrows * k) return;
    int64_t r = e / k;
    int nu = (int)(e - r * k);
    const int c = row_cl[r];
    const double *bx = box + 8 * (size_t)c;
    const double diam = bx[6];
    const double delta = omega_scale * diam / eta;
    double L[3], H[3];
    for (int d = 0; d < 3; ++d) {
        L[d] = bx[d] - delta;
        H[d] = bx[3 + d] + delta;
    }
    const int f = nu / (m * m), ij = nu - f * m * m, i = ij / m, j = ij - i * m;
    const int ax = f >> 1;
    const double side = (f & 1) ? 1.0 : -1.0;
    const int b1 = ax == 0 ? 1 : 0, b2 = ax == 2 ? 1 : 2;
    double z[3], n[3] = {0, 0, 0};
    z[ax] = (f & 1) ? H[ax] : L[ax];
    z[b1] = L[b1] + g.x[i] * (H[b1] - L[b1]);
    z[b2] = L[b2] + g.x[j] * (H[b2] - L[b2]);
    n[ax] = side;
    const double w = g.w[i] * g.w[j] * (H[b1] - L[b1]) * (H[b2] - L[b2]);
    const double *pts = qA + (size_t)row_tri[r] * PA * 4;
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
    double *out = A + row_out[r];
    out[nu] = sw * sg * INV4PI_D;
    out[nu + k] = -diam * sw * sd * INV4PI_D;
}

hipError_t launch_green_A(const double *qA, int PA, const double *box, const int32_t *row_tri,
                          const int32_t *row_cl, const int64_t *row_out, int64_t nrows, int m, const double *glx,
                          const double *glw, double eta, double omega_scale, double *A, hipStream_t s)
{
    if (nrows == 0) return hipSuccess;
    GLRule g{};
    for (int i = 0; i < m; ++i) {
        g.x[i] = glx[i];
        g.w[i] = glw[i];
    }
    int64_t tot = nrows * 6 * m * m;
    dim3 grid((unsigned)((tot + 255) / 256)), blk(256);
    switch (PA) {
#define CASE(PP)                                                                                     \
    case PP:                                                                                         \
        hipLaunchKernelGGL((k_green_A<PP>), grid, blk, 0, s, qA, box, row_tri, row_cl, row_out, nrows, m, \
                           g, eta, omega_scale, A);                                                  \
        break;
        CASE(1) CASE(4) CASE(9) CASE(16) CASE(25) CASE(36) CASE(64) CASE(100) CASE(144)
#undef CASE
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------- cross approx --
// Full pivoting on the explicit rows x cols matrix R (initially A, updated in
// place in global memory; the working set of one cluster stays in L2):
//   while ||R||_F > eps ||A||_F and r < min(rows, cols):
//     (p, q) = argmax |R_ij| (ties: smallest row-major index)
//     u = R[:, q], v = R[p, :] / R[p, q];  R <- R - u v^T (row p, column q set to 0)
// U collects u (rows x maxr, row-major); with L = U[I, :] (lower triangular
// in pivot order) the interpolation matrix is V = U L^{-1}; rows I of V are
// set to the unit vectors.
constexpr int ACA_THREADS = 256;
constexpr int ACA_MAXCOLS = 512;   // 2k = 12 m^2 <= 432 for green_m <= 6

struct ArgMax {
    double v;
    int64_t i;
};

__device__ __forceinline__ bool better(double v, int64_t i, double bv, int64_t bi)
{
    return v > bv || (v == bv && i < bi);
}

__device__ void block_reduce(double &s, double &mv, int64_t &mi, double *sh_s, double *sh_v, int64_t *sh_i)
{
    const int tid = threadIdx.x;
    // wavefront reduction
    for (int off = 32; off > 0; off >>= 1) {
        double os = __shfl_xor(s, off, 64);
        double ov = __shfl_xor(mv, off, 64);
        int64_t oi = __shfl_xor(mi, off, 64);
        s += os;
        if (better(ov, oi, mv, mi)) {
            mv = ov;
            mi = oi;
        }
    }
    const int w = tid >> 6, l = tid & 63;
    if (l == 0) {
        sh_s[w] = s;
        sh_v[w] = mv;
        sh_i[w] = mi;
    }
    __syncthreads();
    if (tid == 0) {
        double ts = 0, tv = -1.0;
        int64_t ti = INT64_MAX;
        for (int k = 0; k < ACA_THREADS / 64; ++k) {
            ts += sh_s[k];
            if (better(sh_v[k], sh_i[k], tv, ti)) {
                tv = sh_v[k];
                ti = sh_i[k];
            }
        }
        sh_s[0] = ts;
        sh_v[0] = tv;
        sh_i[0] = ti;
    }
    __syncthreads();
    s = sh_s[0];
    mv = sh_v[0];
    mi = sh_i[0];
    __syncthreads();
}

__global__ void __launch_bounds__(ACA_THREADS) k_aca(double *Rall, double *Uall, double *Vall, const int64_t *a_off,
                                                     const int64_t *u_off, const int32_t *rows_arr, int cols,
                                                     double eps, int maxr_cap, int32_t *rank_out, int32_t *piv_out,
                                                     int32_t *pivc_out)
{
    __shared__ double sh_s[ACA_THREADS / 64], sh_v[ACA_THREADS / 64];
    __shared__ int64_t sh_i[ACA_THREADS / 64];
    __shared__ double vrow[ACA_MAXCOLS];
    __shared__ int32_t pivr[ACA_MAXCOLS], pivc[ACA_MAXCOLS];
    const int c = blockIdx.x, tid = threadIdx.x;
    const int rows = rows_arr[c];
    const int rmax = min(rows, cols);
    double *R = Rall + a_off[c];
    double *U = Uall + u_off[c];     // rows x rmax, row-major
    double *V = Vall + u_off[c];     // rows x rmax (stride rmax)
    const int64_t tot = (int64_t)rows * cols;

    double s = 0, mv = -1.0;
    int64_t mi = INT64_MAX;
    for (int64_t e = tid; e < tot; e += ACA_THREADS) {
        double a = R[e];
        s += a * a;
        if (better(fabs(a), e, mv, mi)) {
            mv = fabs(a);
            mi = e;
        }
    }
    block_reduce(s, mv, mi, sh_s, sh_v, sh_i);
    const double nA2 = s;
    const double tol2 = eps * eps * nA2;
    double nR2 = s;
    int r = 0;
    while (r < rmax && r < maxr_cap && nR2 > tol2) {
        const int64_t e = mi;
        const int p = (int)(e / cols), q = (int)(e - (int64_t)p * cols);
        const double piv = R[e];
        if (piv == 0.0) break;
        // u = R[:, q] -> U[:, r];  v = R[p, :] / piv
        for (int i = tid; i < rows; i += ACA_THREADS) U[(int64_t)i * rmax + r] = R[(int64_t)i * cols + q];
        for (int j = tid; j < cols; j += ACA_THREADS) vrow[j] = R[(int64_t)p * cols + j] / piv;
        if (tid == 0) {
            pivr[r] = p;
            pivc[r] = q;
        }
        __syncthreads();
        s = 0;
        mv = -1.0;
        mi = INT64_MAX;
        for (int64_t e2 = tid; e2 < tot; e2 += ACA_THREADS) {
            const int i = (int)(e2 / cols), j = (int)(e2 - (int64_t)i * cols);
            double v;
            if (i == p || j == q) {
                v = 0.0;
            } else {
                v = R[e2] - U[(int64_t)i * rmax + r] * vrow[j];
            }
            R[e2] = v;
            s += v * v;
            if (better(fabs(v), e2, mv, mi)) {
                mv = fabs(v);
                mi = e2;
            }
        }
        block_reduce(s, mv, mi, sh_s, sh_v, sh_i);
        nR2 = s;
        ++r;
    }
    if (tid == 0) rank_out[c] = r;
    for (int k = tid; k < r; k += ACA_THREADS) {
        piv_out[(int64_t)c * maxr_cap + k] = pivr[k];
        pivc_out[(int64_t)c * maxr_cap + k] = pivc[k];
    }
    __syncthreads();
    // V = U L^{-1}, L[j][k] = U[piv_j][k] (lower triangular): back substitution per row
    for (int i = tid; i < rows; i += ACA_THREADS) {
        double *vi = V + (int64_t)i * rmax;
        const double *ui = U + (int64_t)i * rmax;
        for (int k = r - 1; k >= 0; --k) {
            double acc = ui[k];
            for (int j = k + 1; j < r; ++j) acc -= vi[j] * U[(int64_t)pivr[j] * rmax + k];
            vi[k] = acc / U[(int64_t)pivr[k] * rmax + k];
        }
    }
    __syncthreads();
    // interpolation property: rows tau~ of V are exactly the unit vectors
    for (int k = tid; k < r; k += ACA_THREADS) {
        double *vi = V + (int64_t)pivr[k] * rmax;
        for (int j = 0; j < r; ++j) vi[j] = (j == k) ? 1.0 : 0.0;
    }
}

// The same cross approximation with the residual held in registers: the
// threads form TR = ACA_RT / cols row groups of cols threads; thread (g, j)
// owns column j of rows g + k TR (k < K).  Each step writes the pivot row and
// column to LDS, then updates the owned entries; the arithmetic (and so the
// pivots) equals k_aca's.
constexpr int ACA_RT = 1024;
constexpr int ACA_RMAXROWS = 1024;   // row groups x K (rows beyond the matrix are zero)
constexpr int ACA_BS_MAXR = 64;      // largest rank of the parallel back substitution

__device__ __forceinline__ bool better32(double v, int i, double bv, int bi)
{
    return v > bv || (v == bv && i < bi);
}

__device__ void block_reduce_rt(double &s, double &mv, int &mi, double *sh_s, double *sh_v, int *sh_i)
{
    const int tid = threadIdx.x;
    for (int off = 32; off > 0; off >>= 1) {
        double os = __shfl_xor(s, off, 64);
        double ov = __shfl_xor(mv, off, 64);
        int oi = __shfl_xor(mi, off, 64);
        s += os;
        if (better32(ov, oi, mv, mi)) {
            mv = ov;
            mi = oi;
        }
    }
    const int w = tid >> 6, l = tid & 63;
    if (l == 0) {
        sh_s[w] = s;
        sh_v[w] = mv;
        sh_i[w] = mi;
    }
    __syncthreads();
    double ts = 0, tv = -1.0;
    int ti = INT32_MAX;
    for (int k = 0; k < ACA_RT / 64; ++k) {
        ts += sh_s[k];
        if (better32(sh_v[k], sh_i[k], tv, ti)) {
            tv = sh_v[k];
            ti = sh_i[k];
        }
    }
    s = ts;
    mv = tv;
    mi = ti;
    // no trailing barrier: the partials are rewritten only after the next
    // barrier of the caller (the pivot row/column barrier)
}

template <int K>
__global__ void __launch_bounds__(ACA_RT) k_aca_reg(const double *Rall, double *Uall, double *Vall,
                                                    const int64_t *a_off, const int64_t *u_off,
                                                    const int32_t *rows_arr, int cols, double eps, int maxr_cap,
                                                    int32_t *rank_out, int32_t *piv_out, int32_t *pivc_out)
{
    __shared__ double sh_s[ACA_RT / 64], sh_v[ACA_RT / 64];
    __shared__ int sh_i[ACA_RT / 64];
    __shared__ double vrow[ACA_MAXCOLS], vq[ACA_MAXCOLS], ucol[ACA_RMAXROWS];
    __shared__ int32_t pivr[ACA_MAXCOLS], pivc[ACA_MAXCOLS];
    __shared__ double Lsh[ACA_BS_MAXR * ACA_BS_MAXR];
    const int c = blockIdx.x, tid = threadIdx.x;
    const int rows = rows_arr[c];
    const int rmax = min(rows, cols);
    const double *R = Rall + a_off[c];
    double *U = Uall + u_off[c];
    double *V = Vall + u_off[c];
    const int TR = ACA_RT / cols;
    const int g = tid / cols, j = tid - g * cols;
    const bool act = g < TR;

    // rows g + k TR beyond the matrix (and inactive threads) hold zeros and
    // never win the pivot search: their index is past every real entry
    for (int i = tid; i < ACA_RMAXROWS; i += ACA_RT) ucol[i] = 0.0;
    const int big = INT32_MAX / 2;
    double x[K];
    double s = 0, mv = -1.0;
    int mi = INT32_MAX;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int i = g + k * TR;
        const bool ok = act && i < rows;
        x[k] = ok ? R[i * cols + j] : 0.0;
        s += x[k] * x[k];
        const int e = ok ? i * cols + j : big;
        if (better32(fabs(x[k]), e, mv, mi)) {
            mv = fabs(x[k]);
            mi = e;
        }
    }
    block_reduce_rt(s, mv, mi, sh_s, sh_v, sh_i);
    const double tol2 = eps * eps * s;
    double nR2 = s;
    int r = 0;
    // two barriers per step: after the pivot row and column reach LDS, and
    // inside the reduction of the updated residual
    while (r < rmax && r < maxr_cap && nR2 > tol2) {
        const int p = mi / cols, q = mi - p * cols;
        // the row-group index is made opaque to the compiler here so that the
        // per-entry indices are recomputed in each step instead of being kept
        // live across steps (they would double the registers per entry)
        int gs = g;
        asm volatile("" : "+v"(gs));
        // pivot row and column to LDS
        if (act) {
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const int i = gs + k * TR;
                if (i == p) vrow[j] = x[k];
                if (j == q) ucol[i] = x[k];
            }
        }
        __syncthreads();
        const double piv = vrow[q];
        if (piv == 0.0) break;
        for (int i = tid; i < rows; i += ACA_RT) U[(int64_t)i * rmax + r] = ucol[i];
        if (tid == 0) {
            pivr[r] = p;
            pivc[r] = q;
        }
        s = 0;
        mv = -1.0;
        mi = INT32_MAX;
        const double vj = act ? vrow[j] / piv : 0.0;
        const bool colq = j == q;
        // the pivot row and column are read before the reduction's barrier,
        // so the next step may overwrite them after it
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int i = gs + k * TR;
            const double v = (i == p || colq) ? 0.0 : x[k] - ucol[i] * vj;
            x[k] = v;
            s += v * v;
            const int e = (act && i < rows) ? i * cols + j : big;
            if (better32(fabs(v), e, mv, mi)) {
                mv = fabs(v);
                mi = e;
            }
        }
        block_reduce_rt(s, mv, mi, sh_s, sh_v, sh_i);
        nR2 = s;
        ++r;
    }
    if (tid == 0) rank_out[c] = r;
    for (int k = tid; k < r; k += ACA_RT) {
        piv_out[(int64_t)c * maxr_cap + k] = pivr[k];
        pivc_out[(int64_t)c * maxr_cap + k] = pivc[k];
    }
    __syncthreads();
    // V = U L^{-1}, L[j][k] = U[piv_j][k] (lower triangular): back substitution
    // per row, k = r-1 .. 0.  Eight threads share a row: thread t holds
    // columns t + 8 s of u_i and v_i in registers, the sum over j > k is
    // split over the eight and combined by shuffles; L is staged in LDS.
    if (r <= ACA_BS_MAXR) {
        for (int e = tid; e < r * r; e += ACA_RT) {
            const int jr = e / r, kc = e - jr * r;
            Lsh[e] = U[(int64_t)pivr[jr] * rmax + kc];
        }
        __syncthreads();
        const int t8 = tid & 7;
        for (int i = tid >> 3; i < rows; i += ACA_RT / 8) {
            double u[ACA_BS_MAXR / 8], v[ACA_BS_MAXR / 8];
#pragma unroll
            for (int sl = 0; sl < ACA_BS_MAXR / 8; ++sl) {
                const int j = t8 + 8 * sl;
                u[sl] = j < r ? U[(int64_t)i * rmax + j] : 0.0;
                v[sl] = 0.0;
            }
            for (int k = r - 1; k >= 0; --k) {
                double acc = 0.0;
#pragma unroll
                for (int sl = 0; sl < ACA_BS_MAXR / 8; ++sl) {
                    const int j = t8 + 8 * sl;
                    if (j > k && j < r) acc += v[sl] * Lsh[j * r + k];
                }
                acc = group_sum<8>(acc);   // the row's eight lanes, DPP
                const int sk = k >> 3;
                if (t8 == (k & 7)) {
#pragma unroll
                    for (int sl = 0; sl < ACA_BS_MAXR / 8; ++sl)
                        if (sl == sk) v[sl] = (u[sl] - acc) / Lsh[k * r + k];
                }
            }
#pragma unroll
            for (int sl = 0; sl < ACA_BS_MAXR / 8; ++sl) {
                const int j = t8 + 8 * sl;
                if (j < r) V[(int64_t)i * rmax + j] = v[sl];
            }
        }
    } else {
        for (int i = tid; i < rows; i += ACA_RT) {
            double *vi = V + (int64_t)i * rmax;
            const double *ui = U + (int64_t)i * rmax;
            for (int k = r - 1; k >= 0; --k) {
                double acc = ui[k];
                for (int jj = k + 1; jj < r; ++jj) acc -= vi[jj] * U[(int64_t)pivr[jj] * rmax + k];
                vi[k] = acc / U[(int64_t)pivr[k] * rmax + k];
            }
        }
    }
    __syncthreads();
    for (int k = tid; k < r; k += ACA_RT) {
        double *vi = V + (int64_t)pivr[k] * rmax;
        for (int jj = 0; jj < r; ++jj) vi[jj] = (jj == k) ? 1.0 : 0.0;
    }
}

hipError_t launch_aca(double *R, double *U, double *V, const int64_t *a_off, const int64_t *u_off,
                      const int32_t *rows, int cols, int nbatch, double eps, int maxr_cap, int32_t *rank_out,
                      int32_t *piv_out, int32_t *pivc_out, int max_rows, hipStream_t s)
{
    if (nbatch == 0) return hipSuccess;
    if (cols > ACA_MAXCOLS || maxr_cap > ACA_MAXCOLS) return hipErrorInvalidValue;
    // register-resident variant when every row group fits K rows
    const int TR = ACA_RT / cols;
    const int need = TR > 0 ? (max_rows + TR - 1) / TR : 1 << 30;
#define ACA_REG(KK)                                                                                   \
    if (need <= KK && KK * TR <= ACA_RMAXROWS) {                                                     \
        hipLaunchKernelGGL(k_aca_reg<KK>, dim3(nbatch), dim3(ACA_RT), 0, s, R, U, V, a_off, u_off, rows, \
                           cols, eps, maxr_cap, rank_out, piv_out, pivc_out);                        \
        return hipGetLastError();                                                                    \
    }
    ACA_REG(8)
    ACA_REG(16)
    ACA_REG(24)
    ACA_REG(32)
    ACA_REG(48)
#undef ACA_REG
    hipLaunchKernelGGL(k_aca, dim3(nbatch), dim3(ACA_THREADS), 0, s, R, U, V, a_off, u_off, rows, cols, eps,
                       maxr_cap, rank_out, piv_out, pivc_out);
    return hipGetLastError();
}

// ------------------------------------------------------------- copy jobs --
// Job k copies rows [row0, row0 + nrows) x cols [0, ncols) of a row-major
// source (leading dimension src_ld) into row-major (dst_ld = ncols) and
// column-major (dst_ld = nrows) FP64 and FP32 destinations.
__global__ void k_copy_jobs(const int64_t *jobs, int njobs, const double *src, double *dr, double *dc, float *fr,
                            float *fc)
{
    const int k = blockIdx.x;
    const int64_t *J = jobs + 6 * k;
    const int64_t so = J[0], ld = J[1], row0 = J[2], nr = J[3], nc = J[4], dof = J[5];
    for (int64_t e = threadIdx.x; e < nr * nc; e += blockDim.x) {
        int64_t i = e / nc, j = e - i * nc;
        double v = src[so + (row0 + i) * ld + j];
        dr[dof + i * nc + j] = v;
        dc[dof + j * nr + i] = v;
        fr[dof + i * nc + j] = (float)v;
        fc[dof + j * nr + i] = (float)v;
    }
}

hipError_t launch_copy_jobs(const int64_t *jobs, int njobs, const double *src, double *dr, double *dc, float *fr,
                            float *fc, hipStream_t s)
{
    if (njobs == 0) return hipSuccess;
    hipLaunchKernelGGL(k_copy_jobs, dim3(njobs), dim3(256), 0, s, jobs, njobs, src, dr, dc, fr, fc);
    return hipGetLastError();
}

}  // namespace gca
