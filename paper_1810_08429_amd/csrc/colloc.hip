// Collocation with the continuous piecewise-linear nodal basis on flat
// triangles (Section 6): blocks of
//     g_ij = int_Gamma g(x_i, y) phi_j(y) dy,   x_i a mesh vertex,
// a single integral over the triangles of the support of phi_j.
//
// One workgroup per block (row vertex subset x column vertex subset).  The
// column subset's merged triangle list (gca_lin_merge, Section 5) is staged
// in LDS with, for every column vertex j, the (triangle, corner) pairs where j
// is a corner, ascending by triangle.  A thread per entry (i, j) adds the
// moments int_t g(x_i, y) lambda_c(y) dy over that list in order (no atomics,
// reproducible bit for bit):
//   - x_i a corner k of t: the Duffy transformation at x_i,
//     y = x_i + u ((a - x_i) + v (b - a)), whose Jacobian 2|t| u cancels the
//     1/|x_i - y| = 1/(u |d(v)|); the barycentric weight of corner c is linear
//     in u (1 - u for c = k, u (1 - v) for c = a, u v for c = b), so the u
//     integral is exact and only v takes the q_s-point Gauss rule:
//         M_c = 2|t| / (4 pi) sum_q w_q omega_c(v_q) / |d(v_q)|,
//     omega_k = 1/2, omega_a = (1 - v)/2, omega_b = v/2 -- equal, up to
//     rounding, to the tensor rule of order q_s on the unit square;
//   - otherwise the regular triangle rule (collapsed Gauss of order q, or the
//     symmetric rule of the same degree) with lambda_c at its points.
// The case is decided from vertex ids, as in the oracle.
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>

#include "devfn.h"
#include "gca_internal.h"
#include "gca_linear.h"

namespace gca {
namespace {

constexpr int CT = 256;                      // threads per workgroup
constexpr int BSET = GCA_LIN_MAX_BLOCK_SET;  // vertices of a row or column subset
constexpr int TMAX = GCA_LIN_MAX_TRIS;       // merged triangles of the column subset
constexpr int DEG = GCA_LIN_MAX_DEGREE;      // triangles around a column vertex
constexpr int QS = 32;                       // Duffy Gauss points at most
constexpr int EPT = (BSET * BSET + CT - 1) / CT;

struct CollRule {
    double s1[16], s2[16];
    double wl[16][3];                        // w_p lambda_c(s_p) on the reference triangle
    double v[QS], wv[QS];                    // Gauss-Legendre on [0, 1] for the Duffy variable
    int np, nq;
};

struct CollArgs {
    const double *xyz;
    const int32_t *tri, *set_vtx, *m_tri, *m_loc, *m_count, *set_off, *blk_row, *blk_col;
    int32_t cap;
    int64_t ld;
    double *out;
    int32_t *status;
    CollRule R;
};

__global__ void __launch_bounds__(CT) k_coll_blocks(CollArgs A)
{
    // per column triangle: its vertices (mesh order), or with rules of up to
    // three points the rule's points (the Duffy case then reads the vertices
    // from xyz)
    __shared__ double px[TMAX][9];
    __shared__ double jac[TMAX];             // 2 |t| / (4 pi)
    __shared__ int tv[TMAX][3];              // their vertex ids
    __shared__ int lst[BSET][DEG];           // (triangle << 2 | corner) of column vertex j, ascending
    __shared__ int lc[BSET];
    __shared__ double rx[BSET][3];           // collocation points
    __shared__ int rv[BSET];
    __shared__ int bad;

    const int b = blockIdx.x, tid = threadIdx.x;
    const int rs = A.blk_row[b], cs = A.blk_col[b];
    const int n = A.set_off[rs + 1] - A.set_off[rs], m = A.set_off[cs + 1] - A.set_off[cs];
    const int nS = A.m_count[cs];
    const int nm = n * m;
    double *out = A.out + (int64_t)b * A.ld;
    if (n > BSET || m > BSET || nS < 0 || nS > TMAX) {
        for (int e = tid; e < nm; e += CT) out[e] = 0.0;
        if (tid == 0) A.status[b] = 2;
        return;
    }
    if (tid == 0) bad = 0;
    const int32_t *ctri = A.m_tri + (int64_t)cs * A.cap;
    const int32_t *cloc = A.m_loc + (int64_t)cs * A.cap * 3;
    constexpr double inv4pi = 0.07957747154594767;
    const bool pts = A.R.np <= 3;
    for (int t = tid; t < nS; t += CT) {
        const int tr = ctri[t];
        double X[9];
        for (int c = 0; c < 3; ++c) {
            const int v = A.tri[3 * tr + c];
            tv[t][c] = v;
            for (int d = 0; d < 3; ++d) X[3 * c + d] = A.xyz[3 * v + d];
        }
        const double ax = X[3] - X[0], ay = X[4] - X[1], az = X[5] - X[2];
        const double bx = X[6] - X[0], by = X[7] - X[1], bz = X[8] - X[2];
        const double cx = ay * bz - az * by, cy = az * bx - ax * bz, cz = ax * by - ay * bx;
        jac[t] = sqrt(cx * cx + cy * cy + cz * cz) * inv4pi;
        if (pts) {
            for (int p = 0; p < A.R.np; ++p)
                for (int d = 0; d < 3; ++d)
                    px[t][3 * p + d] = X[d] + A.R.s1[p] * (X[3 + d] - X[d]) + A.R.s2[p] * (X[6 + d] - X[3 + d]);
        } else {
            for (int e = 0; e < 9; ++e) px[t][e] = X[e];
        }
    }
    for (int i = tid; i < n; i += CT) {
        const int v = A.set_vtx[A.set_off[rs] + i];
        rv[i] = v;
        for (int d = 0; d < 3; ++d) rx[i][d] = A.xyz[3 * v + d];
    }
    // per column vertex: its (triangle, corner) pairs, ascending by triangle
    for (int j = tid; j < m; j += CT) {
        int c = 0;
        for (int t = 0; t < nS; ++t)
            for (int k = 0; k < 3; ++k)
                if (cloc[3 * t + k] == j) {
                    if (c < DEG) lst[j][c] = t << 2 | k;
                    ++c;
                }
        if (c > DEG) bad = 1;
        lc[j] = c > DEG ? DEG : c;
    }
    __syncthreads();
    const CollRule &R = A.R;
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
        const int e = tid + k * CT;
        if (e >= nm) break;
        const int i = e / m, j = e - i * m;
        const double x0 = rx[i][0], x1 = rx[i][1], x2 = rx[i][2];
        const int vi = rv[i];
        double acc = 0.0;
        for (int l = 0; l < lc[j]; ++l) {
            const int t = lst[j][l] >> 2, c = lst[j][l] & 3;
            const int ks = tv[t][0] == vi ? 0 : (tv[t][1] == vi ? 1 : (tv[t][2] == vi ? 2 : -1));
            double s = 0.0;
            if (ks >= 0) {
                // Duffy at corner ks: d(v) = (P_a - P_k) + v (P_b - P_a)
                const int ka = ks == 2 ? 0 : ks + 1, kb = ka == 2 ? 0 : ka + 1;
                auto vtx = [&](int k) { return pts ? A.xyz + 3 * (size_t)tv[t][k] : (const double *)px[t] + 3 * k; };
                const double *Pk = vtx(ks), *Pa = vtx(ka), *Pb = vtx(kb);
                const double e0 = Pa[0] - Pk[0], e1 = Pa[1] - Pk[1], e2 = Pa[2] - Pk[2];
                const double f0 = Pb[0] - Pa[0], f1 = Pb[1] - Pa[1], f2 = Pb[2] - Pa[2];
                const int role = c == ks ? 0 : (c == ka ? 1 : 2);
                for (int q = 0; q < R.nq; ++q) {
                    const double v = R.v[q];
                    const double d0 = e0 + v * f0, d1 = e1 + v * f1, d2 = e2 + v * f2;
                    const double om = role == 0 ? 0.5 : (role == 1 ? 0.5 * (1.0 - v) : 0.5 * v);
                    s += R.wv[q] * om * rsq<double>(d0 * d0 + d1 * d1 + d2 * d2);
                }
            } else if (pts) {
                for (int p = 0; p < R.np; ++p) {
                    const double d0 = x0 - px[t][3 * p], d1 = x1 - px[t][3 * p + 1], d2 = x2 - px[t][3 * p + 2];
                    s += R.wl[p][c] * rsq<double>(d0 * d0 + d1 * d1 + d2 * d2);
                }
            } else {
                const double *X = px[t];
                for (int p = 0; p < R.np; ++p) {
                    const double a1 = R.s1[p], a2 = R.s2[p];
                    const double y0 = X[0] + a1 * (X[3] - X[0]) + a2 * (X[6] - X[3]);
                    const double y1 = X[1] + a1 * (X[4] - X[1]) + a2 * (X[7] - X[4]);
                    const double y2 = X[2] + a1 * (X[5] - X[2]) + a2 * (X[8] - X[5]);
                    const double d0 = x0 - y0, d1 = x1 - y1, d2 = x2 - y2;
                    s += R.wl[p][c] * rsq<double>(d0 * d0 + d1 * d1 + d2 * d2);
                }
            }
            acc += s * jac[t];
        }
        out[e] = bad ? 0.0 : acc;
    }
    if (tid == 0) A.status[b] = bad ? 2 : 0;
}

}  // namespace
}  // namespace gca

using namespace gca;

extern "C" gca_status gca_coll_blocks(const double *xyz, const int32_t *tri, const int32_t *set_vtx,
                                      const int32_t *m_tri, const int32_t *m_loc, const int32_t *m_count,
                                      int32_t cap, const int32_t *set_off, const int32_t *blk_row,
                                      const int32_t *blk_col, int32_t nblk, int64_t ld, int32_t q, int32_t sym,
                                      int32_t q_s, double *out, int32_t *status, void *stream)
{
    clear_error();
    if (nblk < 0 || ld < 0) return set_error(GCA_EINVAL, "nblk and ld must be >= 0");
    if (cap < 1 || cap > GCA_LIN_MAX_GATHER) return set_error(GCA_EINVAL, "cap out of range");
    if (sym != 0 && sym != 1) return set_error(GCA_EINVAL, "sym must be 0 or 1");
    if (q_s < 1 || q_s > QS) return set_error(GCA_EINVAL, "q_s must be in [1, 32]");
    TriRule r;
    if (q < 1 || !tri_rule(q, sym != 0, r) || r.np > 16) return set_error(GCA_EINVAL, "unsupported rule order");
    if (nblk == 0) return GCA_OK;
    if (!xyz || !tri || !set_vtx || !m_tri || !m_loc || !m_count || !set_off || !blk_row || !blk_col || !out ||
        !status)
        return set_error(GCA_EINVAL, "NULL pointer");
    CollArgs a{xyz, tri, set_vtx, m_tri, m_loc, m_count, set_off, blk_row, blk_col, cap, ld, out, status, {}};
    for (int p = 0; p < r.np; ++p) {
        a.R.s1[p] = r.s1[p];
        a.R.s2[p] = r.s2[p];
        a.R.wl[p][0] = r.w[p] * (1.0 - r.s1[p]);
        a.R.wl[p][1] = r.w[p] * (r.s1[p] - r.s2[p]);
        a.R.wl[p][2] = r.w[p] * r.s2[p];
    }
    a.R.np = r.np;
    gauss_legendre01(q_s, a.R.v, a.R.wv);
    a.R.nq = q_s;
    hipLaunchKernelGGL(k_coll_blocks, dim3(nblk), dim3(CT), 0, (hipStream_t)stream, a);
    GCA_HIP_TRY(hipGetLastError());
    return GCA_OK;
}
