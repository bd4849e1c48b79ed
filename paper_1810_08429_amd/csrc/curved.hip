// Galerkin moments of curved (quadratic) triangle pairs (Section 6): the
// double integral over the reference triangles with both Gramians, the
// mapped nodal weights l_a, the single- or double-layer kernel.
//
// Geometry of a triangle, once per pair: its six nodes relative to the first
// corner and the normal n = dPhi/ds1 x dPhi/ds2 at the six nodes.  n is a
// quadratic polynomial in s (dPhi is linear), so the quadratic interpolation
// of its nodal values gives it exactly at every quadrature point (the
// evaluation the paper proposes): 18 FMAs per point instead of the 36 of the
// two derivatives and the cross product.  gamma = |n|.
//
// One kernel, one thread per pair, every pair written once:
//   - a pair without a common corner: the regular rule of P points on both
//     triangles in its own lane (the column points kept in registers);
//   - then the touching pairs of the wavefront (ballot), one after the other
//     by the whole wavefront: the 4D Sauter-Schwab maps (ssmap.h), lanes over
//     (region, xi, e1, e2) and e3 inside, differences formed relative to the
//     shared corner, the lanes' partial sums combined in a fixed order.
// FP64 throughout.
#include <hip/hip_runtime.h>

#include <cmath>

#include "devfn.h"
#include "gca_curved.h"
#include "gca_internal.h"
#include "ssmap.h"

namespace gca {
namespace {

constexpr int CP = 16;   // points of a regular rule at most
constexpr int CQ = 32;   // Gauss points per Sauter-Schwab variable at most
constexpr double INV4PI = 0.07957747154594767;

struct CurvRule {
    double s1[CP], s2[CP], w[CP];
    double wl[CP][3];          // w_p l_a(s_p)
    double gx[CQ], gw[CQ];     // Gauss-Legendre on [0, 1], order qs
    int qs;
};

struct CurvArgs {
    const double *nodes;
    const int32_t *tri;
    int64_t nt;
    const int32_t *I, *J;
    int64_t m;
    double *out;
    CurvRule R;
};

struct CGeo {
    double x0[3];
    double r[5][3];            // nodes 1..5 minus node 0
    double n[6][3];            // the normal at the six nodes
};

__device__ __forceinline__ int edge_slot(int a, int b)
{
    const int lo = a < b ? a : b, hi = a < b ? b : a;
    return lo == 0 ? (hi == 1 ? 3 : 5) : 4;
}

// Triangle t with its corners in the order (p0, p1, p2); the edge nodes follow.
__device__ void load_geo(const CurvArgs &A, int64_t t, int p0, int p1, int p2, CGeo &G)
{
    const int32_t *T = A.tri + 6 * t;
    const int src[6] = {p0, p1, p2, edge_slot(p0, p1), edge_slot(p1, p2), edge_slot(p2, p0)};
    double R[6][3];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const int64_t v = T[src[k]];
#pragma unroll
        for (int d = 0; d < 3; ++d) R[k][d] = A.nodes[3 * v + d];
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        G.x0[d] = R[0][d];
#pragma unroll
        for (int k = 5; k >= 0; --k) R[k][d] -= R[0][d];
    }
#pragma unroll
    for (int k = 0; k < 5; ++k)
#pragma unroll
        for (int d = 0; d < 3; ++d) G.r[k][d] = R[k + 1][d];
    // reference coordinates (s1, s2) of the nodes
    const double ns1[6] = {0.0, 1.0, 1.0, 0.5, 1.0, 0.5}, ns2[6] = {0.0, 0.0, 1.0, 0.0, 0.5, 0.5};
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const double l0 = 1.0 - ns1[k], l1 = ns1[k] - ns2[k], l2 = ns2[k];
        double a[3], b[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            // dPhi/dl_c of the shape functions, then d/ds1 = d/dl1 - d/dl0, d/ds2 = d/dl2 - d/dl1
            const double d0 = (4 * l0 - 1) * R[0][d] + 4 * l1 * R[3][d] + 4 * l2 * R[5][d];
            const double d1 = (4 * l1 - 1) * R[1][d] + 4 * l0 * R[3][d] + 4 * l2 * R[4][d];
            const double d2 = (4 * l2 - 1) * R[2][d] + 4 * l1 * R[4][d] + 4 * l0 * R[5][d];
            a[d] = d1 - d0;
            b[d] = d2 - d1;
        }
        G.n[k][0] = a[1] * b[2] - a[2] * b[1];
        G.n[k][1] = a[2] * b[0] - a[0] * b[2];
        G.n[k][2] = a[0] * b[1] - a[1] * b[0];
    }
}

// Phi(s) - X0 and n(s) by the quadratic shape functions.
__device__ __forceinline__ void curv_point(const CGeo &G, double s1, double s2, double *rel, double *n)
{
    const double l0 = 1.0 - s1, l1 = s1 - s2, l2 = s2;
    const double N0 = l0 * (2 * l0 - 1), N1 = l1 * (2 * l1 - 1), N2 = l2 * (2 * l2 - 1);
    const double N3 = 4 * l0 * l1, N4 = 4 * l1 * l2, N5 = 4 * l2 * l0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        rel[d] = N1 * G.r[0][d] + N2 * G.r[1][d] + N3 * G.r[2][d] + N4 * G.r[3][d] + N5 * G.r[4][d];
        n[d] = N0 * G.n[0][d] + N1 * G.n[1][d] + N2 * G.n[2][d] + N3 * G.n[3][d] + N4 * G.n[4][d] +
               N5 * G.n[5][d];
    }
}

__device__ __forceinline__ double dot3(const double *a, const double *b)
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

// A pair without a common corner, by one thread.
template <int P, int OP, int BASIS>
__device__ void regular_pair(const CurvArgs &A, int64_t t, int64_t s, double *out)
{
    const CurvRule &R = A.R;
    double yy[P][3], yk[P][3];   // column points minus the row triangle's X0; gamma (OP 0) or n (OP 1)
    double s0[3];
    {
        CGeo Gs;
        load_geo(A, s, 0, 1, 2, Gs);
#pragma unroll
        for (int q = 0; q < P; ++q) {
            double n[3];
            curv_point(Gs, R.s1[q], R.s2[q], yy[q], n);
            if (OP == 0) yk[q][0] = sqrt(dot3(n, n));
            else
#pragma unroll
                for (int d = 0; d < 3; ++d) yk[q][d] = n[d];
        }
#pragma unroll
        for (int d = 0; d < 3; ++d) s0[d] = Gs.x0[d];
    }
    {
        CGeo Gt;
        load_geo(A, t, 0, 1, 2, Gt);
        // x - y = (Phi_t - X0_t) - (Phi_s - X0_s) + (X0_t - X0_s)
#pragma unroll
        for (int q = 0; q < P; ++q)
#pragma unroll
            for (int d = 0; d < 3; ++d) yy[q][d] -= Gt.x0[d] - s0[d];
        double M[9], sum = 0.0;
#pragma unroll
        for (int e = 0; e < 9; ++e) M[e] = 0.0;
#pragma unroll
        for (int p = 0; p < P; ++p) {
            double rx[3], nx[3];
            curv_point(Gt, R.s1[p], R.s2[p], rx, nx);
            const double gx = sqrt(dot3(nx, nx));
            double u0 = 0.0, u1 = 0.0, u2 = 0.0;
#pragma unroll
            for (int q = 0; q < P; ++q) {
                const double dx = rx[0] - yy[q][0], dy = rx[1] - yy[q][1], dz = rx[2] - yy[q][2];
                const double r2 = dx * dx + dy * dy + dz * dz;
                const double ir = rsq<double>(r2);
                double kv;
                if (OP == 0) kv = ir * yk[q][0];
                else kv = (yk[q][0] * dx + yk[q][1] * dy + yk[q][2] * dz) * ir * ir * ir;
                if (BASIS) {
                    u0 += R.wl[q][0] * kv;
                    u1 += R.wl[q][1] * kv;
                    u2 += R.wl[q][2] * kv;
                } else {
                    u0 += R.w[q] * kv;
                }
            }
            if (BASIS) {
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const double wa = R.wl[p][a] * gx;
                    M[3 * a + 0] += wa * u0;
                    M[3 * a + 1] += wa * u1;
                    M[3 * a + 2] += wa * u2;
                }
            } else {
                sum += R.w[p] * gx * u0;
            }
        }
        if (BASIS) {
#pragma unroll
            for (int e = 0; e < 9; ++e) out[e] = M[e] * INV4PI;
        } else {
            out[0] = sum * INV4PI;
        }
    }
}

__device__ __forceinline__ double wave_sum(double v)
{
    v = group_sum<16>(v);
    v += __shfl_xor(v, 16);
    v += __shfl_xor(v, 32);
    return v;
}

// The pairs of a wavefront: pair base + lane is (t, s); invalid ids give NaN,
// pairs without a common corner take regular_pair in their own lane, then the
// touching ones (ballot) are integrated one after the other by the whole
// wavefront.  Every lane of the wavefront must call it.
template <int P, int OP, int BASIS>
__device__ void wave_pairs(const CurvArgs &A, int64_t base, int t, int s, bool live)
{
    const int lane = threadIdx.x & 63;
    bool tch = false;
    if (live) {
        double *out = A.out + (BASIS ? 9 * (base + lane) : base + lane);
        if (t < 0 || t >= A.nt || s < 0 || s >= A.nt) {
            for (int e = 0; e < (BASIS ? 9 : 1); ++e) out[e] = __builtin_nan("");
        } else {
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = 0; b < 3; ++b) tch |= A.tri[6 * (int64_t)t + a] == A.tri[6 * (int64_t)s + b];
            if (!tch) regular_pair<P, OP, BASIS>(A, t, s, out);
        }
    }
    uint64_t mask = __ballot(tch);
    const CurvRule &R = A.R;
    const int q = R.qs, q3 = q * q * q;
    while (mask) {
        const int l = __ffsll((unsigned long long)mask) - 1;
        mask &= mask - 1;
        const int64_t tt = __shfl(t, l), ss = __shfl(s, l);
        const int32_t *V = A.tri + 6 * tt, *W = A.tri + 6 * ss;
        // shared corners and the rule's corner order (as the piecewise-constant entries)
        int nsh = 0, a0 = 0, b0 = 0, a1 = 0, b1 = 0;
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b)
                if (V[a] == W[b]) {
                    if (nsh == 0) { a0 = a; b0 = b; }
                    else { a1 = a; b1 = b; }
                    ++nsh;
                }
        int kase, pa0, pa1, pb0, pb1;
        if (nsh == 3) {
            kase = SS_IDENT;
            pa0 = pb0 = 0;
            pa1 = pb1 = 1;
        } else if (nsh == 2) {
            kase = SS_EDGE;
            const bool lo0 = V[a0] < V[a1];
            pa0 = lo0 ? a0 : a1;
            pa1 = lo0 ? a1 : a0;
            pb0 = lo0 ? b0 : b1;
            pb1 = lo0 ? b1 : b0;
        } else {
            kase = SS_VERT;
            pa0 = a0;
            pa1 = a0 == 2 ? 0 : a0 + 1;
            pb0 = b0;
            pb1 = b0 == 2 ? 0 : b0 + 1;
        }
        const int pa2 = 3 - pa0 - pa1, pb2 = 3 - pb0 - pb1;
        // the normal of s in its mesh orientation: an odd reordering flips it
        const double sgn = ((pb0 > pb1) + (pb0 > pb2) + (pb1 > pb2)) & 1 ? -1.0 : 1.0;
        CGeo Gt, Gs;
        load_geo(A, tt, pa0, pa1, pa2, Gt);
        load_geo(A, ss, pb0, pb1, pb2, Gs);
        int ia[3], ib[3];   // rule corner of mesh corner c
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            ia[c] = pa0 == c ? 0 : (pa1 == c ? 1 : 2);
            ib[c] = pb0 == c ? 0 : (pb1 == c ? 1 : 2);
        }
        double M[9], sum = 0.0;
#pragma unroll
        for (int e = 0; e < 9; ++e) M[e] = 0.0;
        for (int o = lane; o < ss_nregions(kase) * q3; o += 64) {
            const int r = o / q3, w = o - r * q3;
            const int i = w / (q * q), j = (w / q) % q, kk = w % q;
            for (int ll = 0; ll < q; ++ll) {
                double x1, x2, y1, y2;
                const double jac = ss_map_full(kase, r, R.gx[i], R.gx[j], R.gx[kk], R.gx[ll], x1, x2, y1, y2);
                const double wt = R.gw[i] * R.gw[j] * R.gw[kk] * R.gw[ll] * jac;
                double rx[3], nx[3], ry[3], ny[3];
                curv_point(Gt, x1, x2, rx, nx);
                curv_point(Gs, y1, y2, ry, ny);
                const double dx = rx[0] - ry[0], dy = rx[1] - ry[1], dz = rx[2] - ry[2];
                const double r2 = dx * dx + dy * dy + dz * dz;
                const double nx2 = dot3(nx, nx);
                double g;
                if (OP == 0) {
                    // gamma_t gamma_s / r = P / sqrt(r2 P), P = |n_t|^2 |n_s|^2
                    const double pp = nx2 * dot3(ny, ny);
                    g = wt * pp * rsq<double>(r2 * pp);
                } else {
                    // gamma_t (n_s . d) / r^3 = |n_t|^2 (n_s . d) / sqrt(|n_t|^2 r2^3)
                    g = wt * sgn * (ny[0] * dx + ny[1] * dy + ny[2] * dz) * nx2 * rsq<double>(nx2 * r2 * r2 * r2);
                }
                if (BASIS) {
                    const double lp0 = 1.0 - x1, lp1 = x1 - x2, lq0 = 1.0 - y1, lq1 = y1 - y2;
                    double lp[3], lq[3];
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        lp[c] = ia[c] == 0 ? lp0 : (ia[c] == 1 ? lp1 : x2);
                        lq[c] = ib[c] == 0 ? lq0 : (ib[c] == 1 ? lq1 : y2);
                    }
#pragma unroll
                    for (int a = 0; a < 3; ++a)
#pragma unroll
                        for (int b = 0; b < 3; ++b) M[3 * a + b] += g * lp[a] * lq[b];
                } else {
                    sum += g;
                }
            }
        }
        if (BASIS) {
#pragma unroll
            for (int e = 0; e < 9; ++e) M[e] = wave_sum(M[e]);
            if (lane == 0)
#pragma unroll
                for (int e = 0; e < 9; ++e) A.out[9 * (base + l) + e] = M[e] * INV4PI;
        } else {
            sum = wave_sum(sum);
            if (lane == 0) A.out[base + l] = sum * INV4PI;
        }
    }
}

// One thread per pair (64 pairs per wavefront, 256 per workgroup).
template <int P, int OP, int BASIS>
__global__ void __launch_bounds__(256) k_curved(CurvArgs A)
{
    const int64_t base = ((int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) * 64;
    const int64_t k = base + (threadIdx.x & 63);
    const bool live = k < A.m;
    wave_pairs<P, OP, BASIS>(A, base, live ? A.I[k] : -1, live ? A.J[k] : -1, live);
}

template <int OP, int BASIS>
hipError_t launch_curved(const CurvArgs &a, int np, hipStream_t s)
{
    const unsigned g = (unsigned)((a.m + 255) / 256);
    switch (np) {
#define CASE(PP)                                                                         \
    case PP:                                                                             \
        hipLaunchKernelGGL((k_curved<PP, OP, BASIS>), dim3(g), dim3(256), 0, s, a);      \
        break;
        CASE(1) CASE(3) CASE(4) CASE(6) CASE(9) CASE(16)
#undef CASE
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace
}  // namespace gca

using namespace gca;

extern "C" gca_status gca_curved_entries(const double *nodes, const int32_t *tri6, int64_t nt, const int32_t *I,
                                         const int32_t *J, int64_t m, int32_t op, int32_t basis, int32_t q,
                                         int32_t sym, int32_t q_s, double *out, void *stream)
{
    clear_error();
    if (m < 0) return set_error(GCA_EINVAL, "m must be >= 0");
    if (nt < 1 || nt > INT32_MAX) return set_error(GCA_EINVAL, "nt out of range");
    if (op != 0 && op != 1) return set_error(GCA_EINVAL, "op must be 0 (single layer) or 1 (double layer)");
    if (basis != 0 && basis != 1) return set_error(GCA_EINVAL, "basis must be 0 (constant) or 1 (nodal)");
    if (sym != 0 && sym != 1) return set_error(GCA_EINVAL, "sym must be 0 or 1");
    if (q_s < 1 || q_s > CQ) return set_error(GCA_EINVAL, "q_s must be in [1, 32]");
    TriRule r;
    if (q < 1 || !tri_rule(q, sym != 0, r) || r.np > CP) return set_error(GCA_EINVAL, "unsupported rule order");
    if (m == 0) return GCA_OK;
    if (!nodes || !tri6 || !I || !J || !out) return set_error(GCA_EINVAL, "NULL pointer");
    CurvArgs a{};
    a.nodes = nodes;
    a.tri = tri6;
    a.nt = nt;
    a.I = I;
    a.J = J;
    a.m = m;
    a.out = out;
    for (int p = 0; p < r.np; ++p) {
        a.R.s1[p] = r.s1[p];
        a.R.s2[p] = r.s2[p];
        a.R.w[p] = r.w[p];
        a.R.wl[p][0] = r.w[p] * (1.0 - r.s1[p]);
        a.R.wl[p][1] = r.w[p] * (r.s1[p] - r.s2[p]);
        a.R.wl[p][2] = r.w[p] * r.s2[p];
    }
    gauss_legendre01(q_s, a.R.gx, a.R.gw);
    a.R.qs = q_s;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = op == 0 ? (basis ? launch_curved<0, 1>(a, r.np, s) : launch_curved<0, 0>(a, r.np, s))
                           : (basis ? launch_curved<1, 1>(a, r.np, s) : launch_curved<1, 0>(a, r.np, s));
    if (e == hipErrorInvalidValue) return set_error(GCA_EINVAL, "unsupported rule size");
    GCA_HIP_TRY(e);
    return GCA_OK;
}
