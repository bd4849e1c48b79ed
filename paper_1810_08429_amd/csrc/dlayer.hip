// Galerkin entries of the double-layer operator on flat triangles with
// piecewise-constant bases (Section 1: the second-kind formulation uses the
// normal derivative of g at y; Section 6: unit normals of the triangles):
//     k_ij = int_{t_i} int_{t_j} n_j . (x - y) / (4 pi |x - y|^3) dy dx,
// n_j the unit normal of t_j from its mesh orientation.
//
// One kernel, one thread per pair, classified on the device from vertex ids
// (as the piecewise-constant entries):
//   - identical pairs are 0 (x - y lies in the plane of t_j);
//   - regular and near-regular pairs (a vertex of one triangle joined by a
//     mesh edge to a vertex of the other): the triangle rule of order q_r /
//     q_nr on both triangles (collapsed Gauss or the symmetric rules), in the
//     pair's own lane;
//   - common vertex / common edge: after a ballot, one wavefront per pair
//     integrates the Sauter-Schwab maps of [0,1]^4 onto T x T (2 / 5 regions)
//     with a q_s-point Gauss rule in every variable, lanes over (region, xi,
//     e1, e2) and e3 inside, the lanes' sums combined in a fixed order; the
//     kernel is O(1/r^2) at the common vertex or edge and the maps' Jacobian
//     (xi^3 times a polynomial) cancels it.
// All in FP64.
#include <hip/hip_runtime.h>

#include "devfn.h"
#include "gca_internal.h"
#include "ssmap.h"

namespace gca {
namespace {

constexpr int DL_RULE = 36;   // points of a triangle rule at most (collapsed order 6)
constexpr int DL_GAUSS = 32;

struct DlRule {
    double s1[DL_RULE], s2[DL_RULE], w[DL_RULE];
    int np;
};

struct DlArgs {
    const double *xyz;           // mesh vertices
    const int32_t *tv;           // per position: the triangle's vertex ids (mesh order)
    const int32_t *iperm;        // original triangle id -> position
    const int64_t *vv_ptr;       // vertex -> vertices joined by a mesh edge (CSR)
    const int32_t *vv;
    int64_t n;
    const int32_t *I, *J;
    int64_t m;
    double *out;
    DlRule rr, rn;
    double gx[DL_GAUSS], gw[DL_GAUSS];
    int q;
};

__device__ __forceinline__ void ldv(const double *xyz, int v, double *o)
{
    o[0] = xyz[3 * (int64_t)v];
    o[1] = xyz[3 * (int64_t)v + 1];
    o[2] = xyz[3 * (int64_t)v + 2];
}

// |(P1 - P0) x (P2 - P1)| of vertices P (9 doubles)
__device__ double jac2(const double *P)
{
    const double ax = P[3] - P[0], ay = P[4] - P[1], az = P[5] - P[2];
    const double bx = P[6] - P[3], by = P[7] - P[4], bz = P[8] - P[5];
    const double cx = ay * bz - az * by, cy = az * bx - ax * bz, cz = ax * by - ay * bx;
    return sqrt(cx * cx + cy * cy + cz * cz);
}

// unit normal (v1 - v0) x (v2 - v0) of the triangle with vertex ids W
__device__ void unit_normal(const double *xyz, const int *W, double *n)
{
    double a[3], b[3], c[3];
    ldv(xyz, W[0], a);
    ldv(xyz, W[1], b);
    ldv(xyz, W[2], c);
    const double e1[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]}, e2[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
    n[0] = e1[1] * e2[2] - e1[2] * e2[1];
    n[1] = e1[2] * e2[0] - e1[0] * e2[2];
    n[2] = e1[0] * e2[1] - e1[1] * e2[0];
    const double l = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    n[0] /= l;
    n[1] /= l;
    n[2] /= l;
}

// n . d / |d|^3 with the refined reciprocal square root
__device__ __forceinline__ double dl_kernel(const double *n, double dx, double dy, double dz)
{
    const double ir = rsq<double>(dx * dx + dy * dy + dz * dz);
    return (n[0] * dx + n[1] * dy + n[2] * dz) * (ir * ir) * ir;
}

__device__ double regular_entry(const DlRule &R, const double *P, const double *Q, const double *n)
{
    double sum = 0.0;
    for (int p = 0; p < R.np; ++p) {
        const double x0 = P[0] + R.s1[p] * (P[3] - P[0]) + R.s2[p] * (P[6] - P[3]);
        const double x1 = P[1] + R.s1[p] * (P[4] - P[1]) + R.s2[p] * (P[7] - P[4]);
        const double x2 = P[2] + R.s1[p] * (P[5] - P[2]) + R.s2[p] * (P[8] - P[5]);
        double inner = 0.0;
        for (int q = 0; q < R.np; ++q) {
            const double y0 = Q[0] + R.s1[q] * (Q[3] - Q[0]) + R.s2[q] * (Q[6] - Q[3]);
            const double y1 = Q[1] + R.s1[q] * (Q[4] - Q[1]) + R.s2[q] * (Q[7] - Q[4]);
            const double y2 = Q[2] + R.s1[q] * (Q[5] - Q[2]) + R.s2[q] * (Q[8] - Q[5]);
            inner += R.w[q] * dl_kernel(n, x0 - y0, x1 - y1, x2 - y2);
        }
        sum += R.w[p] * inner;
    }
    return sum;
}

__device__ __forceinline__ double wave_sum(double v)
{
    v = group_sum<16>(v);
    v += __shfl_xor(v, 16);
    v += __shfl_xor(v, 32);
    return v;
}

constexpr int DL_WAVES = 4;
constexpr double INV4PI_DL = 0.07957747154594767;

__global__ void __launch_bounds__(64 * DL_WAVES) k_dl_pairs(DlArgs a)
{
    const int lane = threadIdx.x & 63;
    const int64_t base = ((int64_t)blockIdx.x * DL_WAVES + (threadIdx.x >> 6)) * 64;
    const int64_t k = base + lane;
    int V[3] = {0, 0, 0}, W[3] = {0, 0, 0};
    bool tch = false;
    if (k < a.m) {
        const int t = a.I[k], s = a.J[k];
        if (t < 0 || t >= a.n || s < 0 || s >= a.n) {
            a.out[k] = __builtin_nan("");
        } else {
            const int pt = a.iperm[t], ps = a.iperm[s];
            for (int c = 0; c < 3; ++c) {
                V[c] = a.tv[3 * (int64_t)pt + c];
                W[c] = a.tv[3 * (int64_t)ps + c];
            }
            int shared = 0;
            for (int x = 0; x < 3; ++x)
                for (int y = 0; y < 3; ++y) shared += V[x] == W[y];
            if (shared == 3) {
                a.out[k] = 0.0;
            } else if (shared > 0) {
                tch = true;
            } else {
                bool nearreg = false;
                for (int x = 0; x < 3 && !nearreg; ++x)
                    for (int64_t e = a.vv_ptr[V[x]]; e < a.vv_ptr[V[x] + 1] && !nearreg; ++e)
                        for (int y = 0; y < 3; ++y) nearreg |= a.vv[e] == W[y];
                double P[9], Q[9], n[3];
                for (int c = 0; c < 3; ++c) {
                    ldv(a.xyz, V[c], P + 3 * c);
                    ldv(a.xyz, W[c], Q + 3 * c);
                }
                unit_normal(a.xyz, W, n);
                a.out[k] = regular_entry(nearreg ? a.rn : a.rr, P, Q, n) * jac2(P) * jac2(Q) * INV4PI_DL;
            }
        }
    }
    uint64_t mask = __ballot(tch);
    const int q = a.q, q3 = q * q * q;
    while (mask) {
        const int l = __ffsll((unsigned long long)mask) - 1;
        mask &= mask - 1;
        int Vs[3], Ws[3];
        for (int c = 0; c < 3; ++c) {
            Vs[c] = __shfl(V[c], l);
            Ws[c] = __shfl(W[c], l);
        }
        // the rule's vertex order: common edge, the shared vertices by
        // ascending id, then the third; common vertex, the shared one, then
        // the cyclic mesh order
        int nsh = 0, sa0 = 0, sb0 = 0, sa1 = 0, sb1 = 0;
        for (int x = 0; x < 3; ++x)
            for (int y = 0; y < 3; ++y)
                if (Vs[x] == Ws[y]) {
                    if (nsh == 0) { sa0 = x; sb0 = y; }
                    else { sa1 = x; sb1 = y; }
                    ++nsh;
                }
        int pa[3], pb[3];
        const int kase = nsh == 2 ? SS_EDGE : SS_VERT;
        if (nsh == 2) {
            const bool lo0 = Vs[sa0] < Vs[sa1];
            pa[0] = lo0 ? sa0 : sa1;
            pa[1] = lo0 ? sa1 : sa0;
            pb[0] = lo0 ? sb0 : sb1;
            pb[1] = lo0 ? sb1 : sb0;
        } else {
            pa[0] = sa0;
            pa[1] = sa0 == 2 ? 0 : sa0 + 1;
            pb[0] = sb0;
            pb[1] = sb0 == 2 ? 0 : sb0 + 1;
        }
        pa[2] = 3 - pa[0] - pa[1];
        pb[2] = 3 - pb[0] - pb[1];
        double P[9], Q[9], n[3];
        for (int c = 0; c < 3; ++c) {
            ldv(a.xyz, Vs[pa[c]], P + 3 * c);
            ldv(a.xyz, Ws[pb[c]], Q + 3 * c);
        }
        unit_normal(a.xyz, Ws, n);
        // both parametrisations relative to the shared vertex P0 = Q0
        const double u1[3] = {P[3] - P[0], P[4] - P[1], P[5] - P[2]}, u2[3] = {P[6] - P[3], P[7] - P[4], P[8] - P[5]};
        const double v1[3] = {Q[3] - Q[0], Q[4] - Q[1], Q[5] - Q[2]}, v2[3] = {Q[6] - Q[3], Q[7] - Q[4], Q[8] - Q[5]};
        double sum = 0.0;
        for (int o = lane; o < ss_nregions(kase) * q3; o += 64) {
            const int r = o / q3, w = o - r * q3;
            const int i = w / (q * q), j = (w / q) % q, kk = w % q;
            for (int ll = 0; ll < q; ++ll) {
                double x1, x2, y1, y2;
                const double jac = ss_map_full(kase, r, a.gx[i], a.gx[j], a.gx[kk], a.gx[ll], x1, x2, y1, y2);
                const double wt = a.gw[i] * a.gw[j] * a.gw[kk] * a.gw[ll] * jac;
                double d[3];
                for (int c = 0; c < 3; ++c) d[c] = (x1 * u1[c] + x2 * u2[c]) - (y1 * v1[c] + y2 * v2[c]);
                sum += wt * dl_kernel(n, d[0], d[1], d[2]);
            }
        }
        sum = wave_sum(sum);
        if (lane == 0) a.out[base + l] = sum * jac2(P) * jac2(Q) * INV4PI_DL;
    }
}

bool fill_rule(int q, bool sym, DlRule &out)
{
    TriRule r;
    if (!tri_rule(q, sym, r) || r.np > DL_RULE) return false;
    for (int p = 0; p < r.np; ++p) {
        out.s1[p] = r.s1[p];
        out.s2[p] = r.s2[p];
        out.w[p] = r.w[p];
    }
    out.np = r.np;
    return true;
}

}  // namespace

hipError_t launch_dl_pairs(const double *xyz, const int32_t *tv, const int32_t *iperm, const int64_t *vv_ptr,
                           const int32_t *vv, int64_t n, const int32_t *I, const int32_t *J, int64_t m, int q_r,
                           int q_nr, int q_s, bool sym, double *out, hipStream_t s)
{
    if (m <= 0) return hipSuccess;
    DlArgs a{};
    a.xyz = xyz;
    a.tv = tv;
    a.iperm = iperm;
    a.vv_ptr = vv_ptr;
    a.vv = vv;
    a.n = n;
    a.I = I;
    a.J = J;
    a.m = m;
    a.out = out;
    if (!fill_rule(q_r, sym, a.rr) || !fill_rule(q_nr, sym, a.rn) || q_s < 1 || q_s > DL_GAUSS)
        return hipErrorInvalidValue;
    gauss_legendre01(q_s, a.gx, a.gw);
    a.q = q_s;
    const int64_t per = 64 * DL_WAVES;
    hipLaunchKernelGGL(k_dl_pairs, dim3((unsigned)((m + per - 1) / per)), dim3(per), 0, s, a);
    return hipGetLastError();
}

}  // namespace gca
