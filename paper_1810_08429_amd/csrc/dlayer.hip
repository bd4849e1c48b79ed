// Galerkin entries of the double-layer operator on flat triangles with
// piecewise-constant bases (Section 1: the second-kind formulation uses the
// normal derivative of g at y; Section 6: unit normals of the triangles):
//     k_ij = int_{t_i} int_{t_j} n_j . (x - y) / (4 pi |x - y|^3) dy dx,
// n_j the unit normal of t_j from its mesh orientation.
//
// One thread per pair; the host classifies the pairs from vertex ids and hands
// every job over as the two triangles' vertices in the order of its rule and
// the normal n_j (168 bytes), grouped by class so that a wavefront runs one
// rule:
//   - regular / near-regular pairs: the triangle rule of order q_r / q_nr on
//     both triangles (collapsed Gauss or the symmetric rules);
//   - common vertex / common edge: the Sauter-Schwab maps of [0,1]^4 onto
//     T x T (2 / 5 regions) with a q_s-point Gauss rule in every variable; the
//     kernel is O(1/r^2) at the common vertex or edge and the maps' Jacobian
//     (xi^3 times a polynomial) cancels it;
//   - identical pairs are 0 (x - y lies in the plane of t_j) and get no job.
// All in FP64.
#include <hip/hip_runtime.h>

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
    const double *job;        // 21 doubles per job: P (3 x 3), Q (3 x 3), n (3)
    const int32_t *kind;      // per job: 0 regular, 1 near-regular, 2 common vertex, 3 common edge
    int64_t m;
    double *out;
    DlRule rr, rn;
    double gx[DL_GAUSS], gw[DL_GAUSS];
    int q;
};

__device__ double jac2(const double *P)
{
    const double ax = P[3] - P[0], ay = P[4] - P[1], az = P[5] - P[2];
    const double bx = P[6] - P[3], by = P[7] - P[4], bz = P[8] - P[5];
    const double cx = ay * bz - az * by, cy = az * bx - ax * bz, cz = ax * by - ay * bx;
    return sqrt(cx * cx + cy * cy + cz * cz);
}

// n . d / |d|^3
__device__ __forceinline__ double dl_kernel(const double *n, double dx, double dy, double dz)
{
    const double r2 = dx * dx + dy * dy + dz * dz;
    return (n[0] * dx + n[1] * dy + n[2] * dz) / (r2 * sqrt(r2));
}

__global__ void __launch_bounds__(128) k_dl_entries(DlArgs a)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.m) return;
    const double *J = a.job + 21 * k;
    const double *P = J, *Q = J + 9, *n = J + 18;
    const int kind = a.kind[k];
    constexpr double inv4pi = 0.07957747154594767;
    double sum = 0.0;
    if (kind <= 1) {
        const DlRule &R = kind == 0 ? a.rr : a.rn;
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
    } else {
        const int edge = kind == 3;
        const int nreg = edge ? 5 : 2;
        // both parametrisations relative to the shared vertex P0 = Q0
        const double pa[3] = {P[3] - P[0], P[4] - P[1], P[5] - P[2]};
        const double pb[3] = {P[6] - P[3], P[7] - P[4], P[8] - P[5]};
        const double qa[3] = {Q[3] - Q[0], Q[4] - Q[1], Q[5] - Q[2]};
        const double qb[3] = {Q[6] - Q[3], Q[7] - Q[4], Q[8] - Q[5]};
        for (int r = 0; r < nreg; ++r)
            for (int i = 0; i < a.q; ++i)
                for (int j = 0; j < a.q; ++j)
                    for (int e = 0; e < a.q; ++e)
                        for (int f = 0; f < a.q; ++f) {
                            double x1, x2, y1, y2;
                            const double jac =
                                ss_map_full(edge ? SS_EDGE : SS_VERT, r, a.gx[i], a.gx[j], a.gx[e], a.gx[f], x1, x2, y1, y2);
                            const double w = a.gw[i] * a.gw[j] * a.gw[e] * a.gw[f] * jac;
                            double d[3];
                            for (int c = 0; c < 3; ++c) d[c] = (x1 * pa[c] + x2 * pb[c]) - (y1 * qa[c] + y2 * qb[c]);
                            sum += w * dl_kernel(n, d[0], d[1], d[2]);
                        }
    }
    a.out[k] = sum * jac2(P) * jac2(Q) * inv4pi;
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

hipError_t launch_dl_entries(const double *job, const int32_t *kind, int64_t m, int q_r, int q_nr, int q_s, bool sym,
                             double *out, hipStream_t s)
{
    if (m <= 0) return hipSuccess;
    DlArgs a{};
    a.job = job;
    a.kind = kind;
    a.m = m;
    a.out = out;
    if (!fill_rule(q_r, sym, a.rr) || !fill_rule(q_nr, sym, a.rn) || q_s < 1 || q_s > DL_GAUSS)
        return hipErrorInvalidValue;
    gauss_legendre01(q_s, a.gx, a.gw);
    a.q = q_s;
    hipLaunchKernelGGL(k_dl_entries, dim3((unsigned)((m + 127) / 128)), dim3(128), 0, s, a);
    return hipGetLastError();
}

}  // namespace gca
