// Adjoint of the H^2 product with respect to the vertex coordinates
// (h2_bilinear_grad): d(a^T G~(X) b)/dX with the structure frozen (tree,
// blocks, boxes, Green points, pivot rows and columns).
//
//   a^T G~ b = sum_near a_i g_ij b_j + sum_far xa_t^T G|t~ x s~ xb_s,
// xa = forward transform of a.  Its derivative has three parts:
//   (i)  pair derivatives of the nearfield entries, weighted a_i b_j + a_j b_i;
//   (ii) pair derivatives of the coupling entries, weighted
//        xa_t[k] xb_s[l] + xb_t[k] xa_s[l];
//   (iii) derivatives of the bases V^ = A^[:, J] A^[I, J]^{-1} through the Green
//        factor A^ of Section 2 (rows depend on the triangles they belong to):
//        Vbar = a (x) cb + b (x) ca at the leaves and xa_son (x) cb + xb_son (x) ca
//        for transfer matrices (cb = backward transform of the coupling output
//        for b), Z = Vbar C^{-T}, Abar[:, J] = Z with (V^T Z) subtracted on the
//        pivot rows, then the derivative of every A^ entry.
// Every triangle gathers its 9 partial derivatives (3 vertices x 3 coordinates)
// from single-writer slots in a fixed order, then every vertex from its
// triangles: the result does not depend on scheduling.
#include <hip/hip_runtime.h>

#include "gca_internal.h"
#include "devfn.h"
#include "mfma.h"

namespace gca {

#define INV4PI_G 0.07957747154594766788

struct Rule {
    double x[32], w[32];
    int q;
};

struct D3 {
    double x, y, z;
};
__device__ __forceinline__ D3 d3(double x, double y, double z) { return {x, y, z}; }
__device__ __forceinline__ D3 operator+(D3 a, D3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ D3 operator-(D3 a, D3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ D3 operator*(double s, D3 a) { return {s * a.x, s * a.y, s * a.z}; }
__device__ __forceinline__ double dot(D3 a, D3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ D3 cross(D3 a, D3 b)
{
    return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ D3 ldv3(const double *xyz, int v) { return {xyz[3 * (size_t)v], xyz[3 * (size_t)v + 1], xyz[3 * (size_t)v + 2]}; }

// J = |e1 x e2|, dJ/de1 = e2 x c^, dJ/de2 = c^ x e1
__device__ inline double jac_grad(D3 e1, D3 e2, D3 &g1, D3 &g2)
{
    D3 c = cross(e1, e2);
    double J = sqrt(dot(c, c));
    D3 ch = (1.0 / J) * c;
    g1 = cross(e2, ch);
    g2 = cross(ch, e1);
    return J;
}

// d ln J / dP_k for the triangle (P0, P1, P2), J = |(P1-P0) x (P2-P1)|
__device__ inline void dlnJ(D3 P0, D3 P1, D3 P2, D3 g[3])
{
    D3 a, b;
    double J = jac_grad(P1 - P0, P2 - P1, a, b);
    g[0] = (-1.0 / J) * a;
    g[1] = (1.0 / J) * (a - b);
    g[2] = (1.0 / J) * b;
}

// f = 1/|v|: accumulate  wt * df/dv = -wt v / |v|^3  and return 1/|v|
__device__ __forceinline__ double inv_and_grad(D3 v, double wt, D3 &acc)
{
    double ri = rsq<double>(dot(v, v));
    acc = acc + (-wt * ri * ri * ri) * v;
    return ri;
}

// ---------------------------------------------- touching pair derivatives --
__constant__ int g_perm[6][3] = {{0, 1, 2}, {1, 2, 0}, {2, 0, 1}, {0, 2, 1}, {1, 0, 2}, {2, 1, 0}};

// Writes d g / d(first triangle's vertex slots) to ga[9] and d g / d(second
// triangle's slots) to gb[9]; shared vertices are attributed to the first.
template <int KIND>
__device__ void touching_grad(const double *xyz, const int32_t *tv, int pa, int pb, int code, const Rule &R,
                              double ga[9], double gb[9])
{
    for (int k = 0; k < 9; ++k) ga[k] = gb[k] = 0;
    const int ca = code & 15, cb = (code >> 4) & 15;
    const int32_t *va = tv + 3 * (size_t)pa, *vb = tv + 3 * (size_t)pb;
    D3 P[3], Q[3];
    for (int k = 0; k < 3; ++k) {
        P[k] = ldv3(xyz, va[g_perm[ca][k]]);
        Q[k] = ldv3(xyz, vb[g_perm[cb][k]]);
    }
    D3 dP[3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}}, dQ[3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    if (KIND == 0) {
        D3 e1 = P[1] - P[0], e2 = P[2] - P[1], j1, j2;
        double J = jac_grad(e1, e2, j1, j2);
        double S = 0;
        D3 s1 = {0, 0, 0}, s2 = {0, 0, 0};
        for (int d = 0; d < R.q; ++d) {
            const double t = R.x[d], w = R.w[d];
            D3 g1 = {0, 0, 0}, g2 = {0, 0, 0}, g3 = {0, 0, 0};
            S += w * inv_and_grad(t * e1 + e2, w, g1);
            S += w * inv_and_grad(e1 + t * e2, w, g2);
            S += w * inv_and_grad((-t) * e1 + (1 - t) * e2, w, g3);
            s1 = s1 + t * g1 + g2 + (-t) * g3;
            s2 = s2 + g1 + t * g2 + (1 - t) * g3;
        }
        const double C = INV4PI_G / 3.0;
        D3 ge1 = C * ((2 * J * S) * j1 + (J * J) * s1);
        D3 ge2 = C * ((2 * J * S) * j2 + (J * J) * s2);
        dP[0] = (-1.0) * ge1;
        dP[1] = ge1 - ge2;
        dP[2] = ge2;
    } else if (KIND == 1) {
        D3 e1 = P[1] - P[0], et = P[2] - P[1], es = Q[2] - P[1];
        D3 jt1, jtt, js1, jss;
        double Jt = jac_grad(e1, et, jt1, jtt), Js = jac_grad(e1, es, js1, jss);
        double S = 0;
        D3 s1 = {0, 0, 0}, st = {0, 0, 0}, ss = {0, 0, 0};
        for (int ia = 0; ia < R.q; ++ia)
            for (int ib = 0; ib < R.q; ++ib) {
                const double h2 = R.x[ia], h3 = R.x[ib], w = R.w[ia] * R.w[ib];
                const double al[5][3] = {{h2, h3, -(1 - h2)},
                                         {h2 * h3, 1.0, -h2 * (1 - h3)},
                                         {-h2, 1 - h2, -h2 * h3},
                                         {-h2 * h3, h2 * (1 - h3), -1.0},
                                         {-h2 * h3, 1 - h2 * h3, -h2}};
                for (int r = 0; r < 5; ++r) {
                    const double wt = w * (r == 0 ? 1.0 : h2);
                    D3 g = {0, 0, 0};
                    S += wt * inv_and_grad(al[r][0] * e1 + al[r][1] * et + al[r][2] * es, wt, g);
                    s1 = s1 + al[r][0] * g;
                    st = st + al[r][1] * g;
                    ss = ss + al[r][2] * g;
                }
            }
        const double C = INV4PI_G / 6.0;
        D3 ge1 = C * ((S * Js) * jt1 + (S * Jt) * js1 + (Jt * Js) * s1);
        D3 get = C * ((S * Js) * jtt + (Jt * Js) * st);
        D3 ges = C * ((S * Jt) * jss + (Jt * Js) * ss);
        dP[0] = (-1.0) * ge1;
        dP[1] = ge1 - get - ges;
        dP[2] = get;
        dQ[2] = ges;
    } else {
        D3 e1t = P[1] - P[0], e2t = P[2] - P[1], e1s = Q[1] - P[0], e2s = Q[2] - Q[1];
        D3 a1, a2, b1, b2;
        double Jt = jac_grad(e1t, e2t, a1, a2), Js = jac_grad(e1s, e2s, b1, b2);
        double S = 0;
        D3 s1t = {0, 0, 0}, s2t = {0, 0, 0}, s1s = {0, 0, 0}, s2s = {0, 0, 0};
        for (int ia = 0; ia < R.q; ++ia)
            for (int ib = 0; ib < R.q; ++ib)
                for (int ic = 0; ic < R.q; ++ic) {
                    const double h1 = R.x[ia], h2 = R.x[ib], h3 = R.x[ic];
                    const double wt = R.w[ia] * R.w[ib] * R.w[ic] * h2;
                    D3 g = {0, 0, 0};
                    S += wt * inv_and_grad(e1t + h1 * e2t + (-h2) * e1s + (-h2 * h3) * e2s, wt, g);
                    s1t = s1t + g;
                    s2t = s2t + h1 * g;
                    s1s = s1s + (-h2) * g;
                    s2s = s2s + (-h2 * h3) * g;
                    g = {0, 0, 0};
                    S += wt * inv_and_grad(h2 * e1t + (h2 * h3) * e2t + (-1.0) * e1s + (-h1) * e2s, wt, g);
                    s1t = s1t + h2 * g;
                    s2t = s2t + (h2 * h3) * g;
                    s1s = s1s + (-1.0) * g;
                    s2s = s2s + (-h1) * g;
                }
        const double C = INV4PI_G / 3.0;
        D3 g1t = C * ((S * Js) * a1 + (Jt * Js) * s1t);
        D3 g2t = C * ((S * Js) * a2 + (Jt * Js) * s2t);
        D3 g1s = C * ((S * Jt) * b1 + (Jt * Js) * s1s);
        D3 g2s = C * ((S * Jt) * b2 + (Jt * Js) * s2s);
        dP[0] = (-1.0) * (g1t + g1s);
        dP[1] = g1t - g2t;
        dP[2] = g2t;
        dQ[1] = g1s - g2s;
        dQ[2] = g2s;
    }
    for (int k = 0; k < 3; ++k) {
        const int sa = g_perm[ca][k], sb = g_perm[cb][k];
        ga[3 * sa + 0] += dP[k].x;
        ga[3 * sa + 1] += dP[k].y;
        ga[3 * sa + 2] += dP[k].z;
        gb[3 * sb + 0] += dQ[k].x;
        gb[3 * sb + 1] += dQ[k].y;
        gb[3 * sb + 2] += dQ[k].z;
    }
}

// coefficient of pair (i, j): a_i b_j + a_j b_i (identical pair: a_i b_i)
template <int KIND>
__global__ void __launch_bounds__(128) k_touching_grad(const double *xyz, const int32_t *tv, const int32_t *pa,
                                                       const int32_t *pb, const int32_t *code, int64_t np, Rule R,
                                                       const double *ap, const double *bp, const int32_t *sa,
                                                       const int32_t *sb, double *gout)
{
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    const int i = pa[p], j = pb[p];
    const double c = (KIND == 0) ? ap[i] * bp[i] : ap[i] * bp[j] + ap[j] * bp[i];
    double ga[9], gb[9];
    touching_grad<KIND>(xyz, tv, i, j, code[p], R, ga, gb);
    double *oa = gout + 9 * (int64_t)sa[p];
    for (int k = 0; k < 9; ++k) oa[k] = c * ga[k];
    if (sb[p] >= 0) {
        double *ob = gout + 9 * (int64_t)sb[p];
        for (int k = 0; k < 9; ++k) ob[k] = c * gb[k];
    }
}

// ------------------------------------------------ regular pair derivatives --
// Point p = (s1, s2) of a triangle rule: barycentric weights of the vertices
// (1 - s1, s1 - s2, s2).
__device__ __forceinline__ void rule_beta(const TriRule &R, int p, double beta[3])
{
    const double s1 = R.s1[p], s2 = R.s2[p];
    beta[0] = 1 - s1;
    beta[1] = s1 - s2;
    beta[2] = s2;
}

// Near-regular pair list: both sides of d g_ij, weighted a_i b_j + a_j b_i.
template <int P>
__global__ void __launch_bounds__(128) k_nearreg_grad(const double *xyz, const int32_t *tv, const double *q,
                                                      const int32_t *pa, const int32_t *pb, int64_t np, TriRule R,
                                                      const double *ap, const double *bp, const int32_t *sa,
                                                      const int32_t *sb, double *gout)
{
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    const int i = pa[p], j = pb[p];
    const double c = ap[i] * bp[j] + ap[j] * bp[i];
    const double *A = q + (size_t)i * P * 4, *B = q + (size_t)j * P * 4;
    double S = 0;
    D3 Ha[P], Hb[P];
    for (int k = 0; k < P; ++k) Ha[k] = Hb[k] = {0, 0, 0};
    for (int bq = 0; bq < P; ++bq) {
        const D3 y = {B[4 * bq], B[4 * bq + 1], B[4 * bq + 2]};
        const double wb = B[4 * bq + 3];
        for (int aq = 0; aq < P; ++aq) {
            const D3 d = D3{A[4 * aq], A[4 * aq + 1], A[4 * aq + 2]} - y;
            const double ri = rsq<double>(dot(d, d));
            const double wab = A[4 * aq + 3] * wb;
            S += wab * ri;
            const D3 f = (wab * ri * ri * ri) * d;
            Ha[aq] = Ha[aq] + f;
            Hb[bq] = Hb[bq] + f;
        }
    }
    const int32_t *vi = tv + 3 * (size_t)i, *vj = tv + 3 * (size_t)j;
    D3 li[3], lj[3];
    dlnJ(ldv3(xyz, vi[0]), ldv3(xyz, vi[1]), ldv3(xyz, vi[2]), li);
    dlnJ(ldv3(xyz, vj[0]), ldv3(xyz, vj[1]), ldv3(xyz, vj[2]), lj);
    double *oa = gout + 9 * (int64_t)sa[p], *ob = gout + 9 * (int64_t)sb[p];
    for (int k = 0; k < 3; ++k) {
        D3 ga = S * li[k], gb = S * lj[k];
        for (int t = 0; t < P; ++t) {
            double beta[3];
            rule_beta(R, t, beta);
            ga = ga - beta[k] * Ha[t];
            gb = gb + beta[k] * Hb[t];
        }
        ga = (c * INV4PI_G) * ga;
        gb = (c * INV4PI_G) * gb;
        oa[3 * k] = ga.x;
        oa[3 * k + 1] = ga.y;
        oa[3 * k + 2] = ga.z;
        ob[3 * k] = gb.x;
        ob[3 * k + 1] = gb.y;
        ob[3 * k + 2] = gb.z;
    }
}

// ------------------------------------------------ block derivatives -------
// One workgroup per (block, orientation); thread per row of the orientation.
// NEAR: rows / cols are leaf triangles, weight a_i b_j + a_j b_i, non-regular
//       pairs masked.  FAR: rows / cols are pivots, weight
//       xa_r[k] xb_c[l] + xb_r[k] xa_c[l].
// Output: 9 values per row at gout + 9 * (slot + row).
template <typename T>
struct GradBlkArgs {
    const int32_t *bt, *bs;
    const int64_t *slot;       // 2 x nblk (row slot, col slot)
    const int32_t *node;
    const double *box;
    const double *q;           // n x P x 4
    const double *xyz;
    const int32_t *tv;
    const int32_t *piv;
    const int64_t *piv_off;
    const int32_t *rank;
    const int64_t *prow_ptr;
    const int32_t *prow_other;
    const T *ca, *cb;          // NEAR: permuted a, b; FAR: forward transforms of a, b
    double *gout;
    int nblk, orient, cw;
    TriRule R;
};

// Threads per row: blocks with at most 32 (64) rows give each row 4 (2)
// threads that take every 4th (2nd) column and sum their accumulators in LDS
// at the end, so small leaves and ranks keep the 128 threads busy.
template <int P>
constexpr int grad_max_split() { return P <= 9 ? 4 : 1; }

template <typename T, int P>
constexpr size_t grad_blk_smem(int cw)
{
    return ((size_t)P * 4 * cw + 2 * cw + (size_t)(grad_max_split<P>() - 1) * 32 * 4 * P) * sizeof(T) + 16;
}

template <typename T, int P, bool NEAR>
__global__ void __launch_bounds__(128, (sizeof(T) == 4 && P <= 6 ? 4 : 1)) k_grad_blocks(GradBlkArgs<T> g)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int b = blockIdx.x, tid = threadIdx.x;
    int t = g.bt[b], s = g.bs[b];
    if (g.orient == 1) {
        if (t == s) return;
        int u = t;
        t = s;
        s = u;
    }
    const int64_t slot = g.slot[2 * b + g.orient];
    const int CW = g.cw;
    T *colp = reinterpret_cast<T *>(smem);   // P x 4 x CW (SoA)
    T *cca = colp + (size_t)P * 4 * CW;     // CW
    T *ccb = cca + CW;
    T *red = ccb + CW;                       // (split - 1) x RW x 4P partial accumulators
    int nr, nc, rb = 0, cb = 0;
    const int32_t *rl = nullptr, *cl = nullptr;
    int64_t ro = 0, co = 0;
    if (NEAR) {
        rb = g.node[5 * t];
        nr = g.node[5 * t + 1] - rb;
        cb = g.node[5 * s];
        nc = g.node[5 * s + 1] - cb;
    } else {
        nr = g.rank[t];
        nc = g.rank[s];
        ro = g.piv_off[t];
        co = g.piv_off[s];
        rl = g.piv + ro;
        cl = g.piv + co;
    }
    constexpr int MAXG = grad_max_split<P>();
    const int G = (MAXG >= 4 && nr <= 32) ? 4 : (MAXG >= 2 && nr <= 64) ? 2 : 1;
    const int RW = (int)blockDim.x / G;
    const int gi = tid / RW, rt = tid - gi * RW;
    const double cx = 0.5 * (g.box[8 * t + 0] + g.box[8 * t + 3]);
    const double cy = 0.5 * (g.box[8 * t + 1] + g.box[8 * t + 4]);
    const double cz = 0.5 * (g.box[8 * t + 2] + g.box[8 * t + 5]);
  for (int r0 = 0; r0 < nr; r0 += RW) {
    const int row = r0 + rt;
    const bool active = row < nr;
    const int pos = active ? (NEAR ? rb + row : rl[row]) : 0;
    T xr[P][3], wr[P];
    T Ga[P], Ha[P][3];
    uint64_t mask = 0;
    T ra = 0, rbv = 0;
    if (active) {
        const double *src = g.q + (size_t)pos * P * 4;
        for (int p = 0; p < P; ++p) {
            xr[p][0] = (T)(src[4 * p] - cx);
            xr[p][1] = (T)(src[4 * p + 1] - cy);
            xr[p][2] = (T)(src[4 * p + 2] - cz);
            wr[p] = (T)src[4 * p + 3];
        }
        ra = NEAR ? g.ca[rb + row] : g.ca[ro + row];
        rbv = NEAR ? g.cb[rb + row] : g.cb[ro + row];
        if (NEAR)
            for (int64_t k = g.prow_ptr[pos]; k < g.prow_ptr[pos + 1]; ++k) {
                int o = g.prow_other[k] - cb;
                if (o >= 0 && o < nc) mask |= (uint64_t)1 << o;
            }
    }
    for (int p = 0; p < P; ++p) {
        Ga[p] = 0;
        Ha[p][0] = Ha[p][1] = Ha[p][2] = 0;
    }
    for (int c0 = 0; c0 < nc; c0 += CW) {
        const int cw = min(CW, nc - c0);
        __syncthreads();
        for (int e = tid; e < cw * P; e += blockDim.x) {
            int j = e / P, p = e - j * P;
            int cpos = NEAR ? cb + c0 + j : cl[c0 + j];
            const double *src = g.q + ((size_t)cpos * P + p) * 4;
            colp[(p * 4 + 0) * CW + j] = (T)(src[0] - cx);
            colp[(p * 4 + 1) * CW + j] = (T)(src[1] - cy);
            colp[(p * 4 + 2) * CW + j] = (T)(src[2] - cz);
            colp[(p * 4 + 3) * CW + j] = (T)src[3];
        }
        for (int j = tid; j < cw; j += blockDim.x) {
            cca[j] = NEAR ? g.ca[cb + c0 + j] : g.ca[co + c0 + j];
            ccb[j] = NEAR ? g.cb[cb + c0 + j] : g.cb[co + c0 + j];
        }
        __syncthreads();
        if (!active) continue;
        for (int j = gi; j < cw; j += G) {
            if (NEAR && ((mask >> (c0 + j)) & 1)) continue;
            const T coef = ra * ccb[j] + rbv * cca[j];
            for (int pb = 0; pb < P; ++pb) {
                const T yx = colp[(pb * 4 + 0) * CW + j], yy = colp[(pb * 4 + 1) * CW + j];
                const T yz = colp[(pb * 4 + 2) * CW + j], yw = coef * colp[(pb * 4 + 3) * CW + j];
#pragma unroll
                for (int pa = 0; pa < P; ++pa) {
                    const T dx = xr[pa][0] - yx, dy = xr[pa][1] - yy, dz = xr[pa][2] - yz;
                    const T ri = (sizeof(T) == 4) ? (T)__builtin_amdgcn_rsqf((float)(dx * dx + dy * dy + dz * dz))
                                                  : (T)rsq<double>((double)(dx * dx + dy * dy + dz * dz));
                    const T tt = yw * ri;
                    Ga[pa] += tt;
                    const T t3 = tt * ri * ri;
                    Ha[pa][0] += t3 * dx;
                    Ha[pa][1] += t3 * dy;
                    Ha[pa][2] += t3 * dz;
                }
            }
        }
    }
    if (G > 1) {
        // the column groups of a row add their sums into group 0 (fixed order)
        __syncthreads();
        if (gi > 0 && active) {
            T *o = red + ((size_t)(gi - 1) * RW + rt) * 4 * P;
            for (int p = 0; p < P; ++p) {
                o[4 * p] = Ga[p];
                o[4 * p + 1] = Ha[p][0];
                o[4 * p + 2] = Ha[p][1];
                o[4 * p + 3] = Ha[p][2];
            }
        }
        __syncthreads();
        if (gi == 0 && active)
            for (int q = 1; q < G; ++q) {
                const T *o = red + ((size_t)(q - 1) * RW + rt) * 4 * P;
                for (int p = 0; p < P; ++p) {
                    Ga[p] += o[4 * p];
                    Ha[p][0] += o[4 * p + 1];
                    Ha[p][1] += o[4 * p + 2];
                    Ha[p][2] += o[4 * p + 3];
                }
            }
    }
    if (active && gi == 0) {
        double S = 0;
        for (int p = 0; p < P; ++p) S += (double)wr[p] * (double)Ga[p];
        const int32_t *v = g.tv + 3 * (size_t)pos;
        D3 lj[3];
        dlnJ(ldv3(g.xyz, v[0]), ldv3(g.xyz, v[1]), ldv3(g.xyz, v[2]), lj);
        double *out = g.gout + 9 * (slot + row);
        for (int k = 0; k < 3; ++k) {
            D3 gk = S * lj[k];
            for (int p = 0; p < P; ++p) {
                double beta[3];
                rule_beta(g.R, p, beta);
                const double wb = beta[k] * (double)wr[p];
                gk = gk - D3{wb * (double)Ha[p][0], wb * (double)Ha[p][1], wb * (double)Ha[p][2]};
            }
            out[3 * k] = INV4PI_G * gk.x;
            out[3 * k + 1] = INV4PI_G * gk.y;
            out[3 * k + 2] = INV4PI_G * gk.z;
        }
    }
  }
}

// --------------------------------------------- basis (Green factor) part --
// Vbar per cluster (rows of A^ x rank), FP64.
template <typename T>
__global__ void k_vbar(const int32_t *node, const int32_t *rank, const int64_t *piv_off, const int64_t *aj_off,
                       const T *ap, const T *bp, const T *xa, const T *xb, const T *ya, const T *yb, double *Vbar)
{
    const int c = blockIdx.x;
    const int r = rank[c];
    const int s0 = node[5 * c + 2], s1 = node[5 * c + 3];
    const T *cbar_a = ya + piv_off[c], *cbar_b = yb + piv_off[c];
    double *out = Vbar + aj_off[c];
    if (s0 < 0) {
        const int beg = node[5 * c], m = node[5 * c + 1] - beg;
        for (int e = threadIdx.x; e < m * r; e += blockDim.x) {
            const int i = e / r, k = e - i * r;
            out[e] = (double)ap[beg + i] * (double)cbar_b[k] + (double)bp[beg + i] * (double)cbar_a[k];
        }
    } else {
        const int r0 = rank[s0], r1 = rank[s1];
        for (int e = threadIdx.x; e < (r0 + r1) * r; e += blockDim.x) {
            const int i = e / r, k = e - i * r;
            const int so = i < r0 ? s0 : s1, jj = i < r0 ? i : i - r0;
            const double xa_ = (double)xa[piv_off[so] + jj], xb_ = (double)xb[piv_off[so] + jj];
            out[e] = xa_ * (double)cbar_b[k] + xb_ * (double)cbar_a[k];
        }
    }
}

// Abar = Z, minus (V^T Z)[k, :] on pivot row I_k (W kept in tmp), all m x r
// row-major; then Abar is written column-major to At (At[l m + i]) through
// LDS tiles, so that the Green-factor derivative kernel reads a column's
// entries of consecutive rows together.  W = V^T Z in 16 x 16 tiles on the
// matrix cores (v_mfma_f64_16x16x4, mfma.h): the four wavefronts take every
// fourth tile, each a sum over the m rows in steps of four.
__global__ void __launch_bounds__(256) k_abar(const int32_t *rank, const int64_t *piv_off, const int32_t *pivrow,
                                              const int64_t *arow_off, const int64_t *aj_off, const double *Vh,
                                              double *Z, double *tmp, double *At)
{
    const int c = blockIdx.x;
    const int r = rank[c];
    const int m = (int)(arow_off[c + 1] - arow_off[c]);
    const double *V = Vh + aj_off[c];
    double *Zc = Z + aj_off[c];
    double *W = tmp + aj_off[c];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63, q = lane & 15, kq = lane >> 4;
    const int nt = (r + 15) >> 4;
    for (int tile = wv; tile < nt * nt; tile += 4) {
        const int k0 = (tile / nt) * 16, l0 = (tile % nt) * 16;
        const int k = k0 + q, l = l0 + q;
        Mfma<double>::acc_t acc = mfma_zero<double>();
        for (int i0 = 0; i0 < m; i0 += 16) {
            // the operands of four steps loaded before their products
            double a[4], b[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int i = i0 + 4 * u + kq;
                a[u] = (i < m && k < r) ? V[(int64_t)i * r + k] : 0.0;
                b[u] = (i < m && l < r) ? Zc[(int64_t)i * r + l] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) acc = Mfma<double>::mma(a[u], b[u], acc);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int kk = k0 + Mfma<double>::row(lane, v);
            if (kk < r && l < r) W[(int64_t)kk * r + l] = acc[v];
        }
    }
    __syncthreads();
    const int32_t *I = pivrow + piv_off[c];
    for (int e = threadIdx.x; e < r * r; e += blockDim.x) {
        const int k = e / r, l = e - k * r;
        Zc[(int64_t)I[k] * r + l] -= W[e];
    }
    __syncthreads();
    __shared__ double tl[32][65];
    double *Ac = At + aj_off[c];
    for (int i0 = 0; i0 < m; i0 += 32)
        for (int l0 = 0; l0 < r; l0 += 64) {
            for (int e = threadIdx.x; e < 32 * 64; e += blockDim.x) {
                const int ii = e >> 6, ll = e & 63;
                tl[ii][ll] = (i0 + ii < m && l0 + ll < r) ? Zc[(int64_t)(i0 + ii) * r + l0 + ll] : 0.0;
            }
            __syncthreads();
            for (int e = threadIdx.x; e < 32 * 64; e += blockDim.x) {
                const int ll = e >> 5, ii = e & 31;
                if (i0 + ii < m && l0 + ll < r) Ac[(int64_t)(l0 + ll) * m + i0 + ii] = tl[ii][ll];
            }
            __syncthreads();
        }
}

// derivative of sum_l Abar[i, l] A^[i, J_l] w.r.t. the row triangle's vertices
// (Abar column-major per cluster: Abar[l m + i])
template <int PA>
__global__ void __launch_bounds__(128, 4) k_abar_grad(const int32_t *rank, const int64_t *piv_off,
                                                   const int32_t *pivcol, const int64_t *arow_off,
                                                   const int32_t *arows, const int64_t *aj_off, const double *box,
                                                   const double *qA, const double *xyz, const int32_t *tv, int m_green,
                                                   double eta, double omega_scale, Rule G_, TriRule RA,
                                                   const double *Abar, double *gout)
{
    const int c = blockIdx.x;
    const int r = rank[c];
    const int64_t ro = arow_off[c];
    const int m = (int)(arow_off[c + 1] - ro);
    const int k = 6 * m_green * m_green;
    const double *bx = box + 8 * (size_t)c;
    const double diam = bx[6], delta = omega_scale * diam / eta;
    double L[3], H[3];
    for (int d = 0; d < 3; ++d) {
        L[d] = bx[d] - delta;
        H[d] = bx[3 + d] + delta;
    }
    // Green column l of the cluster: point z, outward normal n, and the scale
    // of the single-layer (> 0) or double-layer (< 0) column
    auto column = [&](int l, double *o) {
        const int col = pivcol[piv_off[c] + l];
        const int nu = col < k ? col : col - k;
        const int f = nu / (m_green * m_green), ij = nu - f * m_green * m_green, gi = ij / m_green,
                  gj = ij - gi * m_green;
        const int ax = f >> 1, b1 = ax == 0 ? 1 : 0, b2 = ax == 2 ? 1 : 2;
        o[3] = o[4] = o[5] = 0.0;
        o[ax] = (f & 1) ? H[ax] : L[ax];
        o[b1] = L[b1] + G_.x[gi] * (H[b1] - L[b1]);
        o[b2] = L[b2] + G_.x[gj] * (H[b2] - L[b2]);
        o[3 + ax] = (f & 1) ? 1.0 : -1.0;
        const double w = G_.w[gi] * G_.w[gj] * (H[b1] - L[b1]) * (H[b2] - L[b2]);
        o[6] = col < k ? sqrt(w) * INV4PI_G : -diam * sqrt(w) * INV4PI_G;
    };
    // Green columns staged in LDS 64 at a time
    constexpr int CMAX = 64, CH = 4;
    __shared__ double colz[CMAX * 7];
    // rows of at most 32 (64): 4 (2) threads per row take every 4th (2nd)
    // Green column; their sums are added in LDS in a fixed order.  A thread
    // takes its columns CH at a time: their weights Abar[i, l] are loaded
    // once, then per row point p (coordinates loaded once per chunk) the sum
    // over the chunk H_p = sum_l grad_x(...) is folded at once into the three
    // vertex gradients with the point's barycentric weights.
    constexpr int MAXG = PA <= 9 ? 4 : 1;
    constexpr int NV = 10;                 // S and the three vertex gradients
    __shared__ double red[(MAXG == 1 ? 1 : 96) * NV];
    const int G = (MAXG >= 4 && m <= 32) ? 4 : (MAXG >= 2 && m <= 64) ? 2 : 1;
    const int RW = (int)blockDim.x / G, gq = threadIdx.x / RW, rt = threadIdx.x - gq * RW;
    for (int i0 = 0; i0 < m; i0 += RW) {
        const int i = i0 + rt;
        const bool active = i < m;
        const int pos = active ? arows[ro + i] : 0;
        const double *pts = qA + (size_t)pos * PA * 4;
        double S = 0;          // sum_p W_p f_p weighted (for the d ln J term)
        D3 gk[3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
        const double *ab = Abar + aj_off[c] + (active ? i : 0);   // column l at ab[l m]
        for (int lb = 0; lb < r; lb += CMAX) {
            const int le = min(r, lb + CMAX);
            __syncthreads();   // the previous block's columns are no longer read
            for (int l = lb + (int)threadIdx.x; l < le; l += blockDim.x) column(l, colz + 7 * (l - lb));
            __syncthreads();
            for (int l0 = lb + gq; l0 < le; l0 += CH * G) {
                // weights of the chunk's columns (0 past the block: those
                // read the block's last column and add exactly 0)
                double om[CH];
                int lz[CH];
#pragma unroll
                for (int u = 0; u < CH; ++u) {
                    const int l = l0 + u * G;
                    om[u] = (active && l < le) ? ab[(int64_t)l * m] : 0.0;
                    lz[u] = 7 * (min(l, le - 1) - lb);
                }
#pragma unroll 1
                for (int p = 0; active && p < PA; ++p) {
                    const double px = pts[4 * p], py = pts[4 * p + 1], pz = pts[4 * p + 2], pw = pts[4 * p + 3];
                    D3 Hs = {0, 0, 0};
#pragma unroll
                    for (int u = 0; u < CH; ++u) {
                        // column point z, normal n and scale (single layer > 0)
                        const double *cz = colz + lz[u];
                        const double scale = cz[6];
                        const D3 d = D3{px - cz[0], py - cz[1], pz - cz[2]};
                        const double ri = rsq<double>(dot(d, d)), ri3 = ri * ri * ri;
                        const double wq = pw * om[u] * scale;
                        if (scale > 0) {
                            S += wq * ri;                               // g = ri / 4 pi
                            Hs = Hs + (-wq * ri3) * d;                  // grad_x ri = -d ri^3
                        } else {
                            const D3 nn = {cz[3], cz[4], cz[5]};
                            const double nd = dot(nn, d);
                            S += wq * nd * ri3;                         // dg/dn = n.d ri^3 / 4 pi
                            Hs = Hs + wq * ri3 * (nn - (3.0 * nd * ri * ri) * d);
                        }
                    }
                    double beta[3];
                    rule_beta(RA, p, beta);
                    for (int kk = 0; kk < 3; ++kk) gk[kk] = gk[kk] + beta[kk] * Hs;
                }
            }
        }
        if (G > 1) {
            __syncthreads();
            if (gq > 0 && active) {
                double *o = red + ((size_t)(gq - 1) * RW + rt) * NV;
                o[0] = S;
                for (int kk = 0; kk < 3; ++kk) {
                    o[1 + 3 * kk] = gk[kk].x;
                    o[2 + 3 * kk] = gk[kk].y;
                    o[3 + 3 * kk] = gk[kk].z;
                }
            }
            __syncthreads();
            if (gq == 0 && active)
                for (int q = 1; q < G; ++q) {
                    const double *o = red + ((size_t)(q - 1) * RW + rt) * NV;
                    S += o[0];
                    for (int kk = 0; kk < 3; ++kk)
                        gk[kk] = gk[kk] + D3{o[1 + 3 * kk], o[2 + 3 * kk], o[3 + 3 * kk]};
                }
        }
        if (gq != 0 || !active) continue;
        const int32_t *v = tv + 3 * (size_t)pos;
        D3 lj[3];
        dlnJ(ldv3(xyz, v[0]), ldv3(xyz, v[1]), ldv3(xyz, v[2]), lj);
        double *out = gout + 9 * (ro + i);
        for (int kk = 0; kk < 3; ++kk) {
            const D3 g = S * lj[kk] + gk[kk];
            out[3 * kk] = g.x;
            out[3 * kk + 1] = g.y;
            out[3 * kk + 2] = g.z;
        }
    }
}

// ------------------------------------------------------------- gathers ----
// Per triangle position: sum of its near-block slots, coupling-slot pivot
// occurrences, pair-list slots and Green-factor rows (fixed order).
__global__ void k_tri_gather(int64_t n, const int32_t *leaf_of, const int32_t *leaf_index, const int32_t *node,
                             const int64_t *nslot_ptr, const int64_t *nslot, const double *gnear,
                             const int64_t *pocc_ptr, const int32_t *pocc, const int32_t *piv_cluster,
                             const int64_t *piv_off, const int64_t *cslot_ptr, const int64_t *cslot,
                             const double *gfar,
                             const int64_t *tptr, const double *gt, const int64_t *nptr, const double *gn,
                             const int64_t *rocc_ptr, const int32_t *rocc, const double *gb, double *dT)
{
    int64_t pos = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (pos >= n) return;
    double acc[9];
    for (int k = 0; k < 9; ++k) acc[k] = 0;
    const int c = leaf_of[pos], li = leaf_index[c];
    const int i = (int)(pos - node[5 * c]);
    for (int64_t q = nslot_ptr[li]; q < nslot_ptr[li + 1]; ++q)
        for (int k = 0; k < 9; ++k) acc[k] += gnear[9 * (nslot[q] + i) + k];
    for (int64_t q = pocc_ptr[pos]; q < pocc_ptr[pos + 1]; ++q) {
        const int gq = pocc[q];
        const int cc = piv_cluster[gq];
        const int kk = (int)(gq - piv_off[cc]);
        for (int64_t u = cslot_ptr[cc]; u < cslot_ptr[cc + 1]; ++u)
            for (int k = 0; k < 9; ++k) acc[k] += gfar[9 * (cslot[u] + kk) + k];
    }
    for (int64_t q = tptr[pos]; q < tptr[pos + 1]; ++q)
        for (int k = 0; k < 9; ++k) acc[k] += gt[9 * q + k];
    for (int64_t q = nptr[pos]; q < nptr[pos + 1]; ++q)
        for (int k = 0; k < 9; ++k) acc[k] += gn[9 * q + k];
    for (int64_t q = rocc_ptr[pos]; q < rocc_ptr[pos + 1]; ++q)
        for (int k = 0; k < 9; ++k) acc[k] += gb[9 * (int64_t)rocc[q] + k];
    for (int k = 0; k < 9; ++k) dT[9 * pos + k] = acc[k];
}

// dxyz[v] += alpha * sum over (triangle position, local slot) incident to v
__global__ void k_vertex_gather(int64_t nv, const int64_t *vptr, const int32_t *vpos, const int32_t *vslot,
                                const double *dT, double alpha, const double *scale, double *dxyz)
{
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nv) return;
    if (scale) alpha *= *scale;
    double a0 = 0, a1 = 0, a2 = 0;
    for (int64_t q = vptr[v]; q < vptr[v + 1]; ++q) {
        const double *t = dT + 9 * (int64_t)vpos[q] + 3 * vslot[q];
        a0 += t[0];
        a1 += t[1];
        a2 += t[2];
    }
    dxyz[3 * v] += alpha * a0;
    dxyz[3 * v + 1] += alpha * a1;
    dxyz[3 * v + 2] += alpha * a2;
}

// ------------------------------------------------------------ launcher ----
static Rule make_rule(const double *x, const double *w, int q)
{
    Rule R{};
    R.q = q;
    for (int i = 0; i < q; ++i) {
        R.x[i] = x[i];
        R.w[i] = w[i];
    }
    return R;
}

template <typename T, bool NEAR>
static hipError_t launch_grad_blocks_P(int P, GradBlkArgs<T> a, hipStream_t s)
{
    if (a.nblk == 0) return hipSuccess;
    switch (P) {
#define CASE(PP)                                                                                        \
    case PP:                                                                                            \
        for (int o = 0; o < 2; ++o) {                                                                   \
            a.orient = o;                                                                               \
            hipLaunchKernelGGL((k_grad_blocks<T, PP, NEAR>), dim3(a.nblk), dim3(128),                     \
                               (grad_blk_smem<T, PP>(a.cw)), s, a);                                      \
        }                                                                                               \
        break;
        CASE(1) CASE(3) CASE(4) CASE(6) CASE(9) CASE(16)
#undef CASE
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_bilinear_grad(gca_h2_s *h, const GradWs &w, hipStream_t s)
{
    const bool f32 = std::is_same<T, float>::value;
    const T *ap = f32 ? (const T *)w.apf : (const T *)w.ap;
    const T *bp = f32 ? (const T *)w.bpf : (const T *)w.bp;
    const T *xa = (const T *)w.xa, *xb = (const T *)w.xb, *ya = (const T *)w.ya, *yb = (const T *)w.yb;
    const bool sym = h->prm.sym_rules != 0;
    TriRule Rr, Rnr, RA, Rc;
    if (!tri_rule(h->prm.q_r, sym, Rr) || !tri_rule(h->prm.q_nr, sym, Rnr) || !tri_rule(h->prm.q_A, false, RA) ||
        !tri_rule(h->prm.q_c, sym, Rc))
        return hipErrorInvalidValue;
    const Rule Rs = make_rule(h->gs_x, h->gs_w, h->prm.q_s);
    const Rule Rg = make_rule(h->gl_x, h->gl_w, h->prm.green_m);
    const int Pr = h->P_r;
    const int Pc = h->P_c;
    hipError_t e;
    // (i) nearfield blocks, both orientations
    {
        GradBlkArgs<T> a{};
        const int nb = (int)h->blk.near_t.size();
        a.bt = h->d_near;
        a.bs = h->d_near + nb;
        a.slot = h->d_near_slot;
        a.node = h->d_node;
        a.box = h->d_box;
        a.q = h->d_qr;
        a.xyz = h->d_xyz;
        a.tv = h->d_tv;
        a.prow_ptr = h->d_prow_ptr;
        a.prow_other = h->d_prow_other;
        a.ca = ap;
        a.cb = bp;
        a.nblk = nb;
        a.cw = 64;
        a.R = Rr;
        a.gout = w.gnear;
        if ((e = launch_grad_blocks_P<T, true>(Pr, a, s)) != hipSuccess) return e;
    }
    // (ii) coupling blocks, both orientations
    {
        GradBlkArgs<T> a{};
        const int nb = (int)h->blk.far_t.size();
        a.bt = h->d_far;
        a.bs = h->d_far + nb;
        a.slot = h->d_far_slot;
        a.node = h->d_node;
        a.box = h->d_box;
        a.q = h->d_qc;
        a.xyz = h->d_xyz;
        a.tv = h->d_tv;
        a.piv = h->d_piv;
        a.piv_off = h->d_piv_off;
        a.rank = h->d_rank;
        a.ca = xa;
        a.cb = xb;
        a.nblk = nb;
        a.cw = 64;
        a.R = Rc;
        a.gout = w.gfar;
        if ((e = launch_grad_blocks_P<T, false>(Pc, a, s)) != hipSuccess) return e;
    }
    // touching and near-regular lists (FP64)
    for (int kind = 0; kind < 3; ++kind) {
        const int64_t b = h->pl.off[kind], np = h->pl.off[kind + 1] - b;
        if (!np) continue;
        dim3 g((unsigned)((np + 127) / 128)), blk(128);
        if (kind == 0)
            hipLaunchKernelGGL(k_touching_grad<0>, g, blk, 0, s, h->d_xyz, h->d_tv, h->d_pa + b, h->d_pb + b,
                               h->d_pcode + b, np, Rs, w.ap, w.bp, h->d_slot_a + b, h->d_slot_b + b, w.gt);
        else if (kind == 1)
            hipLaunchKernelGGL(k_touching_grad<1>, g, blk, 0, s, h->d_xyz, h->d_tv, h->d_pa + b, h->d_pb + b,
                               h->d_pcode + b, np, Rs, w.ap, w.bp, h->d_slot_a + b, h->d_slot_b + b, w.gt);
        else
            hipLaunchKernelGGL(k_touching_grad<2>, g, blk, 0, s, h->d_xyz, h->d_tv, h->d_pa + b, h->d_pb + b,
                               h->d_pcode + b, np, Rs, w.ap, w.bp, h->d_slot_a + b, h->d_slot_b + b, w.gt);
    }
    {
        const int64_t b = h->pl.off[3], np = h->pl.off[4] - b;
        const int Pnr = h->P_nr;
        if (np) {
            dim3 g((unsigned)((np + 127) / 128)), blk(128);
            switch (Pnr) {
#define CASE(PP)                                                                                          \
    case PP:                                                                                              \
        hipLaunchKernelGGL((k_nearreg_grad<PP>), g, blk, 0, s, h->d_xyz, h->d_tv, h->d_qnr, h->d_pa + b,   \
                           h->d_pb + b, np, Rnr, w.ap, w.bp, h->d_slot_a + b, h->d_slot_b + b, w.gn);       \
        break;
                CASE(1) CASE(3) CASE(4) CASE(6) CASE(9) CASE(16) CASE(25)
#undef CASE
            default:
                return hipErrorInvalidValue;
            }
        }
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // (iii) bases: Vbar, Z = Vbar C^{-T}, Abar, Green-factor row derivatives
    const unsigned nc = (unsigned)h->nc;
    hipLaunchKernelGGL(k_vbar<T>, dim3(nc), dim3(256), 0, s, h->d_node, h->d_rank, h->d_piv_off, h->fz.d_aj_off, ap,
                       bp, xa, xb, ya, yb, h->fz.d_Vbar);
    if ((e = launch_frozen_adjoint_solve(h, s)) != hipSuccess) return e;
    // Abar column-major into the Vbar buffer (Vbar is consumed by now)
    hipLaunchKernelGGL(k_abar, dim3(nc), dim3(256), 0, s, h->d_rank, h->d_piv_off, h->fz.d_pivrow,
                       h->fz.d_arow_off, h->fz.d_aj_off, h->fz.d_Vh, h->fz.d_Z, h->fz.d_tmp, h->fz.d_Vbar);
    const int PA = h->prm.q_A * h->prm.q_A;
    switch (PA) {
#define CASE(PP)                                                                                              \
    case PP:                                                                                                  \
        hipLaunchKernelGGL((k_abar_grad<PP>), dim3(nc), dim3(128), 0, s, h->d_rank, h->d_piv_off, h->fz.d_pivcol, \
                           h->fz.d_arow_off, h->fz.d_arows, h->fz.d_aj_off, h->d_box, h->d_qA, h->d_xyz, h->d_tv, \
                           h->prm.green_m, h->prm.eta, h->prm.omega_scale, Rg, RA, h->fz.d_Vbar, w.gb);            \
        break;
        CASE(1) CASE(4) CASE(9) CASE(16) CASE(25) CASE(36)
#undef CASE
    default:
        return hipErrorInvalidValue;
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_tri_gather, dim3((unsigned)((h->n + 127) / 128)), dim3(128), 0, s, h->n, w.leaf_of,
                       w.leaf_index, h->d_node, h->d_nslot_ptr, h->d_nslot, w.gnear, w.pocc_ptr, w.pocc,
                       w.piv_cluster, h->d_piv_off, h->d_cslot_ptr, h->d_cslot, w.gfar, h->d_tptr, w.gt, h->d_nptr,
                       w.gn, w.rocc_ptr, w.rocc, w.gb, w.dT);
    return hipGetLastError();
}
template hipError_t launch_bilinear_grad<float>(gca_h2_s *, const GradWs &, hipStream_t);
template hipError_t launch_bilinear_grad<double>(gca_h2_s *, const GradWs &, hipStream_t);

hipError_t launch_vertex_gather(gca_h2_s *h, const GradWs &w, double alpha, const double *scale, double *dxyz,
                                hipStream_t s)
{
    hipLaunchKernelGGL(k_vertex_gather, dim3((unsigned)((h->nv + 127) / 128)), dim3(128), 0, s, h->nv, w.vptr,
                       w.vpos, w.vslot, w.dT, alpha, scale, dxyz);
    return hipGetLastError();
}

}  // namespace gca
