// Continuous piecewise-linear nodal basis on flat triangles (Section 5):
// merged per-vertex triangle lists of vertex subsets, and Galerkin blocks of
// the linear basis assembled triangle pair by triangle pair.
//
// Merge (one workgroup per subset): the subset's sets T_i are gathered as keys
// (triangle << 32 | corner << 16 | local index), sorted in LDS by a bitonic
// network, and each run of equal triangles becomes one row whose corners take
// the local indices present in the run and -1 (bottom) elsewhere -- the result
// the mergesort with combination of Section 5 defines (rows ascending by
// triangle, one row per triangle).
//
// Blocks (one 512-thread workgroup per block): every merged triangle of the
// row and the column subset is staged once in LDS, and the corners with a
// local vertex are numbered (row corners rho, column corners kappa).  The
// column triangles are taken in chunks whose corners fit the LDS buffer; for
// every pair (t, s) of a chunk one thread evaluates the kernel at the P x P
// point pairs once and forms the nine corner moments
//     M_ab = |J_t| |J_s| / (4 pi) sum_p sum_q w_p lambda_a(x_p) g(x_p, y_q) w_q lambda_b(y_q),
// keeping those whose two corners are local at (rho, kappa).  Every block
// entry (i, j) then adds them over the corners rho of its vertex i and kappa
// of its vertex j in ascending order, so the block is reproducible bit for
// bit without atomics.
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "devfn.h"
#include "gca_internal.h"
#include "gca_linear.h"
#include "ssmap.h"

namespace gca {
namespace {

constexpr int LT = 256;                          // threads per workgroup
constexpr int LMAX = GCA_LIN_MAX_GATHER;
constexpr int NSET = GCA_LIN_MAX_SET;
constexpr int BSET = GCA_LIN_MAX_BLOCK_SET;
constexpr int TMAX = GCA_LIN_MAX_TRIS;
constexpr int DEG = GCA_LIN_MAX_DEGREE;
constexpr int MV = 3680;                         // FP64 corner moments per chunk (28.75 KiB)
constexpr int LB = 512;                          // threads per workgroup of the block kernel
constexpr uint64_t PAD = ~0ull;

// Exclusive prefix sum over a workgroup of NT threads; *total receives the
// sum.  Every thread must call it.
template <int NT = LT>
__device__ int wg_exscan(int v, int *sh, int *total)
{
    const int tid = threadIdx.x;
    sh[tid] = v;
    __syncthreads();
    for (int d = 1; d < NT; d <<= 1) {
        const int add = tid >= d ? sh[tid - d] : 0;
        __syncthreads();
        sh[tid] += add;
        __syncthreads();
    }
    const int incl = sh[tid];
    *total = sh[NT - 1];
    __syncthreads();
    return incl - v;
}

__global__ void __launch_bounds__(LT) k_lin_merge(const int32_t *__restrict__ vt_off,
                                                  const int32_t *__restrict__ vt_list,
                                                  const int32_t *__restrict__ tri,
                                                  const int32_t *__restrict__ set_off,
                                                  const int32_t *__restrict__ set_vtx, int32_t cap,
                                                  int32_t *__restrict__ out_tri, int32_t *__restrict__ out_loc,
                                                  int32_t *__restrict__ out_count)
{
    __shared__ uint64_t key[LMAX];
    __shared__ int base[NSET + 1];
    __shared__ int sh[LT];
    const int k = blockIdx.x, tid = threadIdx.x;
    const int s0 = set_off[k], n = set_off[k + 1] - s0;
    if (n < 0 || n > NSET) {
        if (tid == 0) out_count[k] = -1;
        return;
    }
    // gather offsets: contiguous local indices per thread, then a scan
    const int per = (n + LT - 1) / LT;
    const int i0 = min(n, tid * per), i1 = min(n, i0 + per);
    int deg = 0;
    for (int i = i0; i < i1; ++i) {
        const int v = set_vtx[s0 + i];
        deg += vt_off[v + 1] - vt_off[v];
    }
    int G;
    int off = wg_exscan(deg, sh, &G);
    if (G > LMAX) {
        if (tid == 0) out_count[k] = -1;
        return;
    }
    for (int i = i0; i < i1; ++i) {
        base[i] = off;
        const int v = set_vtx[s0 + i];
        off += vt_off[v + 1] - vt_off[v];
    }
    __syncthreads();
    for (int i = tid; i < n; i += LT) {
        const int v = set_vtx[s0 + i];
        const int e0 = vt_off[v], e1 = vt_off[v + 1];
        for (int e = e0; e < e1; ++e) {
            const int t = vt_list[e];
            const int c = tri[3 * t] == v ? 0 : (tri[3 * t + 1] == v ? 1 : 2);
            key[base[i] + (e - e0)] = ((uint64_t)(uint32_t)t << 32) | ((uint64_t)c << 16) | (uint64_t)i;
        }
    }
    int np2 = 1;
    while (np2 < G) np2 <<= 1;
    for (int x = G + tid; x < np2; x += LT) key[x] = PAD;
    __syncthreads();
    // bitonic sort, ascending
    for (int size = 2; size <= np2; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int x = tid; x < np2; x += LT) {
                const int y = x ^ stride;
                if (y > x) {
                    const uint64_t a = key[x], b = key[y];
                    const bool up = (x & size) == 0;
                    if ((a > b) == up) {
                        key[x] = b;
                        key[y] = a;
                    }
                }
            }
            __syncthreads();
        }
    }
    // one row per run of equal triangles: heads counted per contiguous chunk
    const int pc = (G + LT - 1) / LT;
    const int r0 = min(G, tid * pc), r1 = min(G, r0 + pc);
    int heads = 0;
    for (int r = r0; r < r1; ++r) heads += (r == 0 || (key[r] >> 32) != (key[r - 1] >> 32));
    int R;
    int row = wg_exscan(heads, sh, &R);
    if (R > cap) {
        if (tid == 0) out_count[k] = -1;
        return;
    }
    const int64_t ob = (int64_t)k * cap;
    for (int r = r0; r < r1; ++r) {
        const uint64_t t = key[r] >> 32;
        if (r > 0 && (key[r - 1] >> 32) == t) continue;
        int loc[3] = {-1, -1, -1};
        for (int u = r; u < G && u < r + 3 && (key[u] >> 32) == t; ++u)
            loc[(key[u] >> 16) & 3] = (int)(key[u] & 0xFFFF);
        out_tri[ob + row] = (int32_t)t;
        for (int c = 0; c < 3; ++c) out_loc[(ob + row) * 3 + c] = loc[c];
        ++row;
    }
    if (tid == 0) out_count[k] = R;
}

struct LinRule {
    double s1[16], s2[16];
    double wl[16][3];   // w_p lambda_a(x_p) on the reference triangle
};

struct LinArgs {
    const double *xyz;
    const int32_t *tri, *m_tri, *m_loc, *m_count, *set_off, *blk_row, *blk_col;
    int32_t cap;
    int64_t ld;
    double *out;
    int32_t *status;
    LinRule R;
    double gx[32], gw[32];   // Gauss-Legendre on [0, 1] of order qs (touching pairs)
    int qs;                  // 0: blocks with a touching pair are reported (status 1)
};

// The nine corner moments M[3 a + b] (a, b corners of t and s in mesh order,
// vertex ids V, W) of a touching pair, without the factor 1 / (4 pi), by one
// wavefront: Sauter-Schwab maps (ssmap.h) with qs Gauss points per variable,
// the rule's vertex order as for the piecewise-constant entries (identical:
// mesh order; common edge: the shared vertices by ascending id, then the
// third; common vertex: the shared one, then the cyclic mesh order), and the
// barycentric weights of the maps' reference points moved back to mesh order.
// Lane l takes the (region, xi, e1, e2) points l, l + 64, ... with the whole
// e3 rule; the lanes' partial moments are summed in a fixed tree, so the
// result does not depend on timing.  Every lane of the wavefront must call it;
// every lane receives M.
__device__ void lin_touch_moments(const LinArgs &A, const int *V, const int *W, double *M)
{
    // shared corners (a0, b0), (a1, b1); private arrays below are indexed by
    // compile-time constants only
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
    int kase, pa0, pa1, pb0, pb1;   // mesh corners of rule vertices 0 and 1
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
    double P[9], Q[9];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        P[d] = A.xyz[3 * V[pa0] + d];
        P[3 + d] = A.xyz[3 * V[pa1] + d];
        P[6 + d] = A.xyz[3 * V[pa2] + d];
        Q[d] = A.xyz[3 * W[pb0] + d];
        Q[3 + d] = A.xyz[3 * W[pb1] + d];
        Q[6 + d] = A.xyz[3 * W[pb2] + d];
    }
    // rule vertex of mesh corner c
    int ia[3], ib[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        ia[c] = pa0 == c ? 0 : (pa1 == c ? 1 : 2);
        ib[c] = pb0 == c ? 0 : (pb1 == c ? 1 : 2);
    }
    const double u1[3] = {P[3] - P[0], P[4] - P[1], P[5] - P[2]}, u2[3] = {P[6] - P[3], P[7] - P[4], P[8] - P[5]};
    const double v1[3] = {Q[3] - Q[0], Q[4] - Q[1], Q[5] - Q[2]}, v2[3] = {Q[6] - Q[3], Q[7] - Q[4], Q[8] - Q[5]};
    double m[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) m[e] = 0.0;
    const int q = A.qs, q3 = q * q * q;
    const int lane = threadIdx.x & 63;
    for (int o = lane; o < ss_nregions(kase) * q3; o += 64) {
        const int r = o / q3, w = o - r * q3;
        const int i = w / (q * q), j = (w / q) % q, k = w % q;
        for (int l = 0; l < q; ++l) {
            double x1, x2, y1, y2;
            const double jac = ss_map_full(kase, r, A.gx[i], A.gx[j], A.gx[k], A.gx[l], x1, x2, y1, y2);
            const double d0 = (x1 * u1[0] + x2 * u2[0]) - (y1 * v1[0] + y2 * v2[0]);
            const double d1 = (x1 * u1[1] + x2 * u2[1]) - (y1 * v1[1] + y2 * v2[1]);
            const double d2 = (x1 * u1[2] + x2 * u2[2]) - (y1 * v1[2] + y2 * v2[2]);
            const double g = A.gw[i] * A.gw[j] * A.gw[k] * A.gw[l] * jac * rsq<double>(d0 * d0 + d1 * d1 + d2 * d2);
            // barycentric weights of the rule's vertices, then in mesh order
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
                for (int b = 0; b < 3; ++b) m[3 * a + b] += g * lp[a] * lq[b];
        }
    }
#pragma unroll
    for (int e = 0; e < 9; ++e) {
        double v = group_sum<16>(m[e]);
        v += __shfl_xor(v, 16);
        v += __shfl_xor(v, 32);
        M[e] = v;
    }
}

// Vertex coordinates (9 FP64) and |J| = twice the area of triangle t.
__device__ __forceinline__ double load_tri(const double *xyz, const int32_t *tri, int t, double *X, int *V)
{
    for (int c = 0; c < 3; ++c) {
        const int v = tri[3 * t + c];
        V[c] = v;
        for (int d = 0; d < 3; ++d) X[3 * c + d] = xyz[3 * v + d];
    }
    const double ax = X[3] - X[0], ay = X[4] - X[1], az = X[5] - X[2];
    const double bx = X[6] - X[3], by = X[7] - X[4], bz = X[8] - X[5];
    const double cx = ay * bz - az * by, cy = az * bx - ax * bz, cz = ax * by - ay * bx;
    return sqrt(cx * cx + cy * cy + cz * cz);
}

// Corner numbering of a merged list: corner (row r, c) with a local vertex
// gets the next number in (row, corner) order, -1 otherwise (map[r][c]);
// base[r] is the first number of row r, base[nrow] the total.  Then the
// per-vertex lists of corner numbers, ascending (the reduction order), and
// *bad when a vertex has more than DEG corners or an index is out of range.
__device__ void corner_lists(const int32_t *loc, int nrow, int nv, int (*map)[3], int *base, int (*vl)[DEG],
                             int *vc, int *sh, int *bad)
{
    const int tid = threadIdx.x;
    const int per = (nrow + LB - 1) / LB;
    const int r0 = min(nrow, tid * per), r1 = min(nrow, r0 + per);
    int cnt = 0;
    for (int r = r0; r < r1; ++r)
        for (int c = 0; c < 3; ++c) cnt += loc[3 * r + c] >= 0;
    int total;
    int k = wg_exscan<LB>(cnt, sh, &total);
    for (int r = r0; r < r1; ++r) {
        base[r] = k;
        for (int c = 0; c < 3; ++c) map[r][c] = loc[3 * r + c] >= 0 ? k++ : -1;
    }
    if (tid == 0) base[nrow] = total;
    for (int i = tid; i < nv; i += LB) vc[i] = 0;
    __syncthreads();
    for (int x = tid; x < 3 * nrow; x += LB) {
        const int l = loc[x];
        if (l >= nv) {
            *bad = 1;
        } else if (l >= 0) {
            const int p = atomicAdd(&vc[l], 1);
            if (p < DEG) vl[l][p] = map[x / 3][x - 3 * (x / 3)];
            else *bad = 1;
        }
    }
    __syncthreads();
    for (int i = tid; i < nv; i += LB) {
        const int c = min(vc[i], DEG);
        for (int a = 1; a < c; ++a) {
            const int v = vl[i][a];
            int b = a - 1;
            while (b >= 0 && vl[i][b] > v) {
                vl[i][b + 1] = vl[i][b];
                --b;
            }
            vl[i][b + 1] = v;
        }
        vc[i] = c;
    }
    __syncthreads();
}

// Stages triangle t: vertex ids, |J|, and either its P quadrature points
// (P <= 3: 3 P doubles) or its vertices (9 doubles).
template <int P>
__device__ __forceinline__ void stage_tri(const LinArgs &A, int t, double *X, int *V, double *jac)
{
    double Y[9];
    *jac = load_tri(A.xyz, A.tri, t, Y, V);
    if constexpr (P <= 3) {
#pragma unroll
        for (int p = 0; p < P; ++p)
#pragma unroll
            for (int d = 0; d < 3; ++d)
                X[3 * p + d] = Y[d] + A.R.s1[p] * (Y[3 + d] - Y[d]) + A.R.s2[p] * (Y[6 + d] - Y[3 + d]);
    } else {
#pragma unroll
        for (int e = 0; e < 9; ++e) X[e] = Y[e];
    }
}

template <int P>
__device__ __forceinline__ void point(const LinArgs &A, const double *X, int p, double *x)
{
    if constexpr (P <= 3) {
#pragma unroll
        for (int d = 0; d < 3; ++d) x[d] = X[3 * p + d];
    } else {
#pragma unroll
        for (int d = 0; d < 3; ++d) x[d] = X[d] + A.R.s1[p] * (X[3 + d] - X[d]) + A.R.s2[p] * (X[6 + d] - X[3 + d]);
    }
}

// The nine corner moments of a pair without a common vertex by the regular
// rule of P points on both triangles (staged points or vertices X, Y),
// without the factor 1 / (4 pi).
template <int P>
__device__ __forceinline__ void regular_moments(const LinArgs &A, const double *X, const double *Y, double *M)
{
    double y[P][3];
#pragma unroll
    for (int q = 0; q < P; ++q) point<P>(A, Y, q, y[q]);
#pragma unroll
    for (int p = 0; p < P; ++p) {
        double x[3];
        point<P>(A, X, p, x);
        double u0 = 0.0, u1 = 0.0, u2 = 0.0;
#pragma unroll
        for (int q = 0; q < P; ++q) {
            const double dx = x[0] - y[q][0], dy = x[1] - y[q][1], dz = x[2] - y[q][2];
            // a pair with a common vertex may give inf / NaN here: such a
            // pair is never stored into a block that is returned
            const double g = rsq<double>(dx * dx + dy * dy + dz * dz);
            u0 += g * A.R.wl[q][0];
            u1 += g * A.R.wl[q][1];
            u2 += g * A.R.wl[q][2];
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            M[3 * a + 0] += A.R.wl[p][a] * u0;
            M[3 * a + 1] += A.R.wl[p][a] * u1;
            M[3 * a + 2] += A.R.wl[p][a] * u2;
        }
    }
}

// Moments M times f into the chunk's slots V[rho * kc + kappa - k0] of the
// row corners rc and column corners cc (-1: not a subset vertex).
__device__ __forceinline__ void store_moments(const double *M, double f, const int *rc, const int *cc, double *V,
                                              int kc, int k0)
{
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int rho = rc[a];
        if (rho < 0) continue;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const int kap = cc[c];
            if (kap >= 0) V[rho * kc + kap - k0] = M[3 * a + c] * f;
        }
    }
}

// EPT block entries per thread (n m <= EPT LB); two workgroups per CU.
// TOUCH = false: every pair by the regular rule; a block with a pair with a
// common vertex is written as zeros with status 1.  TOUCH = true (launched
// after it, on the same stream): only the blocks with status 1, again, the
// touching pairs queued in LDS round by round and integrated by the
// Sauter-Schwab rules, one wavefront per pair.
template <int P, int EPT, bool TOUCH>
__global__ void __launch_bounds__(LB, 2) k_lin_blocks(LinArgs A)
{
    __shared__ double px[2][TMAX][9];      // points (P <= 3) or vertices of every row / column triangle
    __shared__ double jac[2][TMAX];
    __shared__ int tv[2][TMAX][3];
    __shared__ int cmap[2][TMAX][3];       // corner numbers (row corners rho, column corners kappa)
    __shared__ int cbase[TMAX + 1];        // first column corner of each column triangle
    __shared__ int rbase[TMAX + 1];
    __shared__ int vl[2][BSET][DEG];
    __shared__ int vc[2][BSET];
    __shared__ int sh[LB];
    __shared__ double V[MV];               // used moments of a chunk: V[rho * kc + kappa - k0]
    __shared__ int bad, touch;
    __shared__ int qp[TOUCH ? LB : 1];     // queued touching pairs of a round: t << 16 | s
    __shared__ int qn;

    const int b = blockIdx.x, tid = threadIdx.x;
    if (TOUCH && A.status[b] != 1) return;
    const int rs = A.blk_row[b], cs = A.blk_col[b];
    const int n = A.set_off[rs + 1] - A.set_off[rs], m = A.set_off[cs + 1] - A.set_off[cs];
    const int nT = A.m_count[rs], nS = A.m_count[cs];
    const int64_t nm = (int64_t)n * m;
    double *out = A.out + (int64_t)b * A.ld;
    if (n > BSET || m > BSET || nm > EPT * LB || nT < 0 || nS < 0 || nT > TMAX || nS > TMAX) {
        for (int64_t e = tid; e < nm; e += LB) out[e] = 0.0;
        if (tid == 0) A.status[b] = 2;
        return;
    }
    if (tid == 0) {
        bad = 0;
        touch = 0;
        qn = 0;
    }
    const int32_t *rtri = A.m_tri + (int64_t)rs * A.cap, *ctri = A.m_tri + (int64_t)cs * A.cap;
    for (int x = tid; x < nT + nS; x += LB) {
        const int side = x >= nT, t = side ? x - nT : x;
        stage_tri<P>(A, (side ? ctri : rtri)[t], px[side][t], tv[side][t], &jac[side][t]);
    }
    corner_lists(A.m_loc + (int64_t)rs * A.cap * 3, nT, n, cmap[0], rbase, vl[0], vc[0], sh, &bad);
    corner_lists(A.m_loc + (int64_t)cs * A.cap * 3, nS, m, cmap[1], cbase, vl[1], vc[1], sh, &bad);
    const int NR = rbase[nT], NC = cbase[nS];

    double acc[EPT];
    int cp[EPT];
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
        acc[k] = 0.0;
        cp[k] = 0;
    }
    // column corners per chunk: at least one whole triangle (NR <= 3 TMAX)
    const int kmax = NR > 0 ? MV / NR : 3 * TMAX;
    constexpr double inv4pi = 0.07957747154594767;   // 1 / (4 pi)
    for (int s0 = 0; s0 < nS;) {
        // last triangle s1 with cbase[s1] - cbase[s0] <= kmax (same for every thread)
        int lo = s0 + 1, hi = nS;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (cbase[mid] - cbase[s0] <= kmax) lo = mid;
            else hi = mid - 1;
        }
        const int s1 = lo, sc = s1 - s0;
        const int k0 = cbase[s0], kc = cbase[s1] - k0;
        if constexpr (!TOUCH) {
            // pair pi = sl * nT + t, advanced by LB without a division per pair
            const int nt1 = max(nT, 1), dsl = LB / nt1, dt = LB - dsl * nt1;
            int sl = tid / nt1, t = tid - sl * nt1;
            for (int pi = tid; pi < sc * nT; pi += LB, t += dt, sl += dsl) {
                if (t >= nT) {
                    t -= nT;
                    ++sl;
                }
                const int s = s0 + sl;
                bool tch = false;
#pragma unroll
                for (int u = 0; u < 3; ++u)
#pragma unroll
                    for (int v = 0; v < 3; ++v) tch |= tv[0][t][u] == tv[1][s][v];
                if (tch) touch = 1;
                double M[9];
#pragma unroll
                for (int e = 0; e < 9; ++e) M[e] = 0.0;
                regular_moments<P>(A, px[0][t], px[1][s], M);
                store_moments(M, jac[0][t] * jac[1][s] * inv4pi, cmap[0][t], cmap[1][s], V, kc, k0);
            }
        } else {
            const int np = sc * nT, wave = tid >> 6;
            for (int base = 0; base < np; base += LB) {
                const int pi = base + tid;
                if (pi < np) {
                    const int sl = pi / nT, t = pi - sl * nT, s = s0 + sl;
                    bool tch = false;
#pragma unroll
                    for (int u = 0; u < 3; ++u)
#pragma unroll
                        for (int v = 0; v < 3; ++v) tch |= tv[0][t][u] == tv[1][s][v];
                    if (tch) {
                        qp[atomicAdd(&qn, 1)] = t << 16 | s;
                    } else {
                        double M[9];
#pragma unroll
                        for (int e = 0; e < 9; ++e) M[e] = 0.0;
                        regular_moments<P>(A, px[0][t], px[1][s], M);
                        store_moments(M, jac[0][t] * jac[1][s] * inv4pi, cmap[0][t], cmap[1][s], V, kc, k0);
                    }
                }
                __syncthreads();
                const int nq = qn;
                for (int e = wave; e < nq; e += LB / 64) {
                    const int t = qp[e] >> 16, s = qp[e] & 0xFFFF;
                    double M[9];
                    lin_touch_moments(A, tv[0][t], tv[1][s], M);
                    if ((tid & 63) == 0)
                        store_moments(M, jac[0][t] * jac[1][s] * inv4pi, cmap[0][t], cmap[1][s], V, kc, k0);
                }
                __syncthreads();
                if (tid == 0) qn = 0;
                __syncthreads();
            }
        }
        __syncthreads();
        // entries: column corners of vertex j inside this chunk, ascending
#pragma unroll
        for (int k = 0; k < EPT; ++k) {
            const int e = tid + k * LB;
            if (e < nm) {
                const int i = e / m, j = e - i * m;
                double a = acc[k];
                int c = cp[k];
                for (; c < vc[1][j]; ++c) {
                    const int kap = vl[1][j][c] - k0;
                    if (kap >= kc) break;
                    for (int r = 0; r < vc[0][i]; ++r) a += V[vl[0][i][r] * kc + kap];
                }
                acc[k] = a;
                cp[k] = c;
            }
        }
        __syncthreads();
        s0 = s1;
    }
    const int st = bad ? 2 : (touch ? 1 : 0);
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
        const int e = tid + k * LB;
        if (e < nm) out[e] = st ? 0.0 : acc[k];
    }
    if (tid == 0) A.status[b] = st;
}

}  // namespace
}  // namespace gca

using namespace gca;

extern "C" {

gca_status gca_lin_vertex_triangles(const int32_t *tri, int64_t nt, int64_t nv, int32_t *off, int32_t *list)
{
    clear_error();
    if (!tri || !off || (nt > 0 && !list)) return set_error(GCA_EINVAL, "NULL pointer");
    if (nt < 0 || nv < 0 || nt > INT32_MAX / 3 || nv >= INT32_MAX) return set_error(GCA_EINVAL, "nt or nv out of range");
    std::vector<int32_t> cnt(nv + 1, 0);
    for (int64_t t = 0; t < nt; ++t) {
        const int32_t a = tri[3 * t], b = tri[3 * t + 1], c = tri[3 * t + 2];
        if (a < 0 || a >= nv || b < 0 || b >= nv || c < 0 || c >= nv)
            return set_error(GCA_EMESH, "vertex id out of range in triangle " + std::to_string(t));
        if (a == b || b == c || a == c)
            return set_error(GCA_EMESH, "triangle " + std::to_string(t) + " repeats a vertex");
        ++cnt[a + 1];
        ++cnt[b + 1];
        ++cnt[c + 1];
    }
    for (int64_t v = 0; v < nv; ++v) cnt[v + 1] += cnt[v];
    std::memcpy(off, cnt.data(), sizeof(int32_t) * (nv + 1));
    for (int64_t t = 0; t < nt; ++t)
        for (int c = 0; c < 3; ++c) list[cnt[tri[3 * t + c]]++] = (int32_t)t;
    return GCA_OK;
}

gca_status gca_lin_merge(const int32_t *vt_off, const int32_t *vt_list, const int32_t *tri, const int32_t *set_off,
                         const int32_t *set_vtx, int32_t nsets, int32_t cap, int32_t *out_tri, int32_t *out_loc,
                         int32_t *out_count, void *stream)
{
    clear_error();
    if (nsets < 0) return set_error(GCA_EINVAL, "nsets must be >= 0");
    if (cap < 1 || cap > GCA_LIN_MAX_GATHER) return set_error(GCA_EINVAL, "cap out of range");
    if (nsets == 0) return GCA_OK;
    if (!vt_off || !vt_list || !tri || !set_off || !set_vtx || !out_tri || !out_loc || !out_count)
        return set_error(GCA_EINVAL, "NULL pointer");
    hipLaunchKernelGGL(k_lin_merge, dim3(nsets), dim3(LT), 0, (hipStream_t)stream, vt_off, vt_list, tri, set_off,
                       set_vtx, cap, out_tri, out_loc, out_count);
    GCA_HIP_TRY(hipGetLastError());
    return GCA_OK;
}

gca_status gca_lin_blocks(const double *xyz, const int32_t *tri, const int32_t *m_tri, const int32_t *m_loc,
                          const int32_t *m_count, int32_t cap, const int32_t *set_off, const int32_t *blk_row,
                          const int32_t *blk_col, int32_t nblk, int64_t ld, int32_t q, int32_t sym, int32_t q_s,
                          double *out, int32_t *status, void *stream)
{
    clear_error();
    if (nblk < 0 || ld < 0) return set_error(GCA_EINVAL, "nblk and ld must be >= 0");
    if (q_s < 0 || q_s > 32) return set_error(GCA_EINVAL, "q_s must be in [0, 32]");
    if (cap < 1 || cap > GCA_LIN_MAX_GATHER) return set_error(GCA_EINVAL, "cap out of range");
    if (sym != 0 && sym != 1) return set_error(GCA_EINVAL, "sym must be 0 or 1");
    TriRule r;
    if (q < 1 || !tri_rule(q, sym != 0, r) || r.np > 16) return set_error(GCA_EINVAL, "unsupported rule order");
    if (nblk == 0) return GCA_OK;
    if (!xyz || !tri || !m_tri || !m_loc || !m_count || !set_off || !blk_row || !blk_col || !out || !status)
        return set_error(GCA_EINVAL, "NULL pointer");
    LinArgs a{xyz, tri, m_tri, m_loc, m_count, set_off, blk_row, blk_col, cap, ld, out, status, {}};
    for (int p = 0; p < r.np; ++p) {
        a.R.s1[p] = r.s1[p];
        a.R.s2[p] = r.s2[p];
        a.R.wl[p][0] = r.w[p] * (1.0 - r.s1[p]);
        a.R.wl[p][1] = r.w[p] * (r.s1[p] - r.s2[p]);
        a.R.wl[p][2] = r.w[p] * r.s2[p];
    }
    a.qs = q_s;
    if (q_s > 0) gauss_legendre01(q_s, a.gx, a.gw);
    hipStream_t s = (hipStream_t)stream;
    // entries per thread from the caller's stride (ld >= n m of every block)
    const int ept = ld <= 2 * LB ? 2 : (ld <= 4 * LB ? 4 : 8);
    switch (r.np * 16 + ept) {
#define CASE(PP, EE)                                                                          \
    case PP * 16 + EE:                                                                        \
        hipLaunchKernelGGL((k_lin_blocks<PP, EE, false>), dim3(nblk), dim3(LB), 0, s, a);     \
        if (q_s > 0) hipLaunchKernelGGL((k_lin_blocks<PP, EE, true>), dim3(nblk), dim3(LB), 0, s, a); \
        break;
#define CASES(PP) CASE(PP, 2) CASE(PP, 4) CASE(PP, 8)
        CASES(1) CASES(3) CASES(4) CASES(6) CASES(9) CASES(16)
#undef CASES
#undef CASE
    default:
        return set_error(GCA_EINVAL, "unsupported rule size");
    }
    GCA_HIP_TRY(hipGetLastError());
    return GCA_OK;
}

}  // extern "C"
