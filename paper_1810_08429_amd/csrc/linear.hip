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
// Blocks (one workgroup per block): the row subset's merged triangles are
// staged in LDS; the column subset's are taken in chunks.  For every pair
// (t, s) of a chunk one thread evaluates the kernel at the P x P point pairs
// once and forms all nine corner moments
//     M_ab = |J_t| |J_s| / (4 pi) sum_p sum_q w_p lambda_a(x_p) g(x_p, y_q) w_q lambda_b(y_q),
// kept in LDS; every block entry (i, j) then adds M[t][s][a][b] over the rows
// t of its vertex i (corner a) and the rows s of its vertex j (corner b) in a
// fixed order, so the block is reproducible bit for bit without atomics.
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "devfn.h"
#include "gca_internal.h"
#include "gca_linear.h"

namespace gca {
namespace {

constexpr int LT = 256;                          // threads per workgroup
constexpr int LMAX = GCA_LIN_MAX_GATHER;
constexpr int NSET = GCA_LIN_MAX_SET;
constexpr int BSET = GCA_LIN_MAX_BLOCK_SET;
constexpr int TMAX = GCA_LIN_MAX_TRIS;
constexpr int DEG = GCA_LIN_MAX_DEGREE;
constexpr int SCMAX = 16;                        // column triangles per chunk
constexpr int MC = 6144;                         // FP64 moments per chunk (48 KiB)
constexpr int EPT = BSET * BSET / LT;            // block entries per thread
constexpr uint64_t PAD = ~0ull;

// Exclusive prefix sum over the workgroup; *total receives the sum.  Every
// thread must call it.
__device__ int wg_exscan(int v, int *sh, int *total)
{
    const int tid = threadIdx.x;
    sh[tid] = v;
    __syncthreads();
    for (int d = 1; d < LT; d <<= 1) {
        const int add = tid >= d ? sh[tid - d] : 0;
        __syncthreads();
        sh[tid] += add;
        __syncthreads();
    }
    const int incl = sh[tid];
    *total = sh[LT - 1];
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
};

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

// Append corner entries (row * 3 + corner) of a merged list to the per-vertex
// lists, then sort each list so that the reduction order is fixed.  Returns
// through *bad when a vertex has more than DEG rows.
__device__ void vertex_lists(const int32_t *loc, int nrow, int nv, int (*vl)[DEG], int *vc, int *bad)
{
    const int tid = threadIdx.x;
    for (int i = tid; i < nv; i += LT) vc[i] = 0;
    __syncthreads();
    for (int x = tid; x < 3 * nrow; x += LT) {
        const int l = loc[x];
        if (l >= 0 && l < nv) {
            const int p = atomicAdd(&vc[l], 1);
            if (p < DEG) vl[l][p] = x;
            else *bad = 1;
        } else if (l >= nv) {
            *bad = 1;
        }
    }
    __syncthreads();
    for (int i = tid; i < nv; i += LT) {
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

template <int P>
__global__ void __launch_bounds__(LT) k_lin_blocks(LinArgs A)
{
    __shared__ double px_r[TMAX][9];
    __shared__ double jac_r[TMAX];
    __shared__ int tv_r[TMAX][3];
    __shared__ double px_c[SCMAX][9];
    __shared__ double jac_c[SCMAX];
    __shared__ int tv_c[SCMAX][3];
    __shared__ int vl[2][BSET][DEG];
    __shared__ int vc[2][BSET];
    __shared__ double mc[MC];
    __shared__ int bad, touch;

    const int b = blockIdx.x, tid = threadIdx.x;
    const int rs = A.blk_row[b], cs = A.blk_col[b];
    const int n = A.set_off[rs + 1] - A.set_off[rs], m = A.set_off[cs + 1] - A.set_off[cs];
    const int nT = A.m_count[rs], nS = A.m_count[cs];
    const int64_t nm = (int64_t)n * m;
    double *out = A.out + (int64_t)b * A.ld;
    if (n > BSET || m > BSET || nT < 0 || nS < 0 || nT > TMAX || nS > TMAX) {
        for (int64_t e = tid; e < nm; e += LT) out[e] = 0.0;
        if (tid == 0) A.status[b] = 2;
        return;
    }
    if (tid == 0) {
        bad = 0;
        touch = 0;
    }
    const int32_t *rtri = A.m_tri + (int64_t)rs * A.cap, *ctri = A.m_tri + (int64_t)cs * A.cap;
    for (int t = tid; t < nT; t += LT) jac_r[t] = load_tri(A.xyz, A.tri, rtri[t], px_r[t], tv_r[t]);
    __syncthreads();
    vertex_lists(A.m_loc + (int64_t)rs * A.cap * 3, nT, n, vl[0], vc[0], &bad);
    vertex_lists(A.m_loc + (int64_t)cs * A.cap * 3, nS, m, vl[1], vc[1], &bad);

    double acc[EPT];
    int cp[EPT];
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
        acc[k] = 0.0;
        cp[k] = 0;
    }
    const int sc_max = max(1, min(SCMAX, MC / (9 * max(nT, 1))));
    constexpr double inv4pi = 0.07957747154594767;   // 1 / (4 pi)
    for (int s0 = 0; s0 < nS; s0 += sc_max) {
        const int sc = min(sc_max, nS - s0);
        for (int sl = tid; sl < sc; sl += LT) jac_c[sl] = load_tri(A.xyz, A.tri, ctri[s0 + sl], px_c[sl], tv_c[sl]);
        __syncthreads();
        // pair moments of this chunk: index sl * nT + t
        for (int pi = tid; pi < sc * nT; pi += LT) {
            const int sl = pi / nT, t = pi - sl * nT;
            bool tch = false;
#pragma unroll
            for (int u = 0; u < 3; ++u)
#pragma unroll
                for (int v = 0; v < 3; ++v) tch |= tv_r[t][u] == tv_c[sl][v];
            if (tch) touch = 1;
            const double *X = px_r[t], *Y = px_c[sl];
            double y[P][3];
#pragma unroll
            for (int q = 0; q < P; ++q)
#pragma unroll
                for (int d = 0; d < 3; ++d)
                    y[q][d] = Y[d] + A.R.s1[q] * (Y[3 + d] - Y[d]) + A.R.s2[q] * (Y[6 + d] - Y[3 + d]);
            double M[9];
#pragma unroll
            for (int e = 0; e < 9; ++e) M[e] = 0.0;
#pragma unroll
            for (int p = 0; p < P; ++p) {
                double x[3];
#pragma unroll
                for (int d = 0; d < 3; ++d)
                    x[d] = X[d] + A.R.s1[p] * (X[3 + d] - X[d]) + A.R.s2[p] * (X[6 + d] - X[3 + d]);
                double u0 = 0.0, u1 = 0.0, u2 = 0.0;
#pragma unroll
                for (int q = 0; q < P; ++q) {
                    const double dx = x[0] - y[q][0], dy = x[1] - y[q][1], dz = x[2] - y[q][2];
                    const double r2 = dx * dx + dy * dy + dz * dz;
                    const double g = tch ? 0.0 : rsq<double>(r2);
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
            const double f = jac_r[t] * jac_c[sl] * inv4pi;
#pragma unroll
            for (int e = 0; e < 9; ++e) mc[9 * pi + e] = M[e] * f;
        }
        __syncthreads();
        // entries: rows of column vertex j inside this chunk, in ascending order
#pragma unroll
        for (int k = 0; k < EPT; ++k) {
            const int e = tid + k * LT;
            if (e < nm) {
                const int i = e / m, j = e - i * m;
                double a = acc[k];
                int c = cp[k];
                for (; c < vc[1][j]; ++c) {
                    const int s3 = vl[1][j][c];
                    const int s = s3 / 3 - s0;
                    if (s >= sc) break;
                    const int bb = s3 - 3 * (s3 / 3);
                    for (int r = 0; r < vc[0][i]; ++r) {
                        const int t3 = vl[0][i][r];
                        const int t = t3 / 3, aa = t3 - 3 * t;
                        a += mc[9 * (s * nT + t) + 3 * aa + bb];
                    }
                }
                acc[k] = a;
                cp[k] = c;
            }
        }
        __syncthreads();
    }
    const int st = bad ? 2 : (touch ? 1 : 0);
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
        const int e = tid + k * LT;
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
                          const int32_t *blk_col, int32_t nblk, int64_t ld, int32_t q, int32_t sym, double *out,
                          int32_t *status, void *stream)
{
    clear_error();
    if (nblk < 0 || ld < 0) return set_error(GCA_EINVAL, "nblk and ld must be >= 0");
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
    hipStream_t s = (hipStream_t)stream;
    switch (r.np) {
#define CASE(PP)                                                                    \
    case PP:                                                                        \
        hipLaunchKernelGGL(k_lin_blocks<PP>, dim3(nblk), dim3(LT), 0, s, a);        \
        break;
        CASE(1) CASE(3) CASE(4) CASE(6) CASE(9) CASE(16)
#undef CASE
    default:
        return set_error(GCA_EINVAL, "unsupported rule size");
    }
    GCA_HIP_TRY(hipGetLastError());
    return GCA_OK;
}

}  // extern "C"
