// Triangle-pair quadrature on gfx950: the Galerkin entries
//     g_ij = int_{t_i} int_{t_j} 1 / (4 pi |x - y|) dy dx          (Eq. G_def)
// for piecewise-constant bases, evaluated in bulk for
//   - inadmissible leaf blocks G|t^ x s^ and coupling blocks G|t~ x s~
//     (LDS-tiled block-row kernels; entries are recomputed and immediately
//     multiplied, Section 8's second and third task), and
//   - one list per Sauter case (identical, common edge, common vertex) plus,
//     when near-regular pairs get their own order, a list of those (Section
//     8: one list per case so that a wavefront never diverges between rules).
//
// Reference triangle T = {0 <= s2 <= s1 <= 1}, chi(s) = P0 + s1 (P1 - P0) +
// s2 (P2 - P1).  Regular pairs use a collapsed Gauss rule of order q on each
// triangle (precomputed per triangle as points and weights times 2|t|).
// Touching pairs use the Sauter-Schwab regularising maps of [0,1]^4 with the
// factors that are polynomial in the variables integrated exactly: for a flat
// pair and the 1/r kernel the integrand of every region is xi^2 eta1 (or
// xi^2 eta1 eta2) times a function of the remaining variables, so the
// identical case reduces to three 1D integrals, the common-edge case to five
// 2D and the common-vertex case to two 3D integrals (Gauss order q_s >= 2
// integrates the removed polynomial factors exactly, so the values equal the
// full 4D tensor rule up to rounding).
#include <hip/hip_runtime.h>

#include "gca_internal.h"
#include "devfn.h"
#include "mfma.h"

namespace gca {

#define INV4PI 0.07957747154594766788

struct GaussQ {
    double x[32], w[32];
    int q;
};

// ------------------------------------------------------ block kernels ------
// Nearfield blocks G|t^ x s^ and coupling blocks G|t~ x s~ are recomputed in
// every product and multiplied at once (Section 8's second and third task).
// A workgroup (256 threads = 4 wavefronts) takes one block row: a row
// cluster and the concatenated columns of all its blocks of the symmetric
// half.  Point sets are staged in LDS relative to a reference point (FP64
// subtract, then rounding to T), so FP32 keeps the relative accuracy of short
// distances.  Entries are computed in wavefront tiles of R x C = 64 lanes and
// multiplied at once: g_ij x_j is summed over the C lanes of a tile row and
// g_ij x_i over the R lanes of a tile column by cross-lane shuffles, then
// added to row and column accumulators that each wavefront owns in LDS.
// Deterministic: a fixed tile order per wavefront, fixed reduction orders, no
// atomics, one writer per partial.
constexpr int BLK_THREADS = 256;
constexpr int BLK_WAVES = BLK_THREADS / 64;

template <typename T>
struct alignas(4 * sizeof(T)) Q4 {
    T x, y, z, w;
};


__host__ __device__ constexpr size_t al16(size_t b) { return (b + 15) & ~(size_t)15; }

// LDS layout of the block kernel (byte offsets, 16-byte aligned sections):
//   mask[rmax] u64 (NEAR) | rowp[rmax][P] Q4 | rown[rmax][P] |
//   colp[CW][P] Q4 | coln[CW][P] | xr[rmax] | xc[CW] |
//   racc[4][rmax] | cacc[4][CW]
// rown / coln are the squared norms of the expanded distance
// |x - y|^2 = |x|^2 + |y|^2 - 2 x.y.
template <typename T>
struct BlkLayout {
    size_t mask, rowp, rown, colp, coln, xr, xc, racc, cacc, total;
    __host__ __device__ BlkLayout(int rmax, int P, int CW, bool near)
    {
        mask = 0;
        rowp = mask + (near ? al16((size_t)rmax * 8) : 0);
        rown = rowp + al16((size_t)rmax * P * sizeof(Q4<T>));
        colp = rown + al16((size_t)rmax * P * sizeof(T));
        coln = colp + al16((size_t)CW * P * sizeof(Q4<T>));
        xr = coln + al16((size_t)CW * P * sizeof(T));
        xc = xr + al16((size_t)rmax * sizeof(T));
        racc = xc + al16((size_t)CW * sizeof(T));
        cacc = racc + al16((size_t)BLK_WAVES * rmax * sizeof(T));
        total = cacc + al16((size_t)BLK_WAVES * CW * sizeof(T));
    }
};

template <typename T>
__device__ __forceinline__ T fmat(T a, T b, T c);
template <>
__device__ __forceinline__ float fmat<float>(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
template <>
__device__ __forceinline__ double fmat<double>(double a, double b, double c) { return __builtin_fma(a, b, c); }

// sum over the collapsed rules of both triangles of w_a w_b / |x_a - y_b|,
// row points and their squared norms in registers, column points (scaled by
// -2) and their squared norms from LDS:
//     |x_a - y_b|^2 = (|x_a|^2 + |y_b|^2) + x_a . (-2 y_b)
// one add and three FMAs per point pair.  All coordinates are relative to
// the row cluster's box centre, so the cancellation is bounded by
// (|x|^2 + |y|^2) / |x - y|^2, a few hundred at most for the regular pairs of
// nearfield blocks and far less for admissible ones.
template <typename T, int P>
__device__ __forceinline__ T block_entry(const Q4<T> (&rp)[P], const T (&rn)[P], const Q4<T> *cp, const T *cn)
{
    T acc = 0;
    auto column_point = [&](int pb) {
        const Q4<T> c = cp[pb];
        const T ny = cn[pb];
        T inner = 0;
#pragma unroll
        for (int pa = 0; pa < P; ++pa) {
            T r2 = rn[pa] + ny;
            r2 = fmat(rp[pa].z, c.z, r2);
            r2 = fmat(rp[pa].y, c.y, r2);
            r2 = fmat(rp[pa].x, c.x, r2);
            inner = fmat(rp[pa].w, rsq<T>(r2), inner);
        }
        acc = fmat(c.w, inner, acc);
    };
    // rules up to 3 x 3 points fully unrolled; larger ones keep the column
    // loop (code size)
    if constexpr (P <= 9) {
#pragma unroll
        for (int pb = 0; pb < P; ++pb) column_point(pb);
    } else {
#pragma unroll 1
        for (int pb = 0; pb < P; ++pb) column_point(pb);
    }
    return acc;
}

// Sum over the lanes congruent modulo S (S = 1 .. 32); every lane receives
// the sum of its class.  Within a row of 16 the class is rotated through
// (row_ror by 8, 4, .., S), then lane ^ 16 and lane ^ 32 join the rows.
template <int S, typename T>
__device__ __forceinline__ T class_sum(T v, int lane)
{
    if constexpr (S <= 8) v += dpp_mov<0x128>(v);   // row_ror:8
    if constexpr (S <= 4) v += dpp_mov<0x124>(v);   // row_ror:4
    if constexpr (S <= 2) v += dpp_mov<0x122>(v);   // row_ror:2
    if constexpr (S <= 1) v += dpp_mov<0x121>(v);   // row_ror:1
    if constexpr (S <= 16) v += xor16_mov(v);
    v += xor32_mov(v, (lane ^ 32) << 2);
    return v;
}

// One pass over the entries of an rw x cw chunk (rows in rowp/rown, columns
// in colp/coln, both in LDS): tiles of R rows x C columns = 64 lanes (C = 8
// or 16 picked for the fewest tile rounds over the 4 wavefronts, then the
// fewest tiles).  Without a mask each wavefront takes a contiguous run of the
// row-major tile list; masked passes interleave the tiles over the
// wavefronts, so that fully masked tiles (skipped at no cost) are spread
// evenly.  Either way consecutive tiles of a wavefront mostly share their
// rows, which stay in registers until the tile row changes.
//
// The lanes of a tile column are R consecutive lanes (row ii = lane % R):
// entry g_ij adds g_ij x_i to the column sum, reduced over those lanes by
// DPP and added to cacc[j] once per tile, and g_ij x_j to a per-lane row sum
// that stays in a register while the tile row is unchanged and is reduced
// over the C lanes of the row (lanes congruent modulo R) into racc[i] when it
// changes.  racc and cacc belong to the calling wavefront.  MASK skips the
// pairs whose bit c0 + j is set in mask[i].  STORE writes the entries
// (masked ones as zeros) to st[i * ld + j] instead, with the columns on
// consecutive lanes.
template <typename T, int P, bool MASK, bool STORE, int LC>
__device__ __forceinline__ void tile_loop(int rw, int cw, int c0, const Q4<T> *rowp, const T *rown,
                                          const Q4<T> *colp, const T *coln, const T *xr, const T *xc,
                                          const uint64_t *mask, T *racc, T *cacc, T *st, int64_t ld, int k0,
                                          int k1, int kstep)
{
    constexpr int C = 1 << LC, R = 64 >> LC;
    const int lane = threadIdx.x & 63;
    const int ii = STORE ? lane >> LC : lane & (R - 1);
    const int jj = STORE ? lane & (C - 1) : lane >> (6 - LC);
    const int nct = (cw + C - 1) >> LC;
    Q4<T> rr[P];
    T rq[P];
    T vacc = 0;
    uint64_t mrow = 0;   // MASK: the lane's row mask word, loaded with the row
    int cur_tr = -1;
    // tile coordinates are wavefront-uniform
    int tr = k0 / nct, tc = k0 - tr * nct;
    auto flush_rows = [&]() {
        const T v = class_sum<R>(vacc, lane);
        const int i = cur_tr * R + ii;
        if (jj == 0 && i < rw) racc[i] += v;
    };
    for (int k = k0; k < k1; k += kstep) {
        const int i = tr * R + ii, j = tc * C + jj;
        if (tr != cur_tr) {
            if (!STORE && cur_tr >= 0) flush_rows();
            vacc = 0;
            cur_tr = tr;
            const int il = min(i, rw - 1);
#pragma unroll
            for (int p = 0; p < P; ++p) {
                rr[p] = rowp[(size_t)il * P + p];
                rq[p] = rown[(size_t)il * P + p];
            }
            if (MASK) mrow = mask[il];
        }
        const bool valid = i < rw && j < cw;
        if (STORE) {
            T g = 0;
            if (valid && !(MASK && ((mrow >> (c0 + j)) & 1)))
                g = block_entry<T, P>(rr, rq, colp + (size_t)j * P, coln + (size_t)j * P) * (T)INV4PI;
            if (valid) st[(int64_t)i * ld + j] = g;
        } else {
            T u = 0;
            if (valid && !(MASK && ((mrow >> (c0 + j)) & 1))) {
                const T g = block_entry<T, P>(rr, rq, colp + (size_t)j * P, coln + (size_t)j * P) * (T)INV4PI;
                vacc = fmat(g, xc[j], vacc);
                u = g * xr[i];
            }
            u = group_sum<R>(u);
            if (ii == 0 && j < cw) cacc[j] += u;
        }
        tc += kstep;
        while (tc >= nct) {
            tc -= nct;
            ++tr;
        }
    }
    if (!STORE && cur_tr >= 0) flush_rows();
}

template <typename T, int P, bool MASK, bool STORE>
__device__ __forceinline__ void tile_pass(int rw, int cw, int c0, const Q4<T> *rowp, const T *rown,
                                          const Q4<T> *colp, const T *coln, const T *xr, const T *xc,
                                          const uint64_t *mask, T *racc, T *cacc, T *st, int64_t ld)
{
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    int lc = 0, best_r = 1 << 30, best_n = 1 << 30;
    for (int l = 3; l <= 4; ++l) {
        const int R = 64 >> l;
        const int n = ((rw + R - 1) / R) * ((cw + (1 << l) - 1) >> l);
        const int rounds = (n + BLK_WAVES - 1) / BLK_WAVES;
        if (rounds < best_r || (rounds == best_r && n < best_n)) {
            best_r = rounds;
            best_n = n;
            lc = l;
        }
    }
    const int k0 = MASK ? wv : (wv * best_n) / BLK_WAVES;
    const int k1 = MASK ? best_n : ((wv + 1) * best_n) / BLK_WAVES;
    const int kstep = MASK ? BLK_WAVES : 1;
    // C = 8 or 16 (R = 8 or 4): the two shapes cover the leaf and rank sizes
    // of the block rows; narrower or wider tiles are not instantiated
    switch (lc) {
#define TL(L)                                                                                                  \
    case L:                                                                                                   \
        tile_loop<T, P, MASK, STORE, L>(rw, cw, c0, rowp, rown, colp, coln, xr, xc, mask, racc, cacc, st, ld, k0, \
                                        k1, kstep);                                                           \
        break;
        TL(3) TL(4)
#undef TL
    }
}

// Wavefronts per SIMD the block kernels are compiled for: as many as the
// registers of a tile allow without spilling (the row points of a lane take
// 5 P values; 512 / waves VGPRs per lane), at most 6 (FP32 nearfield), 5
// (FP32 coupling; 6 spills at 4 points) or 3 (FP64).  Measured on the
// level-8 sphere: FP32 3x3 nearfield 3.98 ms with the compiler's own choice
// (103 VGPRs), 3.46 ms at 5, 3.79 ms at 6; FP32 6-point nearfield 1.81 ms at
// 5, 1.70 ms at 6; FP64 3x3 nearfield 9.15 ms at 4 (88 bytes of spills),
// 8.91 ms at 3, 8.82 ms at 2.
constexpr int blk_waves(int word_bytes, int P, int base, int cap)
{
    const int need = 5 * P * (word_bytes / 4) + base;
    const int w = 512 / need;
    return w < 1 ? 1 : (w > cap ? cap : w);
}
template <typename T, int P>
constexpr int near_waves() { return blk_waves((int)sizeof(T), P, 48, sizeof(T) == 8 ? 3 : 6); }
template <typename T, int P>
constexpr int far_waves() { return blk_waves((int)sizeof(T), P, 64, sizeof(T) == 8 ? 3 : 5); }

// ------------------------------------------------ coupling block rows ------
// One workgroup per row cluster t with coupling blocks (t, s), t < s (a block
// row of the symmetric half).  The columns of all its blocks are concatenated
// -- column k is pivot entry col_e[k] of cluster col_s[k] -- so the row points
// are staged once and the tiles of the whole block row are balanced over the
// workgroup.  Row partials  sum_k g_ik x_k  go to part[g_rslot + i], the
// column partial of column k to part[col_out[k]] (one writer each).
// Coordinates are taken relative to the centre c_t of t's box.  The FP32 path
// reads the pivots' points from pq32, stored relative to their own
// cluster's centre, and shifts the columns by c_s - c_t (FP64 difference,
// rounded once); admissibility keeps |x - y| >= dist(t, s) >= diam / (2 eta),
// so the cancellation in |x|^2 + |y|^2 - 2 x.y stays within a few dozen FP32
// ulps of |x - y|^2.
template <typename T>
struct FarArgs {
    const int32_t *g_t;       // ng: row cluster of each group
    const int64_t *g_ptr;     // ng + 1: column range of each group
    const int64_t *g_rslot;   // ng: first row-partial slot
    const int32_t *col_e;     // pivot entry (piv_off[s] + j) of each column
    const int32_t *col_s;     // cluster of each column
    const int64_t *col_out;   // column-partial slot of each column
    const int32_t *rank;
    const int64_t *piv_off;
    const int32_t *piv;       // FP64 path: pivot positions
    const double *box;        // nc x 8
    const double *q;          // FP64 path: n x P x 4
    const float *pq32;        // FP32 path: sum(rank) x P x 4
    const T *xh;
    T *part;
    T *store;                 // STORE: entries, row-major per group at g_soff
    const int64_t *g_soff;
    int ng;
    int rmax;
    int cw;
};

template <typename T, int P, bool STORE>
__global__ void __launch_bounds__(BLK_THREADS, (far_waves<T, P>()))
    k_far_rows(FarArgs<T> a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr bool F32 = sizeof(T) == 4;
    const int g = blockIdx.x;
    const int tid = threadIdx.x, wv = tid >> 6;
    const int t = a.g_t[g];
    const int64_t kb = a.g_ptr[g];
    const int nc = (int)(a.g_ptr[g + 1] - kb);
    const int nr = a.rank[t];
    const int64_t xro = a.piv_off[t];
    const int64_t rslot = a.g_rslot[g];
    const int rmax = a.rmax, CW = a.cw;
    const BlkLayout<T> L(rmax, P, CW, false);
    Q4<T> *rowp = reinterpret_cast<Q4<T> *>(smem + L.rowp);
    T *rown = reinterpret_cast<T *>(smem + L.rown);
    Q4<T> *colp = reinterpret_cast<Q4<T> *>(smem + L.colp);
    T *coln = reinterpret_cast<T *>(smem + L.coln);
    T *xr = reinterpret_cast<T *>(smem + L.xr);
    T *xc = reinterpret_cast<T *>(smem + L.xc);
    T *racc = reinterpret_cast<T *>(smem + L.racc);
    T *cacc = reinterpret_cast<T *>(smem + L.cacc);
    const double cx = 0.5 * (a.box[8 * t + 0] + a.box[8 * t + 3]);
    const double cy = 0.5 * (a.box[8 * t + 1] + a.box[8 * t + 4]);
    const double cz = 0.5 * (a.box[8 * t + 2] + a.box[8 * t + 5]);

    for (int e = tid; e < BLK_WAVES * rmax; e += BLK_THREADS) racc[e] = 0;
    for (int e = tid; e < BLK_WAVES * CW; e += BLK_THREADS) cacc[e] = 0;
    for (int r0 = 0; r0 < nr; r0 += rmax) {
        const int rw = min(rmax, nr - r0);
        if (r0 > 0) __syncthreads();
        for (int e = tid; e < rw * P; e += BLK_THREADS) {
            const int i = e / P, p = e - i * P;
            if (F32) {
                const float4 v = reinterpret_cast<const float4 *>(a.pq32)[(size_t)(xro + r0 + i) * P + p];
                rowp[e] = Q4<T>{(T)v.x, (T)v.y, (T)v.z, (T)v.w};
                rown[e] = (T)(v.x * v.x + v.y * v.y + v.z * v.z);
            } else {
                const double *src = a.q + ((size_t)a.piv[xro + r0 + i] * P + p) * 4;
                const T x = (T)(src[0] - cx), y = (T)(src[1] - cy), z = (T)(src[2] - cz);
                rowp[e] = Q4<T>{x, y, z, (T)src[3]};
                rown[e] = x * x + y * y + z * z;
            }
        }
        // the store variant gets no vectors (xh is null there)
        if (!STORE)
            for (int i = tid; i < rw; i += BLK_THREADS) xr[i] = a.xh[xro + r0 + i];
        for (int c0 = 0; c0 < nc; c0 += CW) {
            const int cw = min(CW, nc - c0);
            __syncthreads();
            for (int e = tid; e < cw * P; e += BLK_THREADS) {
                const int j = e / P, p = e - j * P;
                const int64_t k = kb + c0 + j;
                const int ce = a.col_e[k];
                if (F32) {
                    const int cs = a.col_s[k];
                    const float ox = (float)(0.5 * (a.box[8 * cs + 0] + a.box[8 * cs + 3]) - cx);
                    const float oy = (float)(0.5 * (a.box[8 * cs + 1] + a.box[8 * cs + 4]) - cy);
                    const float oz = (float)(0.5 * (a.box[8 * cs + 2] + a.box[8 * cs + 5]) - cz);
                    const float4 v = reinterpret_cast<const float4 *>(a.pq32)[(size_t)ce * P + p];
                    const float y0 = v.x + ox, y1 = v.y + oy, y2 = v.z + oz;
                    colp[e] = Q4<T>{(T)(-2 * y0), (T)(-2 * y1), (T)(-2 * y2), (T)v.w};
                    coln[e] = (T)(y0 * y0 + y1 * y1 + y2 * y2);
                } else {
                    const double *src = a.q + ((size_t)a.piv[ce] * P + p) * 4;
                    const T y0 = (T)(src[0] - cx), y1 = (T)(src[1] - cy), y2 = (T)(src[2] - cz);
                    colp[e] = Q4<T>{-2 * y0, -2 * y1, -2 * y2, (T)src[3]};
                    coln[e] = y0 * y0 + y1 * y1 + y2 * y2;
                }
            }
            if (!STORE)
                for (int j = tid; j < cw; j += BLK_THREADS) xc[j] = a.xh[a.col_e[kb + c0 + j]];
            __syncthreads();
            tile_pass<T, P, false, STORE>(rw, cw, 0, rowp, rown, colp, coln, xr, xc, nullptr, racc + wv * rmax,
                                               cacc + wv * CW,
                                               STORE ? a.store + a.g_soff[g] + (int64_t)r0 * nc + c0 : nullptr, nc);
            __syncthreads();
            if (STORE) continue;
            for (int j = tid; j < cw; j += BLK_THREADS) {
                T c = 0;
#pragma unroll
                for (int w = 0; w < BLK_WAVES; ++w) {
                    c += cacc[w * CW + j];
                    cacc[w * CW + j] = 0;
                }
                const int64_t o = a.col_out[kb + c0 + j];
                if (r0 == 0)
                    a.part[o] = c;
                else
                    a.part[o] += c;
            }
        }
        if (STORE) continue;
        for (int i = tid; i < rw; i += BLK_THREADS) {
            T r = 0;
#pragma unroll
            for (int w = 0; w < BLK_WAVES; ++w) {
                r += racc[w * rmax + i];
                racc[w * rmax + i] = 0;
            }
            a.part[rslot + r0 + i] = r;
        }
    }
}

// ------------------------------------------------ nearfield block rows -----
// One workgroup per leaf t with nearfield blocks (t, s), t <= s: the columns of
// all its blocks are concatenated (diagonal block first), the row points are
// staged once and the tiles of the whole block row are balanced over the
// workgroup.  Pairs listed in the row CSR (touching pairs, and near-regular
// pairs when they have their own order) and the lower triangle of the
// diagonal block are skipped by a precomputed mask, one word per row and
// chunk of NEAR_CW columns, so every unordered pair is evaluated once.  Row
// partials go to part[g_rslot + i], the column partial of column k to
// part[col_out[k]].  Coordinates relative to the centre of t's box (FP64
// subtract, then rounding to T).
template <typename T>
struct NearArgs {
    const int32_t *g_t;
    const int64_t *g_ptr;
    const int64_t *g_rslot;
    const int64_t *g_moff;
    const int32_t *col_pos;
    const int64_t *col_out;
    const uint64_t *mask;
    const int32_t *node;      // nc x 5
    const double *box;        // nc x 8
    const double *q;          // n x P x 4 (FP64 path)
    const double *cent;       // FP32 path: n x 4, reference point of each triangle
    const float *qloc;        // FP32 path: n x P x 4, points relative to it (x, y, z, w)
    const T *xp;              // permuted x
    T *part;
    T *store;                 // STORE: entries, row-major per group at g_soff
    const int64_t *g_soff;
    int ng;
    int rmax;                 // >= largest leaf
    int cw;                   // column sub-chunk (divides NEAR_CW)
};

template <typename T, int P, bool STORE>
__global__ void __launch_bounds__(BLK_THREADS, (near_waves<T, P>()))
    k_near_rows(NearArgs<T> a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int CW = a.cw;
    const int g = blockIdx.x;
    const int tid = threadIdx.x, wv = tid >> 6;
    const int t = a.g_t[g];
    const int64_t kb = a.g_ptr[g];
    const int nc = (int)(a.g_ptr[g + 1] - kb);
    const int rb = a.node[5 * t + 0], nr = a.node[5 * t + 1] - rb;
    const int64_t rslot = a.g_rslot[g];
    const uint64_t *gm = a.mask + a.g_moff[g];
    const int rmax = a.rmax;
    // expanded distances around t's box centre in both precisions; the FP32
    // points are formed from each triangle's reference point (FP64 offset to
    // the centre, rounded once) plus its FP32 local points
    const BlkLayout<T> L(rmax, P, CW, true);
    uint64_t *mask = reinterpret_cast<uint64_t *>(smem + L.mask);
    Q4<T> *rowp = reinterpret_cast<Q4<T> *>(smem + L.rowp);
    T *rown = reinterpret_cast<T *>(smem + L.rown);
    Q4<T> *colp = reinterpret_cast<Q4<T> *>(smem + L.colp);
    T *coln = reinterpret_cast<T *>(smem + L.coln);
    T *xr = reinterpret_cast<T *>(smem + L.xr);
    T *xc = reinterpret_cast<T *>(smem + L.xc);
    T *racc = reinterpret_cast<T *>(smem + L.racc);
    T *cacc = reinterpret_cast<T *>(smem + L.cacc);
    const double cx = 0.5 * (a.box[8 * t + 0] + a.box[8 * t + 3]);
    const double cy = 0.5 * (a.box[8 * t + 1] + a.box[8 * t + 4]);
    const double cz = 0.5 * (a.box[8 * t + 2] + a.box[8 * t + 5]);
    // point p of triangle `pos` relative to t's box centre, and its weight
    auto point = [&](int pos, int p) {
        if constexpr (sizeof(T) == 4) {
            const double *c = a.cent + 4 * (size_t)pos;
            const float4 v = reinterpret_cast<const float4 *>(a.qloc)[(size_t)pos * P + p];
            return Q4<T>{(T)(c[0] - cx) + v.x, (T)(c[1] - cy) + v.y, (T)(c[2] - cz) + v.z, v.w};
        } else {
            const double *src = a.q + ((size_t)pos * P + p) * 4;
            return Q4<T>{src[0] - cx, src[1] - cy, src[2] - cz, src[3]};
        }
    };

    for (int e = tid; e < BLK_WAVES * rmax; e += BLK_THREADS) racc[e] = 0;
    for (int e = tid; e < BLK_WAVES * CW; e += BLK_THREADS) cacc[e] = 0;
    for (int e = tid; e < nr * P; e += BLK_THREADS) {
        const int i = e / P, p = e - i * P;
        const Q4<T> v = point(rb + i, p);
        rowp[e] = v;
        rown[e] = v.x * v.x + v.y * v.y + v.z * v.z;
    }
    // the store variant gets no vectors (xp is null there)
    if (!STORE)
        for (int i = tid; i < nr; i += BLK_THREADS) xr[i] = a.xp[rb + i];
    for (int c0 = 0; c0 < nc; c0 += CW) {
        const int cw = min(CW, nc - c0);
        const int ch = c0 / NEAR_CW, cb = c0 - ch * NEAR_CW;   // mask word and bit offset
        __syncthreads();
        for (int e = tid; e < cw * P; e += BLK_THREADS) {
            const int j = e / P, p = e - j * P;
            const Q4<T> v = point(a.col_pos[kb + c0 + j], p);
            colp[e] = Q4<T>{-2 * v.x, -2 * v.y, -2 * v.z, v.w};
            coln[e] = v.x * v.x + v.y * v.y + v.z * v.z;
        }
        if (!STORE)
            for (int j = tid; j < cw; j += BLK_THREADS) xc[j] = a.xp[a.col_pos[kb + c0 + j]];
        for (int i = tid; i < nr; i += BLK_THREADS) mask[i] = gm[(size_t)ch * nr + i];
        __syncthreads();
        tile_pass<T, P, true, STORE>(nr, cw, cb, rowp, rown, colp, coln, xr, xc, mask, racc + wv * rmax,
                                           cacc + wv * CW, STORE ? a.store + a.g_soff[g] + c0 : nullptr, nc);
        __syncthreads();
        if (STORE) continue;
        for (int j = tid; j < cw; j += BLK_THREADS) {
            T c = 0;
#pragma unroll
            for (int w = 0; w < BLK_WAVES; ++w) {
                c += cacc[w * CW + j];
                cacc[w * CW + j] = 0;
            }
            a.part[a.col_out[kb + c0 + j]] = c;
        }
    }
    if (STORE) return;
    for (int i = tid; i < nr; i += BLK_THREADS) {
        T r = 0;
#pragma unroll
        for (int w = 0; w < BLK_WAVES; ++w) r += racc[w * rmax + i];
        a.part[rslot + i] = r;
    }
}

// Reference point of every triangle (the mean of its regular-rule points, FP64)
// and the points relative to it (FP64 subtract, one rounding to FP32), for
// the FP32 nearfield blocks.
__global__ void k_local_points(const double *q, int P, int64_t n, double *cent, float *qloc)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double *src = q + (size_t)i * P * 4;
    double c[3] = {0, 0, 0};
    for (int p = 0; p < P; ++p)
        for (int d = 0; d < 3; ++d) c[d] += src[4 * p + d];
    for (int d = 0; d < 3; ++d) c[d] /= P;
    for (int d = 0; d < 3; ++d) cent[4 * i + d] = c[d];
    cent[4 * i + 3] = 0;
    for (int p = 0; p < P; ++p) {
        float4 v;
        v.x = (float)(src[4 * p + 0] - c[0]);
        v.y = (float)(src[4 * p + 1] - c[1]);
        v.z = (float)(src[4 * p + 2] - c[2]);
        v.w = (float)src[4 * p + 3];
        reinterpret_cast<float4 *>(qloc)[(size_t)i * P + p] = v;
    }
}

hipError_t launch_local_points(gca_h2_s *h, hipStream_t s)
{
    const int P = h->P_r;
    hipLaunchKernelGGL(k_local_points, dim3((unsigned)((h->n + 127) / 128)), dim3(128), 0, s, h->d_qr, P, h->n,
                       h->d_cent, h->d_qloc32);
    return hipGetLastError();
}

// FP32 copies of the pivots' quadrature points relative to their cluster's
// centre (FP64 subtract, one rounding): entry e = piv_off[c] + k of cluster c.
__global__ void k_pivot_points(const int32_t *piv_cluster, const int32_t *piv, const double *box, const double *q,
                               int P, int64_t n_entries, float *out)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n_entries * P) return;
    const int64_t k = e / P;
    const int p = (int)(e - k * P);
    const int c = piv_cluster[k];
    const double *src = q + ((size_t)piv[k] * P + p) * 4;
    float4 v;
    v.x = (float)(src[0] - 0.5 * (box[8 * c + 0] + box[8 * c + 3]));
    v.y = (float)(src[1] - 0.5 * (box[8 * c + 1] + box[8 * c + 4]));
    v.z = (float)(src[2] - 0.5 * (box[8 * c + 2] + box[8 * c + 5]));
    v.w = (float)src[3];
    reinterpret_cast<float4 *>(out)[e] = v;
}

hipError_t launch_pivot_points(gca_h2_s *h, hipStream_t s)
{
    const int P = h->P_c;
    const int64_t ne = h->n_piv_total;
    if (ne == 0) return hipSuccess;
    const int64_t total = ne * P;
    hipLaunchKernelGGL(k_pivot_points, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, h->d_piv_cluster,
                       h->d_piv, h->d_box, h->d_qc, P, ne, h->d_pq32);
    return hipGetLastError();
}

template <typename T>
static size_t blk_smem(int rmax, int P, int cw, bool near)
{
    return BlkLayout<T>(rmax, P, cw, near).total;
}

// LDS budget per workgroup of the block kernel: the widest column chunk
// (multiple of 8, at most 128) whose arrays fit it.  The budget trades fewer
// chunks against more resident workgroups per CU (160 KB of LDS each).
constexpr int BLK_LDS_KB = 40;
template <typename T>
static int blk_cw(int rmax, int P, bool near)
{
    for (int cw = 128; cw >= 8; cw -= 8)
        if (blk_smem<T>(rmax, P, cw, near) <= BLK_LDS_KB * 1024) return cw;
    for (int cw = 64; cw >= 8; cw -= 8)
        if (blk_smem<T>(rmax, P, cw, near) <= 64 * 1024) return cw;
    return 0;
}

template <typename T, bool STORE>
static hipError_t near_rows(gca_h2_s *h, const T *xp, T *npart, T *store, hipStream_t s)
{
    const int ng = h->n_near_groups;
    if (ng == 0) return hipSuccess;
    if (STORE ? store == nullptr : (xp == nullptr || npart == nullptr)) return hipErrorInvalidValue;
    const int P = h->P_r;
    NearArgs<T> a{};
    a.g_t = h->d_ng_t;
    a.g_ptr = h->d_ng_ptr;
    a.g_rslot = h->d_ng_rslot;
    a.g_moff = h->d_ng_moff;
    a.col_pos = h->d_ncol_pos;
    a.col_out = h->d_ncol_out;
    a.mask = h->d_nmask;
    a.node = h->d_node;
    a.box = h->d_box;
    a.q = h->d_qr;
    a.cent = h->d_cent;
    a.qloc = h->d_qloc32;
    a.xp = xp;
    a.part = npart;
    a.store = store;
    a.g_soff = h->d_ng_soff;
    a.ng = ng;
    a.rmax = h->max_leaf;
    if (a.rmax > 64) return hipErrorInvalidValue;
    a.cw = NEAR_CW;
    while (a.cw > 8 && BlkLayout<T>(a.rmax, P, a.cw, true).total > 64 * 1024) a.cw /= 2;
    const size_t sm = BlkLayout<T>(a.rmax, P, a.cw, true).total;
    if (sm > 64 * 1024) return hipErrorInvalidValue;
    switch (P) {
#define CASE(PP)                                                                              \
    case PP:                                                                                  \
        hipLaunchKernelGGL((k_near_rows<T, PP, STORE>), dim3(ng), dim3(BLK_THREADS), sm, s, a); \
        break;
        CASE(1) CASE(3) CASE(4) CASE(6) CASE(9) CASE(16) CASE(25) CASE(36)
#undef CASE
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T, bool STORE>
static hipError_t far_rows(gca_h2_s *h, const T *xh, T *cpart, T *store, hipStream_t s)
{
    const int ng = h->n_far_groups;
    if (ng == 0) return hipSuccess;
    if (STORE ? store == nullptr : (xh == nullptr || cpart == nullptr)) return hipErrorInvalidValue;
    const int P = h->P_c;   // the coupling rule
    FarArgs<T> a{};
    a.g_t = h->d_fg_t;
    a.g_ptr = h->d_fg_ptr;
    a.g_rslot = h->d_fg_rslot;
    a.col_e = h->d_fcol_e;
    a.col_s = h->d_fcol_s;
    a.col_out = h->d_fcol_out;
    a.rank = h->d_rank;
    a.piv_off = h->d_piv_off;
    a.piv = h->d_piv;
    a.box = h->d_box;
    a.q = h->d_qc;
    a.pq32 = h->d_pq32;
    a.xh = xh;
    a.part = cpart;
    a.store = store;
    a.g_soff = h->d_fg_soff;
    a.ng = ng;
    a.rmax = std::max(1, std::min(64, h->max_rank));
    a.cw = blk_cw<T>(a.rmax, P, false);
    if (a.cw == 0) return hipErrorInvalidValue;
    const size_t sm = blk_smem<T>(a.rmax, P, a.cw, false);
    switch (P) {
#define CASE(PP)                                                                              \
    case PP:                                                                                  \
        hipLaunchKernelGGL((k_far_rows<T, PP, STORE>), dim3(ng), dim3(BLK_THREADS), sm, s, a);  \
        break;
        CASE(1) CASE(3) CASE(4) CASE(6) CASE(9) CASE(16) CASE(25) CASE(36)
#undef CASE
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_near(gca_h2_s *h, const T *xp, T *npart, hipStream_t s)
{
    return near_rows<T, false>(h, xp, npart, nullptr, s);
}

template <typename T>
hipError_t launch_far_blocks(gca_h2_s *h, const T *xh, T *cpart, hipStream_t s)
{
    return far_rows<T, false>(h, xh, cpart, nullptr, s);
}

template <typename T>
hipError_t launch_store_blocks(gca_h2_s *h, T *far_store, T *near_store, hipStream_t s)
{
    hipError_t e = far_rows<T, true>(h, nullptr, nullptr, far_store, s);
    if (e != hipSuccess) return e;
    return near_rows<T, true>(h, nullptr, nullptr, near_store, s);
}

// ------------------------------------ block rows, 16 right-hand sides ------
// The batched product (h2_matvec with nrhs > 1) evaluates every entry once
// for NB = 16 right-hand sides.  Per chunk of a block row the workgroup
// writes the entries of the chunk (rows x columns, masked pairs as 0) into
// an LDS tile with the wavefront tiles of the single-vector kernels, then
// applies the tile on the matrix cores: wavefront w multiplies the 16 rows
// 16w.. by the chunk's columns of X (row partials, accumulated over the
// chunks) and the transposed tile's 16 columns 16w.. by the rows of X (column
// partials of the chunk).  Vectors and partials hold the NB values of a row
// or slot contiguously.  Deterministic: fixed chunk and K order, one writer
// per partial.
// Column chunk of the batched block rows: 32 in FP32 (27 KB of LDS per
// workgroup instead of 40 at 64, so five workgroups fit a CU instead of
// three; 16-column product 6.27 -> 6.13 ms) and in FP64 (16 is slower).
#ifndef GCA_NB_CW32
#define GCA_NB_CW32 32
#endif
#ifndef GCA_NB_CW64
#define GCA_NB_CW64 32
#endif
template <typename T>
constexpr int nb_cw() { return sizeof(T) == 4 ? GCA_NB_CW32 : GCA_NB_CW64; }

// LDS layout (16-byte aligned sections): mask[64] (near) | rowp[64][P] |
// rown[64][P] | colp[CW][P] | coln[CW][P] | xr[64][NB] | xc[CW][NB] |
// gs[64][CW + 1]
template <typename T>
struct NbLayout {
    size_t mask, rowp, rown, colp, coln, xr, xc, gs, total;
    int gld;
    __host__ __device__ NbLayout(int P, int CW, bool near)
    {
        mask = 0;
        rowp = mask + (near ? al16(64 * 8) : 0);
        rown = rowp + al16((size_t)64 * P * sizeof(Q4<T>));
        colp = rown + al16((size_t)64 * P * sizeof(T));
        coln = colp + al16((size_t)CW * P * sizeof(Q4<T>));
        xr = coln + al16((size_t)CW * P * sizeof(T));
        xc = xr + al16((size_t)64 * NB * sizeof(T));
        gs = xc + al16((size_t)CW * NB * sizeof(T));
        gld = CW + 1;
        total = gs + al16((size_t)64 * gld * sizeof(T));
    }
};

// acc (rows 16w.. of the tile) += gs[16w.., 0..kw) xc[0..kw) (kw: a multiple of 4)
template <typename T>
__device__ __forceinline__ void nb_rows(typename Mfma<T>::acc_t &acc, const T *gs, int gld, const T *xc, int w,
                                        int kw)
{
    const int lane = threadIdx.x & 63, i = 16 * w + (lane & 15), k = lane >> 4;
    for (int k0 = 0; k0 < kw; k0 += 4)
        acc = Mfma<T>::mma(gs[i * gld + k0 + k], xc[(k0 + k) * NB + (lane & 15)], acc);
}

// gs[0..kr, 16w..]^T xr[0..kr) (kr: a multiple of 4)
template <typename T>
__device__ __forceinline__ typename Mfma<T>::acc_t nb_cols(const T *gs, int gld, const T *xr, int w, int kr)
{
    const int lane = threadIdx.x & 63, j = 16 * w + (lane & 15), k = lane >> 4;
    typename Mfma<T>::acc_t acc = mfma_zero<T>();
    for (int k0 = 0; k0 < kr; k0 += 4)
        acc = Mfma<T>::mma(gs[(k0 + k) * gld + j], xr[(k0 + k) * NB + (lane & 15)], acc);
    return acc;
}

template <typename T>
constexpr int nb_waves() { return sizeof(T) == 4 ? 4 : 3; }

// Nearfield block rows for NB right-hand sides: xp and part hold NB values
// per position / slot.
template <typename T, int P>
__global__ void __launch_bounds__(BLK_THREADS, (nb_waves<T>())) k_near_rows_nb(NearArgs<T> a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int CW = a.cw;
    const int g = blockIdx.x;
    const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
    const int t = a.g_t[g];
    const int64_t kb = a.g_ptr[g];
    const int nc = (int)(a.g_ptr[g + 1] - kb);
    const int rb = a.node[5 * t + 0], nr = a.node[5 * t + 1] - rb;
    const int64_t rslot = a.g_rslot[g];
    const uint64_t *gm = a.mask + a.g_moff[g];
    const NbLayout<T> L(P, CW, true);
    uint64_t *mask = reinterpret_cast<uint64_t *>(smem + L.mask);
    Q4<T> *rowp = reinterpret_cast<Q4<T> *>(smem + L.rowp);
    T *rown = reinterpret_cast<T *>(smem + L.rown);
    Q4<T> *colp = reinterpret_cast<Q4<T> *>(smem + L.colp);
    T *coln = reinterpret_cast<T *>(smem + L.coln);
    T *xr = reinterpret_cast<T *>(smem + L.xr);
    T *xc = reinterpret_cast<T *>(smem + L.xc);
    T *gs = reinterpret_cast<T *>(smem + L.gs);
    const int gld = L.gld;
    const double cx = 0.5 * (a.box[8 * t + 0] + a.box[8 * t + 3]);
    const double cy = 0.5 * (a.box[8 * t + 1] + a.box[8 * t + 4]);
    const double cz = 0.5 * (a.box[8 * t + 2] + a.box[8 * t + 5]);
    auto point = [&](int pos, int p) {
        if constexpr (sizeof(T) == 4) {
            const double *c = a.cent + 4 * (size_t)pos;
            const float4 v = reinterpret_cast<const float4 *>(a.qloc)[(size_t)pos * P + p];
            return Q4<T>{(T)(c[0] - cx) + v.x, (T)(c[1] - cy) + v.y, (T)(c[2] - cz) + v.z, v.w};
        } else {
            const double *src = a.q + ((size_t)pos * P + p) * 4;
            return Q4<T>{src[0] - cx, src[1] - cy, src[2] - cz, src[3]};
        }
    };
    for (int e = tid; e < nr * P; e += BLK_THREADS) {
        const int i = e / P, p = e - i * P;
        const Q4<T> v = point(rb + i, p);
        rowp[e] = v;
        rown[e] = v.x * v.x + v.y * v.y + v.z * v.z;
    }
    // rows beyond nr read as zero by the column products
    for (int e = tid; e < 64 * NB; e += BLK_THREADS) xr[e] = e < nr * NB ? a.xp[(int64_t)rb * NB + e] : (T)0;
    typename Mfma<T>::acc_t racc = mfma_zero<T>();
    const int kr = (nr + 3) & ~3;
    for (int c0 = 0; c0 < nc; c0 += CW) {
        const int cw = min(CW, nc - c0);
        const int ch = c0 / NEAR_CW, cb = c0 - ch * NEAR_CW;
        __syncthreads();
        for (int e = tid; e < cw * P; e += BLK_THREADS) {
            const int j = e / P, p = e - j * P;
            const Q4<T> v = point(a.col_pos[kb + c0 + j], p);
            colp[e] = Q4<T>{-2 * v.x, -2 * v.y, -2 * v.z, v.w};
            coln[e] = v.x * v.x + v.y * v.y + v.z * v.z;
        }
        for (int e = tid; e < CW * NB; e += BLK_THREADS) {
            const int j = e / NB;
            xc[e] = j < cw ? a.xp[(int64_t)a.col_pos[kb + c0 + j] * NB + (e - j * NB)] : (T)0;
        }
        for (int i = tid; i < nr; i += BLK_THREADS) mask[i] = gm[(size_t)ch * nr + i];
        for (int e = tid; e < 64 * gld; e += BLK_THREADS) gs[e] = 0;
        __syncthreads();
        tile_pass<T, P, true, true>(nr, cw, cb, rowp, rown, colp, coln, nullptr, nullptr, mask, nullptr, nullptr,
                                     gs, gld);
        __syncthreads();
        if (16 * wv < nr) nb_rows<T>(racc, gs, gld, xc, wv, (cw + 3) & ~3);
        if (16 * wv < cw) {
            const typename Mfma<T>::acc_t cacc = nb_cols<T>(gs, gld, xr, wv, kr);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int j = 16 * wv + Mfma<T>::row(lane, v);
                if (j < cw) a.part[a.col_out[kb + c0 + j] * NB + (lane & 15)] = cacc[v];
            }
        }
    }
    if (16 * wv < nr) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = 16 * wv + Mfma<T>::row(lane, v);
            if (i < nr) a.part[(rslot + i) * NB + (lane & 15)] = racc[v];
        }
    }
}

// Coupling block rows for NB right-hand sides: xh and part hold NB values
// per pivot entry / slot; row blocks of 64 pivots.
template <typename T, int P>
__global__ void __launch_bounds__(BLK_THREADS, (nb_waves<T>())) k_far_rows_nb(FarArgs<T> a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr bool F32 = sizeof(T) == 4;
    const int CW = a.cw;
    const int g = blockIdx.x;
    const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
    const int t = a.g_t[g];
    const int64_t kb = a.g_ptr[g];
    const int nc = (int)(a.g_ptr[g + 1] - kb);
    const int nr = a.rank[t];
    const int64_t xro = a.piv_off[t];
    const int64_t rslot = a.g_rslot[g];
    const NbLayout<T> L(P, CW, false);
    Q4<T> *rowp = reinterpret_cast<Q4<T> *>(smem + L.rowp);
    T *rown = reinterpret_cast<T *>(smem + L.rown);
    Q4<T> *colp = reinterpret_cast<Q4<T> *>(smem + L.colp);
    T *coln = reinterpret_cast<T *>(smem + L.coln);
    T *xr = reinterpret_cast<T *>(smem + L.xr);
    T *xc = reinterpret_cast<T *>(smem + L.xc);
    T *gs = reinterpret_cast<T *>(smem + L.gs);
    const int gld = L.gld;
    const double cx = 0.5 * (a.box[8 * t + 0] + a.box[8 * t + 3]);
    const double cy = 0.5 * (a.box[8 * t + 1] + a.box[8 * t + 4]);
    const double cz = 0.5 * (a.box[8 * t + 2] + a.box[8 * t + 5]);
    for (int r0 = 0; r0 < nr; r0 += 64) {
        const int rw = min(64, nr - r0);
        if (r0 > 0) __syncthreads();
        for (int e = tid; e < rw * P; e += BLK_THREADS) {
            const int i = e / P, p = e - i * P;
            if (F32) {
                const float4 v = reinterpret_cast<const float4 *>(a.pq32)[(size_t)(xro + r0 + i) * P + p];
                rowp[e] = Q4<T>{(T)v.x, (T)v.y, (T)v.z, (T)v.w};
                rown[e] = (T)(v.x * v.x + v.y * v.y + v.z * v.z);
            } else {
                const double *src = a.q + ((size_t)a.piv[xro + r0 + i] * P + p) * 4;
                const T x = (T)(src[0] - cx), y = (T)(src[1] - cy), z = (T)(src[2] - cz);
                rowp[e] = Q4<T>{x, y, z, (T)src[3]};
                rown[e] = x * x + y * y + z * z;
            }
        }
        for (int e = tid; e < 64 * NB; e += BLK_THREADS)
            xr[e] = e < rw * NB ? a.xh[(xro + r0) * NB + e] : (T)0;
        typename Mfma<T>::acc_t racc = mfma_zero<T>();
        const int kr = (rw + 3) & ~3;
        for (int c0 = 0; c0 < nc; c0 += CW) {
            const int cw = min(CW, nc - c0);
            __syncthreads();
            for (int e = tid; e < cw * P; e += BLK_THREADS) {
                const int j = e / P, p = e - j * P;
                const int64_t k = kb + c0 + j;
                const int ce = a.col_e[k];
                if (F32) {
                    const int cs = a.col_s[k];
                    const float ox = (float)(0.5 * (a.box[8 * cs + 0] + a.box[8 * cs + 3]) - cx);
                    const float oy = (float)(0.5 * (a.box[8 * cs + 1] + a.box[8 * cs + 4]) - cy);
                    const float oz = (float)(0.5 * (a.box[8 * cs + 2] + a.box[8 * cs + 5]) - cz);
                    const float4 v = reinterpret_cast<const float4 *>(a.pq32)[(size_t)ce * P + p];
                    const float y0 = v.x + ox, y1 = v.y + oy, y2 = v.z + oz;
                    colp[e] = Q4<T>{(T)(-2 * y0), (T)(-2 * y1), (T)(-2 * y2), (T)v.w};
                    coln[e] = (T)(y0 * y0 + y1 * y1 + y2 * y2);
                } else {
                    const double *src = a.q + ((size_t)a.piv[ce] * P + p) * 4;
                    const T y0 = (T)(src[0] - cx), y1 = (T)(src[1] - cy), y2 = (T)(src[2] - cz);
                    colp[e] = Q4<T>{-2 * y0, -2 * y1, -2 * y2, (T)src[3]};
                    coln[e] = y0 * y0 + y1 * y1 + y2 * y2;
                }
            }
            for (int e = tid; e < CW * NB; e += BLK_THREADS) {
                const int j = e / NB;
                xc[e] = j < cw ? a.xh[(int64_t)a.col_e[kb + c0 + j] * NB + (e - j * NB)] : (T)0;
            }
            for (int e = tid; e < 64 * gld; e += BLK_THREADS) gs[e] = 0;
            __syncthreads();
            tile_pass<T, P, false, true>(rw, cw, 0, rowp, rown, colp, coln, nullptr, nullptr, nullptr, nullptr,
                                          nullptr, gs, gld);
            __syncthreads();
            if (16 * wv < rw) nb_rows<T>(racc, gs, gld, xc, wv, (cw + 3) & ~3);
            if (16 * wv < cw) {
                const typename Mfma<T>::acc_t cacc = nb_cols<T>(gs, gld, xr, wv, kr);
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int j = 16 * wv + Mfma<T>::row(lane, v);
                    if (j < cw) {
                        T *o = a.part + a.col_out[kb + c0 + j] * NB + (lane & 15);
                        *o = r0 == 0 ? cacc[v] : *o + cacc[v];
                    }
                }
            }
        }
        if (16 * wv < rw) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = 16 * wv + Mfma<T>::row(lane, v);
                if (i < rw) a.part[(rslot + r0 + i) * NB + (lane & 15)] = racc[v];
            }
        }
    }
}

template <typename T>
hipError_t launch_near_nb(gca_h2_s *h, const T *xp, T *npart, hipStream_t s)
{
    const int ng = h->n_near_groups;
    if (ng == 0) return hipSuccess;
    if (xp == nullptr || npart == nullptr) return hipErrorInvalidValue;
    const int P = h->P_r;
    NearArgs<T> a{};
    a.g_t = h->d_ng_t;
    a.g_ptr = h->d_ng_ptr;
    a.g_rslot = h->d_ng_rslot;
    a.g_moff = h->d_ng_moff;
    a.col_pos = h->d_ncol_pos;
    a.col_out = h->d_ncol_out;
    a.mask = h->d_nmask;
    a.node = h->d_node;
    a.box = h->d_box;
    a.q = h->d_qr;
    a.cent = h->d_cent;
    a.qloc = h->d_qloc32;
    a.xp = xp;
    a.part = npart;
    a.ng = ng;
    a.rmax = h->max_leaf;
    if (a.rmax > 64) return hipErrorInvalidValue;
    a.cw = nb_cw<T>();
    while (a.cw > 16 && NbLayout<T>(P, a.cw, true).total > 64 * 1024) a.cw /= 2;
    const size_t sm = NbLayout<T>(P, a.cw, true).total;
    if (sm > 64 * 1024) return hipErrorInvalidValue;
    switch (P) {
#define CASE(PP)                                                                                  \
    case PP:                                                                                      \
        hipLaunchKernelGGL((k_near_rows_nb<T, PP>), dim3(ng), dim3(BLK_THREADS), sm, s, a);         \
        break;
        CASE(1) CASE(3) CASE(4) CASE(6) CASE(9)
#undef CASE
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_far_blocks_nb(gca_h2_s *h, const T *xh, T *cpart, hipStream_t s)
{
    const int ng = h->n_far_groups;
    if (ng == 0) return hipSuccess;
    if (xh == nullptr || cpart == nullptr) return hipErrorInvalidValue;
    const int P = h->P_c;
    FarArgs<T> a{};
    a.g_t = h->d_fg_t;
    a.g_ptr = h->d_fg_ptr;
    a.g_rslot = h->d_fg_rslot;
    a.col_e = h->d_fcol_e;
    a.col_s = h->d_fcol_s;
    a.col_out = h->d_fcol_out;
    a.rank = h->d_rank;
    a.piv_off = h->d_piv_off;
    a.piv = h->d_piv;
    a.box = h->d_box;
    a.q = h->d_qc;
    a.pq32 = h->d_pq32;
    a.xh = xh;
    a.part = cpart;
    a.ng = ng;
    a.rmax = 64;
    a.cw = nb_cw<T>();
    while (a.cw > 16 && NbLayout<T>(P, a.cw, false).total > 64 * 1024) a.cw /= 2;
    const size_t sm = NbLayout<T>(P, a.cw, false).total;
    if (sm > 64 * 1024) return hipErrorInvalidValue;
    switch (P) {
#define CASE(PP)                                                                                 \
    case PP:                                                                                     \
        hipLaunchKernelGGL((k_far_rows_nb<T, PP>), dim3(ng), dim3(BLK_THREADS), sm, s, a);         \
        break;
        CASE(1) CASE(3) CASE(4) CASE(6) CASE(9)
#undef CASE
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}
template hipError_t launch_near_nb<float>(gca_h2_s *, const float *, float *, hipStream_t);
template hipError_t launch_near_nb<double>(gca_h2_s *, const double *, double *, hipStream_t);
template hipError_t launch_far_blocks_nb<float>(gca_h2_s *, const float *, float *, hipStream_t);
template hipError_t launch_far_blocks_nb<double>(gca_h2_s *, const double *, double *, hipStream_t);

// ----------------------------------------------------- stored block rows ---
// Product with block rows stored by the STORE kernels: G_g (nr x nc,
// row-major at g_soff) gives the row partials G_g x_cols and the column
// partials G_g^T x_rows from one read of every entry.  Wavefront w streams
// the rows i = w mod 4 (each a contiguous run of nc entries, lanes over
// columns): the row sum is reduced across the wavefront (DPP, then two
// cross-row moves), the
// column sums stay in registers (up to APPLY_CB columns at a time) and are
// combined over the four wavefronts in LDS.  One writer per partial slot.
constexpr int APPLY_K = 4;                 // column registers per lane
constexpr int APPLY_CB = 64 * APPLY_K;     // columns per pass
template <typename T>
constexpr int apply_rows() { return 4; }   // rows per wavefront step (FP64 at 2: 2.01 ms per stored product, at 4: 1.93)

template <typename T>
struct ApplyArgs {
    const int32_t *g_t;
    const int64_t *g_ptr;
    const int64_t *g_rslot;
    const int64_t *g_soff;
    const int32_t *col_idx;   // coupling: pivot entry (into xh); nearfield: position (into xp)
    const int64_t *col_out;
    const int32_t *node;
    const int32_t *rank;
    const int64_t *piv_off;
    const T *x;               // coupling: xh; nearfield: permuted x
    const T *G;
    T *part;
};

template <typename T, bool NEARG>
__global__ void __launch_bounds__(BLK_THREADS) k_rows_apply(ApplyArgs<T> a)
{
    __shared__ T cacc[BLK_WAVES][APPLY_CB];
    const int g = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int t = a.g_t[g];
    const int64_t kb = a.g_ptr[g];
    const int nc = (int)(a.g_ptr[g + 1] - kb);
    int nr;
    const T *xrow;
    if (NEARG) {
        const int rb = a.node[5 * t];
        nr = a.node[5 * t + 1] - rb;
        xrow = a.x + rb;
    } else {
        nr = a.rank[t];
        xrow = a.x + a.piv_off[t];
    }
    const T *G = a.G + a.g_soff[g];
    const int64_t rslot = a.g_rslot[g];
    for (int cb = 0; cb < nc; cb += APPLY_CB) {
        const int cw = min(APPLY_CB, nc - cb);
        T xc[APPLY_K], ca[APPLY_K];
#pragma unroll
        for (int k = 0; k < APPLY_K; ++k) {
            const int j = lane + 64 * k;
            xc[k] = j < cw ? a.x[a.col_idx[kb + cb + j]] : (T)0;
            ca[k] = 0;
        }
        // APPLY_R rows per step so that their loads are in flight together
        constexpr int APPLY_R = apply_rows<T>();
        for (int i0 = wv; i0 < nr; i0 += APPLY_R * BLK_WAVES) {
            T gr[APPLY_R][APPLY_K], xi[APPLY_R];
#pragma unroll
            for (int q = 0; q < APPLY_R; ++q) {
                const int i = i0 + q * BLK_WAVES;
                const bool ok = i < nr;
                xi[q] = ok ? xrow[i] : (T)0;
                const T *Gi = G + (int64_t)(ok ? i : i0) * nc + cb;
#pragma unroll
                for (int k = 0; k < APPLY_K; ++k) {
                    const int j = lane + 64 * k;
                    gr[q][k] = (ok && j < cw) ? Gi[j] : (T)0;
                }
            }
#pragma unroll
            for (int q = 0; q < APPLY_R; ++q) {
                T v = 0;
#pragma unroll
                for (int k = 0; k < APPLY_K; ++k) {
                    v += gr[q][k] * xc[k];
                    ca[k] += gr[q][k] * xi[q];
                }
                v = class_sum<1>(v, lane);   // DPP within rows of 16, then lane ^ 16, lane ^ 32
                const int i = i0 + q * BLK_WAVES;
                if (lane == 0 && i < nr) {
                    if (cb == 0)
                        a.part[rslot + i] = v;
                    else
                        a.part[rslot + i] += v;
                }
            }
        }
#pragma unroll
        for (int k = 0; k < APPLY_K; ++k) cacc[wv][lane + 64 * k] = ca[k];
        __syncthreads();
        for (int j = tid; j < cw; j += BLK_THREADS) {
            T c = 0;
#pragma unroll
            for (int w = 0; w < BLK_WAVES; ++w) c += cacc[w][j];
            a.part[a.col_out[kb + cb + j]] = c;
        }
        __syncthreads();
    }
}

template <typename T>
hipError_t launch_apply_stored(gca_h2_s *h, bool nearfield, const T *x, const T *G, T *part, hipStream_t s)
{
    ApplyArgs<T> a{};
    a.node = h->d_node;
    a.rank = h->d_rank;
    a.piv_off = h->d_piv_off;
    a.x = x;
    a.G = G;
    a.part = part;
    int ng;
    if (nearfield) {
        ng = h->n_near_groups;
        a.g_t = h->d_ng_t;
        a.g_ptr = h->d_ng_ptr;
        a.g_rslot = h->d_ng_rslot;
        a.g_soff = h->d_ng_soff;
        a.col_idx = h->d_ncol_pos;
        a.col_out = h->d_ncol_out;
    } else {
        ng = h->n_far_groups;
        a.g_t = h->d_fg_t;
        a.g_ptr = h->d_fg_ptr;
        a.g_rslot = h->d_fg_rslot;
        a.g_soff = h->d_fg_soff;
        a.col_idx = h->d_fcol_e;
        a.col_out = h->d_fcol_out;
    }
    if (ng == 0) return hipSuccess;
    if (nearfield)
        hipLaunchKernelGGL((k_rows_apply<T, true>), dim3(ng), dim3(BLK_THREADS), 0, s, a);
    else
        hipLaunchKernelGGL((k_rows_apply<T, false>), dim3(ng), dim3(BLK_THREADS), 0, s, a);
    return hipGetLastError();
}

template hipError_t launch_near<float>(gca_h2_s *, const float *, float *, hipStream_t);
template hipError_t launch_near<double>(gca_h2_s *, const double *, double *, hipStream_t);
template hipError_t launch_far_blocks<float>(gca_h2_s *, const float *, float *, hipStream_t);
template hipError_t launch_far_blocks<double>(gca_h2_s *, const double *, double *, hipStream_t);
template hipError_t launch_store_blocks<float>(gca_h2_s *, float *, float *, hipStream_t);
template hipError_t launch_store_blocks<double>(gca_h2_s *, double *, double *, hipStream_t);
template hipError_t launch_apply_stored<float>(gca_h2_s *, bool, const float *, const float *, float *,
                                               hipStream_t);
template hipError_t launch_apply_stored<double>(gca_h2_s *, bool, const double *, const double *, double *,
                                                hipStream_t);

// ------------------------------------------------------- touching pairs --
// FP64 by default.  T = float (the mixed product): vertices are read and the
// edge vectors and surface elements formed in FP64, then the Gauss loops run
// in FP32 -- the dimension-reduced integrands below are smooth, so FP32 only
// adds rounding of the order of 1e-7 relative to the pair's value.

__constant__ int c_perm[6][3] = {{0, 1, 2}, {1, 2, 0}, {2, 0, 1}, {0, 2, 1}, {1, 0, 2}, {2, 1, 0}};

template <typename T = double>
struct V3 {
    T x, y, z;
};
template <typename T>
__device__ __forceinline__ V3<T> vsub(V3<double> a, V3<double> b)
{
    return {(T)(a.x - b.x), (T)(a.y - b.y), (T)(a.z - b.z)};
}
// the Sauter-Schwab integrands are evaluated at interior Gauss points, where
// the squared distances are positive and finite
template <typename T>
__device__ __forceinline__ T vrnorm(T x, T y, T z) { return rsq<T>(x * x + y * y + z * z); }
template <typename T>
__device__ __forceinline__ double cross_norm(V3<T> a, V3<T> b)
{
    const double ax = a.x, ay = a.y, az = a.z, bx = b.x, by = b.y, bz = b.z;
    double cx = ay * bz - az * by, cy = az * bx - ax * bz, cz = ax * by - ay * bx;
    return sqrt(cx * cx + cy * cy + cz * cz);
}

__device__ __forceinline__ V3<double> ldv(const double *xyz, int v)
{
    return {xyz[3 * (size_t)v], xyz[3 * (size_t)v + 1], xyz[3 * (size_t)v + 2]};
}

// Ordered vertices of a triangle: code indexes c_perm.
__device__ __forceinline__ void tri_vertices(const double *xyz, const int32_t *tv, int pos, int code, V3<double> P[3])
{
    const int32_t *v = tv + 3 * (size_t)pos;
    P[0] = ldv(xyz, v[c_perm[code][0]]);
    P[1] = ldv(xyz, v[c_perm[code][1]]);
    P[2] = ldv(xyz, v[c_perm[code][2]]);
}

// identical triangles: J^2/(4 pi) * (1/3) * sum_d w_d [ 1/|eta e1 + e2| + 1/|e1 + eta e2| + 1/|-eta e1 + (1-eta) e2| ]
// NQ > 0: the Gauss order as a compile-time constant (loops unrolled, the
// points' loop-invariant parts formed once); NQ = 0: g.q at run time.
template <int NQ, typename T = double>
__device__ double ss_identical(const V3<double> P[3], const GaussQ &g)
{
    const V3<T> e1 = vsub<T>(P[1], P[0]), e2 = vsub<T>(P[2], P[1]);
    const double J = cross_norm(vsub<double>(P[1], P[0]), vsub<double>(P[2], P[1]));
    T s = 0;
    const int q = NQ ? NQ : g.q;
#pragma unroll
    for (int d = 0; d < q; ++d) {
        const T t = (T)g.x[d];
        T a = vrnorm<T>(t * e1.x + e2.x, t * e1.y + e2.y, t * e1.z + e2.z);
        T b = vrnorm<T>(e1.x + t * e2.x, e1.y + t * e2.y, e1.z + t * e2.z);
        T c = vrnorm<T>(-t * e1.x + (1 - t) * e2.x, -t * e1.y + (1 - t) * e2.y, -t * e1.z + (1 - t) * e2.z);
        s += (T)g.w[d] * (a + b + c);
    }
    return J * J * INV4PI * (double)s * (1.0 / 3.0);
}

// common edge P0 P1 (same parametrisation on both triangles): five 2D integrals
template <int NQ, typename T = double>
__device__ double ss_edge(const V3<double> P[3], const V3<double> Q[3], const GaussQ &g)
{
    const V3<T> e1 = vsub<T>(P[1], P[0]), et = vsub<T>(P[2], P[1]), es = vsub<T>(Q[2], Q[1]);
    const V3<double> d1 = vsub<double>(P[1], P[0]);
    const double Jt = cross_norm(d1, vsub<double>(P[2], P[1])), Js = cross_norm(d1, vsub<double>(Q[2], Q[1]));
    T s = 0;
    const int q = NQ ? NQ : g.q;
#pragma unroll
    for (int ia = 0; ia < q; ++ia) {
        const T h2 = (T)g.x[ia];
        T sb = 0;
#pragma unroll
        for (int ib = 0; ib < q; ++ib) {
            const T h3 = (T)g.x[ib];
            // region 1 (no eta2 factor)
            T r1 = vrnorm<T>(h2 * e1.x + h3 * et.x - (1 - h2) * es.x, h2 * e1.y + h3 * et.y - (1 - h2) * es.y,
                             h2 * e1.z + h3 * et.z - (1 - h2) * es.z);
            T r2 = vrnorm<T>(h2 * h3 * e1.x + et.x - h2 * (1 - h3) * es.x,
                             h2 * h3 * e1.y + et.y - h2 * (1 - h3) * es.y,
                             h2 * h3 * e1.z + et.z - h2 * (1 - h3) * es.z);
            T r3 = vrnorm<T>(-h2 * e1.x + (1 - h2) * et.x - h2 * h3 * es.x,
                             -h2 * e1.y + (1 - h2) * et.y - h2 * h3 * es.y,
                             -h2 * e1.z + (1 - h2) * et.z - h2 * h3 * es.z);
            T r4 = vrnorm<T>(-h2 * h3 * e1.x + h2 * (1 - h3) * et.x - es.x,
                             -h2 * h3 * e1.y + h2 * (1 - h3) * et.y - es.y,
                             -h2 * h3 * e1.z + h2 * (1 - h3) * et.z - es.z);
            T r5 = vrnorm<T>(-h2 * h3 * e1.x + (1 - h2 * h3) * et.x - h2 * es.x,
                             -h2 * h3 * e1.y + (1 - h2 * h3) * et.y - h2 * es.y,
                             -h2 * h3 * e1.z + (1 - h2 * h3) * et.z - h2 * es.z);
            sb += (T)g.w[ib] * (r1 + h2 * (r2 + r3 + r4 + r5));
        }
        s += (T)g.w[ia] * sb;
    }
    return Jt * Js * INV4PI * (double)s * (1.0 / 6.0);
}

// common vertex P0 = Q0: two 3D integrals
template <int NQ, typename T = double>
__device__ double ss_vertex(const V3<double> P[3], const V3<double> Q[3], const GaussQ &g)
{
    const V3<T> e1t = vsub<T>(P[1], P[0]), e2t = vsub<T>(P[2], P[1]);
    const V3<T> e1s = vsub<T>(Q[1], Q[0]), e2s = vsub<T>(Q[2], Q[1]);
    const double Jt = cross_norm(vsub<double>(P[1], P[0]), vsub<double>(P[2], P[1]));
    const double Js = cross_norm(vsub<double>(Q[1], Q[0]), vsub<double>(Q[2], Q[1]));
    T s = 0;
    const int q = NQ ? NQ : g.q;
#pragma unroll
    for (int ia = 0; ia < q; ++ia) {
        const T h1 = (T)g.x[ia];
        // x-side points (1, eta1) and y-side points (1, eta1)
        const T ax = e1t.x + h1 * e2t.x, ay = e1t.y + h1 * e2t.y, az = e1t.z + h1 * e2t.z;
        const T bx = e1s.x + h1 * e2s.x, by = e1s.y + h1 * e2s.y, bz = e1s.z + h1 * e2s.z;
        T sa = 0;
#pragma unroll
        for (int ib = 0; ib < q; ++ib) {
            const T h2 = (T)g.x[ib];
            T sb = 0;
#pragma unroll
            for (int ic = 0; ic < q; ++ic) {
                const T h3 = (T)g.x[ic];
                const T cx = e1s.x + h3 * e2s.x, cy = e1s.y + h3 * e2s.y, cz = e1s.z + h3 * e2s.z;
                const T dx = e1t.x + h3 * e2t.x, dy = e1t.y + h3 * e2t.y, dz = e1t.z + h3 * e2t.z;
                T r1 = vrnorm<T>(ax - h2 * cx, ay - h2 * cy, az - h2 * cz);
                T r2 = vrnorm<T>(h2 * dx - bx, h2 * dy - by, h2 * dz - bz);
                sb += (T)g.w[ic] * (r1 + r2);
            }
            sa += (T)g.w[ib] * h2 * sb;
        }
        s += (T)g.w[ia] * sa;
    }
    return Jt * Js * INV4PI * (double)s * (1.0 / 3.0);
}

template <int KIND, int NQ, typename T = double>
__device__ double touching_value(const double *xyz, const int32_t *tv, int pa, int pb, int code, const GaussQ &g)
{
    V3<double> P[3], Q[3];
    tri_vertices(xyz, tv, pa, code & 15, P);
    if (KIND == 0) return ss_identical<NQ, T>(P, g);
    tri_vertices(xyz, tv, pb, (code >> 4) & 15, Q);
    if (KIND == 1) return ss_edge<NQ, T>(P, Q, g);
    return ss_vertex<NQ, T>(P, Q, g);
}

// Value of pair p goes to out[sa[p]] and out[sb[p]] (sb < 0: none) when slot
// maps are given (row CSR of the product), else to out[p].  T: the type of
// the Gauss loops (values are stored in FP64 either way).
template <int KIND, typename T = double>
__global__ void __launch_bounds__(256) k_touching(const double *xyz, const int32_t *tv, const int32_t *pa,
                                                  const int32_t *pb, const int32_t *code, int64_t np,
                                                  GaussQ g, const int32_t *sa, const int32_t *sb, double *out)
{
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    // the default Sauter-Schwab order 4 with unrolled loops
    const double v = g.q == 4 ? touching_value<KIND, 4, T>(xyz, tv, pa[p], pb[p], code[p], g)
                              : touching_value<KIND, 0, T>(xyz, tv, pa[p], pb[p], code[p], g);
    if (sa) {
        out[sa[p]] = v;
        if (sb[p] >= 0) out[sb[p]] = v;
    } else {
        out[p] = v;
    }
}

static GaussQ make_gq(const double *x, const double *w, int q)
{
    GaussQ g{};
    g.q = q;
    for (int i = 0; i < q; ++i) {
        g.x[i] = x[i];
        g.w[i] = w[i];
    }
    return g;
}

template <typename T>
static hipError_t touching_lists(gca_h2_s *h, double *tval, hipStream_t s)
{
    GaussQ g = make_gq(h->gs_x, h->gs_w, h->prm.q_s);
    for (int kind = 0; kind < 3; ++kind) {
        int64_t b = h->pl.off[kind], e = h->pl.off[kind + 1];
        int64_t np = e - b;
        if (np == 0) continue;
        dim3 grid((unsigned)((np + 255) / 256)), blk(256);
        if (kind == 0)
            hipLaunchKernelGGL((k_touching<0, T>), grid, blk, 0, s, h->d_xyz, h->d_tv, h->d_pa + b, h->d_pb + b,
                               h->d_pcode + b, np, g, h->d_tslot_a + b, h->d_tslot_b + b, tval);
        else if (kind == 1)
            hipLaunchKernelGGL((k_touching<1, T>), grid, blk, 0, s, h->d_xyz, h->d_tv, h->d_pa + b, h->d_pb + b,
                               h->d_pcode + b, np, g, h->d_tslot_a + b, h->d_tslot_b + b, tval);
        else
            hipLaunchKernelGGL((k_touching<2, T>), grid, blk, 0, s, h->d_xyz, h->d_tv, h->d_pa + b, h->d_pb + b,
                               h->d_pcode + b, np, g, h->d_tslot_a + b, h->d_tslot_b + b, tval);
        hipError_t err = hipGetLastError();
        if (err != hipSuccess) return err;
    }
    return hipSuccess;
}

hipError_t launch_touching(gca_h2_s *h, double *tval, hipStream_t s, bool fp32)
{
    return fp32 ? touching_lists<float>(h, tval, s) : touching_lists<double>(h, tval, s);
}

// ------------------------------------------------------ near-regular pairs --
// Disjoint pairs joined by a mesh edge get the regular rule of order q_nr.
// Points relative to the first point of the first triangle (FP64), then T.
template <typename T, int P>
__device__ T regular_pair(const double *q, int pa, int pb)
{
    const double *A = q + (size_t)pa * P * 4;
    const double *B = q + (size_t)pb * P * 4;
    const double ox = A[0], oy = A[1], oz = A[2];
    T ax[P], ay[P], az[P], aw[P];
#pragma unroll
    for (int i = 0; i < P; ++i) {
        ax[i] = (T)(A[4 * i] - ox);
        ay[i] = (T)(A[4 * i + 1] - oy);
        az[i] = (T)(A[4 * i + 2] - oz);
        aw[i] = (T)A[4 * i + 3];
    }
    T acc = 0;
    for (int j = 0; j < P; ++j) {
        const T bx = (T)(B[4 * j] - ox), by = (T)(B[4 * j + 1] - oy), bz = (T)(B[4 * j + 2] - oz);
        const T bw = (T)B[4 * j + 3];
        T inner = 0;
#pragma unroll
        for (int i = 0; i < P; ++i) {
            const T dx = ax[i] - bx, dy = ay[i] - by, dz = az[i] - bz;
            inner += aw[i] * rsq<T>(dx * dx + dy * dy + dz * dz);
        }
        acc += bw * inner;
    }
    return acc * (T)INV4PI;
}

template <typename T, int P>
__global__ void __launch_bounds__(256) k_nearreg(const double *q, const int32_t *pa, const int32_t *pb, int64_t np,
                                                 const int32_t *sa, const int32_t *sb, T *out)
{
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    const T v = regular_pair<T, P>(q, pa[p], pb[p]);
    if (sa) {
        out[sa[p]] = v;
        if (sb[p] >= 0) out[sb[p]] = v;
    } else {
        out[p] = v;
    }
}

template <typename T>
static hipError_t launch_regular_list(int P, const double *q, const int32_t *pa, const int32_t *pb, int64_t np,
                                      const int32_t *sa, const int32_t *sb, T *out, hipStream_t s)
{
    if (np == 0) return hipSuccess;
    dim3 grid((unsigned)((np + 255) / 256)), blk(256);
    switch (P) {
#define CASE(PP)                                                                              \
    case PP:                                                                                  \
        hipLaunchKernelGGL((k_nearreg<T, PP>), grid, blk, 0, s, q, pa, pb, np, sa, sb, out);   \
        break;
        CASE(1) CASE(3) CASE(4) CASE(6) CASE(9) CASE(16) CASE(25) CASE(36) CASE(49)
#undef CASE
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_nearreg(gca_h2_s *h, T *nval, hipStream_t s)
{
    int64_t b = h->pl.off[3], e = h->pl.off[4];
    return launch_regular_list<T>(h->P_nr, h->d_qnr, h->d_pa + b, h->d_pb + b, e - b,
                                  h->d_slot_a + b, h->d_slot_b + b, nval, s);
}

template hipError_t launch_nearreg<float>(gca_h2_s *, float *, hipStream_t);
template hipError_t launch_nearreg<double>(gca_h2_s *, double *, hipStream_t);

// ---------------------------------------------------- single entries ------
// Entries for a list of pairs already sorted into classes by the host:
// touching (codes), near-regular and regular pairs go through the same
// device functions as the matrix-vector product.
hipError_t launch_entry_jobs(gca_h2_s *h, const EntryJobs &j, double *tmp64, float *tmp32, int precision,
                             hipStream_t s)
{
    GaussQ g = make_gq(h->gs_x, h->gs_w, h->prm.q_s);
    const bool f32 = precision != GCA_FP64 && h->prm.ss_fp32;   // FP32 Gauss loops (opt-in, mixed only)
    for (int kind = 0; kind < 3; ++kind) {
        int64_t b = j.off[kind], np = j.off[kind + 1] - b;
        if (!np) continue;
        dim3 grid((unsigned)((np + 255) / 256)), blk(256);
#define TOUCH(K)                                                                                        \
    if (f32)                                                                                            \
        hipLaunchKernelGGL((k_touching<K, float>), grid, blk, 0, s, h->d_xyz, h->d_tv, j.pa + b, j.pb + b, \
                           j.code + b, np, g, nullptr, nullptr, tmp64 + b);                             \
    else                                                                                                \
        hipLaunchKernelGGL((k_touching<K, double>), grid, blk, 0, s, h->d_xyz, h->d_tv, j.pa + b, j.pb + b, \
                           j.code + b, np, g, nullptr, nullptr, tmp64 + b);
        if (kind == 0) {
            TOUCH(0)
        } else if (kind == 1) {
            TOUCH(1)
        } else {
            TOUCH(2)
        }
#undef TOUCH
    }
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    const int Pnr = h->P_nr, Pr = h->P_r;
    if (precision == GCA_FP64) {
        err = launch_regular_list<double>(Pnr, h->d_qnr, j.pa + j.off[3], j.pb + j.off[3], j.off[4] - j.off[3],
                                          nullptr, nullptr, tmp64 + j.off[3], s);
        if (err != hipSuccess) return err;
        err = launch_regular_list<double>(Pr, h->d_qr, j.pa + j.off[4], j.pb + j.off[4], j.off[5] - j.off[4],
                                          nullptr, nullptr, tmp64 + j.off[4], s);
    } else {
        err = launch_regular_list<float>(Pnr, h->d_qnr, j.pa + j.off[3], j.pb + j.off[3], j.off[4] - j.off[3],
                                         nullptr, nullptr, tmp32 + j.off[3], s);
        if (err != hipSuccess) return err;
        err = launch_regular_list<float>(Pr, h->d_qr, j.pa + j.off[4], j.pb + j.off[4], j.off[5] - j.off[4],
                                         nullptr, nullptr, tmp32 + j.off[4], s);
    }
    return err;
}

}  // namespace gca
