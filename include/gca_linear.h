/*
 * gca_linear.h -- C-ABI of libgca for the continuous piecewise-linear nodal
 * basis on flat triangles (Section 5).
 *
 * With nodal basis functions phi_i (one per vertex, linear on every triangle,
 * one at vertex i and zero at all other vertices) the Galerkin entry
 *     g_ij = sum_{t in T_i} sum_{s in T_j} int_t phi_i(x) int_s g(x, y) phi_j(y) dy dx,
 *     g(x, y) = 1 / (4 pi |x - y|),
 * runs over the sets T_i, T_j of triangles in the two supports (Section 5).
 * The compression needs such entries only on index subsets (the pivot sets
 * and the clusters of Sections 2-4), so the library
 *   1. unites the sets T_i of each vertex subset into one list sorted by
 *      triangle, every row carrying the subset-local index of each corner's
 *      vertex or "bottom" (the mergesort of Section 5, worked example), and
 *   2. assembles a block G|rows x cols triangle pair by triangle pair: the
 *      kernel values at the quadrature points of a pair serve all nine
 *      combinations of its corners' nodal functions (Section 5).
 *
 * Conventions are those of gca.h: GCA_OK or a negative gca_status, arguments
 * validated before device work is queued, device pointers owned by the
 * caller, work queued on the given stream without synchronisation.
 */
#ifndef GCA_LINEAR_H
#define GCA_LINEAR_H

#include <stdint.h>

#include "gca.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Limits of the device kernels (per subset and per block). */
#define GCA_LIN_MAX_GATHER 2048 /* sum of |T_i| over one subset */
#define GCA_LIN_MAX_SET 1024    /* vertices in one subset (merge) */
#define GCA_LIN_MAX_BLOCK_SET 64 /* vertices in a row or column subset of a block */
#define GCA_LIN_MAX_TRIS 192    /* merged triangles of a block's row or column subset */
#define GCA_LIN_MAX_DEGREE 16   /* |T_i| of a vertex in a block subset */

/* The sets T_i (Section 5) of an nv-vertex mesh, on the host.
 * tri: host int32, nt x 3 vertex ids (row-major).
 * off: host int32, nv + 1 entries, written: T_i is list[off[i] .. off[i+1]).
 * list: host int32, 3 nt entries, written: triangle ids, ascending within
 *       each T_i (a triangle is listed once per distinct corner vertex).
 * Errors: GCA_EINVAL (NULL pointers, nt < 0, nv < 0), GCA_EMESH (a vertex id
 * out of range, or a triangle with a repeated vertex). */
gca_status gca_lin_vertex_triangles(const int32_t *tri, int64_t nt, int64_t nv, int32_t *off,
                                    int32_t *list);

/* Merged triangle lists of nsets vertex subsets (Section 5, the mergesort and
 * its combination rule), one workgroup per subset.
 * vt_off, vt_list: device int32, the sets T_i as written by
 *       gca_lin_vertex_triangles (nv + 1 and 3 nt entries).
 * tri: device int32, nt x 3 vertex ids.
 * set_off: device int32, nsets + 1 entries; set_vtx: device int32 vertex ids;
 *       subset k is set_vtx[set_off[k] .. set_off[k+1]), the local index of a
 *       vertex is its position there (vertices distinct within a subset).
 * cap: rows reserved per subset in the outputs (1 .. GCA_LIN_MAX_GATHER).
 * out_tri: device int32, nsets x cap: triangle ids of subset k at
 *       out_tri[k cap + r], r < out_count[k], ascending;
 * out_loc: device int32, nsets x cap x 3: local index of corner c of that
 *       triangle at out_loc[(k cap + r) 3 + c], or -1 (bottom) when the
 *       corner's vertex is not in the subset;
 * out_count: device int32, nsets: rows of subset k, or -1 when the subset
 *       exceeds GCA_LIN_MAX_SET vertices, its sets T_i exceed
 *       GCA_LIN_MAX_GATHER entries, or its rows exceed cap (its rows are then
 *       not written).  Vertex ids are not range-checked on the device: they
 *       must lie in [0, nv).
 * Errors: GCA_EINVAL (NULL pointers, nsets < 0, cap out of range), GCA_EHIP. */
gca_status gca_lin_merge(const int32_t *vt_off, const int32_t *vt_list, const int32_t *tri,
                         const int32_t *set_off, const int32_t *set_vtx, int32_t nsets, int32_t cap,
                         int32_t *out_tri, int32_t *out_loc, int32_t *out_count, void *stream);

/* Dense FP64 blocks G|rows x cols of the linear-basis Galerkin matrix by
 * triangle-pair assembly (Section 5) over the merged lists of
 * gca_lin_merge, one workgroup per block, the regular rule of order q on both
 * triangles of every pair (collapsed Gauss, q = 1..4; or, sym = 1, the
 * symmetric rules of degree 2 q - 2, q = 2, 3).  Pairs of triangles with a
 * common vertex (identical, common edge, common vertex) take, when q_s > 0,
 * the Sauter-Schwab rules with q_s Gauss points per variable and the nodal
 * weights (Sections 6 and 8's touching cases, Section 5's basis).
 * xyz: device FP64, nv x 3 vertex coordinates; tri: device int32, nt x 3.
 * m_tri, m_loc, m_count, cap: the outputs of gca_lin_merge and its cap;
 * set_off: device int32, the subsets given to gca_lin_merge (sizes n, m).
 * blk_row, blk_col: device int32, nblk subset ids: block b is rows subset
 *       blk_row[b] x columns subset blk_col[b].
 * q_s: 0 .. 32; 0 leaves touching pairs out (see status 1).
 * out: device FP64, nblk x ld: block b row-major at out[b ld + i m + j]
 *       (ld >= n m of every block; the rest of the stride is not written).
 * status: device int32, nblk: 0 ok; 1 (q_s = 0 only) a triangle of the row
 *       list and one of the column list share a vertex (the block is written
 *       as zeros); 2 a limit above is exceeded or a merge count is -1 (block
 *       written as zeros where it fits, else not at all).
 * Errors: GCA_EINVAL (NULL pointers, nblk < 0, ld < 0, unsupported q / sym /
 * q_s), GCA_EHIP. */
gca_status gca_lin_blocks(const double *xyz, const int32_t *tri, const int32_t *m_tri,
                          const int32_t *m_loc, const int32_t *m_count, int32_t cap,
                          const int32_t *set_off, const int32_t *blk_row, const int32_t *blk_col,
                          int32_t nblk, int64_t ld, int32_t q, int32_t sym, int32_t q_s, double *out,
                          int32_t *status, void *stream);

/* Dense FP64 blocks of the collocation matrix of the linear nodal basis
 * (Section 6: g_ij = int g(x_i, y) phi_j(y) dy with x_i a mesh vertex, a single
 * integral), one workgroup per block.  Rows: the vertices of row subset
 * blk_row[b] (set_vtx[set_off[r] ..], the collocation points; no merge
 * needed); columns: the nodal functions of the vertices of column subset
 * blk_col[b], integrated over that subset's merged triangle list
 * (gca_lin_merge).  A triangle with the collocation point as a corner takes the
 * Duffy transformation at that corner with q_s Gauss points (1 .. 32; the
 * radial variable is integrated exactly); the others the regular rule of order
 * q (collapsed Gauss q = 1..4, or sym = 1: the symmetric rules q = 2, 3).
 * Arguments as in gca_lin_blocks; set_vtx: device int32, the subsets' vertex
 * ids given to gca_lin_merge.  out: block b row-major at out[b ld + i m + j]
 * (ld >= n m of every block).  status: 0 ok; 2 a subset exceeds
 * GCA_LIN_MAX_BLOCK_SET vertices, the column list exceeds GCA_LIN_MAX_TRIS
 * triangles or its merge count is -1, or a column vertex lies in more than
 * GCA_LIN_MAX_DEGREE of them (block written as zeros).
 * Errors: GCA_EINVAL (NULL pointers, nblk < 0, ld < 0, unsupported q / sym /
 * q_s), GCA_EHIP. */
gca_status gca_coll_blocks(const double *xyz, const int32_t *tri, const int32_t *set_vtx,
                           const int32_t *m_tri, const int32_t *m_loc, const int32_t *m_count, int32_t cap,
                           const int32_t *set_off, const int32_t *blk_row, const int32_t *blk_col,
                           int32_t nblk, int64_t ld, int32_t q, int32_t sym, int32_t q_s, double *out,
                           int32_t *status, void *stream);

/* ---- GCA-H^2 with the nodal basis (Sections 2-5 over the vertices) ----
 *
 * The index set is the vertices (one nodal function each).  The cluster tree
 * splits the vertex positions at the median of the longest extent of their
 * bounding box (ties by vertex id); a cluster's box, used by the
 * admissibility condition max(diam t, diam s) <= 2 eta dist(t, s) and by the
 * Green points of Section 2, encloses the supports of its functions (every
 * triangle of T_i).  The Green factor A of a cluster has one row per vertex:
 * the integrals of g(x, z_nu) and of the normal derivative against phi_i over
 * its support (collapsed Gauss of order q_A on every triangle, the nodal
 * weight); full-pivot ACA and the nested bases follow Sections 3-4 as for the
 * piecewise-constant basis.  The coupling matrices G|t~ x s~ (the rule of
 * order q_c on both triangles) and the nearfield blocks (order q_r, touching
 * pairs by Sauter-Schwab with q_s points per variable) are assembled once by
 * the pair-wise kernels above and stored; the product is FP64. */
typedef struct gca_lin_h2_s *gca_lin_h2;

/* Builds the approximation.  mesh: host arrays (copied).  leaf: vertices per
 * leaf cluster, 1..64.  p: eta, eps, omega_scale, green_m, q_A, q_r, q_s,
 * q_c (0: q_r), sym_rules, alloc / free / alloc_ctx as for gca_build (q_nr,
 * ss_fp32 and serial are not used; q_r and q_c: 1..4, or 2, 3 with
 * sym_rules).  Synchronises the stream.  *out: a handle, gca_lin_destroy.
 * Errors: GCA_EINVAL, GCA_EMESH, GCA_ENOMEM, GCA_EHIP, GCA_EINTERNAL (a pivot
 * or leaf chunk outside the pair-wise kernels' limits). */
gca_status gca_lin_build(const gca_mesh *mesh, int32_t leaf, const gca_params *p, void *stream, gca_lin_h2 *out);

/* y = G~ x for the nodal basis: x, y device FP64 vectors of n_v entries in the
 * original vertex order (y may not alias x); queued on the stream.  Calls
 * on one handle share its work vectors: do not overlap them.
 * Errors: GCA_EINVAL, GCA_EHIP. */
gca_status gca_lin_matvec(gca_lin_h2 h, const double *x, double *y, void *stream);

/* info[8] = {n_v, clusters, coupling blocks, nearfield blocks (both
 * orientations), largest rank, sum of the ranks, stored coupling entries,
 * stored nearfield entries}.  Errors: GCA_EINVAL. */
gca_status gca_lin_info(gca_lin_h2 h, int64_t *info);

/* Host arrays: perm[n_v] (cluster position -> vertex id), ranks[clusters]
 * (pre-order), pivots[sum of ranks] (vertex ids, cluster by cluster in
 * pre-order, each in pivot order).  Errors: GCA_EINVAL. */
gca_status gca_lin_export(gca_lin_h2 h, int32_t *perm, int32_t *ranks, int32_t *pivots);

/* Frees the handle and its device memory (synchronises the device). */
void gca_lin_destroy(gca_lin_h2 h);

#ifdef __cplusplus
}
#endif

#endif /* GCA_LINEAR_H */
