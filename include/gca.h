/*
 * gca.h -- C-ABI of libgca: Green cross approximation (GCA) H^2-matrix
 * compression of the Laplace single-layer Galerkin matrix on MI355X (gfx950).
 *
 * The operator (Section 1, Eq. G_def) is
 *     g_ij = int_{t_i} int_{t_j} 1 / (4 pi |x - y|) dy dx
 * for piecewise-constant basis functions, one per flat triangle t_i
 * (Section 2).  The library builds the GCA-H^2 approximation of Sections 2-4
 * (Green quadrature on the boundary of a box around each cluster, cross
 * approximation of the resulting thin factor, nested bases with transfer
 * matrices) and applies it with coupling and nearfield blocks recomputed on
 * the fly by triangle-pair quadrature (one list per Sauter case, Section 8).
 *
 * Conventions for every call:
 *   - return value: GCA_OK (0) or a negative gca_status; nothing throws or
 *     aborts; gca_last_error() gives a thread-local message for the last
 *     non-OK status;
 *   - arguments are validated before any device work is queued;
 *   - "host" pointers are plain CPU memory, read during the call only;
 *     "device" pointers are HIP device memory owned by the caller;
 *   - stream arguments are hipStream_t (NULL = the default stream); calls that
 *     take a stream queue their work on it and return without synchronising
 *     unless stated otherwise;
 *   - vectors are indexed in the ORIGINAL triangle order of the mesh.
 */
#ifndef GCA_H
#define GCA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GCA_OK = 0,
    GCA_EINVAL = -1,     /* invalid argument */
    GCA_ENOMEM = -2,     /* device or host allocation failed */
    GCA_EHIP = -3,       /* a HIP runtime call or kernel launch failed */
    GCA_EMESH = -4,      /* invalid mesh (index out of range, zero-area or
                            duplicate triangle, non-manifold edge) */
    GCA_ENOTSPD = -5,    /* CG met a non-positive curvature p^T G p <= 0 */
    GCA_ENOCONV = -6,    /* iterative solve did not reach its tolerance */
    GCA_EINTERNAL = -7
} gca_status;

/* Arithmetic of a matrix-vector product.
 * GCA_FP64 : every quadrature, transfer and accumulation in FP64.
 * GCA_MIXED: regular-pair quadrature (nearfield and coupling), kernel
 *            evaluation and basis transfers in FP32 with FP32 accumulation;
 *            touching pairs (Sauter-Schwab) in FP64 (edge vectors, surface
 *            elements, Gauss loops and values), unless the handle was built
 *            with gca_params.ss_fp32 = 1, which runs their Gauss loops in
 *            FP32 on FP64 edge vectors (values still kept in FP64). */
typedef enum { GCA_FP64 = 0, GCA_MIXED = 1 } gca_precision;

/* Element type of the vectors of h2_matvec (x and y alike). */
typedef enum { GCA_F64 = 0, GCA_F32 = 1 } gca_dtype;

/* Device memory callbacks.  alloc returns `bytes` bytes of device memory
 * (aligned to at least 256 bytes) usable on `stream`, or NULL when it cannot;
 * free releases a block that alloc returned, once no queued work uses it.
 * `stream` is the hipStream_t of the call that allocates (build, store,
 * solve, gradient, energy, entries; NULL = the default stream) and, for free,
 * NULL: the library synchronises the device before it frees.  ctx is
 * gca_params.alloc_ctx, passed through unchanged. */
typedef void *(*gca_alloc_fn)(size_t bytes, void *stream, void *ctx);
typedef void (*gca_free_fn)(void *ptr, void *stream, void *ctx);

/* Flat triangle mesh (host memory).  xyz: nv x 3 vertex coordinates (FP64,
 * row-major); tri: nt x 3 vertex indices (0-based, row-major).  Copied during
 * the call that receives it. */
typedef struct {
    int64_t nv, nt;
    const double *xyz;
    const int32_t *tri;
} gca_mesh;

/* Parameters of the approximation (Section 2: admissibility parameter eta;
 * Green quadrature order; Section 3: cross-approximation tolerance). */
typedef struct {
    double eta;          /* admissible iff max(diam t, diam s) <= 2 eta dist(t, s) */
    double eps;          /* ACA stop: ||R||_F <= eps ||A||_F                       */
    double omega_scale;  /* omega = cluster box enlarged by omega_scale*diam/eta per side */
    int32_t green_m;     /* Gauss points per direction on each box face (k = 6 m^2) */
    int32_t q_A;         /* triangle rule order of the Green factor A            */
    int32_t q_r;         /* regular pair rule order (per triangle: q_r^2 points)  */
    int32_t q_nr;        /* order for near-regular pairs (vertices joined by an edge) */
    int32_t q_s;         /* Sauter-Schwab order (>= 2) for touching pairs         */
    int32_t q_c;         /* regular rule order for the coupling entries G|t~ x s~
                            (admissible blocks); 0 means q_c = q_r              */
    int32_t sym_rules;   /* 0: the disjoint pairs (regular, near-regular, coupling)
                            use the collapsed Gauss rule of their order on each
                            triangle (q^2 points, the disjoint case of Sauter's
                            rules, Section 8); 1: the fully symmetric rule of the
                            same polynomial degree 2q - 2 (q = 2: 3 points, q = 3:
                            6 points), which needs q_r, q_nr, q_c in {2, 3}.  The
                            Green factor keeps the collapsed rule of order q_A. */
    int32_t ss_fp32;     /* 0 (default): touching pairs in FP64 in both products;
                            1: the mixed product runs the Sauter-Schwab Gauss
                            loops in FP32 (FP64 edge vectors and values)       */
    int32_t serial;      /* 0 (default): a product overlaps its phases on two
                            side streams of the handle (touching values; the
                            transform chain with the coupling blocks) beside
                            the nearfield blocks on the caller's stream;
                            1: every phase on the caller's stream in order, so
                            each kernel has the chip to itself (per-kernel
                            measurement)                                     */
    gca_alloc_fn alloc;  /* device memory of the handle and of every call on it;
                            NULL (with free NULL): hipMalloc / hipFree          */
    gca_free_fn free;    /* NULL exactly when alloc is NULL                      */
    void *alloc_ctx;     /* passed to alloc and free                             */
} gca_params;

#define GCA_NPHASE 9

typedef struct gca_tree_s *gca_tree;   /* host object; gca_tree_destroy */
typedef struct gca_h2_s *gca_h2;       /* owns its device memory; gca_destroy */

/* Statistics of a built approximation (gca_stats). */
typedef struct {
    int64_t n, nv, n_clusters, n_leaves, depth;
    int64_t n_far, n_near;               /* admissible / inadmissible leaf blocks, both orders */
    int64_t n_far_sym, n_near_sym;       /* the halves computed (t < s, t <= s) */
    int64_t n_ident, n_edge, n_vert, n_nearreg;   /* pair lists (unordered) */
    int64_t coupling_entries;            /* sum over t < s admissible of |t~| |s~| */
    int64_t near_pairs;                  /* pairs evaluated by the nearfield-block kernel (t <= s blocks, full tiles) */
    int64_t near_regular_pairs;          /* unordered regular pairs inside near blocks (algorithmic count) */
    int64_t rank_min, rank_max;
    double rank_mean;
    int64_t basis_bytes_fp64;            /* leaf V + transfers E, FP64 */
    double build_ms;                     /* wall time of gca_build (host + device, synchronised) */
    double setup_ms[8];                  /* parts of build_ms: 0 mesh checks + adjacency,
                                            1 pair lists, 2 block tree + list checks,
                                            3 geometry upload + quadrature points,
                                            4 nested basis (Green factor + ACA, all levels),
                                            5 block slots, lists and workspaces, 6-7 unused */
    double phase_ms[GCA_NPHASE + 1];     /* last product's last right-hand side, HIP events
                                            around each phase on the stream it runs on:
                                            0 permute in, 1 forward transform,
                                            2 coupling-block quadrature, 3 coupling reduction,
                                            4 backward transform, 5 nearfield-block quadrature,
                                            6 near-regular list, 7 touching lists (6 and 7 only
                                            for the first right-hand side), 8 gather,
                                            9 total (wall time of the product on the caller's
                                            stream).  Unless gca_params.serial, phases 1-4 (one
                                            side stream) and 7 (another) run beside 5-6, so
                                            0-8 need not add up to 9 and a phase's time is its
                                            duration while it shares the chip */
    int64_t store_entries_far;           /* entries of the stored coupling block rows */
    int64_t store_entries_near;          /* entries of the stored nearfield block rows (masked pairs as zeros) */
    int32_t stored_mask;                 /* precisions with stored block rows (gca_store_blocks) */
    int32_t reserved_i;
    int64_t basis_entries_leaf;          /* entries of the leaf bases V (sum |t^| r_t) */
    int64_t basis_entries_transfer;      /* entries of the transfer matrices E (sum r_t r_parent) */
} gca_stats_t;

/* Default parameters: eta 2, eps 1e-6, omega_scale 0.25, green_m 3, q_A 3,
 * q_r 3, q_nr 3, q_s 4, q_c 3, sym_rules 0, ss_fp32 0, serial 0, no allocator
 * callbacks (hipMalloc / hipFree).  With q_nr == q_r near-regular pairs are
 * integrated by the regular rule inside the nearfield blocks (no separate
 * list). */
void gca_params_default(gca_params *p);

/* Cluster tree over the triangles (Section 4's binary subdivision of index
 * sets into disjoint sons).  Splitting rule: the bounding box of the triangle
 * centroids ((v0+v1)+v2)/3 is cut along its longest axis (lowest axis on
 * ties) at the median: triangles sorted by that centroid coordinate (ties by
 * original id), the first floor(#/2) form the first son.  Clusters with at
 * most leaf_size triangles are leaves.  Each cluster has the axis-parallel
 * bounding box of all vertices of its triangles (Section 2).  Host only.
 * Errors: GCA_EINVAL (null pointers, leaf_size < 1), GCA_EMESH. */
gca_status gca_tree_build(const gca_mesh *mesh, int32_t leaf_size, gca_tree *out);

/* Sizes of a tree: number of clusters (pre-order numbering, root 0) and depth. */
gca_status gca_tree_info(gca_tree t, int64_t *n_clusters, int64_t *depth);

/* Copies the tree to host arrays (any pointer may be NULL):
 * perm[nt]            cluster order -> original triangle id;
 * nodes[5*nc]         begin, end, son0, son1, level (sons -1 for leaves);
 * boxes[7*nc]         lo xyz, hi xyz, diam. */
gca_status gca_tree_export(gca_tree t, int32_t *perm, int32_t *nodes, double *boxes);

void gca_tree_destroy(gca_tree t);

/* Block partition of I x I for admissibility parameter eta (Section 2):
 * admissible iff dist(t, s) > 0 and max(diam t, diam s) <= 2 eta dist(t, s)
 * (axis-parallel boxes); otherwise split every non-leaf member, and keep
 * inadmissible pairs of leaves as nearfield blocks.  Returns the symmetric
 * halves: admissible blocks with t < s and inadmissible leaf blocks with
 * t <= s (each stands for itself and its transpose).  Host only.
 * far / near: host arrays of 2 x capacity int32 (t[0..n), s[0..n)), or NULL
 * to query the counts; n_far / n_near receive the counts.  If a capacity is
 * too small nothing is written to that array and GCA_EINVAL is returned. */
gca_status gca_block_tree(gca_tree t, double eta, int64_t far_capacity, int32_t *far, int64_t *n_far,
                          int64_t near_capacity, int32_t *near, int64_t *n_near);

/* Builds the GCA-H^2 approximation (Sections 2-4, Section 8's three tasks):
 * block tree by admissibility, Green points per cluster, the factor A of
 * Section 2 at the leaves and at the sons' pivots for every parent,
 * full-pivot cross approximation (FP64) giving tau~, leaf bases V and
 * transfer matrices E, and the per-case pair lists for the nearfield.
 * The mesh must be the one the tree was built from.  Synchronises `stream`
 * before returning (one small read-back per tree level).
 * Errors: GCA_EINVAL (parameters), GCA_EMESH, GCA_ENOMEM, GCA_EHIP. */
gca_status gca_build(const gca_mesh *mesh, gca_tree tree, const gca_params *p,
                     void *stream, gca_h2 *out);

/* y = G~ x (Section 4's H^2 representation applied by forward transform,
 * coupling with entries G|t~ x s~ recomputed, backward transform, and
 * nearfield blocks G|t^ x s^ recomputed).  x, y: device, nt x nrhs,
 * column-major with leading dimension ld >= nt, elements of type `dtype`
 * (GCA_F64 double, GCA_F32 float; the product's own arithmetic is set by
 * `precision`, not by dtype: FP32 vectors are widened on entry and the result
 * rounded to FP32 on exit); y is overwritten; x and y must not overlap.
 * precision: gca_precision.  Unless the handle was built with
 * gca_params.serial = 1, the touching-pair values and the transform chain
 * (forward transform, coupling blocks, backward transform) run on two side
 * streams owned by the handle, forked from and joined back into `stream`
 * within the call's work, so `stream` orders the whole product.
 * nrhs > 1: the right-hand sides are taken 16 at a time and every block entry
 * is evaluated once per 16 (the transfer, coupling and nearfield products of
 * the 16 columns on the matrix cores); the first such call in a precision
 * allocates that precision's batched workspaces, held by the handle
 * (16 x (2 n + 2 sum of ranks + partial slots) values, plus 16 n doubles for
 * the mixed product).  nrhs = 1, and products of a precision whose blocks are
 * stored (gca_store_blocks), allocate nothing and go one column at a time.
 * Errors: GCA_EINVAL (null handle or pointers, nrhs < 1, ld < nt, aliasing,
 * unknown dtype or precision), GCA_EHIP. */
gca_status h2_matvec(gca_h2 h, const void *x, void *y, int64_t nrhs, int64_t ld, int32_t dtype,
                     int32_t precision, void *stream);

/* Electrostatic energy of a density u (the single-layer system of Section 1):
 *     E = 1/2 u^T G~ u,   and optionally   g = scale * G~ u
 * (g is dE/du, the gradient of the energy with respect to the density, times
 * scale).  u: device FP64, nt entries, original triangle order.  e: device
 * FP64 scalar receiving E, or NULL.  g: device FP64, nt entries, or NULL.
 * scale: device FP64 scalar, or NULL for 1 (the incoming cotangent of E in a
 * reverse-mode chain).  The product is the one of h2_matvec in `precision`;
 * the dot product is FP64 in a fixed reduction order.  The first call
 * allocates a workspace of nt + 1025 doubles held by the handle.
 * Errors: GCA_EINVAL (null handle or u, both e and g NULL, g overlapping u,
 * unknown precision), GCA_ENOMEM, GCA_EHIP. */
gca_status gca_energy(gca_h2 h, const double *u, const double *scale, double *e, double *g, int32_t precision,
                      void *stream);

/* gca_energy for callers that cannot allocate device memory (work under
 * stream capture, tight serving or optimisation loops, hosts that forbid
 * allocation): the same computation, arguments, checks and results as
 * gca_energy, but its workspace (the dot-product partials and, when g is
 * NULL, the product G~ u) lies in a fixed device array of the library,
 * (1025 + GCA_NOALLOC_MAX_N) doubles = 520 KiB per GPU, held until the process
 * ends.  Allocates nothing (no hipMalloc, no allocator callback).  With g NULL
 * the handle's n must not exceed GCA_NOALLOC_MAX_N (GCA_EINVAL otherwise; pass
 * g, which then receives G~ u, for larger n).  All calls on one GPU share the
 * array: calls that overlap in time on one GPU (different streams, or host
 * threads without ordering) race on it and must be serialised by the caller.
 * Errors: those of gca_energy except GCA_ENOMEM. */
#define GCA_NOALLOC_MAX_N 65536
gca_status gca_energy_noalloc(gca_h2 h, const double *u, const double *scale, double *e, double *g,
                              int32_t precision, void *stream);

/* Stored-block mode (the paper's GPU setup computes and keeps the coupling
 * matrices G|t~ x s~ and the nearfield blocks G|t^ x s^, Section 8's second
 * and third task): computes the entries of every coupling and nearfield block
 * row of the symmetric halves once, with the same quadrature as the
 * recomputing product, and keeps them in device memory for the precisions
 * whose bit is set in `which` (bit GCA_FP64 = 1, bit GCA_MIXED = 2; FP32
 * entries for the mixed product).  Products in a stored precision then read
 * the entries (one pass over (store_entries_far + store_entries_near) x 4 or 8
 * bytes) instead of recomputing them, and reuse the touching and
 * near-regular list values computed here.  which = 0 releases the storage.
 * gca_update_geometry recomputes stored entries; h2_bilinear_grad always
 * recomputes.  Synchronises the stream.
 * Errors: GCA_EINVAL (null handle, unknown bits), GCA_ENOMEM (nothing is
 * stored then), GCA_EHIP. */
gca_status gca_store_blocks(gca_h2 h, int32_t which, void *stream);

/* The stored block entries of one precision (after gca_store_blocks with
 * its bit), for inspection and element-wise checks of the block kernels:
 * kind 0 the coupling blocks G|t~ x s~ of the admissible pairs t < s
 * (Section 4's coupling matrices, Section 8's second task), kind 1 the
 * nearfield blocks G|t^ x s^ of the inadmissible leaf pairs t <= s (Section
 * 8's third task).  Entry k is g(rows[k], cols[k]) with original triangle
 * ids; nearfield entries that the pair lists own (touching pairs, and
 * near-regular pairs when q_nr != q_r) and the lower triangle of diagonal
 * blocks are stored as 0.  rows, cols (int32), vals (FP64; FP32 entries
 * widened): host arrays of capacity entries, or all three NULL to query
 * *count (the number of stored entries of that kind; count may be NULL).
 * Synchronises the stream.
 * Errors: GCA_EINVAL (null handle, unknown precision or kind, blocks of that
 * precision not stored, capacity below the count, only some arrays given),
 * GCA_EHIP. */
gca_status gca_block_entries(gca_h2 h, int32_t precision, int32_t kind, int64_t capacity, int32_t *rows,
                             int32_t *cols, double *vals, int64_t *count, void *stream);

/* Solves G~ u = f by conjugate gradients on the mixed-precision product
 * (inner iterations, stopped when the inner residual falls below
 * inner_rtol times its start) inside FP64 iterative refinement: each outer
 * step forms r = f - G~ u with the FP64 product and adds the inner
 * correction.  Stops when ||f - G~ u||_2 <= rtol ||f||_2 (FP64 product).
 * The solved equation is the one the paper's boundary element method leads
 * to (Section 1; the single-layer system for exterior electrostatics).
 * f, u: device FP64, n entries, original triangle order; u is overwritten
 * (the start is u = 0); f and u must not overlap.
 * iters_out (host, may be NULL): [0] outer refinement steps, [1] inner CG
 * iterations in total.  relres_out (host, may be NULL): final relative
 * FP64 residual.  Synchronises the stream once per iteration.
 * Errors: GCA_EINVAL; GCA_ENOTSPD if CG meets p^T G~ p <= 0; GCA_ENOCONV if
 * max_outer steps do not reach rtol (u then holds the last iterate);
 * GCA_ENOMEM; GCA_EHIP. */
gca_status gca_solve_refined(gca_h2 h, const double *f, double *u, double rtol, int32_t max_outer,
                             double inner_rtol, int32_t max_inner, int32_t *iters_out, double *relres_out,
                             void *stream);

/* Moves the vertices to xyz (host, nv x 3, same mesh topology) keeping the
 * structure of the approximation frozen: cluster tree, block partition,
 * boxes omega, Green points, and every cluster's pivot rows I and Green
 * columns J.  Leaf bases and transfer matrices are recomputed as
 * V^ = A^[:, J] A^[I, J]^{-1} from the Green factor of Section 2 at the new
 * triangle positions (equal to the cross-approximation basis when xyz is the
 * mesh of gca_build).  The energy and product of the frozen approximation are
 * then smooth functions of xyz, which is what h2_bilinear_grad
 * differentiates.  Synchronises the stream.  Errors: GCA_EINVAL, GCA_ENOMEM,
 * GCA_EHIP. */
gca_status gca_update_geometry(gca_h2 h, const double *xyz, void *stream);

/* Adjoint of the product with respect to the vertex coordinates:
 *     dxyz += alpha * scale * d(a^T G~(X) b) / dX
 * with the structure frozen (tree, blocks, boxes, Green points, pivot rows I
 * and Green columns J of every cluster; the bases are the functions
 * V^ = A^[:, J] A^[I, J]^{-1} of the vertex positions that gca_update_geometry
 * evaluates).  Terms: derivatives of every nearfield and coupling entry
 * (recomputed, not stored), of the touching pairs' Sauter-Schwab rules, and of
 * the Green factor rows through the interpolation chain of Sections 3-4.
 * For the energy E = 1/2 u^T G~ u pass a = b = u, alpha = 1/2.
 * a, b: device FP64, n entries, original triangle order; scale: device FP64
 * scalar or NULL for 1 (an incoming cotangent that stays on the device);
 * dxyz: device FP64, nv x 3 row-major, accumulated.  precision: GCA_FP64, or
 * GCA_MIXED (FP32 nearfield / coupling derivatives and transfers; touching
 * pairs and bases in FP64).  The first call allocates the adjoint's
 * workspaces and index maps (held by the handle).  Stream-ordered, no
 * synchronisation after the first call.
 * Errors: GCA_EINVAL, GCA_ENOMEM, GCA_EHIP. */
gca_status h2_bilinear_grad(gca_h2 h, const double *a, const double *b, double alpha, const double *scale,
                            double *dxyz, int32_t precision, void *stream);

/* Galerkin entries g_{I[k], J[k]} (Eq. G_def) for m pairs, computed by the
 * same device quadrature the matrix-vector product uses (the pair's Sauter
 * case decides the rule; touching pairs follow the handle's ss_fp32 in the
 * mixed precision).  I, J: device int32 original triangle ids; out: device
 * FP64, m values.  Classifies the pairs on the host (copies I and J back and
 * synchronises the stream); the device workspace of 24 bytes per pair is held
 * by the handle and grown when a call needs more.
 * Errors: GCA_EINVAL, GCA_ENOMEM, GCA_EHIP. */
gca_status gca_entries(gca_h2 h, const int32_t *I, const int32_t *J, int64_t m,
                       double *out, int32_t precision, void *stream);

/* Galerkin entries of the double-layer operator for m pairs (Section 1: the
 * second-kind formulation uses the normal derivative of g at y; Section 6:
 * unit normals of the triangles):
 *     k_ij = int_{t_i} int_{t_j} n_j . (x - y) / (4 pi |x - y|^3) dy dx,
 * n_j the unit normal of t_j from its mesh orientation (v1 - v0) x (v2 - v0).
 * Not symmetric.  The pair's Sauter case decides the rule, as for g_ij:
 * identical pairs are 0 (x - y lies in the plane of t_j); common edge and
 * common vertex pairs use the Sauter-Schwab maps with q_s Gauss points in
 * each of the four variables; the others the regular rules of order q_r /
 * q_nr of the handle.  FP64.  I, J: device int32 original triangle ids (an id
 * outside [0, n) gives NaN); out: device FP64, m values.  The pairs are
 * classified on the device and the work is queued on the stream without
 * synchronisation; the first call uploads the mesh's vertex adjacency (for
 * the near-regular class), held by the handle.
 * Errors: GCA_EINVAL, GCA_ENOMEM, GCA_EHIP. */
gca_status gca_dl_entries(gca_h2 h, const int32_t *I, const int32_t *J, int64_t m, double *out, void *stream);

/* Copies the nested basis to host arrays for inspection (any may be NULL):
 * ranks[nc]                   |tau~| per cluster (pre-order numbering);
 * pivots[sum ranks]           original triangle ids of tau~, clusters in
 *                             pre-order, each in pivot order;
 * basis[sum over leaves |tau^| * rank + sum over non-root clusters rank(son) *
 *       rank(parent)]        leaf V (rows in cluster order, row-major) then
 *                             transfer matrices E (row-major), clusters in
 *                             pre-order.  Synchronises the device. */
gca_status gca_basis_export(gca_h2 h, int32_t *ranks, int32_t *pivots, double *basis);

/* Sizes for gca_basis_export: total pivots and total basis entries. */
gca_status gca_basis_sizes(gca_h2 h, int64_t *n_pivots, int64_t *n_basis);

gca_status gca_stats(gca_h2 h, gca_stats_t *out);

/* Phase times (ms, HIP events on the stream of each product) of the last
 * min(max_products, 64, products so far) single-right-hand-side products,
 * oldest first: out[q * (GCA_NPHASE + 1) + k], k as in gca_stats_t.phase_ms
 * (each phase timed on the stream it ran on).  out may be NULL to query
 * *count.  Synchronises with the last product. */
gca_status gca_phase_times(gca_h2 h, int64_t max_products, double *out, int64_t *count);

void gca_destroy(gca_h2 h);

/* Thread-local message describing the last non-OK status ("" if none). */
const char *gca_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* GCA_H */
