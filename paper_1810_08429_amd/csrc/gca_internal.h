// Internal declarations of libgca (host structures, device buffers, kernel
// launchers).  Not part of the public interface (include/gca.h).
#pragma once

#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <cstdint>
#include <functional>
#include <string>
#include <thread>
#include <vector>

#include "../../include/gca.h"

namespace gca {

// ------------------------------------------------------- host threading --
// Host worker count: the hardware threads, at most 16.
inline int host_threads()
{
    return (int)std::max<unsigned>(1, std::min<unsigned>(16, std::thread::hardware_concurrency()));
}

// f(i0, i1) over [0, n) in contiguous chunks on host_threads() threads.
// Results must not depend on which thread runs which chunk.
template <class F>
void parallel_for(int64_t n, F &&f, int64_t min_chunk = 1024)
{
    if (n <= 0) return;
    const int nthr = host_threads();
    const int64_t nchunk = std::max<int64_t>(1, std::min<int64_t>(4 * nthr, (n + min_chunk - 1) / min_chunk));
    if (nchunk == 1) {
        f((int64_t)0, n);
        return;
    }
    std::atomic<int64_t> next{0};
    auto worker = [&]() {
        for (;;) {
            const int64_t c = next.fetch_add(1);
            if (c >= nchunk) break;
            f(n * c / nchunk, n * (c + 1) / nchunk);
        }
    };
    std::vector<std::thread> th;
    for (int t = 1; t < std::min<int64_t>(nthr, nchunk); ++t) th.emplace_back(worker);
    worker();
    for (auto &x : th) x.join();
}

// ---------------------------------------------------------------- errors --
gca_status set_error(gca_status s, const std::string &msg);
void clear_error();

#define GCA_HIP_TRY(expr)                                                        \
    do {                                                                         \
        hipError_t e_ = (expr);                                                  \
        if (e_ != hipSuccess)                                                    \
            return ::gca::set_error(GCA_EHIP, std::string(#expr " failed: ") +   \
                                                  hipGetErrorString(e_));        \
    } while (0)

#define GCA_TRY(expr)                                                            \
    do {                                                                         \
        gca_status s_ = (expr);                                                  \
        if (s_ != GCA_OK) return s_;                                             \
    } while (0)

// --------------------------------------------------------------- geometry --
struct Mesh {
    int64_t nv = 0, nt = 0;
    std::vector<double> xyz;    // nv x 3
    std::vector<int32_t> tri;   // nt x 3
};

// Copies the mesh and checks coordinates, indices and areas; with topology
// also duplicate triangles and non-manifold edges.
gca_status mesh_copy_validate(const gca_mesh *m, Mesh &out, bool topology = true);

// Adjacency needed for the pair classes (Section 8: identical / common edge /
// common vertex / disjoint, plus "near-regular" disjoint pairs that contain a
// mesh edge between them).
struct Adjacency {
    std::vector<int64_t> vt_ptr;   // vertex -> triangles
    std::vector<int32_t> vt;
    std::vector<int64_t> vv_ptr;   // vertex -> vertices joined by an edge
    std::vector<int32_t> vv;
};
gca_status build_adjacency(const Mesh &m, Adjacency &adj);

// -------------------------------------------------------------- clustering --
struct Node {
    int32_t begin, end, son[2], parent, level;
    double lo[3], hi[3], diam;
};

}  // namespace gca

struct gca_tree_s {
    int64_t nt = 0, nv = 0;
    int32_t leaf = 0;
    std::vector<int32_t> perm;      // cluster position -> original triangle id
    std::vector<gca::Node> nodes;   // pre-order
    int32_t depth = 0;
    std::vector<double> mesh_xyz;   // the mesh the tree was built from (to check gca_build)
    std::vector<int32_t> mesh_tri;
};

namespace gca {

gca_status tree_build(const Mesh &m, int32_t leaf, gca_tree_s &t);
// The tree over the vertices (the nodal basis of Section 5): points the
// vertices, boxes those of the supports (every triangle of T_v, given as the
// CSR vt_ptr / vt); perm maps positions to vertex ids.
gca_status tree_build_vertices(const Mesh &m, const std::vector<int64_t> &vt_ptr, const std::vector<int32_t> &vt,
                               int32_t leaf, gca_tree_s &t);

// Block partition (Section 2 admissibility) as symmetric halves.
struct Blocks {
    std::vector<int32_t> far_t, far_s;     // admissible, t < s
    std::vector<int32_t> near_t, near_s;   // inadmissible leaf pairs, t <= s
    int64_t n_far_full = 0, n_near_full = 0;
};
void block_tree(const gca_tree_s &t, double eta, Blocks &b);

// Pairs that the regular rule does not handle, in cluster positions.
// kind: 0 identical, 1 common edge, 2 common vertex, 3 near-regular.
// The first triangle is the one with the smaller ORIGINAL id; for touching
// pairs `code` packs the vertex orders (see kernels) of first | second << 4.
struct PairLists {
    std::vector<int32_t> a, b, code;   // positions of first / second, order code
    int64_t off[5] = {0, 0, 0, 0, 0};  // class ranges in the concatenated list
    // row CSR over positions: for position i, entries (other position, pair id)
    std::vector<int64_t> row_ptr;
    std::vector<int32_t> row_other, row_pair;
    // value CSRs used by the product: touching pairs (classes 0-2) and
    // near-regular pairs (class 3) separately; pair p writes its value to
    // slot_a[p] (row of its first triangle) and slot_b[p] (row of the second,
    // -1 for identical pairs)
    std::vector<int64_t> t_ptr, n_ptr;
    std::vector<int32_t> t_other, n_other;
    std::vector<int32_t> slot_a, slot_b;
};
// with_nearreg = false: near-regular pairs use the regular rule (q_nr == q_r)
// and stay in the nearfield blocks, so no list is built for them.  With
// with_nearreg, near_ok(position a, position b) tells whether a near-regular
// pair lies in a nearfield block (only those are listed; a near-regular pair
// of an admissible block is represented by that block like every other pair
// of it); NULL lists them all.
gca_status build_pair_lists(const Mesh &m, const Adjacency &adj, const gca_tree_s &t, bool with_nearreg,
                            PairLists &pl, const std::function<bool(int32_t, int32_t)> &near_ok = nullptr);
int classify_pair(const Mesh &m, const Adjacency &adj, int32_t i, int32_t j, int32_t *code);
const char *last_error_cstr();

// Gauss-Legendre on [0,1] (ascending nodes).
void gauss_legendre01(int q, double *x, double *w);

// ------------------------------------------------------------- device data --
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

}  // namespace gca

namespace gca {
// Frozen-structure basis data (pivot rows / columns fixed): device copies of
// the per-cluster row lists and workspaces of the refresh and the adjoint.
struct Frozen {
    bool ready = false;
    bool basis_current = false;      // LU factors and V^ hold for the current geometry
    int32_t *d_batch = nullptr;      // cluster ids 0..nc-1
    int32_t *d_pivrow = nullptr, *d_pivcol = nullptr;
    int64_t *d_arow_off = nullptr;
    int32_t *d_arows = nullptr;
    int64_t *d_aj_off = nullptr, *d_c_off = nullptr;
    int64_t *d_roff = nullptr;       // nc + 1: prefix sums of the ranks (cluster order)
    std::vector<int64_t> aj_off, c_off;
    int64_t n_aj = 0, n_c = 0;
    double *d_AJ = nullptr, *d_Vh = nullptr, *d_tmp = nullptr, *d_LU = nullptr;
    double *d_Vbar = nullptr, *d_Z = nullptr;
    double *d_Cinv = nullptr;        // C^{-1} = A^[I, J]^{-1} per cluster (r x r at c_off)
    int32_t *d_perm = nullptr;
    int64_t *d_copy_jobs = nullptr;  // V / E copies from d_Vh
    int32_t n_vjobs = 0, n_ejobs = 0;
};
}  // namespace gca

namespace gca {
// Workspaces and index maps of h2_bilinear_grad (allocated by its first call).
struct GradWs {
    bool ready = false;
    double *ap = nullptr, *bp = nullptr;        // permuted a, b (FP64)
    float *apf = nullptr, *bpf = nullptr;       // permuted a, b (mixed)
    void *xa = nullptr, *xb = nullptr, *ya = nullptr, *yb = nullptr;   // n_piv of T (sized for FP64)
    void *cpart = nullptr;                      // coupling partials (sized for FP64)
    double *gnear = nullptr, *gfar = nullptr;   // 9 per near / coupling slot entry
    double *gt = nullptr, *gn = nullptr;        // 9 per pair-CSR entry
    double *gb = nullptr;                       // 9 per row of every cluster's A^
    double *dT = nullptr;                       // 9 per triangle position
    int32_t *leaf_of = nullptr, *leaf_index = nullptr;
    int64_t *pocc_ptr = nullptr;                // position -> occurrences as a pivot
    int32_t *pocc = nullptr, *piv_cluster = nullptr;
    int64_t *rocc_ptr = nullptr;                // position -> occurrences as a row of some A^
    int32_t *rocc = nullptr;
    int64_t *vptr = nullptr;                    // vertex -> (position, local slot)
    int32_t *vpos = nullptr, *vslot = nullptr;
};
}  // namespace gca

struct gca_h2_s {
    gca_params prm{};
    gca::Frozen fz;
    gca::GradWs gw;
    int64_t n = 0, nv = 0, nc = 0;
    int32_t depth = 0;
    gca_tree_s tree;                 // private copy
    gca::Mesh mesh;
    gca::Adjacency adj;
    gca::Blocks blk;
    gca::PairLists pl;

    int32_t PA_rows = 0;             // Green-factor points per row if not q_A^2 (the nodal basis)

    // host copies of the basis structure
    std::vector<int32_t> rank;       // per cluster
    std::vector<int64_t> piv_off;    // per cluster offset into pivots / xhat
    std::vector<int32_t> pivots;     // positions, per cluster in pivot order
    std::vector<int32_t> pivrow;     // per pivot: local row index in the cluster's A (pivot order)
    std::vector<int32_t> pivcol;     // per pivot: Green column of the factor A (pivot order)
    std::vector<int64_t> arow_off;   // per cluster: offset of its row list in arows
    std::vector<int32_t> arows;      // rows of each cluster's A (leaf: its triangles; parent: sons' pivots)
    std::vector<int64_t> v_off;      // leaf V offsets (entries)
    std::vector<int64_t> e_off;      // E offsets for non-root clusters (entries)
    int64_t n_piv = 0, n_v = 0, n_e = 0;

    // device memory (all owned)
    std::vector<void *> allocs;
    double *d_xyz = nullptr;         // nv x 3
    int32_t *d_tv = nullptr;         // n x 3 vertex ids, cluster order
    int32_t *d_perm = nullptr;       // position -> original id
    int32_t *d_iperm = nullptr;      // original id -> position
    double *d_qr = nullptr;          // n x Pr x 4 (x, y, z, w*J), regular rule
    double *d_qnr = nullptr;         // n x Pnr x 4, near-regular rule
    double *d_qA = nullptr;          // n x PA x 4 (may alias d_qr)
    double *d_qc = nullptr;          // n x Pc x 4, coupling rule (may alias d_qr)
    double *d_cent = nullptr;        // n x 4: reference point per triangle (mean of its d_qr points)
    float *d_qloc32 = nullptr;       // n x Pr x 4: d_qr points relative to it (FP32), weights
    double *d_box = nullptr;         // nc x 8: lo, hi, diam, 0

    int32_t *d_piv = nullptr;        // pivot positions
    int64_t *d_piv_off = nullptr;    // nc
    int32_t *d_rank = nullptr;       // nc
    double *d_V = nullptr;           // leaf bases, row-major |t^| x r   (FP64)
    double *d_Vt = nullptr;          // leaf bases, column-major        (FP64)
    double *d_E = nullptr;           // transfers, row-major r' x r     (FP64)
    double *d_Et = nullptr;          // transfers, column-major         (FP64)
    float *d_Vf = nullptr, *d_Vtf = nullptr, *d_Ef = nullptr, *d_Etf = nullptr;
    int64_t *d_v_off = nullptr, *d_e_off = nullptr;

    // clusters by level (for the level-wise transfer launches)
    std::vector<std::vector<int32_t>> level_clusters;
    std::vector<int32_t *> d_level_clusters;
    std::vector<int32_t> leaves;
    int32_t *d_leaves = nullptr;
    int32_t *d_node = nullptr;       // nc x 5: begin, end, son0, son1, parent

    // coupling blocks (t < s)
    int32_t *d_far = nullptr;        // 2 x n_far_sym
    int64_t *d_far_slot = nullptr;   // 2 x n_far_sym: partial-slot offsets (row, col)
    int64_t *d_cslot_ptr = nullptr;  // nc + 1: per cluster CSR of partial slots
    int64_t *d_cslot = nullptr;
    int64_t n_cslot_total = 0;       // size of the coupling partial buffer
    int32_t max_rank = 0;

    // coupling block rows (product path): one group per row cluster t with
    // blocks (t, s); the columns of its blocks are concatenated
    int32_t n_far_groups = 0;
    int32_t *d_fg_t = nullptr;       // ng: row cluster
    int64_t *d_fg_ptr = nullptr;     // ng + 1: column ranges
    int64_t *d_fg_rslot = nullptr;   // ng: row-partial slot
    int32_t *d_fcol_e = nullptr;     // per column: pivot entry piv_off[s] + j
    int32_t *d_fcol_s = nullptr;     // per column: cluster s
    int64_t *d_fcol_out = nullptr;   // per column: column-partial slot
    int64_t *d_fg_soff = nullptr;    // ng: offset of the group's stored entries (rank_t x columns)
    int64_t n_far_store = 0;         // stored coupling entries
    int64_t *d_gslot_ptr = nullptr;  // nc + 1: per cluster CSR of partial slots
    int64_t *d_gslot = nullptr;
    int64_t n_gslot_total = 0;
    int64_t n_piv_total = 0;         // sum of ranks
    int32_t *d_piv_cluster = nullptr;   // per pivot entry: its cluster
    float *d_pq32 = nullptr;         // per pivot entry: Pr x (x, y, z, w) relative to its cluster's centre

    // near blocks (t <= s)
    int32_t *d_near = nullptr;       // 2 x n_near_sym
    int64_t *d_near_slot = nullptr;  // 2 x n_near_sym (col slot -1 on diagonal)
    int64_t *d_nslot_ptr = nullptr;  // n_leaves + 1 (leaf index order)
    int64_t *d_nslot = nullptr;
    int64_t n_nslot_total = 0;
    int32_t max_leaf = 0;

    // nearfield block rows (product path): one group per leaf t with its
    // blocks (t, s), t <= s, diagonal first; columns concatenated
    int32_t n_near_groups = 0;
    int32_t *d_ng_t = nullptr;       // ng: row leaf
    int64_t *d_ng_ptr = nullptr;     // ng + 1: column ranges
    int64_t *d_ng_rslot = nullptr;   // ng: row-partial slot
    int64_t *d_ng_moff = nullptr;    // ng + 1: mask ranges (chunk-major, one word per row)
    int32_t *d_ncol_pos = nullptr;   // per column: position
    int64_t *d_ncol_out = nullptr;   // per column: column-partial slot
    uint64_t *d_nmask = nullptr;     // per (group, chunk, row): pairs owned by the list kernels
    int64_t *d_ng_soff = nullptr;    // ng: offset of the group's stored entries (rows x columns)
    int64_t n_near_store = 0;        // stored nearfield entries (masked pairs as zeros)
    int64_t *d_gnslot_ptr = nullptr; // n_leaves + 1 (leaf index order)
    int64_t *d_gnslot = nullptr;
    int64_t n_gnslot_total = 0;

    // pair lists
    int32_t *d_pa = nullptr, *d_pb = nullptr, *d_pcode = nullptr;
    int64_t *d_prow_ptr = nullptr;
    int32_t *d_prow_other = nullptr;
    int64_t *d_tptr = nullptr, *d_nptr = nullptr;
    int32_t *d_tother = nullptr, *d_nother = nullptr;
    int32_t *d_slot_a = nullptr, *d_slot_b = nullptr;
    // touching values of the product (FP64) in a leaf-ELL layout: leaf li
    // owns tell_k[li] x nr columns from tell_off[li], entry (k, i) is the k-th
    // touching partner of its row i (padding: value 0, partner = the row);
    // pair p writes to tslot_a[p] and tslot_b[p] (-1: identical pair)
    double *d_tval = nullptr;
    int64_t *d_tell_off = nullptr;
    int32_t *d_tell_k = nullptr, *d_tell_other = nullptr;
    int32_t *d_tslot_a = nullptr, *d_tslot_b = nullptr;
    double *d_nval = nullptr;        // near-regular values, row CSR (FP64 path)
    float *d_nvalf = nullptr;        // near-regular values, row CSR (mixed path)

    // stored block rows (gca_store_blocks): entries of the coupling and the
    // nearfield block rows per precision; the product then reads them
    double *d_far_g64 = nullptr, *d_near_g64 = nullptr;
    float *d_far_g32 = nullptr, *d_near_g32 = nullptr;
    int32_t stored_mask = 0;         // bits GCA_FP64 / GCA_MIXED

    // workspaces of the batched product (h2_matvec with nrhs > 1), one set
    // per precision (index 0 FP64, 1 FP32), allocated by the first batched
    // product of that precision: x and its FP64 copy (n x NB), pivot vectors
    // xh, yh (n_piv x NB), coupling and nearfield partials (slots x NB)
    struct Batch {
        void *xb = nullptr, *xh = nullptr, *yh = nullptr, *cpart = nullptr, *npart = nullptr;
        double *xb64 = nullptr;
    } batch[2];

    // solver workspaces (allocated by the first solve)
    double *d_sv = nullptr;          // 5 x n: r, d, res, p, q
    double *d_dotp = nullptr;        // dot partials (1024) + result (first solve or energy)
    double *d_ews = nullptr;         // energy: the product G~ u when the caller wants E only
    void *d_ent = nullptr;           // gca_entries: pair arrays and values, 24 bytes per pair
    size_t ent_cap = 0;              // pairs d_ent holds
    int64_t *d_vv_ptr = nullptr;     // gca_dl_entries: the vertex adjacency (first call)
    int32_t *d_vv = nullptr;
    hipStream_t cur_stream = nullptr;   // stream of the call in progress (given to the alloc callback)

    // per-matvec workspaces
    double *d_xp = nullptr;          // permuted input (FP64) n
    float *d_xpf = nullptr;
    double *d_xh = nullptr, *d_yh = nullptr;       // n_piv
    float *d_xhf = nullptr, *d_yhf = nullptr;
    double *d_cpart = nullptr;       // coupling partials
    float *d_cpartf = nullptr;
    double *d_npart = nullptr;       // near partials
    float *d_npartf = nullptr;

    // Green rule (m points per direction on a face)
    double gl_x[32], gl_w[32];
    double gs_x[32], gs_w[32];       // Sauter-Schwab order q_s

    // points per triangle of the regular, near-regular and coupling rules
    int P_r = 0, P_nr = 0, P_c = 0;
    static constexpr int RING = 64;  // products whose phase events are retained
    // ev[slot][k] = (start, end) of phase k on the stream it ran on;
    // ev_tot[slot] brackets the whole product on the caller's stream
    hipEvent_t ev[RING][GCA_NPHASE][2] = {};
    hipEvent_t ev_tot[RING][2] = {};
    int64_t n_products = 0;
    bool events = false;
    bool timed = false;              // phase events hold a recorded product
    // Unless prm.serial, a product runs on three streams (non-blocking,
    // default priority): the touching values on s_side (forked at the start
    // of a product, joined before the gather) and the transform chain
    // (forward transform, coupling blocks and their reduction, backward
    // transform) on s_chain (forked after the permutation of x, joined before
    // the gather), beside the nearfield blocks on the caller's stream.
    hipStream_t s_side = nullptr, s_chain = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    hipEvent_t ev_cfork = nullptr, ev_cjoin = nullptr;
    gca_stats_t st{};
};

namespace gca {

constexpr int NEAR_CW = 64;          // column chunk of the nearfield block rows (one mask word)
constexpr int NB = 16;               // right-hand sides of a batched product (N of the 16 x 16 MFMA tiles)

// ---------------------------------------------------------- kernel launchers --
// All launchers enqueue on `s` and return the launch status.
// A rule on the reference triangle {0 <= s2 <= s1 <= 1}: point
// P0 + s1 (P1 - P0) + s2 (P2 - P1), weight w times |(P1 - P0) x (P2 - P1)|;
// the weights sum to 1/2.
// index of the touching phase in the phase times
constexpr int TOUCH_PHASE = 7;

struct TriRule {
    int np;
    double s1[64], s2[64], w[64];
};
// Collapsed Gauss rule of order q, or (sym) the symmetric rule of the same
// degree 2q - 2 (q = 2: 3 points, q = 3: 6 points).  False if unsupported.
bool tri_rule(int q, bool sym, TriRule &r);

// Fills the leaf-ELL partner table of the touching values (padding: the row
// itself) and the ELL slot of both rows of every touching pair, from the row
// CSR (d_tptr, d_tother, d_slot_a/b); pos_li: leaf index of every position,
// qmap: scratch of one int32 per CSR entry.
hipError_t launch_touching_ell(gca_h2_s *h, const int32_t *pos_li, int32_t *qmap, int64_t ntouch, hipStream_t s);
hipError_t launch_tri_points(const double *xyz, const int32_t *tv, int64_t n, const TriRule &rule,
                             double *out, hipStream_t s);
hipError_t launch_green_A(const double *qA, int PA, const double *box, const int32_t *row_tri,
                          const int32_t *row_cl, const int64_t *row_out, int64_t nrows, int m, const double *glx,
                          const double *glw, double eta, double omega_scale, double *A, hipStream_t s);
hipError_t launch_aca(double *R, double *U, double *V, const int64_t *a_off, const int64_t *u_off,
                      const int32_t *rows, int cols, int nbatch, double eps, int maxr_cap, int32_t *rank_out,
                      int32_t *piv_out, int32_t *pivc_out, int max_rows, hipStream_t s);
hipError_t launch_copy_jobs(const int64_t *jobs, int njobs, const double *src, double *dr, double *dc, float *fr,
                            float *fc, hipStream_t s);

// xp = x in cluster order (x: FP32 when xf32, else FP64), xp64 (if not NULL)
// the same values in FP64
template <typename T>
hipError_t launch_permute_in(const void *x, bool xf32, const int32_t *perm, int64_t n, T *xp, double *xp64,
                             hipStream_t s);
template <typename T>
hipError_t launch_forward(gca_h2_s *h, const T *xp, T *xh, hipStream_t s);
template <typename T>
hipError_t launch_far_blocks(gca_h2_s *h, const T *xh, T *cpart, hipStream_t s);
template <typename T>
hipError_t launch_coupling_reduce(gca_h2_s *h, const int64_t *slot_ptr, const int64_t *slots, const T *cpart,
                                  T *yh, hipStream_t s);
hipError_t launch_pivot_points(gca_h2_s *h, hipStream_t s);
hipError_t launch_local_points(gca_h2_s *h, hipStream_t s);
template <typename T>
hipError_t launch_backward(gca_h2_s *h, T *yh, hipStream_t s);
template <typename T>
hipError_t launch_store_blocks(gca_h2_s *h, T *far_store, T *near_store, hipStream_t s);
template <typename T>
hipError_t launch_apply_stored(gca_h2_s *h, bool nearfield, const T *x, const T *G, T *part, hipStream_t s);
template <typename T>
hipError_t launch_near(gca_h2_s *h, const T *xp, T *npart, hipStream_t s);

// batched product (16 right-hand sides; vectors and partials row-major x 16):
// block rows on the matrix cores (quad.hip) and the transforms, reduction,
// permutation and gather (multi.hip)
template <typename T>
hipError_t launch_near_nb(gca_h2_s *h, const T *xb, T *npart, hipStream_t s);
template <typename T>
hipError_t launch_far_blocks_nb(gca_h2_s *h, const T *xhb, T *cpart, hipStream_t s);
template <typename T>
hipError_t launch_permute_in_nb(const void *x, bool xf32, int64_t ld, int nrhs, const int32_t *iperm, int64_t n,
                                T *xb, double *xb64, hipStream_t s);
template <typename T>
hipError_t launch_forward_nb(gca_h2_s *h, const T *xb, T *xhb, hipStream_t s);
template <typename T>
hipError_t launch_coupling_reduce_nb(gca_h2_s *h, const T *cpart, T *yhb, hipStream_t s);
template <typename T>
hipError_t launch_backward_nb(gca_h2_s *h, T *yhb, hipStream_t s);
template <typename T>
hipError_t launch_gather_nb(gca_h2_s *h, const T *xb, const double *xb64, const T *yhb, const T *npart,
                            const T *nval, void *y, bool yf32, int64_t ld, int nrhs, hipStream_t s);
// Touching-pair values (FP64 table); fp32: the Gauss loops in FP32.
hipError_t launch_touching(gca_h2_s *h, double *tval, hipStream_t s, bool fp32 = false);
template <typename T>
hipError_t launch_nearreg(gca_h2_s *h, T *nval, hipStream_t s);
// y (FP32 when yf32, else FP64) in the original order
template <typename T>
hipError_t launch_gather(gca_h2_s *h, const T *xp, const double *xp64, const T *yh, const T *npart,
                         const T *nval, void *y, bool yf32, hipStream_t s);

// vector kernels of the solver (solve.hip)
// *out = factor * sum a[i] b[i] (fixed reduction order; partial: 1024 doubles)
hipError_t launch_dot(const double *a, const double *b, int64_t n, double *partial, double *out, hipStream_t s,
                      double factor = 1.0);
// Double-layer entries (dlayer.hip) of m pairs (original triangle ids I, J) classified on
// the device: tv / iperm the handle's position tables, vv_ptr / vv the vertex
// adjacency (near-regular class); ids out of range give NaN.
hipError_t launch_dl_pairs(const double *xyz, const int32_t *tv, const int32_t *iperm, const int64_t *vv_ptr,
                           const int32_t *vv, int64_t n, const int32_t *I, const int32_t *J, int64_t m, int q_r,
                           int q_nr, int q_s, bool sym, double *out, hipStream_t s);

// doubles of a dot-product workspace: 1024 partials + one result slot
constexpr size_t DOT_PARTIALS = 1025;

// gca_energy after its workspaces exist: argument checks (GCA_OK or the
// status already recorded), and the product, dot and scaling on stream s with
// dotp (DOT_PARTIALS doubles) and ews (n doubles, used only when g is NULL)
gca_status energy_check(const gca_h2_s *h, const double *u, const double *e, const double *g, int32_t precision);
gca_status energy_run(gca_h2_s *h, const double *u, const double *scale, double *e, double *g, int32_t precision,
                      hipStream_t s, double *dotp, double *ews);
// y = (scale ? *scale : 1) * x  (scale: device scalar)
hipError_t launch_scale(const double *scale, const double *x, double *y, int64_t n, hipStream_t s);
hipError_t launch_axpby(double alpha, const double *x, double beta, double *y, int64_t n, hipStream_t s);
hipError_t launch_cg_update(double alpha, const double *p, const double *q, double *d, double *r, int64_t n,
                            hipStream_t s);
hipError_t launch_sub(const double *a, const double *b, double *out, int64_t n, hipStream_t s);
hipError_t launch_fill(double *y, double v, int64_t n, hipStream_t s);

// frozen-structure basis (adjoint.hip)
hipError_t launch_frozen_basis(gca_h2_s *h, hipStream_t s);
hipError_t launch_frozen_adjoint_solve(gca_h2_s *h, hipStream_t s);

// adjoint (grad.hip)
template <typename T>
hipError_t launch_bilinear_grad(gca_h2_s *h, const GradWs &w, hipStream_t s);
// dxyz += alpha * (scale ? *scale : 1) * (vertex sums of the triangle derivatives)
hipError_t launch_vertex_gather(gca_h2_s *h, const GradWs &w, double alpha, const double *scale, double *dxyz,
                                hipStream_t s);

// Entries for pairs sorted by class on the host (gca_entries).
struct EntryJobs {
    const int32_t *pa, *pb, *code;
    int64_t off[6];   // 0 identical, 1 edge, 2 vertex, 3 near-regular, 4 regular, 5 end
};
hipError_t launch_entry_jobs(gca_h2_s *h, const EntryJobs &j, double *tmp64, float *tmp32, int precision,
                             hipStream_t s);

// Shared with the nodal-basis handle (capi.cpp): device memory owned by the
// handle until it is freed, the parameter checks, the level-wise basis
// construction (rows per cluster from the tree, Green points from d_box,
// PA_rows points per row in d_qA).
gca_status handle_alloc(gca_h2_s *h, void **p, size_t bytes);
void handle_free_all(gca_h2_s *h);
gca_status params_check(const gca_params *p);
gca_status basis_build(gca_h2_s *h, hipStream_t s);

// Stored blocks of the nodal-basis handle (lin_h2.hip): block b has rows
// [row0, row0 + nr) of its target (row0 = 0: whole blocks), G column-major
// nr x nc at goff[b], columns src[srcoff[b] + j]; its row sums go to
// part[poff[b] + i].  Target g (cluster tgt[g]) then adds those of its blocks
// sub_ptr[g] .. sub_ptr[g+1] in order.  FAR: yh[piv_off[t] + i] = sum; else
// y[perm[begin + i]] = V_t yh_t + sum (the gather).
struct LinApply {
    int32_t ntarget = 0;
    int64_t nsub = 0;
    int32_t *tgt = nullptr;
    int64_t *sub_ptr = nullptr;
    int32_t *sub_meta = nullptr;   // 3 per sub-block: nr, nc, row0
    int64_t *goff = nullptr, *srcoff = nullptr;
    int64_t *poff = nullptr;       // per sub-block: its rows' partial sums in part
    double *G = nullptr, *part = nullptr;
};
// the row sums of every sub-block (one wavefront each), then per target
hipError_t launch_lin_sub(const LinApply &a, const double *src, hipStream_t s);
hipError_t launch_lin_reduce(const gca_h2_s *h, const LinApply &a, bool far, double *yh, double *y, hipStream_t s);
// out[dst[b] + j ldo + i] = in[b ld + i nc + j] for the nb sub-blocks of a batch
// (meta: nr, nc, ldo per sub-block; transposed into their blocks)
hipError_t launch_lin_compact(const double *in, int64_t ld, int32_t nb, const int32_t *meta, const int64_t *goff,
                              double *out, hipStream_t s);

}  // namespace gca
