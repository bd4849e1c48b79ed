// The nodal-basis GCA-H^2 handle (include/gca_linear.h): Sections 2-4 over
// the index set of Section 5 (one continuous piecewise-linear basis function
// per vertex).
//
// Build: the vertex tree (points the vertices, boxes those of the supports),
// the block tree, the Green factor rows of every vertex (the triangles of its
// support with the collapsed rule of order q_A and the nodal weights, padded
// to PA points), then the level-wise ACA and nested bases of the
// piecewise-constant handle (basis_build).  The coupling matrices G|t~ x s~
// and the nearfield blocks are assembled once by the pair-wise kernels of
// Section 5 (gca_lin_merge, gca_lin_blocks) on chunks of the pivot and leaf
// vertex sets and stored; the product applies them between the transforms.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <string>

#include "gca_internal.h"
#include "gca_linear.h"

using namespace gca;

struct gca_lin_h2_s {
    gca_h2_s h;                      // vertex tree, basis, transfers, level lists
    std::vector<int32_t> far_t, far_s, near_t, near_s;   // both orientations
    LinApply far, near;
    int64_t n_far_store = 0, n_near_store = 0;
    double *d_xp = nullptr, *d_xh = nullptr, *d_yh = nullptr;
    // the transform chain and the coupling blocks run on s_side beside the
    // nearfield blocks on the caller's stream
    hipStream_t s_side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
};

namespace {

constexpr int CHUNK_V = GCA_LIN_MAX_BLOCK_SET;   // vertices of a chunk at most
constexpr int CHUNK_T = GCA_LIN_MAX_TRIS;        // sum of |T_v| over a chunk at most (merged rows)
constexpr int BATCH = 2048;                      // sub-blocks per assembly launch
// product sub-blocks: a stored block is applied in column pieces of about
// PIECE entries (at least 8 columns), one wavefront each, so that the large
// coupling blocks are shared by several wavefronts
constexpr int64_t PIECE = 4096;

template <typename T>
gca_status alloc_n(gca_h2_s *h, T **p, size_t n)
{
    void *q = nullptr;
    GCA_TRY(handle_alloc(h, &q, std::max<size_t>(n, 1) * sizeof(T)));
    *p = (T *)q;
    return GCA_OK;
}

template <typename T>
gca_status put(gca_h2_s *h, T **p, const std::vector<T> &v, hipStream_t s)
{
    GCA_TRY(alloc_n(h, p, v.size()));
    if (!v.empty()) GCA_HIP_TRY(hipMemcpyAsync(*p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
    return GCA_OK;
}

// Splits an ordered vertex list into consecutive chunks of at most CHUNK_V
// vertices and CHUNK_T support triangles; returns the chunk starts (and the
// end).
std::vector<int32_t> chunks_of(const std::vector<int32_t> &vs, const std::vector<int64_t> &vt_ptr)
{
    std::vector<int32_t> cut{0};
    if (vs.empty()) return cut;   // no chunk
    int64_t tri = 0;
    for (size_t k = 0; k < vs.size(); ++k) {
        const int64_t d = vt_ptr[vs[k] + 1] - vt_ptr[vs[k]];
        if ((int64_t)k - cut.back() >= CHUNK_V || tri + d > CHUNK_T) {
            cut.push_back((int32_t)k);
            tri = 0;
        }
        tri += d;
    }
    cut.push_back((int32_t)vs.size());
    return cut;
}

gca_status build_lin(const gca_mesh *mesh, int32_t leaf, const gca_params *p, hipStream_t s, gca_lin_h2_s *L)
{
    gca_h2_s *h = &L->h;
    GCA_TRY(params_check(p));
    if (leaf < 1 || leaf > CHUNK_V) return set_error(GCA_EINVAL, "leaf_size must be in [1, 64]");
    gca_params prm = *p;
    if (prm.q_c == 0) prm.q_c = prm.q_r;
    TriRule rr, rc, ra;
    if (!tri_rule(prm.q_r, prm.sym_rules != 0, rr) || rr.np > 16 || !tri_rule(prm.q_c, prm.sym_rules != 0, rc) ||
        rc.np > 16)
        return set_error(GCA_EINVAL, "the nodal-basis blocks need q_r, q_c in 1..4 (symmetric rules: 2, 3)");
    if (prm.q_s < 1 || prm.q_s > 32) return set_error(GCA_EINVAL, "q_s must be in [1, 32]");
    if (!tri_rule(prm.q_A, false, ra)) return set_error(GCA_EINVAL, "unsupported q_A");
    h->prm = prm;
    h->cur_stream = s;
    GCA_TRY(mesh_copy_validate(mesh, h->mesh, true));
    const Mesh &m = h->mesh;
    const int64_t nv = m.nv, nt = m.nt;
    // the sets T_v (ascending triangle ids)
    std::vector<int32_t> voff32(nv + 1), vlist(3 * nt);
    GCA_TRY(gca_lin_vertex_triangles(m.tri.data(), nt, nv, voff32.data(), vlist.data()));
    std::vector<int64_t> vt_ptr(voff32.begin(), voff32.end());
    int maxdeg = 0;
    for (int64_t v = 0; v < nv; ++v) {
        if (vt_ptr[v + 1] == vt_ptr[v]) return set_error(GCA_EMESH, "vertex " + std::to_string(v) + " has no triangle");
        maxdeg = std::max<int>(maxdeg, (int)(vt_ptr[v + 1] - vt_ptr[v]));
    }
    GCA_TRY(tree_build_vertices(m, vt_ptr, vlist, leaf, h->tree));
    h->n = nv;
    h->nv = nv;
    h->nc = (int64_t)h->tree.nodes.size();
    h->depth = h->tree.depth;
    const auto &nodes = h->tree.nodes;
    const int nc = (int)h->nc;
    block_tree(h->tree, prm.eta, h->blk);
    for (size_t b = 0; b < h->blk.far_t.size(); ++b) {
        L->far_t.push_back(h->blk.far_t[b]);
        L->far_s.push_back(h->blk.far_s[b]);
        L->far_t.push_back(h->blk.far_s[b]);
        L->far_s.push_back(h->blk.far_t[b]);
    }
    for (size_t b = 0; b < h->blk.near_t.size(); ++b) {
        L->near_t.push_back(h->blk.near_t[b]);
        L->near_s.push_back(h->blk.near_s[b]);
        if (h->blk.near_t[b] != h->blk.near_s[b]) {
            L->near_t.push_back(h->blk.near_s[b]);
            L->near_s.push_back(h->blk.near_t[b]);
        }
    }
    h->level_clusters.assign(h->depth + 1, {});
    h->leaves.clear();
    for (int c = 0; c < nc; ++c) {
        h->level_clusters[nodes[c].level].push_back(c);
        if (nodes[c].son[0] < 0) h->leaves.push_back(c);
    }
    gauss_legendre01(prm.green_m, h->gl_x, h->gl_w);

    // positions, boxes, tree arrays
    std::vector<int32_t> perm(h->tree.perm.begin(), h->tree.perm.end());
    std::vector<double> box(8 * (size_t)nc, 0.0);
    std::vector<int32_t> nodearr(5 * (size_t)nc);
    for (int c = 0; c < nc; ++c) {
        for (int d = 0; d < 3; ++d) {
            box[8 * c + d] = nodes[c].lo[d];
            box[8 * c + 3 + d] = nodes[c].hi[d];
        }
        box[8 * c + 6] = nodes[c].diam;
        nodearr[5 * c + 0] = nodes[c].begin;
        nodearr[5 * c + 1] = nodes[c].end;
        nodearr[5 * c + 2] = nodes[c].son[0];
        nodearr[5 * c + 3] = nodes[c].son[1];
        nodearr[5 * c + 4] = nodes[c].parent;
    }
    GCA_TRY(put(h, &h->d_perm, perm, s));
    GCA_TRY(put(h, &h->d_box, box, s));
    GCA_TRY(put(h, &h->d_node, nodearr, s));
    h->d_level_clusters.assign(h->level_clusters.size(), nullptr);
    for (size_t l = 0; l < h->level_clusters.size(); ++l) GCA_TRY(put(h, &h->d_level_clusters[l], h->level_clusters[l], s));

    // Green-factor rows: the collapsed rule of order q_A on every triangle of
    // the support with the weight w |J| lambda of the vertex's corner; padded
    // with zero weights at the vertex itself (PA points per row)
    const int need = maxdeg * ra.np;
    int PA = 0;
    for (int c : {1, 4, 9, 16, 25, 36, 64, 100, 144})
        if (c >= need) {
            PA = c;
            break;
        }
    if (!PA) return set_error(GCA_EINVAL, "vertex degree times the q_A rule exceeds 144 Green-factor points");
    h->PA_rows = PA;
    std::vector<double> qa((size_t)nv * PA * 4, 0.0);
    parallel_for(nv, [&](int64_t p0, int64_t p1) {
        for (int64_t pos = p0; pos < p1; ++pos) {
            const int32_t v = perm[pos];
            double *o = &qa[(size_t)pos * PA * 4];
            int k = 0;
            for (int64_t q = vt_ptr[v]; q < vt_ptr[v + 1]; ++q) {
                const int32_t t = vlist[q];
                const double *P0 = &m.xyz[3 * (int64_t)m.tri[3 * t]], *P1 = &m.xyz[3 * (int64_t)m.tri[3 * t + 1]],
                             *P2 = &m.xyz[3 * (int64_t)m.tri[3 * t + 2]];
                const int c = m.tri[3 * t] == v ? 0 : (m.tri[3 * t + 1] == v ? 1 : 2);
                const double a0 = P1[0] - P0[0], a1 = P1[1] - P0[1], a2 = P1[2] - P0[2];
                const double b0 = P2[0] - P1[0], b1 = P2[1] - P1[1], b2 = P2[2] - P1[2];
                const double cx = a1 * b2 - a2 * b1, cy = a2 * b0 - a0 * b2, cz = a0 * b1 - a1 * b0;
                const double J = std::sqrt(cx * cx + cy * cy + cz * cz);
                for (int r = 0; r < ra.np; ++r, ++k) {
                    const double s1 = ra.s1[r], s2 = ra.s2[r];
                    const double lam = c == 0 ? 1.0 - s1 : (c == 1 ? s1 - s2 : s2);
                    for (int d = 0; d < 3; ++d) o[4 * k + d] = P0[d] + s1 * (P1[d] - P0[d]) + s2 * (P2[d] - P1[d]);
                    o[4 * k + 3] = ra.w[r] * J * lam;
                }
            }
            for (; k < PA; ++k)
                for (int d = 0; d < 3; ++d) o[4 * k + d] = m.xyz[3 * (int64_t)v + d];
        }
    });
    GCA_TRY(put(h, &h->d_qA, qa, s));
    GCA_HIP_TRY(hipStreamSynchronize(s));
    std::vector<double>().swap(qa);
    GCA_TRY(basis_build(h, s));
    GCA_TRY(put(h, &h->d_piv, h->pivots, s));
    GCA_TRY(put(h, &h->d_piv_off, h->piv_off, s));
    GCA_TRY(put(h, &h->d_rank, h->rank, s));
    GCA_TRY(put(h, &h->d_v_off, h->v_off, s));
    GCA_TRY(put(h, &h->d_e_off, h->e_off, s));

    // vertex subsets: the pivots of every cluster (pivot order) and the
    // vertices of every leaf (position order), in chunks
    std::vector<int32_t> set_off{0}, set_vtx;
    std::vector<std::vector<int32_t>> fch(nc), nch(nc);   // chunk starts per cluster / leaf
    std::vector<int32_t> fset0(nc, -1), nset0(nc, -1);    // first subset id
    for (int c = 0; c < nc; ++c) {
        std::vector<int32_t> vs;
        for (int k = 0; k < h->rank[c]; ++k) vs.push_back(perm[h->pivots[h->piv_off[c] + k]]);
        fch[c] = chunks_of(vs, vt_ptr);
        fset0[c] = (int32_t)set_off.size() - 1;
        for (size_t q = 0; q + 1 < fch[c].size(); ++q) {
            set_vtx.insert(set_vtx.end(), vs.begin() + fch[c][q], vs.begin() + fch[c][q + 1]);
            set_off.push_back((int32_t)set_vtx.size());
        }
    }
    for (int c : h->leaves) {
        std::vector<int32_t> vs(perm.begin() + nodes[c].begin, perm.begin() + nodes[c].end);
        nch[c] = chunks_of(vs, vt_ptr);
        nset0[c] = (int32_t)set_off.size() - 1;
        for (size_t q = 0; q + 1 < nch[c].size(); ++q) {
            set_vtx.insert(set_vtx.end(), vs.begin() + nch[c][q], vs.begin() + nch[c][q + 1]);
            set_off.push_back((int32_t)set_vtx.size());
        }
    }
    const int32_t nsets = (int32_t)set_off.size() - 1;
    int32_t *d_set_off, *d_set_vtx, *d_voff, *d_vlist, *d_tri, *d_mtri, *d_mloc, *d_mcnt;
    double *d_xyz;
    GCA_TRY(put(h, &d_set_off, set_off, s));
    GCA_TRY(put(h, &d_set_vtx, set_vtx, s));
    GCA_TRY(put(h, &d_voff, voff32, s));
    GCA_TRY(put(h, &d_vlist, vlist, s));
    GCA_TRY(put(h, &d_tri, m.tri, s));
    GCA_TRY(put(h, &d_xyz, m.xyz, s));
    h->d_xyz = d_xyz;
    GCA_TRY(alloc_n(h, &d_mtri, (size_t)std::max(nsets, 1) * CHUNK_T));
    GCA_TRY(alloc_n(h, &d_mloc, (size_t)std::max(nsets, 1) * CHUNK_T * 3));
    GCA_TRY(alloc_n(h, &d_mcnt, (size_t)std::max(nsets, 1)));
    if (nsets > 0) {
        GCA_TRY(gca_lin_merge(d_voff, d_vlist, d_tri, d_set_off, d_set_vtx, nsets, CHUNK_T, d_mtri, d_mloc, d_mcnt, s));
        std::vector<int32_t> cnt(nsets);
        GCA_HIP_TRY(hipMemcpyAsync(cnt.data(), d_mcnt, 4 * (size_t)nsets, hipMemcpyDeviceToHost, s));
        GCA_HIP_TRY(hipStreamSynchronize(s));
        for (int32_t c : cnt)
            if (c < 0) return set_error(GCA_EINTERNAL, "a vertex chunk exceeds the merged-list limits");
    }

    // sub-blocks per target, assembled in batches and compacted into the store
    double *d_tmp;
    int32_t *d_status, *d_br, *d_bc, *d_meta;
    int64_t *d_goff;
    GCA_TRY(alloc_n(h, &d_tmp, (size_t)BATCH * CHUNK_V * CHUNK_V));
    GCA_TRY(alloc_n(h, &d_status, BATCH));
    GCA_TRY(alloc_n(h, &d_br, BATCH));
    GCA_TRY(alloc_n(h, &d_bc, BATCH));
    GCA_TRY(alloc_n(h, &d_meta, 3 * (size_t)BATCH));
    GCA_TRY(alloc_n(h, &d_goff, BATCH));
    auto assemble = [&](bool farb, LinApply &A, int64_t &nstore) -> gca_status {
        const auto &bt = farb ? L->far_t : L->near_t;
        const auto &bs = farb ? L->far_s : L->near_s;
        const auto &ch = farb ? fch : nch;
        const auto &set0 = farb ? fset0 : nset0;
        // targets: every cluster (coupling) or every leaf (nearfield); blocks
        // of a target in (source, column chunk, row chunk) order
        std::vector<int32_t> tg = farb ? std::vector<int32_t>() : h->leaves;
        if (farb) {
            tg.resize(nc);
            std::iota(tg.begin(), tg.end(), 0);
        }
        std::vector<int32_t> tpos(nc, -1);
        for (size_t g = 0; g < tg.size(); ++g) tpos[tg[g]] = (int32_t)g;
        std::vector<std::vector<int32_t>> per(tg.size());
        for (size_t b = 0; b < bt.size(); ++b) per[tpos[bt[b]]].push_back(bs[b]);
        // stored blocks: every block (t, u) whole, column-major with leading
        // dimension the rows of t; assembled in chunk sub-blocks (the pair-wise
        // kernels' limits) that the compaction puts in place, and applied in
        // column pieces with a partial-sum slot each
        std::vector<int64_t> sub_ptr{0}, goff, srcoff, poff, dst;
        std::vector<int32_t> meta, smeta, br, bc;
        int64_t off = 0, prow = 0;
        for (size_t g = 0; g < tg.size(); ++g) {
            const int t = tg[g];
            const int nrt = ch[t].back();
            std::sort(per[g].begin(), per[g].end());
            for (int u : per[g]) {
                const int ncu = ch[u].back();
                const int wmax = (int)std::max<int64_t>(8, PIECE / std::max(nrt, 1));
                for (int c0 = 0; c0 < ncu; c0 += wmax) {
                    meta.insert(meta.end(), {nrt, std::min(wmax, ncu - c0), 0});
                    goff.push_back(off + (int64_t)c0 * nrt);
                    poff.push_back(prow);
                    srcoff.push_back((farb ? h->piv_off[u] : nodes[u].begin) + c0);
                    prow += nrt;
                }
                for (size_t cb = 0; cb + 1 < ch[u].size(); ++cb)
                    for (size_t rb = 0; rb + 1 < ch[t].size(); ++rb) {
                        const int nr = ch[t][rb + 1] - ch[t][rb], ncol = ch[u][cb + 1] - ch[u][cb];
                        smeta.insert(smeta.end(), {nr, ncol, nrt});
                        dst.push_back(off + (int64_t)ch[u][cb] * nrt + ch[t][rb]);
                        br.push_back(set0[t] + (int32_t)rb);
                        bc.push_back(set0[u] + (int32_t)cb);
                    }
                off += (int64_t)nrt * ncu;
            }
            sub_ptr.push_back((int64_t)goff.size());
        }
        nstore = off;
        A.ntarget = (int32_t)tg.size();
        A.nsub = (int64_t)goff.size();
        GCA_TRY(put(h, &A.tgt, tg, s));
        GCA_TRY(put(h, &A.poff, poff, s));
        GCA_TRY(alloc_n(h, &A.part, (size_t)prow));
        GCA_TRY(put(h, &A.sub_ptr, sub_ptr, s));
        GCA_TRY(put(h, &A.sub_meta, meta, s));
        GCA_TRY(put(h, &A.goff, goff, s));
        GCA_TRY(put(h, &A.srcoff, srcoff, s));
        GCA_TRY(alloc_n(h, &A.G, (size_t)off));
        const int q = farb ? prm.q_c : prm.q_r;
        std::vector<int32_t> st(BATCH);
        for (size_t b0 = 0; b0 < dst.size(); b0 += BATCH) {
            const int32_t nb = (int32_t)std::min<size_t>(BATCH, dst.size() - b0);
            GCA_HIP_TRY(hipMemcpyAsync(d_br, br.data() + b0, 4 * (size_t)nb, hipMemcpyHostToDevice, s));
            GCA_HIP_TRY(hipMemcpyAsync(d_bc, bc.data() + b0, 4 * (size_t)nb, hipMemcpyHostToDevice, s));
            GCA_HIP_TRY(hipMemcpyAsync(d_meta, smeta.data() + 3 * b0, 12 * (size_t)nb, hipMemcpyHostToDevice, s));
            GCA_HIP_TRY(hipMemcpyAsync(d_goff, dst.data() + b0, 8 * (size_t)nb, hipMemcpyHostToDevice, s));
            GCA_TRY(gca_lin_blocks(d_xyz, d_tri, d_mtri, d_mloc, d_mcnt, CHUNK_T, d_set_off, d_br, d_bc, nb,
                                   (int64_t)CHUNK_V * CHUNK_V, q, prm.sym_rules != 0, farb ? 0 : prm.q_s, d_tmp,
                                   d_status, s));
            GCA_HIP_TRY(launch_lin_compact(d_tmp, (int64_t)CHUNK_V * CHUNK_V, nb, d_meta, d_goff, A.G, s));
            GCA_HIP_TRY(hipMemcpyAsync(st.data(), d_status, 4 * (size_t)nb, hipMemcpyDeviceToHost, s));
            GCA_HIP_TRY(hipStreamSynchronize(s));
            for (int32_t k = 0; k < nb; ++k)
                if (st[k] != 0)
                    return set_error(GCA_EINTERNAL, std::string(farb ? "coupling" : "nearfield") +
                                                        " sub-block status " + std::to_string(st[k]));
        }
        return GCA_OK;
    };
    GCA_TRY(assemble(true, L->far, L->n_far_store));
    GCA_TRY(assemble(false, L->near, L->n_near_store));
    GCA_TRY(alloc_n(h, &L->d_xp, (size_t)nv));
    GCA_TRY(alloc_n(h, &L->d_xh, (size_t)std::max<int64_t>(h->n_piv, 1)));
    GCA_TRY(alloc_n(h, &L->d_yh, (size_t)std::max<int64_t>(h->n_piv, 1)));
    GCA_HIP_TRY(hipStreamCreateWithFlags(&L->s_side, hipStreamNonBlocking));
    GCA_HIP_TRY(hipEventCreateWithFlags(&L->ev_fork, hipEventDisableTiming));
    GCA_HIP_TRY(hipEventCreateWithFlags(&L->ev_join, hipEventDisableTiming));
    GCA_HIP_TRY(hipStreamSynchronize(s));
    return GCA_OK;
}

void destroy_lin(gca_lin_h2_s *L)
{
    (void)hipDeviceSynchronize();
    if (L->ev_fork) (void)hipEventDestroy(L->ev_fork);
    if (L->ev_join) (void)hipEventDestroy(L->ev_join);
    if (L->s_side) (void)hipStreamDestroy(L->s_side);
    handle_free_all(&L->h);
    delete L;
}

}  // namespace

extern "C" {

gca_status gca_lin_build(const gca_mesh *mesh, int32_t leaf, const gca_params *p, void *stream, gca_lin_h2 *out)
{
    clear_error();
    if (!out) return set_error(GCA_EINVAL, "out is NULL");
    *out = nullptr;
    if (!mesh || !p) return set_error(GCA_EINVAL, "NULL pointer");
    auto *L = new (std::nothrow) gca_lin_h2_s;
    if (!L) return set_error(GCA_ENOMEM, "out of host memory");
    const gca_status st = build_lin(mesh, leaf, p, (hipStream_t)stream, L);
    if (st != GCA_OK) {
        destroy_lin(L);
        return st;
    }
    *out = L;
    return GCA_OK;
}

gca_status gca_lin_matvec(gca_lin_h2 L, const double *x, double *y, void *stream)
{
    clear_error();
    if (!L || !x || !y) return set_error(GCA_EINVAL, "NULL pointer");
    gca_h2_s *h = &L->h;
    const hipStream_t s = (hipStream_t)stream;
    const hipStream_t c = L->s_side;
    GCA_HIP_TRY(launch_permute_in<double>(x, false, h->d_perm, h->n, L->d_xp, nullptr, s));
    GCA_HIP_TRY(hipEventRecord(L->ev_fork, s));
    GCA_HIP_TRY(hipStreamWaitEvent(c, L->ev_fork, 0));
    GCA_HIP_TRY(launch_forward<double>(h, L->d_xp, L->d_xh, c));
    GCA_HIP_TRY(launch_lin_sub(L->far, L->d_xh, c));
    GCA_HIP_TRY(launch_lin_reduce(h, L->far, true, L->d_yh, nullptr, c));
    GCA_HIP_TRY(launch_backward<double>(h, L->d_yh, c));
    GCA_HIP_TRY(hipEventRecord(L->ev_join, c));
    GCA_HIP_TRY(launch_lin_sub(L->near, L->d_xp, s));
    GCA_HIP_TRY(hipStreamWaitEvent(s, L->ev_join, 0));
    GCA_HIP_TRY(launch_lin_reduce(h, L->near, false, L->d_yh, y, s));
    return GCA_OK;
}

gca_status gca_lin_info(gca_lin_h2 L, int64_t *info)
{
    clear_error();
    if (!L || !info) return set_error(GCA_EINVAL, "NULL pointer");
    const gca_h2_s *h = &L->h;
    int32_t mr = 0;
    for (int32_t r : h->rank) mr = std::max(mr, r);
    const int64_t v[8] = {h->n, h->nc, (int64_t)L->far_t.size(), (int64_t)L->near_t.size(), mr, h->n_piv,
                          L->n_far_store, L->n_near_store};
    std::memcpy(info, v, sizeof(v));
    return GCA_OK;
}

gca_status gca_lin_export(gca_lin_h2 L, int32_t *perm, int32_t *ranks, int32_t *pivots)
{
    clear_error();
    if (!L || !perm || !ranks || !pivots) return set_error(GCA_EINVAL, "NULL pointer");
    const gca_h2_s *h = &L->h;
    for (int64_t q = 0; q < h->n; ++q) perm[q] = h->tree.perm[q];
    for (int64_t c = 0; c < h->nc; ++c) ranks[c] = h->rank[c];
    for (int64_t k = 0; k < h->n_piv; ++k) pivots[k] = h->tree.perm[h->pivots[k]];
    return GCA_OK;
}

void gca_lin_destroy(gca_lin_h2 L)
{
    if (L) destroy_lin(L);
}

}  // extern "C"
