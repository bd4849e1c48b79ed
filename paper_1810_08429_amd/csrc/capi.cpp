// C-ABI of libgca (include/gca.h): argument checks, device memory, the
// level-wise basis construction (Sections 2-4) and the matrix-vector product.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <numeric>
#include <unordered_set>

#include "gca_internal.h"

using namespace gca;

namespace {

// Device memory of a handle: the caller's callbacks, or hipMalloc / hipFree.
void *dev_alloc(gca_h2_s *h, size_t bytes)
{
    bytes = std::max<size_t>(bytes, 256);
    if (h->prm.alloc) return h->prm.alloc(bytes, (void *)h->cur_stream, h->prm.alloc_ctx);
    void *q = nullptr;
    return hipMalloc(&q, bytes) == hipSuccess ? q : nullptr;
}

void dev_free(gca_h2_s *h, void *p)
{
    if (!p) return;
    if (h->prm.free)
        h->prm.free(p, nullptr, h->prm.alloc_ctx);
    else
        (void)hipFree(p);
}

gca_status alloc_error(size_t bytes, const char *what)
{
    return set_error(GCA_ENOMEM, std::string("device allocation of ") + std::to_string(bytes) + " bytes (" + what +
                                     ") failed");
}

// count elements owned by the handle until gca_destroy
template <typename T>
gca_status dalloc(gca_h2_s *h, T **p, size_t count)
{
    *p = nullptr;
    if (count == 0) count = 1;
    void *q = dev_alloc(h, count * sizeof(T));
    if (!q) return alloc_error(count * sizeof(T), "handle");
    h->allocs.push_back(q);
    *p = static_cast<T *>(q);
    return GCA_OK;
}

template <typename T>
gca_status upload(T *dst, const std::vector<T> &src, hipStream_t s)
{
    if (src.empty()) return GCA_OK;
    GCA_HIP_TRY(hipMemcpyAsync(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, s));
    GCA_HIP_TRY(hipStreamSynchronize(s));
    return GCA_OK;
}

template <typename T>
gca_status upload_new(gca_h2_s *h, T **dst, const std::vector<T> &src, hipStream_t s)
{
    GCA_TRY(dalloc(h, dst, src.size()));
    return upload(*dst, src, s);
}

void free_stored(gca_h2_s *h)
{
    if (h->d_far_g64 || h->d_near_g64 || h->d_far_g32 || h->d_near_g32) (void)hipDeviceSynchronize();
    for (void **p : {(void **)&h->d_far_g64, (void **)&h->d_near_g64, (void **)&h->d_far_g32,
                     (void **)&h->d_near_g32}) {
        dev_free(h, *p);
        *p = nullptr;
    }
}

void free_all(gca_h2_s *h)
{
    (void)hipDeviceSynchronize();
    free_stored(h);
    dev_free(h, h->d_ent);
    h->d_ent = nullptr;
    h->ent_cap = 0;
    for (void *p : h->allocs) dev_free(h, p);
    h->allocs.clear();
    if (h->events) {
        for (auto &r : h->ev)
            for (auto &pr : r)
                for (auto &e : pr) (void)hipEventDestroy(e);
        for (auto &r : h->ev_tot)
            for (auto &e : r) (void)hipEventDestroy(e);
        (void)hipEventDestroy(h->ev_fork);
        (void)hipEventDestroy(h->ev_join);
        (void)hipEventDestroy(h->ev_cfork);
        (void)hipEventDestroy(h->ev_cjoin);
        (void)hipStreamDestroy(h->s_side);
        (void)hipStreamDestroy(h->s_chain);
        h->s_side = nullptr;
        h->s_chain = nullptr;
    }
    h->events = false;
}

gca_status check_params(const gca_params *p)
{
    if (!p) return set_error(GCA_EINVAL, "params is NULL");
    if (!(p->eta > 0) || !std::isfinite(p->eta)) return set_error(GCA_EINVAL, "eta must be positive and finite");
    if (!(p->eps >= 0) || !(p->eps < 1)) return set_error(GCA_EINVAL, "eps must be in [0, 1)");
    if (!(p->omega_scale > 0) || !std::isfinite(p->omega_scale))
        return set_error(GCA_EINVAL, "omega_scale must be positive and finite");
    if (p->green_m < 1 || p->green_m > 6) return set_error(GCA_EINVAL, "green_m must be in [1, 6]");
    if (p->q_A < 1 || p->q_A > 6) return set_error(GCA_EINVAL, "q_A must be in [1, 6]");
    if (p->q_r < 1 || p->q_r > 6) return set_error(GCA_EINVAL, "q_r must be in [1, 6]");
    if (p->q_nr < 1 || p->q_nr > 7) return set_error(GCA_EINVAL, "q_nr must be in [1, 7]");
    if (p->q_s < 2 || p->q_s > 32) return set_error(GCA_EINVAL, "q_s must be in [2, 32]");
    if (p->ss_fp32 != 0 && p->ss_fp32 != 1) return set_error(GCA_EINVAL, "ss_fp32 must be 0 or 1");
    if (p->serial != 0 && p->serial != 1) return set_error(GCA_EINVAL, "serial must be 0 or 1");
    if ((p->alloc == nullptr) != (p->free == nullptr))
        return set_error(GCA_EINVAL, "alloc and free callbacks must be given together");
    if (p->q_c < 0 || p->q_c > 6) return set_error(GCA_EINVAL, "q_c must be in 1..6 (0: same as q_r)");
    if (p->sym_rules != 0 && p->sym_rules != 1) return set_error(GCA_EINVAL, "sym_rules must be 0 or 1");
    if (p->sym_rules) {
        const int qc = p->q_c ? p->q_c : p->q_r;
        for (int q : {p->q_r, p->q_nr, qc})
            if (q != 2 && q != 3) return set_error(GCA_EINVAL, "sym_rules needs q_r, q_nr and q_c in {2, 3}");
    }
    return GCA_OK;
}

double now_ms()
{
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Basis construction, one tree level at a time from the leaves to the root.
gca_status build_basis(gca_h2_s *h, hipStream_t s)
{
    const gca_params &p = h->prm;
    const int k = 6 * p.green_m * p.green_m, cols = 2 * k;
    const int PA = h->PA_rows > 0 ? h->PA_rows : p.q_A * p.q_A;
    const auto &nodes = h->tree.nodes;
    const int nc = (int)h->nc;
    std::vector<std::vector<int32_t>> piv(nc);   // pivot positions per cluster
    std::vector<std::vector<int32_t>> arows_c(nc), prow_c(nc), pcol_c(nc);
    h->rank.assign(nc, 0);

    struct LevelWs {
        double *V = nullptr;                // rows x min(rows, cols) per cluster
        std::vector<int64_t> u_off;         // per batch entry
        std::vector<int32_t> rows, rstride;
    };
    std::vector<LevelWs> lw(h->level_clusters.size());
    std::vector<void *> temp;
    auto tmp_alloc = [&](void **q, size_t bytes) -> gca_status {
        *q = dev_alloc(h, bytes);
        if (!*q) return alloc_error(bytes, "basis workspace");
        temp.push_back(*q);
        return GCA_OK;
    };
    auto cleanup = [&]() {
        (void)hipStreamSynchronize(s);
        for (void *q : temp) dev_free(h, q);
        temp.clear();
    };
    // workspaces shared by the levels (the leaf level is the largest): the
    // Green factor A and the cross-approximation columns U
    struct Grow {
        void *p = nullptr;
        size_t cap = 0;
    } wA, wU;
    auto grow = [&](Grow &g, size_t bytes) -> gca_status {
        if (bytes <= g.cap) return GCA_OK;
        void *q = nullptr;
        GCA_TRY(tmp_alloc(&q, bytes));
        g.p = q;
        g.cap = bytes;
        return GCA_OK;
    };
    gca_status st = GCA_OK;
    for (int l = (int)h->level_clusters.size() - 1; l >= 0 && st == GCA_OK; --l) {
        const auto &cl = h->level_clusters[l];
        const int nb = (int)cl.size();
        if (!nb) continue;
        std::vector<int32_t> row_tri, row_cl, rows(nb);
        std::vector<int64_t> row_out, a_off(nb), u_off(nb);
        int64_t atot = 0, utot = 0;
        for (int bi = 0; bi < nb; ++bi) {
            const Node &nd = nodes[cl[bi]];
            std::vector<int32_t> rr;
            if (nd.son[0] < 0) {
                for (int32_t q = nd.begin; q < nd.end; ++q) rr.push_back(q);
            } else {
                rr = piv[nd.son[0]];
                rr.insert(rr.end(), piv[nd.son[1]].begin(), piv[nd.son[1]].end());
            }
            rows[bi] = (int32_t)rr.size();
            a_off[bi] = atot;
            u_off[bi] = utot;
            for (size_t r = 0; r < rr.size(); ++r) {
                row_tri.push_back(rr[r]);
                row_cl.push_back(cl[bi]);
                row_out.push_back(atot + (int64_t)r * cols);
            }
            atot += (int64_t)rr.size() * cols;
            utot += (int64_t)rr.size() * std::min<int64_t>((int64_t)rr.size(), cols);
            piv[cl[bi]] = rr;   // row list for now; replaced by the pivots below
        }
        double *dA, *dU, *dV;
        int32_t *d_rows, *d_rowtri, *d_rowcl, *d_rank, *d_pivl, *d_pivc;
        int64_t *d_rowout, *d_aoff, *d_uoff;
        if ((st = grow(wA, atot * sizeof(double))) != GCA_OK) break;
        if ((st = grow(wU, utot * sizeof(double))) != GCA_OK) break;
        dA = (double *)wA.p;
        dU = (double *)wU.p;
        if ((st = tmp_alloc((void **)&dV, utot * sizeof(double))) != GCA_OK) break;
        if ((st = tmp_alloc((void **)&d_rows, nb * 4)) != GCA_OK) break;
        if ((st = tmp_alloc((void **)&d_rowtri, row_tri.size() * 4)) != GCA_OK) break;
        if ((st = tmp_alloc((void **)&d_rowcl, row_cl.size() * 4)) != GCA_OK) break;
        if ((st = tmp_alloc((void **)&d_rank, nb * 4)) != GCA_OK) break;
        if ((st = tmp_alloc((void **)&d_pivl, (size_t)nb * cols * 4)) != GCA_OK) break;
        if ((st = tmp_alloc((void **)&d_pivc, (size_t)nb * cols * 4)) != GCA_OK) break;
        if ((st = tmp_alloc((void **)&d_rowout, row_out.size() * 8)) != GCA_OK) break;
        if ((st = tmp_alloc((void **)&d_aoff, nb * 8)) != GCA_OK) break;
        if ((st = tmp_alloc((void **)&d_uoff, nb * 8)) != GCA_OK) break;
        if ((st = upload(d_rows, rows, s)) != GCA_OK) break;
        if ((st = upload(d_rowtri, row_tri, s)) != GCA_OK) break;
        if ((st = upload(d_rowcl, row_cl, s)) != GCA_OK) break;
        if ((st = upload(d_rowout, row_out, s)) != GCA_OK) break;
        if ((st = upload(d_aoff, a_off, s)) != GCA_OK) break;
        if ((st = upload(d_uoff, u_off, s)) != GCA_OK) break;
        hipError_t e = launch_green_A(h->d_qA, PA, h->d_box, d_rowtri, d_rowcl, d_rowout, (int64_t)row_tri.size(),
                                      p.green_m, h->gl_x, h->gl_w, p.eta, p.omega_scale, dA, s);
        if (e == hipSuccess)
            e = launch_aca(dA, dU, dV, d_aoff, d_uoff, d_rows, cols, nb, p.eps, cols, d_rank, d_pivl, d_pivc,
                           *std::max_element(rows.begin(), rows.end()), s);
        if (e != hipSuccess) {
            st = set_error(GCA_EHIP, std::string("basis kernels: ") + hipGetErrorString(e));
            break;
        }
        std::vector<int32_t> rk(nb), pl((size_t)nb * cols), pc((size_t)nb * cols);
        e = hipMemcpyAsync(rk.data(), d_rank, nb * 4, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipMemcpyAsync(pl.data(), d_pivl, (size_t)nb * cols * 4, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipMemcpyAsync(pc.data(), d_pivc, (size_t)nb * cols * 4, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) {
            st = set_error(GCA_EHIP, std::string("basis read-back: ") + hipGetErrorString(e));
            break;
        }
        for (int bi = 0; bi < nb; ++bi) {
            const int c = cl[bi];
            std::vector<int32_t> rr = piv[c], pv(rk[bi]);
            for (int r = 0; r < rk[bi]; ++r) pv[r] = rr[pl[(size_t)bi * cols + r]];
            arows_c[c] = rr;
            prow_c[c].assign(pl.begin() + (size_t)bi * cols, pl.begin() + (size_t)bi * cols + rk[bi]);
            pcol_c[c].assign(pc.begin() + (size_t)bi * cols, pc.begin() + (size_t)bi * cols + rk[bi]);
            piv[c] = pv;
            h->rank[c] = rk[bi];
        }
        lw[l].V = dV;
        lw[l].u_off = u_off;
        lw[l].rows = rows;
        lw[l].rstride.resize(nb);
        for (int bi = 0; bi < nb; ++bi) lw[l].rstride[bi] = std::min(rows[bi], cols);
    }
    if (st != GCA_OK) {
        cleanup();
        return st;
    }
    // final layouts: pivots, leaf V, transfers E
    h->piv_off.assign(nc, 0);
    h->pivots.clear();
    for (int c = 0; c < nc; ++c) {
        h->piv_off[c] = (int64_t)h->pivots.size();
        h->pivots.insert(h->pivots.end(), piv[c].begin(), piv[c].end());
    }
    h->n_piv = (int64_t)h->pivots.size();
    h->pivrow.clear();
    h->pivcol.clear();
    h->arow_off.assign(nc + 1, 0);
    h->arows.clear();
    for (int c = 0; c < nc; ++c) {
        h->pivrow.insert(h->pivrow.end(), prow_c[c].begin(), prow_c[c].end());
        h->pivcol.insert(h->pivcol.end(), pcol_c[c].begin(), pcol_c[c].end());
        h->arow_off[c] = (int64_t)h->arows.size();
        h->arows.insert(h->arows.end(), arows_c[c].begin(), arows_c[c].end());
    }
    h->arow_off[nc] = (int64_t)h->arows.size();
    h->v_off.assign(nc, 0);
    h->e_off.assign(nc, 0);
    int64_t nv_ = 0, ne_ = 0;
    for (int c = 0; c < nc; ++c) {
        const Node &nd = nodes[c];
        if (nd.son[0] < 0) {
            h->v_off[c] = nv_;
            nv_ += (int64_t)(nd.end - nd.begin) * h->rank[c];
        }
        if (nd.parent >= 0) {
            h->e_off[c] = ne_;
            ne_ += (int64_t)h->rank[c] * h->rank[nd.parent];
        }
    }
    h->n_v = nv_;
    h->n_e = ne_;
    h->max_rank = 0;
    for (int c = 0; c < nc; ++c) h->max_rank = std::max(h->max_rank, h->rank[c]);
    GCA_TRY(dalloc(h, &h->d_V, nv_));
    GCA_TRY(dalloc(h, &h->d_Vt, nv_));
    GCA_TRY(dalloc(h, &h->d_Vf, nv_));
    GCA_TRY(dalloc(h, &h->d_Vtf, nv_));
    GCA_TRY(dalloc(h, &h->d_E, ne_));
    GCA_TRY(dalloc(h, &h->d_Et, ne_));
    GCA_TRY(dalloc(h, &h->d_Ef, ne_));
    GCA_TRY(dalloc(h, &h->d_Etf, ne_));
    for (int l = 0; l < (int)h->level_clusters.size(); ++l) {
        const auto &cl = h->level_clusters[l];
        std::vector<int64_t> vjobs, ejobs;   // 6 per job
        for (size_t bi = 0; bi < cl.size(); ++bi) {
            const int c = cl[bi];
            const Node &nd = nodes[c];
            const int64_t so = lw[l].u_off[bi], ld = lw[l].rstride[bi];
            if (nd.son[0] < 0) {
                vjobs.insert(vjobs.end(), {so, ld, 0, (int64_t)lw[l].rows[bi], (int64_t)h->rank[c], h->v_off[c]});
            } else {
                const int s0 = nd.son[0], s1 = nd.son[1];
                ejobs.insert(ejobs.end(), {so, ld, 0, (int64_t)h->rank[s0], (int64_t)h->rank[c], h->e_off[s0]});
                ejobs.insert(ejobs.end(),
                             {so, ld, (int64_t)h->rank[s0], (int64_t)h->rank[s1], (int64_t)h->rank[c], h->e_off[s1]});
            }
        }
        for (int which = 0; which < 2; ++which) {
            const auto &jobs = which ? ejobs : vjobs;
            if (jobs.empty()) continue;
            int64_t *dj;
            if ((st = tmp_alloc((void **)&dj, jobs.size() * 8)) != GCA_OK) break;
            if ((st = upload(dj, jobs, s)) != GCA_OK) break;
            hipError_t e = which ? launch_copy_jobs(dj, (int)(jobs.size() / 6), lw[l].V, h->d_E, h->d_Et, h->d_Ef,
                                                    h->d_Etf, s)
                                 : launch_copy_jobs(dj, (int)(jobs.size() / 6), lw[l].V, h->d_V, h->d_Vt, h->d_Vf,
                                                    h->d_Vtf, s);
            if (e != hipSuccess) {
                st = set_error(GCA_EHIP, std::string("basis copy: ") + hipGetErrorString(e));
                break;
            }
        }
        if (st != GCA_OK) break;
    }
    if (st == GCA_OK) {
        hipError_t e = hipStreamSynchronize(s);
        if (e != hipSuccess) st = set_error(GCA_EHIP, std::string("basis copy sync: ") + hipGetErrorString(e));
    }
    cleanup();
    return st;
}

gca_status build_impl(const gca_mesh *mesh, gca_tree tree, const gca_params *p, hipStream_t s, gca_h2_s *h)
{
    const double t0 = now_ms();
    GCA_TRY(check_params(p));
    h->prm = *p;
    h->cur_stream = s;
    if (h->prm.q_c == 0) h->prm.q_c = h->prm.q_r;
    // the topology checks ran when the tree was built from this same mesh
    GCA_TRY(mesh_copy_validate(mesh, h->mesh, false));
    if (tree->nt != h->mesh.nt || tree->nv != h->mesh.nv || tree->mesh_xyz != h->mesh.xyz ||
        tree->mesh_tri != h->mesh.tri)
        return set_error(GCA_EINVAL, "the tree was built from a different mesh");
    if (tree->leaf > 64) return set_error(GCA_EINVAL, "leaf_size must be <= 64 (one wavefront per leaf row set)");
    h->tree = *tree;
    h->n = h->mesh.nt;
    h->nv = h->mesh.nv;
    h->nc = (int64_t)h->tree.nodes.size();
    h->depth = h->tree.depth;
    const auto &nodes = h->tree.nodes;
    const int nc = (int)h->nc;
    const int64_t n = h->n;

    double tm[8] = {0};
    double tl = now_ms();
    auto lap = [&](int k) {
        double t = now_ms();
        tm[k] += t - tl;
        tl = t;
    };
    GCA_TRY(build_adjacency(h->mesh, h->adj));
    lap(0);
    block_tree(h->tree, p->eta, h->blk);

    // clusters by level, leaves, leaf of each position
    h->level_clusters.assign(h->depth + 1, {});
    h->leaves.clear();
    std::vector<int32_t> leaf_of(n, -1), leaf_index(nc, -1);
    h->max_leaf = 0;
    for (int c = 0; c < nc; ++c) {
        h->level_clusters[nodes[c].level].push_back(c);
        if (nodes[c].son[0] < 0) {
            leaf_index[c] = (int32_t)h->leaves.size();
            h->leaves.push_back(c);
            for (int32_t q = nodes[c].begin; q < nodes[c].end; ++q) leaf_of[q] = c;
            h->max_leaf = std::max(h->max_leaf, nodes[c].end - nodes[c].begin);
        }
    }
    // the nearfield partners of every leaf (sorted): a pair of positions lies
    // in an inadmissible leaf block iff its leaves are partners
    const size_t nl = h->leaves.size();
    std::vector<int64_t> nptr(nl + 1, 0);
    for (size_t b = 0; b < h->blk.near_t.size(); ++b) nptr[leaf_index[h->blk.near_t[b]] + 1]++;
    for (size_t l = 0; l < nl; ++l) nptr[l + 1] += nptr[l];
    std::vector<int32_t> partner(nptr[nl]);
    {
        std::vector<int64_t> fill(nptr.begin(), nptr.end() - 1);
        for (size_t b = 0; b < h->blk.near_t.size(); ++b)
            partner[fill[leaf_index[h->blk.near_t[b]]]++] = h->blk.near_s[b];
    }
    for (size_t l = 0; l < nl; ++l) std::sort(partner.begin() + nptr[l], partner.begin() + nptr[l + 1]);
    auto in_near = [&](int32_t pa, int32_t pb) {
        const int32_t la = leaf_of[pa], lb = leaf_of[pb];
        const int32_t t = std::min(la, lb), u = std::max(la, lb);
        const int32_t li = leaf_index[t];
        return std::binary_search(partner.begin() + nptr[li], partner.begin() + nptr[li + 1], u);
    };
    lap(2);
    // near-regular pairs of admissible blocks are left to those blocks
    GCA_TRY(build_pair_lists(h->mesh, h->adj, h->tree, p->q_nr != p->q_r, h->pl, in_near));
    lap(1);
    // every listed pair lies in an inadmissible leaf block: touching pairs
    // because the boxes of the supports share the common vertex (distance 0,
    // never admissible), near-regular pairs by the filter above
    {
        std::atomic<bool> bad{false};
        parallel_for((int64_t)h->pl.a.size(), [&](int64_t q0, int64_t q1) {
            for (int64_t q = q0; q < q1; ++q)
                if (!in_near(h->pl.a[q], h->pl.b[q])) bad = true;
        });
        if (bad) return set_error(GCA_EINTERNAL, "a listed pair lies outside the nearfield blocks");
    }
    lap(2);

    gauss_legendre01(p->green_m, h->gl_x, h->gl_w);
    gauss_legendre01(p->q_s, h->gs_x, h->gs_w);

    // geometry
    std::vector<int32_t> tv(3 * n), perm(n), iperm(n);
    for (int64_t q = 0; q < n; ++q) {
        int32_t t = h->tree.perm[q];
        perm[q] = t;
        iperm[t] = (int32_t)q;
        for (int k = 0; k < 3; ++k) tv[3 * q + k] = h->mesh.tri[3 * (int64_t)t + k];
    }
    GCA_TRY(upload_new(h, &h->d_xyz, h->mesh.xyz, s));
    GCA_TRY(upload_new(h, &h->d_tv, tv, s));
    GCA_TRY(upload_new(h, &h->d_perm, perm, s));
    GCA_TRY(upload_new(h, &h->d_iperm, iperm, s));
    std::vector<double> box(8 * (size_t)nc);
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
    GCA_TRY(upload_new(h, &h->d_box, box, s));
    GCA_TRY(upload_new(h, &h->d_node, nodearr, s));
    GCA_TRY(upload_new(h, &h->d_leaves, h->leaves, s));
    h->d_level_clusters.assign(h->level_clusters.size(), nullptr);
    for (size_t l = 0; l < h->level_clusters.size(); ++l)
        GCA_TRY(upload_new(h, &h->d_level_clusters[l], h->level_clusters[l], s));

    // triangle quadrature points: the regular-pair rules (collapsed Gauss or
    // symmetric, by sym_rules) and the collapsed rule of the Green factor
    const bool sym = p->sym_rules != 0;
    auto tri_pts = [&](int q, bool sy, double **out, int *np) -> gca_status {
        TriRule r;
        if (!tri_rule(q, sy, r)) return set_error(GCA_EINVAL, "unsupported triangle rule");
        if (np) *np = r.np;
        GCA_TRY(dalloc(h, out, (size_t)n * r.np * 4));
        GCA_HIP_TRY(launch_tri_points(h->d_xyz, h->d_tv, n, r, *out, s));
        return GCA_OK;
    };
    GCA_TRY(tri_pts(p->q_r, sym, &h->d_qr, &h->P_r));
    GCA_TRY(dalloc(h, &h->d_cent, (size_t)n * 4));
    GCA_TRY(dalloc(h, &h->d_qloc32, (size_t)n * h->P_r * 4));
    GCA_HIP_TRY(launch_local_points(h, s));
    if (p->q_nr == p->q_r) {
        h->d_qnr = h->d_qr;
        h->P_nr = h->P_r;
    } else {
        GCA_TRY(tri_pts(p->q_nr, sym, &h->d_qnr, &h->P_nr));
    }
    if (p->q_A == p->q_r && !sym)
        h->d_qA = h->d_qr;
    else
        GCA_TRY(tri_pts(p->q_A, false, &h->d_qA, nullptr));
    if (h->prm.q_c == p->q_r) {
        h->d_qc = h->d_qr;
        h->P_c = h->P_r;
    } else {
        GCA_TRY(tri_pts(h->prm.q_c, sym, &h->d_qc, &h->P_c));
    }

    GCA_HIP_TRY(hipStreamSynchronize(s));
    lap(3);
    // nested basis (Green factor + cross approximation, level by level)
    GCA_TRY(build_basis(h, s));
    lap(4);
    GCA_TRY(upload_new(h, &h->d_piv, h->pivots, s));
    GCA_TRY(upload_new(h, &h->d_piv_off, h->piv_off, s));
    GCA_TRY(upload_new(h, &h->d_rank, h->rank, s));
    GCA_TRY(upload_new(h, &h->d_v_off, h->v_off, s));
    GCA_TRY(upload_new(h, &h->d_e_off, h->e_off, s));

    // coupling blocks and their partial slots
    {
        const size_t nb = h->blk.far_t.size();
        std::vector<int32_t> far(2 * nb);
        std::vector<int64_t> slot(2 * nb);
        std::vector<std::vector<int64_t>> per(nc);
        int64_t off = 0;
        for (size_t b = 0; b < nb; ++b) {
            const int t = h->blk.far_t[b], u = h->blk.far_s[b];
            far[b] = t;
            far[nb + b] = u;
            slot[2 * b] = off;
            per[t].push_back(off);
            off += h->rank[t];
            slot[2 * b + 1] = off;
            per[u].push_back(off);
            off += h->rank[u];
        }
        h->n_cslot_total = off;
        std::vector<int64_t> ptr(nc + 1, 0), flat;
        for (int c = 0; c < nc; ++c) {
            ptr[c + 1] = ptr[c] + (int64_t)per[c].size();
            flat.insert(flat.end(), per[c].begin(), per[c].end());
        }
        GCA_TRY(upload_new(h, &h->d_far, far, s));
        GCA_TRY(upload_new(h, &h->d_far_slot, slot, s));
        GCA_TRY(upload_new(h, &h->d_cslot_ptr, ptr, s));
        GCA_TRY(upload_new(h, &h->d_cslot, flat, s));
    }
    // block rows of the coupling half for the product: blocks grouped by row
    // cluster, groups launched in decreasing order of work
    {
        const size_t nb = h->blk.far_t.size();
        std::vector<int64_t> bptr(nc + 1, 0);
        for (size_t b = 0; b < nb; ++b) bptr[h->blk.far_t[b] + 1]++;
        for (int c = 0; c < nc; ++c) bptr[c + 1] += bptr[c];
        std::vector<int32_t> bcol(nb);
        {
            std::vector<int64_t> fill(bptr.begin(), bptr.end() - 1);
            for (size_t b = 0; b < nb; ++b) bcol[fill[h->blk.far_t[b]]++] = h->blk.far_s[b];
        }
        std::vector<int32_t> gt;
        std::vector<int64_t> work;
        for (int c = 0; c < nc; ++c)
            if (bptr[c + 1] > bptr[c]) {
                int64_t w = 0;
                for (int64_t q = bptr[c]; q < bptr[c + 1]; ++q) w += (int64_t)h->rank[c] * h->rank[bcol[q]];
                gt.push_back(c);
                work.push_back(w);
            }
        std::vector<int32_t> order(gt.size());
        for (size_t k = 0; k < order.size(); ++k) order[k] = (int32_t)k;
        std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return work[a] > work[b]; });
        const size_t ng = gt.size();
        // offsets (serial), then the column arrays (parallel over groups)
        std::vector<int32_t> fg_t(ng);
        std::vector<int64_t> fg_ptr(ng + 1, 0), fg_rslot(ng), fg_cslot(ng);
        int64_t off = 0;
        for (size_t k = 0; k < ng; ++k) {
            const int t = gt[order[k]];
            fg_t[k] = t;
            fg_rslot[k] = off;
            off += h->rank[t];
            int64_t cols = 0;
            for (int64_t q = bptr[t]; q < bptr[t + 1]; ++q) cols += h->rank[bcol[q]];
            fg_cslot[k] = off;
            off += cols;
            fg_ptr[k + 1] = fg_ptr[k] + cols;
        }
        h->n_gslot_total = off;
        h->n_far_groups = (int32_t)ng;
        std::vector<int64_t> fg_soff(ng);
        h->n_far_store = 0;
        for (size_t k = 0; k < ng; ++k) {
            fg_soff[k] = h->n_far_store;
            h->n_far_store += (int64_t)h->rank[fg_t[k]] * (fg_ptr[k + 1] - fg_ptr[k]);
        }
        std::vector<int32_t> col_e(fg_ptr[ng]), col_s(fg_ptr[ng]);
        std::vector<int64_t> col_out(fg_ptr[ng]);
        parallel_for((int64_t)ng, [&](int64_t k0, int64_t k1) {
            for (int64_t k = k0; k < k1; ++k) {
                const int t = fg_t[k];
                int64_t kk = fg_ptr[k];
                for (int64_t q = bptr[t]; q < bptr[t + 1]; ++q) {
                    const int u = bcol[q];
                    for (int j = 0; j < h->rank[u]; ++j, ++kk) {
                        col_e[kk] = (int32_t)(h->piv_off[u] + j);
                        col_s[kk] = u;
                        col_out[kk] = fg_cslot[k] + (kk - fg_ptr[k]);
                    }
                }
            }
        }, 64);
        // per cluster: its row slot (as a row cluster) and its column slots
        std::vector<int64_t> ptr(nc + 1, 0);
        for (size_t k = 0; k < ng; ++k) {
            const int t = fg_t[k];
            ptr[t + 1]++;
            for (int64_t q = bptr[t]; q < bptr[t + 1]; ++q) ptr[bcol[q] + 1]++;
        }
        for (int c = 0; c < nc; ++c) ptr[c + 1] += ptr[c];
        std::vector<int64_t> flat(ptr[nc]);
        {
            std::vector<int64_t> fill(ptr.begin(), ptr.end() - 1);
            for (size_t k = 0; k < ng; ++k) {
                const int t = fg_t[k];
                flat[fill[t]++] = fg_rslot[k];
                int64_t o = fg_cslot[k];
                for (int64_t q = bptr[t]; q < bptr[t + 1]; ++q) {
                    flat[fill[bcol[q]]++] = o;
                    o += h->rank[bcol[q]];
                }
            }
        }
        if (ng > 0) {
            GCA_TRY(upload_new(h, &h->d_fg_t, fg_t, s));
            GCA_TRY(upload_new(h, &h->d_fg_ptr, fg_ptr, s));
            GCA_TRY(upload_new(h, &h->d_fg_rslot, fg_rslot, s));
            GCA_TRY(upload_new(h, &h->d_fcol_e, col_e, s));
            GCA_TRY(upload_new(h, &h->d_fcol_s, col_s, s));
            GCA_TRY(upload_new(h, &h->d_fcol_out, col_out, s));
            GCA_TRY(upload_new(h, &h->d_fg_soff, fg_soff, s));
        }
        GCA_TRY(upload_new(h, &h->d_gslot_ptr, ptr, s));
        GCA_TRY(upload_new(h, &h->d_gslot, flat, s));
        // FP32 pivot points relative to their cluster's centre
        h->n_piv_total = h->n_piv;
        std::vector<int32_t> pc((size_t)h->n_piv_total);
        for (int c = 0; c < nc; ++c)
            for (int64_t k = h->piv_off[c]; k < h->piv_off[c] + h->rank[c]; ++k) pc[(size_t)k] = c;
        if (h->n_piv_total > 0) {
            GCA_TRY(upload_new(h, &h->d_piv_cluster, pc, s));
            GCA_TRY(dalloc(h, &h->d_pq32, (size_t)h->n_piv_total * h->P_c * 4));
            GCA_HIP_TRY(launch_pivot_points(h, s));
        }
    }
    // near blocks and their partial slots
    {
        const size_t nb = h->blk.near_t.size();
        std::vector<int32_t> nearv(2 * nb);
        std::vector<int64_t> slot(2 * nb);
        std::vector<std::vector<int64_t>> per(h->leaves.size());
        int64_t off = 0;
        for (size_t b = 0; b < nb; ++b) {
            const int t = h->blk.near_t[b], u = h->blk.near_s[b];
            nearv[b] = t;
            nearv[nb + b] = u;
            slot[2 * b] = off;
            per[leaf_index[t]].push_back(off);
            off += nodes[t].end - nodes[t].begin;
            if (t != u) {
                slot[2 * b + 1] = off;
                per[leaf_index[u]].push_back(off);
                off += nodes[u].end - nodes[u].begin;
            } else {
                slot[2 * b + 1] = -1;
            }
        }
        h->n_nslot_total = off;
        std::vector<int64_t> ptr(h->leaves.size() + 1, 0), flat;
        for (size_t c = 0; c < h->leaves.size(); ++c) {
            ptr[c + 1] = ptr[c] + (int64_t)per[c].size();
            flat.insert(flat.end(), per[c].begin(), per[c].end());
        }
        GCA_TRY(upload_new(h, &h->d_near, nearv, s));
        GCA_TRY(upload_new(h, &h->d_near_slot, slot, s));
        GCA_TRY(upload_new(h, &h->d_nslot_ptr, ptr, s));
        GCA_TRY(upload_new(h, &h->d_nslot, flat, s));
    }
    // block rows of the nearfield half for the product: the blocks (t, s),
    // t <= s, of each leaf t with the diagonal block first; the columns of a
    // row are the concatenated positions of its leaves s.  Pairs of the row
    // CSR (touching, and near-regular when they have their own order) and the
    // lower triangle of the diagonal block are masked per row and chunk of
    // NEAR_CW columns.
    {
        const size_t nb = h->blk.near_t.size();
        std::vector<int64_t> bptr(nc + 1, 0);
        for (size_t b = 0; b < nb; ++b) bptr[h->blk.near_t[b] + 1]++;
        for (int c = 0; c < nc; ++c) bptr[c + 1] += bptr[c];
        std::vector<int32_t> bcol(nb);
        {
            std::vector<int64_t> fill(bptr.begin(), bptr.end() - 1);
            for (size_t b = 0; b < nb; ++b) bcol[fill[h->blk.near_t[b]]++] = h->blk.near_s[b];
            // diagonal block first, the others in ascending order
            for (int c = 0; c < nc; ++c)
                std::sort(bcol.begin() + bptr[c], bcol.begin() + bptr[c + 1], [c](int32_t x, int32_t y) {
                    if ((x == c) != (y == c)) return x == c;
                    return x < y;
                });
        }
        auto rows_of = [&](int c) { return nodes[c].end - nodes[c].begin; };
        std::vector<int32_t> gt;
        std::vector<int64_t> work;
        for (int c = 0; c < nc; ++c)
            if (bptr[c + 1] > bptr[c]) {
                if (bcol[bptr[c]] != c) return set_error(GCA_EINTERNAL, "leaf without its diagonal nearfield block");
                int64_t w = 0;
                for (int64_t q = bptr[c]; q < bptr[c + 1]; ++q) w += (int64_t)rows_of(c) * rows_of(bcol[q]);
                gt.push_back(c);
                work.push_back(w);
            }
        std::vector<int32_t> order(gt.size());
        for (size_t k = 0; k < order.size(); ++k) order[k] = (int32_t)k;
        std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return work[a] > work[b]; });
        const size_t ng = gt.size();
        std::vector<int32_t> g_t(ng);
        std::vector<int64_t> g_ptr(ng + 1, 0), g_rslot(ng), g_cslot(ng), g_moff(ng + 1, 0);
        int64_t off = 0;
        for (size_t k = 0; k < ng; ++k) {
            const int t = gt[order[k]];
            g_t[k] = t;
            g_rslot[k] = off;
            off += rows_of(t);
            int64_t cols = 0;
            for (int64_t q = bptr[t]; q < bptr[t + 1]; ++q) cols += rows_of(bcol[q]);
            g_cslot[k] = off;
            off += cols;
            g_ptr[k + 1] = g_ptr[k] + cols;
            g_moff[k + 1] = g_moff[k] + ((cols + NEAR_CW - 1) / NEAR_CW) * rows_of(t);
        }
        h->n_gnslot_total = off;
        h->n_near_groups = (int32_t)ng;
        std::vector<int64_t> g_soff(ng);
        h->n_near_store = 0;
        for (size_t k = 0; k < ng; ++k) {
            g_soff[k] = h->n_near_store;
            h->n_near_store += (int64_t)rows_of(g_t[k]) * (g_ptr[k + 1] - g_ptr[k]);
        }
        std::vector<int32_t> col_pos(g_ptr[ng]);
        std::vector<int64_t> col_out(g_ptr[ng]);
        std::vector<uint64_t> masks(g_moff[ng], 0);
        parallel_for((int64_t)ng, [&](int64_t k0, int64_t k1) {
            for (int64_t k = k0; k < k1; ++k) {
                const int t = g_t[k];
                const int rb = nodes[t].begin, nr = rows_of(t);
                int64_t kk = g_ptr[k];
                for (int64_t q = bptr[t]; q < bptr[t + 1]; ++q) {
                    const int u = bcol[q];
                    for (int32_t pos = nodes[u].begin; pos < nodes[u].end; ++pos, ++kk) {
                        col_pos[kk] = pos;
                        col_out[kk] = g_cslot[k] + (kk - g_ptr[k]);
                    }
                }
                uint64_t *m = masks.data() + g_moff[k];
                for (int i = 0; i < nr; ++i) {
                    // diagonal block (first segment): each unordered pair once, j > i;
                    // its column partial is the mirrored entry's row contribution
                    for (int j = 0; j <= i; ++j) m[(size_t)((j / NEAR_CW) * nr + i)] |= (uint64_t)1 << (j % NEAR_CW);
                    const int pos = rb + i;
                    for (int64_t e = h->pl.row_ptr[pos]; e < h->pl.row_ptr[pos + 1]; ++e) {
                        const int o = h->pl.row_other[e];
                        int64_t col0 = 0;
                        for (int64_t q = bptr[t]; q < bptr[t + 1]; ++q) {
                            const Node &nu = nodes[bcol[q]];
                            if (o >= nu.begin && o < nu.end) {
                                const int64_t col = col0 + (o - nu.begin);
                                m[(size_t)((col / NEAR_CW) * nr + i)] |= (uint64_t)1 << (col % NEAR_CW);
                                break;
                            }
                            col0 += nu.end - nu.begin;
                        }
                    }
                }
            }
        }, 64);
        // per leaf: its row slot and its column slots (leaf index order)
        const size_t nl = h->leaves.size();
        std::vector<int64_t> ptr(nl + 1, 0);
        for (size_t k = 0; k < ng; ++k) {
            const int t = g_t[k];
            ptr[leaf_index[t] + 1]++;
            for (int64_t q = bptr[t]; q < bptr[t + 1]; ++q) ptr[leaf_index[bcol[q]] + 1]++;
        }
        for (size_t l = 0; l < nl; ++l) ptr[l + 1] += ptr[l];
        std::vector<int64_t> flat(ptr[nl]);
        {
            std::vector<int64_t> fill(ptr.begin(), ptr.end() - 1);
            for (size_t k = 0; k < ng; ++k) {
                const int t = g_t[k];
                flat[fill[leaf_index[t]]++] = g_rslot[k];
                int64_t o = g_cslot[k];
                for (int64_t q = bptr[t]; q < bptr[t + 1]; ++q) {
                    flat[fill[leaf_index[bcol[q]]]++] = o;
                    o += rows_of(bcol[q]);
                }
            }
        }
        if (ng > 0) {
            GCA_TRY(upload_new(h, &h->d_ng_t, g_t, s));
            GCA_TRY(upload_new(h, &h->d_ng_ptr, g_ptr, s));
            GCA_TRY(upload_new(h, &h->d_ng_rslot, g_rslot, s));
            GCA_TRY(upload_new(h, &h->d_ng_moff, g_moff, s));
            GCA_TRY(upload_new(h, &h->d_ncol_pos, col_pos, s));
            GCA_TRY(upload_new(h, &h->d_ncol_out, col_out, s));
            GCA_TRY(upload_new(h, &h->d_nmask, masks, s));
            GCA_TRY(upload_new(h, &h->d_ng_soff, g_soff, s));
        }
        GCA_TRY(upload_new(h, &h->d_gnslot_ptr, ptr, s));
        GCA_TRY(upload_new(h, &h->d_gnslot, flat, s));
    }
    // pair lists
    GCA_TRY(upload_new(h, &h->d_pa, h->pl.a, s));
    GCA_TRY(upload_new(h, &h->d_pb, h->pl.b, s));
    GCA_TRY(upload_new(h, &h->d_pcode, h->pl.code, s));
    GCA_TRY(upload_new(h, &h->d_prow_ptr, h->pl.row_ptr, s));
    GCA_TRY(upload_new(h, &h->d_prow_other, h->pl.row_other, s));
    GCA_TRY(upload_new(h, &h->d_tptr, h->pl.t_ptr, s));
    GCA_TRY(upload_new(h, &h->d_nptr, h->pl.n_ptr, s));
    GCA_TRY(upload_new(h, &h->d_tother, h->pl.t_other, s));
    GCA_TRY(upload_new(h, &h->d_nother, h->pl.n_other, s));
    GCA_TRY(upload_new(h, &h->d_slot_a, h->pl.slot_a, s));
    GCA_TRY(upload_new(h, &h->d_slot_b, h->pl.slot_b, s));
    {
        // leaf-ELL layout of the touching values: the gather's lanes (rows of a
        // leaf) read their k-th partners from consecutive addresses
        const auto &nodes = h->tree.nodes;
        const size_t nl = h->leaves.size();
        std::vector<int64_t> ell_off(nl + 1, 0);
        std::vector<int32_t> ell_k(nl, 0);
        for (size_t li = 0; li < nl; ++li) {
            const Node &nd = nodes[h->leaves[li]];
            int32_t kmax = 0;
            for (int64_t pos = nd.begin; pos < nd.end; ++pos)
                kmax = std::max<int32_t>(kmax, (int32_t)(h->pl.t_ptr[pos + 1] - h->pl.t_ptr[pos]));
            ell_k[li] = kmax;
            ell_off[li + 1] = ell_off[li] + (int64_t)kmax * (nd.end - nd.begin);
        }
        if (ell_off[nl] > INT32_MAX) return set_error(GCA_EINVAL, "touching value table exceeds 2^31 entries");
        std::vector<int32_t> pos_li(std::max<int64_t>(n, 1));
        for (size_t li = 0; li < nl; ++li) {
            const Node &nd = nodes[h->leaves[li]];
            for (int64_t pos = nd.begin; pos < nd.end; ++pos) pos_li[pos] = (int32_t)li;
        }
        const int64_t ntouch = h->pl.off[3];
        int32_t *d_pos_li = nullptr, *d_qmap = nullptr;
        GCA_TRY(upload_new(h, &h->d_tell_off, ell_off, s));
        GCA_TRY(upload_new(h, &h->d_tell_k, ell_k, s));
        GCA_TRY(upload_new(h, &d_pos_li, pos_li, s));
        GCA_TRY(dalloc(h, &h->d_tell_other, (size_t)std::max<int64_t>(ell_off[nl], 1)));
        GCA_TRY(dalloc(h, &d_qmap, std::max<size_t>(h->pl.t_other.size(), 1)));
        GCA_TRY(dalloc(h, &h->d_tslot_a, (size_t)std::max<int64_t>(ntouch, 1)));
        GCA_TRY(dalloc(h, &h->d_tslot_b, (size_t)std::max<int64_t>(ntouch, 1)));
        GCA_HIP_TRY(launch_touching_ell(h, d_pos_li, d_qmap, ntouch, s));
        GCA_TRY(dalloc(h, &h->d_tval, (size_t)std::max<int64_t>(ell_off[nl], 1)));
        // padding entries stay zero
        GCA_HIP_TRY(hipMemsetAsync(h->d_tval, 0, sizeof(double) * std::max<int64_t>(ell_off[nl], 1), s));
    }
    GCA_TRY(dalloc(h, &h->d_nval, h->pl.n_other.size()));
    GCA_TRY(dalloc(h, &h->d_nvalf, h->pl.n_other.size()));

    // workspaces of the matrix-vector product
    GCA_TRY(dalloc(h, &h->d_xp, n));
    GCA_TRY(dalloc(h, &h->d_xpf, n));
    GCA_TRY(dalloc(h, &h->d_xh, h->n_piv));
    GCA_TRY(dalloc(h, &h->d_yh, h->n_piv));
    GCA_TRY(dalloc(h, &h->d_xhf, h->n_piv));
    GCA_TRY(dalloc(h, &h->d_yhf, h->n_piv));
    GCA_TRY(dalloc(h, &h->d_cpart, h->n_gslot_total));
    GCA_TRY(dalloc(h, &h->d_cpartf, h->n_gslot_total));
    GCA_TRY(dalloc(h, &h->d_npart, h->n_gnslot_total));
    GCA_TRY(dalloc(h, &h->d_npartf, h->n_gnslot_total));
    for (auto &r : h->ev)
        for (auto &pr : r)
            for (auto &e : pr) GCA_HIP_TRY(hipEventCreate(&e));
    for (auto &r : h->ev_tot)
        for (auto &e : r) GCA_HIP_TRY(hipEventCreate(&e));
    GCA_HIP_TRY(hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming));
    GCA_HIP_TRY(hipEventCreateWithFlags(&h->ev_join, hipEventDisableTiming));
    GCA_HIP_TRY(hipEventCreateWithFlags(&h->ev_cfork, hipEventDisableTiming));
    GCA_HIP_TRY(hipEventCreateWithFlags(&h->ev_cjoin, hipEventDisableTiming));
    GCA_HIP_TRY(hipStreamCreateWithFlags(&h->s_side, hipStreamNonBlocking));
    GCA_HIP_TRY(hipStreamCreateWithFlags(&h->s_chain, hipStreamNonBlocking));
    h->events = true;
    GCA_HIP_TRY(hipStreamSynchronize(s));
    lap(5);

    // statistics
    gca_stats_t &st = h->st;
    st = gca_stats_t{};
    st.n = n;
    st.nv = h->nv;
    st.n_clusters = nc;
    st.n_leaves = (int64_t)h->leaves.size();
    st.depth = h->depth;
    st.n_far = h->blk.n_far_full;
    st.n_near = h->blk.n_near_full;
    st.n_far_sym = (int64_t)h->blk.far_t.size();
    st.n_near_sym = (int64_t)h->blk.near_t.size();
    st.n_ident = h->pl.off[1] - h->pl.off[0];
    st.n_edge = h->pl.off[2] - h->pl.off[1];
    st.n_vert = h->pl.off[3] - h->pl.off[2];
    st.n_nearreg = h->pl.off[4] - h->pl.off[3];
    for (size_t b = 0; b < h->blk.far_t.size(); ++b)
        st.coupling_entries += (int64_t)h->rank[h->blk.far_t[b]] * h->rank[h->blk.far_s[b]];
    int64_t unordered = 0;
    for (size_t b = 0; b < h->blk.near_t.size(); ++b) {
        const Node &a = nodes[h->blk.near_t[b]], &c = nodes[h->blk.near_s[b]];
        const int64_t na = a.end - a.begin, ncc = c.end - c.begin;
        st.near_pairs += na * ncc;
        unordered += (h->blk.near_t[b] == h->blk.near_s[b]) ? na * (na + 1) / 2 : na * ncc;
    }
    // every non-regular pair (touching or near-regular) lies in a near block
    st.near_regular_pairs = unordered - (int64_t)h->pl.a.size();
    st.rank_min = INT64_MAX;
    double rs = 0;
    for (int c = 0; c < nc; ++c) {
        st.rank_min = std::min<int64_t>(st.rank_min, h->rank[c]);
        st.rank_max = std::max<int64_t>(st.rank_max, h->rank[c]);
        rs += h->rank[c];
    }
    st.rank_mean = rs / nc;
    st.basis_bytes_fp64 = 8 * (h->n_v + h->n_e);
    st.build_ms = now_ms() - t0;
    for (int k = 0; k < 8; ++k) st.setup_ms[k] = tm[k];
    return GCA_OK;
}

// One product y = G~ x on stream s.  x, y: FP32 when vf32, else FP64.
// first: the touching (and near-regular list) values are recomputed; later
// right-hand sides of the same call reuse them.  Unless prm.serial, the
// touching values run on s_side and the transform chain on s_chain beside the
// nearfield blocks (both forked from s and joined into s before the gather);
// serial keeps every phase on s in order, so each kernel has the chip alone.
template <typename T>
hipError_t matvec_one(gca_h2_s *h, const void *x, void *y, bool vf32, bool first, hipStream_t s)
{
    const bool f32 = std::is_same<T, float>::value;
    const bool ss32 = f32 && h->prm.ss_fp32;   // FP32 Gauss loops of the Sauter-Schwab rules
    T *xp = f32 ? (T *)h->d_xpf : (T *)h->d_xp;
    T *xh = f32 ? (T *)h->d_xhf : (T *)h->d_xh;
    T *yh = f32 ? (T *)h->d_yhf : (T *)h->d_yh;
    T *cpart = f32 ? (T *)h->d_cpartf : (T *)h->d_cpart;
    T *npart = f32 ? (T *)h->d_npartf : (T *)h->d_npart;
    T *nval = f32 ? (T *)h->d_nvalf : (T *)h->d_nval;
    hipError_t e;
    const int slot = (int)(h->n_products % gca_h2_s::RING);
    // phase k between beg(k) and fin(k) on the stream it runs on
    auto beg = [&](int k, hipStream_t st) {
        if (h->events) (void)hipEventRecord(h->ev[slot][k][0], st);
    };
    auto fin = [&](int k, hipStream_t st) {
        if (h->events) (void)hipEventRecord(h->ev[slot][k][1], st);
    };
    const T *far_g = f32 ? (const T *)h->d_far_g32 : (const T *)h->d_far_g64;
    const T *near_g = f32 ? (const T *)h->d_near_g32 : (const T *)h->d_near_g64;
    const bool stored = far_g != nullptr;
    const bool par = h->events && !h->prm.serial;
    const bool touch = first && !stored;      // stored mode: computed with the blocks
    const bool side = touch && par;
    const hipStream_t cs = par ? h->s_chain : s;
    if (h->events) (void)hipEventRecord(h->ev_tot[slot][0], s);
    if (side) {
        // touching values depend on the geometry only; the fork orders them
        // after earlier products on s (whose gathers read the same table)
        if ((e = hipEventRecord(h->ev_fork, s)) != hipSuccess) return e;
        if ((e = hipStreamWaitEvent(h->s_side, h->ev_fork, 0)) != hipSuccess) return e;
        beg(TOUCH_PHASE, h->s_side);
        if ((e = launch_touching(h, h->d_tval, h->s_side, ss32)) != hipSuccess) return e;
        fin(TOUCH_PHASE, h->s_side);
        if ((e = hipEventRecord(h->ev_join, h->s_side)) != hipSuccess) return e;
    }
    beg(0, s);
    if ((e = launch_permute_in<T>(x, vf32, h->d_perm, h->n, xp, f32 ? h->d_xp : nullptr, s)) != hipSuccess) return e;
    fin(0, s);
    if (par) {
        if ((e = hipEventRecord(h->ev_cfork, s)) != hipSuccess) return e;
        if ((e = hipStreamWaitEvent(h->s_chain, h->ev_cfork, 0)) != hipSuccess) return e;
    }
    beg(1, cs);
    if ((e = launch_forward<T>(h, xp, xh, cs)) != hipSuccess) return e;
    fin(1, cs);
    beg(2, cs);
    if (stored) {
        if ((e = launch_apply_stored<T>(h, false, xh, far_g, cpart, cs)) != hipSuccess) return e;
    } else if ((e = launch_far_blocks<T>(h, xh, cpart, cs)) != hipSuccess) {
        return e;
    }
    fin(2, cs);
    beg(3, cs);
    if ((e = launch_coupling_reduce<T>(h, h->d_gslot_ptr, h->d_gslot, cpart, yh, cs)) != hipSuccess) return e;
    fin(3, cs);
    beg(4, cs);
    if ((e = launch_backward<T>(h, yh, cs)) != hipSuccess) return e;
    fin(4, cs);
    if (par && (e = hipEventRecord(h->ev_cjoin, h->s_chain)) != hipSuccess) return e;
    beg(5, s);
    if (stored) {
        if ((e = launch_apply_stored<T>(h, true, xp, near_g, npart, s)) != hipSuccess) return e;
    } else if ((e = launch_near<T>(h, xp, npart, s)) != hipSuccess) {
        return e;
    }
    fin(5, s);
    beg(6, s);
    if (touch && (e = launch_nearreg<T>(h, nval, s)) != hipSuccess) return e;
    fin(6, s);
    if (side) {
        if ((e = hipStreamWaitEvent(s, h->ev_join, 0)) != hipSuccess) return e;
    } else {
        beg(TOUCH_PHASE, s);
        if (touch && (e = launch_touching(h, h->d_tval, s, ss32)) != hipSuccess) return e;
        fin(TOUCH_PHASE, s);
    }
    if (par && (e = hipStreamWaitEvent(s, h->ev_cjoin, 0)) != hipSuccess) return e;
    beg(8, s);
    if ((e = launch_gather<T>(h, xp, h->d_xp, yh, npart, nval, y, vf32, s)) != hipSuccess) return e;
    fin(8, s);
    if (h->events) (void)hipEventRecord(h->ev_tot[slot][1], s);
    h->timed = h->events;
    h->n_products++;
    return hipSuccess;
}

// The batched product needs the block kernels' rules to be instantiated
// for NB right-hand sides (up to 9 points per triangle) and recomputed
// blocks (stored block rows are applied one right-hand side at a time).
bool batch_supported(const gca_h2_s *h, bool f32)
{
    auto ok = [](int P) { return P == 1 || P == 3 || P == 4 || P == 6 || P == 9; };
    const bool stored = f32 ? h->d_far_g32 != nullptr : h->d_far_g64 != nullptr;
    return !stored && ok(h->P_r) && ok(h->P_c) && h->max_leaf <= 64;
}

// Workspaces of the batched product in precision T, allocated on first use.
template <typename T>
gca_status batch_workspace(gca_h2_s *h, gca_h2_s::Batch *&w)
{
    const bool f32 = std::is_same<T, float>::value;
    w = &h->batch[f32 ? 1 : 0];
    if (w->xb) return GCA_OK;
    T *xb = nullptr, *xh = nullptr, *yh = nullptr, *cp = nullptr, *np = nullptr;
    double *x64 = nullptr;
    GCA_TRY(dalloc(h, &xb, (size_t)h->n * NB));
    if (f32) GCA_TRY(dalloc(h, &x64, (size_t)h->n * NB));
    GCA_TRY(dalloc(h, &xh, (size_t)std::max<int64_t>(h->n_piv, 1) * NB));
    GCA_TRY(dalloc(h, &yh, (size_t)std::max<int64_t>(h->n_piv, 1) * NB));
    GCA_TRY(dalloc(h, &cp, (size_t)std::max<int64_t>(h->n_gslot_total, 1) * NB));
    GCA_TRY(dalloc(h, &np, (size_t)std::max<int64_t>(h->n_gnslot_total, 1) * NB));
    w->xh = xh;
    w->yh = yh;
    w->cpart = cp;
    w->npart = np;
    w->xb64 = f32 ? x64 : (double *)xb;
    w->xb = xb;
    return GCA_OK;
}

// One product for nrhs <= NB right-hand sides (columns of x and y with
// leading dimension ld): every block entry is evaluated once and applied to
// all of them; transfers, coupling and nearfield products on the matrix
// cores.  Streams and phase events as in matvec_one (one ring slot per call).
template <typename T>
hipError_t matvec_batch(gca_h2_s *h, gca_h2_s::Batch &w, const void *x, void *y, int nrhs, int64_t ld, bool vf32,
                        bool first, hipStream_t s)
{
    const bool f32 = std::is_same<T, float>::value;
    const bool ss32 = f32 && h->prm.ss_fp32;
    T *xb = (T *)w.xb, *xh = (T *)w.xh, *yh = (T *)w.yh, *cpart = (T *)w.cpart, *npart = (T *)w.npart;
    T *nval = f32 ? (T *)h->d_nvalf : (T *)h->d_nval;
    hipError_t e;
    const int slot = (int)(h->n_products % gca_h2_s::RING);
    auto beg = [&](int k, hipStream_t st) {
        if (h->events) (void)hipEventRecord(h->ev[slot][k][0], st);
    };
    auto fin = [&](int k, hipStream_t st) {
        if (h->events) (void)hipEventRecord(h->ev[slot][k][1], st);
    };
    const bool par = h->events && !h->prm.serial;
    const bool side = first && par;
    const hipStream_t cs = par ? h->s_chain : s;
    if (h->events) (void)hipEventRecord(h->ev_tot[slot][0], s);
    if (side) {
        if ((e = hipEventRecord(h->ev_fork, s)) != hipSuccess) return e;
        if ((e = hipStreamWaitEvent(h->s_side, h->ev_fork, 0)) != hipSuccess) return e;
        beg(TOUCH_PHASE, h->s_side);
        if ((e = launch_touching(h, h->d_tval, h->s_side, ss32)) != hipSuccess) return e;
        fin(TOUCH_PHASE, h->s_side);
        if ((e = hipEventRecord(h->ev_join, h->s_side)) != hipSuccess) return e;
    }
    beg(0, s);
    if ((e = launch_permute_in_nb<T>(x, vf32, ld, nrhs, h->d_iperm, h->n, xb, f32 ? w.xb64 : nullptr, s)) !=
        hipSuccess)
        return e;
    fin(0, s);
    if (par) {
        if ((e = hipEventRecord(h->ev_cfork, s)) != hipSuccess) return e;
        if ((e = hipStreamWaitEvent(h->s_chain, h->ev_cfork, 0)) != hipSuccess) return e;
    }
    beg(1, cs);
    if ((e = launch_forward_nb<T>(h, xb, xh, cs)) != hipSuccess) return e;
    fin(1, cs);
    beg(2, cs);
    if ((e = launch_far_blocks_nb<T>(h, xh, cpart, cs)) != hipSuccess) return e;
    fin(2, cs);
    beg(3, cs);
    if ((e = launch_coupling_reduce_nb<T>(h, cpart, yh, cs)) != hipSuccess) return e;
    fin(3, cs);
    beg(4, cs);
    if ((e = launch_backward_nb<T>(h, yh, cs)) != hipSuccess) return e;
    fin(4, cs);
    if (par && (e = hipEventRecord(h->ev_cjoin, h->s_chain)) != hipSuccess) return e;
    beg(5, s);
    if ((e = launch_near_nb<T>(h, xb, npart, s)) != hipSuccess) return e;
    fin(5, s);
    beg(6, s);
    if (first && (e = launch_nearreg<T>(h, nval, s)) != hipSuccess) return e;
    fin(6, s);
    if (side) {
        if ((e = hipStreamWaitEvent(s, h->ev_join, 0)) != hipSuccess) return e;
    } else {
        beg(TOUCH_PHASE, s);
        if (first && (e = launch_touching(h, h->d_tval, s, ss32)) != hipSuccess) return e;
        fin(TOUCH_PHASE, s);
    }
    if (par && (e = hipStreamWaitEvent(s, h->ev_cjoin, 0)) != hipSuccess) return e;
    beg(8, s);
    if ((e = launch_gather_nb<T>(h, xb, w.xb64, yh, npart, nval, y, vf32, ld, nrhs, s)) != hipSuccess) return e;
    fin(8, s);
    if (h->events) (void)hipEventRecord(h->ev_tot[slot][1], s);
    h->timed = h->events;
    h->n_products++;
    return hipSuccess;
}

// Device data of the frozen-structure basis, built on first use.
gca_status frozen_setup(gca_h2_s *h, hipStream_t s)
{
    Frozen &fz = h->fz;
    if (fz.ready) return GCA_OK;
    const int nc = (int)h->nc;
    std::vector<int32_t> batch(nc);
    for (int c = 0; c < nc; ++c) batch[c] = c;
    fz.aj_off.assign(nc, 0);
    fz.c_off.assign(nc, 0);
    std::vector<int64_t> roff(nc + 1, 0);
    int64_t aj = 0, cc = 0;
    for (int c = 0; c < nc; ++c) {
        const int64_t m = h->arow_off[c + 1] - h->arow_off[c];
        fz.aj_off[c] = aj;
        fz.c_off[c] = cc;
        aj += m * h->rank[c];
        cc += (int64_t)h->rank[c] * h->rank[c];
        roff[c + 1] = roff[c] + h->rank[c];
    }
    fz.n_aj = aj;
    fz.n_c = cc;
    GCA_TRY(upload_new(h, &fz.d_batch, batch, s));
    GCA_TRY(upload_new(h, &fz.d_pivrow, h->pivrow, s));
    GCA_TRY(upload_new(h, &fz.d_pivcol, h->pivcol, s));
    GCA_TRY(upload_new(h, &fz.d_arow_off, h->arow_off, s));
    GCA_TRY(upload_new(h, &fz.d_arows, h->arows, s));
    GCA_TRY(upload_new(h, &fz.d_aj_off, fz.aj_off, s));
    GCA_TRY(upload_new(h, &fz.d_c_off, fz.c_off, s));
    GCA_TRY(upload_new(h, &fz.d_roff, roff, s));
    GCA_TRY(dalloc(h, &fz.d_AJ, aj));
    GCA_TRY(dalloc(h, &fz.d_Vh, aj));
    GCA_TRY(dalloc(h, &fz.d_tmp, aj));
    GCA_TRY(dalloc(h, &fz.d_Vbar, aj));
    GCA_TRY(dalloc(h, &fz.d_Z, aj));
    GCA_TRY(dalloc(h, &fz.d_LU, cc));
    GCA_TRY(dalloc(h, &fz.d_Cinv, cc));
    GCA_TRY(dalloc(h, &fz.d_perm, h->n_piv));
    // copies of V^ into the leaf bases and transfer matrices
    std::vector<int64_t> vj, ej;
    for (int c = 0; c < nc; ++c) {
        const Node &nd = h->tree.nodes[c];
        const int64_t r = h->rank[c];
        if (nd.son[0] < 0) {
            vj.insert(vj.end(), {fz.aj_off[c], r, 0, (int64_t)(nd.end - nd.begin), r, h->v_off[c]});
        } else {
            const int s0 = nd.son[0], s1 = nd.son[1];
            ej.insert(ej.end(), {fz.aj_off[c], r, 0, (int64_t)h->rank[s0], r, h->e_off[s0]});
            ej.insert(ej.end(), {fz.aj_off[c], r, (int64_t)h->rank[s0], (int64_t)h->rank[s1], r, h->e_off[s1]});
        }
    }
    fz.n_vjobs = (int32_t)(vj.size() / 6);
    fz.n_ejobs = (int32_t)(ej.size() / 6);
    vj.insert(vj.end(), ej.begin(), ej.end());
    GCA_TRY(upload_new(h, &fz.d_copy_jobs, vj, s));
    fz.ready = true;
    return GCA_OK;
}

// Workspaces and index maps of the adjoint, built on first use.
gca_status grad_setup(gca_h2_s *h, hipStream_t s)
{
    GradWs &w = h->gw;
    if (w.ready) return GCA_OK;
    const int64_t n = h->n, nv = h->nv;
    const int nc = (int)h->nc;
    GCA_TRY(dalloc(h, &w.ap, n));
    GCA_TRY(dalloc(h, &w.bp, n));
    GCA_TRY(dalloc(h, &w.apf, n));
    GCA_TRY(dalloc(h, &w.bpf, n));
    double *tmp;
    GCA_TRY(dalloc(h, &tmp, h->n_piv));
    w.xa = tmp;
    GCA_TRY(dalloc(h, &tmp, h->n_piv));
    w.xb = tmp;
    GCA_TRY(dalloc(h, &tmp, h->n_piv));
    w.ya = tmp;
    GCA_TRY(dalloc(h, &tmp, h->n_piv));
    w.yb = tmp;
    GCA_TRY(dalloc(h, &tmp, h->n_gslot_total));
    w.cpart = tmp;
    GCA_TRY(dalloc(h, &w.gnear, 9 * (size_t)h->n_nslot_total));
    GCA_TRY(dalloc(h, &w.gfar, 9 * (size_t)h->n_cslot_total));
    GCA_TRY(dalloc(h, &w.gt, 9 * h->pl.t_other.size()));
    GCA_TRY(dalloc(h, &w.gn, 9 * h->pl.n_other.size()));
    GCA_TRY(dalloc(h, &w.gb, 9 * h->arows.size()));
    GCA_TRY(dalloc(h, &w.dT, 9 * (size_t)n));
    const auto &nodes = h->tree.nodes;
    std::vector<int32_t> leaf_of(n), leaf_index(nc, -1);
    for (size_t li = 0; li < h->leaves.size(); ++li) {
        const int c = h->leaves[li];
        leaf_index[c] = (int32_t)li;
        for (int32_t q = nodes[c].begin; q < nodes[c].end; ++q) leaf_of[q] = c;
    }
    GCA_TRY(upload_new(h, &w.leaf_of, leaf_of, s));
    GCA_TRY(upload_new(h, &w.leaf_index, leaf_index, s));
    auto csr = [&](const std::vector<int32_t> &key, int64_t nkey, std::vector<int64_t> &ptr,
                   std::vector<int32_t> &val) {
        ptr.assign(nkey + 1, 0);
        for (int32_t k : key) ptr[k + 1]++;
        for (int64_t i = 0; i < nkey; ++i) ptr[i + 1] += ptr[i];
        val.assign(key.size(), 0);
        std::vector<int64_t> f(ptr.begin(), ptr.end() - 1);
        for (size_t q = 0; q < key.size(); ++q) val[f[key[q]]++] = (int32_t)q;
    };
    std::vector<int64_t> ptr;
    std::vector<int32_t> val;
    csr(h->pivots, n, ptr, val);
    GCA_TRY(upload_new(h, &w.pocc_ptr, ptr, s));
    GCA_TRY(upload_new(h, &w.pocc, val, s));
    std::vector<int32_t> pc(h->n_piv);
    for (int c = 0; c < nc; ++c)
        for (int k = 0; k < h->rank[c]; ++k) pc[h->piv_off[c] + k] = c;
    GCA_TRY(upload_new(h, &w.piv_cluster, pc, s));
    csr(h->arows, n, ptr, val);
    GCA_TRY(upload_new(h, &w.rocc_ptr, ptr, s));
    GCA_TRY(upload_new(h, &w.rocc, val, s));
    // vertex -> (position, slot)
    std::vector<int32_t> vkey(3 * n);
    for (int64_t q = 0; q < n; ++q)
        for (int k = 0; k < 3; ++k) vkey[3 * q + k] = h->mesh.tri[3 * (int64_t)h->tree.perm[q] + k];
    csr(vkey, nv, ptr, val);
    std::vector<int32_t> vpos(val.size()), vslot(val.size());
    for (size_t q = 0; q < val.size(); ++q) {
        vpos[q] = val[q] / 3;
        vslot[q] = val[q] % 3;
    }
    GCA_TRY(upload_new(h, &w.vptr, ptr, s));
    GCA_TRY(upload_new(h, &w.vpos, vpos, s));
    GCA_TRY(upload_new(h, &w.vslot, vslot, s));
    w.ready = true;
    return GCA_OK;
}

template <typename T>
hipError_t grad_device(gca_h2_s *h, const double *a, const double *b, double alpha, const double *scale,
                       double *dxyz, hipStream_t s)
{
    GradWs &w = h->gw;
    const bool f32 = std::is_same<T, float>::value;
    T *ap = f32 ? (T *)w.apf : (T *)w.ap, *bp = f32 ? (T *)w.bpf : (T *)w.bp;
    T *xa = (T *)w.xa, *xb = (T *)w.xb, *ya = (T *)w.ya, *yb = (T *)w.yb, *cp = (T *)w.cpart;
    hipError_t e;
    // the factors of C = A^[I, J] and V^ depend only on the geometry: computed
    // by the first gradient after a build, and by every geometry update
    if (!h->fz.basis_current) {
        if ((e = launch_frozen_basis(h, s)) != hipSuccess) return e;
        h->fz.basis_current = true;
    }
    if ((e = launch_permute_in<T>(a, false, h->d_perm, h->n, ap, f32 ? w.ap : nullptr, s)) != hipSuccess) return e;
    if ((e = launch_permute_in<T>(b, false, h->d_perm, h->n, bp, f32 ? w.bp : nullptr, s)) != hipSuccess) return e;
    if ((e = launch_forward<T>(h, ap, xa, s)) != hipSuccess) return e;
    if ((e = launch_forward<T>(h, bp, xb, s)) != hipSuccess) return e;
    if ((e = launch_far_blocks<T>(h, xa, cp, s)) != hipSuccess) return e;
    if ((e = launch_coupling_reduce<T>(h, h->d_gslot_ptr, h->d_gslot, cp, ya, s)) != hipSuccess) return e;
    if ((e = launch_far_blocks<T>(h, xb, cp, s)) != hipSuccess) return e;
    if ((e = launch_coupling_reduce<T>(h, h->d_gslot_ptr, h->d_gslot, cp, yb, s)) != hipSuccess) return e;
    if ((e = launch_backward<T>(h, ya, s)) != hipSuccess) return e;
    if ((e = launch_backward<T>(h, yb, s)) != hipSuccess) return e;
    if ((e = launch_bilinear_grad<T>(h, w, s)) != hipSuccess) return e;
    return launch_vertex_gather(h, w, alpha, scale, dxyz, s);
}

// Computes and stores the coupling and nearfield block rows (and the list
// values) for the precisions in `which` (bit GCA_FP64, bit GCA_MIXED).
gca_status store_impl(gca_h2_s *h, int32_t which, hipStream_t s)
{
    free_stored(h);
    if (which == 0) return GCA_OK;
    auto alloc = [&](void **p, size_t bytes) -> gca_status {
        *p = dev_alloc(h, bytes);
        if (!*p) {
            free_stored(h);
            return alloc_error(bytes, "stored blocks");
        }
        return GCA_OK;
    };
    double *f64 = nullptr, *n64 = nullptr;
    float *f32 = nullptr, *n32 = nullptr;
    if (which & (1 << GCA_FP64)) {
        GCA_TRY(alloc((void **)&f64, (size_t)h->n_far_store * 8));
        h->d_far_g64 = f64;
        GCA_TRY(alloc((void **)&n64, (size_t)h->n_near_store * 8));
        h->d_near_g64 = n64;
        GCA_HIP_TRY(launch_store_blocks<double>(h, f64, n64, s));
    }
    if (which & (1 << GCA_MIXED)) {
        GCA_TRY(alloc((void **)&f32, (size_t)h->n_far_store * 4));
        h->d_far_g32 = f32;
        GCA_TRY(alloc((void **)&n32, (size_t)h->n_near_store * 4));
        h->d_near_g32 = n32;
        GCA_HIP_TRY(launch_store_blocks<float>(h, f32, n32, s));
    }
    GCA_HIP_TRY(launch_touching(h, h->d_tval, s));
    if (h->d_qnr != h->d_qr) {
        GCA_HIP_TRY(launch_nearreg<double>(h, h->d_nval, s));
        GCA_HIP_TRY(launch_nearreg<float>(h, h->d_nvalf, s));
    }
    GCA_HIP_TRY(hipStreamSynchronize(s));
    return GCA_OK;
}

// Phase times (ms) of the product in ring slot `slot`: out[k] for the
// phases, out[GCA_NPHASE] the whole product.
gca_status phase_ms_of(gca_h2_s *h, int slot, double *out)
{
    float ms;
    for (int k = 0; k < GCA_NPHASE; ++k) {
        GCA_HIP_TRY(hipEventElapsedTime(&ms, h->ev[slot][k][0], h->ev[slot][k][1]));
        out[k] = ms;
    }
    GCA_HIP_TRY(hipEventElapsedTime(&ms, h->ev_tot[slot][0], h->ev_tot[slot][1]));
    out[GCA_NPHASE] = ms;
    return GCA_OK;
}

}  // namespace

extern "C" {

gca_status gca_store_blocks(gca_h2 h, int32_t which, void *stream)
{
    clear_error();
    if (!h) return set_error(GCA_EINVAL, "handle is NULL");
    if (which & ~((1 << GCA_FP64) | (1 << GCA_MIXED))) return set_error(GCA_EINVAL, "unknown precision bits");
    h->cur_stream = (hipStream_t)stream;
    gca_status st = store_impl(h, which, (hipStream_t)stream);
    h->stored_mask = st == GCA_OK ? which : 0;
    return st;
}


void gca_params_default(gca_params *p)
{
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->eta = 2.0;
    p->eps = 1e-6;
    p->omega_scale = 0.25;
    p->green_m = 3;
    p->q_A = 3;
    p->q_r = 3;
    p->q_nr = 3;
    p->q_s = 4;
    p->q_c = 3;
    p->ss_fp32 = 0;
    p->serial = 0;
    p->alloc = nullptr;
    p->free = nullptr;
    p->alloc_ctx = nullptr;
}

const char *gca_last_error(void) { return last_error_cstr(); }

gca_status gca_tree_build(const gca_mesh *mesh, int32_t leaf_size, gca_tree *out)
{
    clear_error();
    if (!out) return set_error(GCA_EINVAL, "out is NULL");
    *out = nullptr;
    if (leaf_size < 1) return set_error(GCA_EINVAL, "leaf_size must be >= 1");
    Mesh m;
    GCA_TRY(mesh_copy_validate(mesh, m));
    auto *t = new (std::nothrow) gca_tree_s;
    if (!t) return set_error(GCA_ENOMEM, "out of host memory");
    gca_status st = tree_build(m, leaf_size, *t);
    if (st != GCA_OK) {
        delete t;
        return st;
    }
    *out = t;
    return GCA_OK;
}

gca_status gca_tree_info(gca_tree t, int64_t *n_clusters, int64_t *depth)
{
    clear_error();
    if (!t) return set_error(GCA_EINVAL, "tree is NULL");
    if (n_clusters) *n_clusters = (int64_t)t->nodes.size();
    if (depth) *depth = t->depth;
    return GCA_OK;
}

gca_status gca_tree_export(gca_tree t, int32_t *perm, int32_t *nodes, double *boxes)
{
    clear_error();
    if (!t) return set_error(GCA_EINVAL, "tree is NULL");
    if (perm) std::copy(t->perm.begin(), t->perm.end(), perm);
    for (size_t c = 0; c < t->nodes.size(); ++c) {
        const Node &nd = t->nodes[c];
        if (nodes) {
            nodes[5 * c + 0] = nd.begin;
            nodes[5 * c + 1] = nd.end;
            nodes[5 * c + 2] = nd.son[0];
            nodes[5 * c + 3] = nd.son[1];
            nodes[5 * c + 4] = nd.level;
        }
        if (boxes) {
            for (int d = 0; d < 3; ++d) {
                boxes[7 * c + d] = nd.lo[d];
                boxes[7 * c + 3 + d] = nd.hi[d];
            }
            boxes[7 * c + 6] = nd.diam;
        }
    }
    return GCA_OK;
}

void gca_tree_destroy(gca_tree t) { delete t; }

gca_status gca_block_tree(gca_tree t, double eta, int64_t far_capacity, int32_t *far, int64_t *n_far,
                          int64_t near_capacity, int32_t *near, int64_t *n_near)
{
    clear_error();
    if (!t) return set_error(GCA_EINVAL, "tree is NULL");
    if (!(eta > 0) || !std::isfinite(eta)) return set_error(GCA_EINVAL, "eta must be positive and finite");
    Blocks b;
    block_tree(*t, eta, b);
    const int64_t nf = (int64_t)b.far_t.size(), nn = (int64_t)b.near_t.size();
    if (n_far) *n_far = nf;
    if (n_near) *n_near = nn;
    gca_status st = GCA_OK;
    if (far) {
        if (far_capacity < nf) {
            st = set_error(GCA_EINVAL, "far capacity too small");
        } else {
            std::copy(b.far_t.begin(), b.far_t.end(), far);
            std::copy(b.far_s.begin(), b.far_s.end(), far + nf);
        }
    }
    if (near) {
        if (near_capacity < nn) {
            st = set_error(GCA_EINVAL, "near capacity too small");
        } else {
            std::copy(b.near_t.begin(), b.near_t.end(), near);
            std::copy(b.near_s.begin(), b.near_s.end(), near + nn);
        }
    }
    return st;
}

gca_status gca_build(const gca_mesh *mesh, gca_tree tree, const gca_params *p, void *stream, gca_h2 *out)
{
    clear_error();
    if (!out) return set_error(GCA_EINVAL, "out is NULL");
    *out = nullptr;
    if (!tree) return set_error(GCA_EINVAL, "tree is NULL");
    auto *h = new (std::nothrow) gca_h2_s;
    if (!h) return set_error(GCA_ENOMEM, "out of host memory");
    gca_status st = build_impl(mesh, tree, p, (hipStream_t)stream, h);
    if (st != GCA_OK) {
        free_all(h);
        delete h;
        return st;
    }
    *out = h;
    return GCA_OK;
}

gca_status h2_matvec(gca_h2 h, const void *x, void *y, int64_t nrhs, int64_t ld, int32_t dtype, int32_t precision,
                     void *stream)
{
    clear_error();
    if (!h) return set_error(GCA_EINVAL, "handle is NULL");
    if (!x || !y) return set_error(GCA_EINVAL, "x or y is NULL");
    if (nrhs < 1) return set_error(GCA_EINVAL, "nrhs must be >= 1");
    if (ld < h->n) return set_error(GCA_EINVAL, "ld must be >= n");
    if (dtype != GCA_F64 && dtype != GCA_F32) return set_error(GCA_EINVAL, "unknown dtype");
    if (precision != GCA_FP64 && precision != GCA_MIXED) return set_error(GCA_EINVAL, "unknown precision");
    const size_t es = dtype == GCA_F32 ? 4 : 8;
    {
        const char *xb = (const char *)x, *xe = xb + ((nrhs - 1) * ld + h->n) * es;
        const char *yb = (const char *)y, *ye = yb + ((nrhs - 1) * ld + h->n) * es;
        if (xb < ye && yb < xe) return set_error(GCA_EINVAL, "x and y overlap");
    }
    hipStream_t s = (hipStream_t)stream;
    const bool vf32 = dtype == GCA_F32;
    const bool f32 = precision == GCA_MIXED;
    if (nrhs > 1 && batch_supported(h, f32)) {
        // NB right-hand sides per pass, every block entry evaluated once per pass
        gca_h2_s::Batch *w = nullptr;
        h->cur_stream = s;
        GCA_TRY(f32 ? batch_workspace<float>(h, w) : batch_workspace<double>(h, w));
        for (int64_t k0 = 0; k0 < nrhs; k0 += NB) {
            const int nb = (int)std::min<int64_t>(NB, nrhs - k0);
            const void *xk = (const char *)x + k0 * ld * es;
            void *yk = (char *)y + k0 * ld * es;
            hipError_t e = f32 ? matvec_batch<float>(h, *w, xk, yk, nb, ld, vf32, k0 == 0, s)
                               : matvec_batch<double>(h, *w, xk, yk, nb, ld, vf32, k0 == 0, s);
            if (e != hipSuccess) return set_error(GCA_EHIP, std::string("batched matvec launch: ") + hipGetErrorString(e));
        }
        return GCA_OK;
    }
    for (int64_t k = 0; k < nrhs; ++k) {
        const void *xk = (const char *)x + k * ld * es;
        void *yk = (char *)y + k * ld * es;
        hipError_t e = precision == GCA_FP64 ? matvec_one<double>(h, xk, yk, vf32, k == 0, s)
                                             : matvec_one<float>(h, xk, yk, vf32, k == 0, s);
        if (e != hipSuccess) return set_error(GCA_EHIP, std::string("matvec launch: ") + hipGetErrorString(e));
    }
    return GCA_OK;
}

gca_status gca_energy(gca_h2 h, const double *u, const double *scale, double *e, double *g, int32_t precision,
                      void *stream)
{
    clear_error();
    GCA_TRY(gca::energy_check(h, u, e, g, precision));
    hipStream_t s = (hipStream_t)stream;
    h->cur_stream = s;
    if (!h->d_dotp) GCA_TRY(dalloc(h, &h->d_dotp, gca::DOT_PARTIALS));
    if (!g && !h->d_ews) GCA_TRY(dalloc(h, &h->d_ews, (size_t)h->n));
    return gca::energy_run(h, u, scale, e, g, precision, s, h->d_dotp, h->d_ews);
}

gca_status gca_entries(gca_h2 h, const int32_t *I, const int32_t *J, int64_t m, double *out, int32_t precision,
                       void *stream)
{
    clear_error();
    if (!h) return set_error(GCA_EINVAL, "handle is NULL");
    if (m < 0) return set_error(GCA_EINVAL, "m must be >= 0");
    if (m == 0) return GCA_OK;
    if (!I || !J || !out) return set_error(GCA_EINVAL, "NULL pointer");
    if (precision != GCA_FP64 && precision != GCA_MIXED) return set_error(GCA_EINVAL, "unknown precision");
    hipStream_t s = (hipStream_t)stream;
    std::vector<int32_t> hi(m), hj(m);
    GCA_HIP_TRY(hipMemcpyAsync(hi.data(), I, m * 4, hipMemcpyDeviceToHost, s));
    GCA_HIP_TRY(hipMemcpyAsync(hj.data(), J, m * 4, hipMemcpyDeviceToHost, s));
    GCA_HIP_TRY(hipStreamSynchronize(s));
    std::vector<int32_t> cls[5], codes[5], idx[5], fa[5], fb[5];
    std::vector<int32_t> iperm(h->n);
    for (int64_t q = 0; q < h->n; ++q) iperm[h->tree.perm[q]] = (int32_t)q;
    for (int64_t k = 0; k < m; ++k) {
        int32_t a = hi[k], b = hj[k];
        if (a < 0 || a >= h->n || b < 0 || b >= h->n) return set_error(GCA_EINVAL, "triangle id out of range");
        if (a > b) std::swap(a, b);
        int32_t code = 0;
        int kind = classify_pair(h->mesh, h->adj, a, b, &code);
        int slot = kind;   // 0 ident, 1 edge, 2 vert, 3 near-regular, 4 regular
        fa[slot].push_back(iperm[a]);
        fb[slot].push_back(iperm[b]);
        codes[slot].push_back(code);
        idx[slot].push_back((int32_t)k);
    }
    std::vector<int32_t> pa, pb, pc, order;
    EntryJobs j{};
    for (int c = 0; c < 5; ++c) {
        j.off[c] = (int64_t)pa.size();
        pa.insert(pa.end(), fa[c].begin(), fa[c].end());
        pb.insert(pb.end(), fb[c].begin(), fb[c].end());
        pc.insert(pc.end(), codes[c].begin(), codes[c].end());
        order.insert(order.end(), idx[c].begin(), idx[c].end());
    }
    j.off[5] = (int64_t)pa.size();
    // workspace held by the handle: pair arrays (3 x int32) and values (FP64 + FP32) per pair
    if ((size_t)m > h->ent_cap) {
        GCA_HIP_TRY(hipStreamSynchronize(s));
        dev_free(h, h->d_ent);
        h->d_ent = nullptr;
        h->ent_cap = 0;
        const size_t cap = std::max<size_t>((size_t)m, 1024);
        h->cur_stream = s;
        h->d_ent = dev_alloc(h, cap * 24);
        if (!h->d_ent) return alloc_error(cap * 24, "entries workspace");
        h->ent_cap = cap;
    }
    double *t64 = (double *)h->d_ent;
    int32_t *dpa = (int32_t *)(t64 + h->ent_cap), *dpb = dpa + h->ent_cap, *dpc = dpb + h->ent_cap;
    float *t32 = (float *)(dpc + h->ent_cap);
    gca_status st = GCA_OK;
    auto fail = [&](hipError_t e, const char *what) {
        st = set_error(GCA_EHIP, std::string(what) + ": " + hipGetErrorString(e));
    };
    hipError_t e = hipMemcpyAsync(dpa, pa.data(), m * 4, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(dpb, pb.data(), m * 4, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(dpc, pc.data(), m * 4, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) fail(e, "entries setup");
    std::vector<double> r64(m);
    std::vector<float> r32(m);
    if (st == GCA_OK) {
        j.pa = dpa;
        j.pb = dpb;
        j.code = dpc;
        e = launch_entry_jobs(h, j, t64, t32, precision, s);
        if (e == hipSuccess) e = hipMemcpyAsync(r64.data(), t64, m * 8, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipMemcpyAsync(r32.data(), t32, m * 4, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) fail(e, "entries kernels");
    }
    if (st == GCA_OK) {
        std::vector<double> res(m);
        for (int64_t q = 0; q < m; ++q) {
            bool f32 = precision == GCA_MIXED && q >= j.off[3];
            res[order[q]] = f32 ? (double)r32[q] : r64[q];
        }
        e = hipMemcpyAsync(out, res.data(), m * 8, hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) fail(e, "entries result");
    }
    return st;
}

gca_status gca_dl_entries(gca_h2 h, const int32_t *I, const int32_t *J, int64_t m, double *out, void *stream)
{
    clear_error();
    if (!h) return set_error(GCA_EINVAL, "handle is NULL");
    if (m < 0) return set_error(GCA_EINVAL, "m must be >= 0");
    if (m == 0) return GCA_OK;
    if (!I || !J || !out) return set_error(GCA_EINVAL, "NULL pointer");
    hipStream_t s = (hipStream_t)stream;
    // the vertex adjacency of the near-regular class, uploaded by the first call
    if (!h->d_vv_ptr) {
        h->cur_stream = s;
        GCA_TRY(upload_new(h, &h->d_vv_ptr, h->adj.vv_ptr, s));
        GCA_TRY(upload_new(h, &h->d_vv, h->adj.vv, s));
    }
    GCA_HIP_TRY(launch_dl_pairs(h->d_xyz, h->d_tv, h->d_iperm, h->d_vv_ptr, h->d_vv, h->n, I, J, m, h->prm.q_r,
                                h->prm.q_nr, h->prm.q_s, h->prm.sym_rules != 0, out, s));
    return GCA_OK;
}

gca_status gca_block_entries(gca_h2 h, int32_t precision, int32_t kind, int64_t capacity, int32_t *rows,
                             int32_t *cols, double *vals, int64_t *count, void *stream)
{
    clear_error();
    if (!h) return set_error(GCA_EINVAL, "handle is NULL");
    if (precision != GCA_FP64 && precision != GCA_MIXED) return set_error(GCA_EINVAL, "unknown precision");
    if (kind != 0 && kind != 1) return set_error(GCA_EINVAL, "kind must be 0 (coupling) or 1 (nearfield)");
    if (!(h->stored_mask & (1 << precision)))
        return set_error(GCA_EINVAL, "the blocks of this precision are not stored (gca_store_blocks)");
    const bool far = kind == 0;
    const int64_t total = far ? h->n_far_store : h->n_near_store;
    if (count) *count = total;
    if (!rows && !cols && !vals) return GCA_OK;
    if (!rows || !cols || !vals) return set_error(GCA_EINVAL, "rows, cols and vals must all be given");
    if (capacity < total) return set_error(GCA_EINVAL, "capacity below the number of stored entries");
    hipStream_t s = (hipStream_t)stream;
    const int ng = far ? h->n_far_groups : h->n_near_groups;
    std::vector<int32_t> g_t(ng);
    std::vector<int64_t> g_ptr(ng + 1, 0), g_soff(ng);
    if (ng > 0) {
        GCA_HIP_TRY(hipMemcpyAsync(g_t.data(), far ? h->d_fg_t : h->d_ng_t, ng * 4, hipMemcpyDeviceToHost, s));
        GCA_HIP_TRY(hipMemcpyAsync(g_ptr.data(), far ? h->d_fg_ptr : h->d_ng_ptr, (ng + 1) * 8,
                                   hipMemcpyDeviceToHost, s));
        GCA_HIP_TRY(hipMemcpyAsync(g_soff.data(), far ? h->d_fg_soff : h->d_ng_soff, ng * 8,
                                   hipMemcpyDeviceToHost, s));
    }
    GCA_HIP_TRY(hipStreamSynchronize(s));
    const int64_t ncol = g_ptr[ng];
    std::vector<int32_t> col(ncol);
    if (ncol > 0)
        GCA_HIP_TRY(hipMemcpyAsync(col.data(), far ? h->d_fcol_e : h->d_ncol_pos, ncol * 4, hipMemcpyDeviceToHost, s));
    std::vector<double> v64;
    std::vector<float> v32;
    if (precision == GCA_FP64) {
        v64.resize(total);
        if (total > 0)
            GCA_HIP_TRY(hipMemcpyAsync(v64.data(), far ? h->d_far_g64 : h->d_near_g64, total * 8,
                                       hipMemcpyDeviceToHost, s));
    } else {
        v32.resize(total);
        if (total > 0)
            GCA_HIP_TRY(hipMemcpyAsync(v32.data(), far ? h->d_far_g32 : h->d_near_g32, total * 4,
                                       hipMemcpyDeviceToHost, s));
    }
    GCA_HIP_TRY(hipStreamSynchronize(s));
    const auto &perm = h->tree.perm;
    const auto &nodes = h->tree.nodes;
    for (int k = 0; k < ng; ++k) {
        const int t = g_t[k];
        const int64_t nc = g_ptr[k + 1] - g_ptr[k];
        const int nr = far ? h->rank[t] : nodes[t].end - nodes[t].begin;
        for (int i = 0; i < nr; ++i) {
            const int rpos = far ? h->pivots[h->piv_off[t] + i] : nodes[t].begin + i;
            for (int64_t j = 0; j < nc; ++j) {
                const int64_t o = g_soff[k] + (int64_t)i * nc + j;
                const int32_t c = col[g_ptr[k] + j];
                rows[o] = perm[rpos];
                cols[o] = perm[far ? h->pivots[c] : c];
                vals[o] = precision == GCA_FP64 ? v64[o] : (double)v32[o];
            }
        }
    }
    return GCA_OK;
}

gca_status gca_solve_refined(gca_h2 h, const double *f, double *u, double rtol, int32_t max_outer,
                             double inner_rtol, int32_t max_inner, int32_t *iters_out, double *relres_out,
                             void *stream)
{
    clear_error();
    if (!h) return set_error(GCA_EINVAL, "handle is NULL");
    if (!f || !u) return set_error(GCA_EINVAL, "f or u is NULL");
    if (!(rtol > 0 && rtol < 1) || !(inner_rtol > 0 && inner_rtol < 1))
        return set_error(GCA_EINVAL, "tolerances must be in (0, 1)");
    if (max_outer < 1 || max_inner < 1) return set_error(GCA_EINVAL, "iteration limits must be >= 1");
    const int64_t n = h->n;
    {
        const char *fb = (const char *)f, *fe = (const char *)(f + n);
        const char *ub = (const char *)u, *ue = (const char *)(u + n);
        if (fb < ue && ub < fe) return set_error(GCA_EINVAL, "f and u overlap");
    }
    hipStream_t s = (hipStream_t)stream;
    h->cur_stream = s;
    if (!h->d_sv) GCA_TRY(dalloc(h, &h->d_sv, 5 * (size_t)n));
    if (!h->d_dotp) GCA_TRY(dalloc(h, &h->d_dotp, gca::DOT_PARTIALS));
    double *r = h->d_sv, *d = r + n, *res = d + n, *p = res + n, *q = p + n;
    double *dres = h->d_dotp + 1024;
    auto dot = [&](const double *a, const double *b, double *out) -> gca_status {
        GCA_HIP_TRY(launch_dot(a, b, n, h->d_dotp, dres, s));
        GCA_HIP_TRY(hipMemcpyAsync(out, dres, sizeof(double), hipMemcpyDeviceToHost, s));
        GCA_HIP_TRY(hipStreamSynchronize(s));
        return GCA_OK;
    };
    auto product = [&](const double *x, double *y, int prec) -> gca_status {
        hipError_t e = prec == GCA_FP64 ? matvec_one<double>(h, x, y, false, true, s)
                                        : matvec_one<float>(h, x, y, false, true, s);
        if (e != hipSuccess) return set_error(GCA_EHIP, std::string("product in solve: ") + hipGetErrorString(e));
        return GCA_OK;
    };
    double ff;
    GCA_TRY(dot(f, f, &ff));
    const double nf = std::sqrt(ff);
    GCA_HIP_TRY(launch_fill(u, 0.0, n, s));
    int32_t outer = 0, inner = 0;
    double relres = nf > 0 ? 1.0 : 0.0;
    if (nf > 0) {
        for (;;) {
            // FP64 refinement residual r = f - G~ u
            GCA_TRY(product(u, q, GCA_FP64));
            GCA_HIP_TRY(launch_sub(f, q, r, n, s));
            double rr;
            GCA_TRY(dot(r, r, &rr));
            relres = std::sqrt(rr) / nf;
            if (relres <= rtol || outer >= max_outer) break;
            ++outer;
            // inner CG on the mixed-precision operator: G~_mixed d = r
            GCA_HIP_TRY(launch_fill(d, 0.0, n, s));
            GCA_HIP_TRY(hipMemcpyAsync(res, r, n * sizeof(double), hipMemcpyDeviceToDevice, s));
            GCA_HIP_TRY(hipMemcpyAsync(p, r, n * sizeof(double), hipMemcpyDeviceToDevice, s));
            double rho = rr;
            const double stop = inner_rtol * std::sqrt(rr);
            for (int it = 0; it < max_inner; ++it) {
                GCA_TRY(product(p, q, GCA_MIXED));
                double pq;
                GCA_TRY(dot(p, q, &pq));
                ++inner;
                if (!(pq > 0))
                    return set_error(GCA_ENOTSPD, "conjugate gradients met p^T G p <= 0 (operator not positive definite)");
                const double alpha = rho / pq;
                GCA_HIP_TRY(launch_cg_update(alpha, p, q, d, res, n, s));
                double rho_new;
                GCA_TRY(dot(res, res, &rho_new));
                if (std::sqrt(rho_new) <= stop) break;
                GCA_HIP_TRY(launch_axpby(1.0, res, rho_new / rho, p, n, s));
                rho = rho_new;
            }
            GCA_HIP_TRY(launch_axpby(1.0, d, 1.0, u, n, s));
        }
    }
    if (iters_out) {
        iters_out[0] = outer;
        iters_out[1] = inner;
    }
    if (relres_out) *relres_out = relres;
    if (relres > rtol)
        return set_error(GCA_ENOCONV, "refinement stopped at relative residual " + std::to_string(relres));
    return GCA_OK;
}

gca_status gca_update_geometry(gca_h2 h, const double *xyz, void *stream)
{
    clear_error();
    if (!h || !xyz) return set_error(GCA_EINVAL, "NULL argument");
    for (int64_t k = 0; k < 3 * h->nv; ++k)
        if (!std::isfinite(xyz[k])) return set_error(GCA_EINVAL, "non-finite vertex coordinate");
    hipStream_t s = (hipStream_t)stream;
    h->cur_stream = s;
    GCA_TRY(frozen_setup(h, s));
    std::copy(xyz, xyz + 3 * h->nv, h->mesh.xyz.begin());
    GCA_TRY(upload(h->d_xyz, h->mesh.xyz, s));
    const bool sym = h->prm.sym_rules != 0;
    auto tri_pts = [&](int q, bool sy, double *out) -> gca_status {
        TriRule r;
        if (!tri_rule(q, sy, r)) return set_error(GCA_EINVAL, "unsupported triangle rule");
        GCA_HIP_TRY(launch_tri_points(h->d_xyz, h->d_tv, h->n, r, out, s));
        return GCA_OK;
    };
    GCA_TRY(tri_pts(h->prm.q_r, sym, h->d_qr));
    GCA_HIP_TRY(launch_local_points(h, s));
    if (h->d_qnr != h->d_qr) GCA_TRY(tri_pts(h->prm.q_nr, sym, h->d_qnr));
    if (h->d_qA != h->d_qr) GCA_TRY(tri_pts(h->prm.q_A, false, h->d_qA));
    if (h->d_qc != h->d_qr) GCA_TRY(tri_pts(h->prm.q_c, sym, h->d_qc));
    if (h->n_piv_total > 0) GCA_HIP_TRY(launch_pivot_points(h, s));
    h->fz.basis_current = false;
    GCA_HIP_TRY(launch_frozen_basis(h, s));
    h->fz.basis_current = true;
    if (h->stored_mask) GCA_TRY(store_impl(h, h->stored_mask, s));
    Frozen &fz = h->fz;
    GCA_HIP_TRY(launch_copy_jobs(fz.d_copy_jobs, fz.n_vjobs, fz.d_Vh, h->d_V, h->d_Vt, h->d_Vf, h->d_Vtf, s));
    GCA_HIP_TRY(launch_copy_jobs(fz.d_copy_jobs + 6 * (int64_t)fz.n_vjobs, fz.n_ejobs, fz.d_Vh, h->d_E, h->d_Et,
                                 h->d_Ef, h->d_Etf, s));
    GCA_HIP_TRY(hipStreamSynchronize(s));
    return GCA_OK;
}

gca_status h2_bilinear_grad(gca_h2 h, const double *a, const double *b, double alpha, const double *scale,
                            double *dxyz, int32_t precision, void *stream)
{
    clear_error();
    if (!h) return set_error(GCA_EINVAL, "handle is NULL");
    if (!a || !b || !dxyz) return set_error(GCA_EINVAL, "NULL vector");
    if (precision != GCA_FP64 && precision != GCA_MIXED) return set_error(GCA_EINVAL, "unknown precision");
    if (!std::isfinite(alpha)) return set_error(GCA_EINVAL, "alpha must be finite");
    hipStream_t s = (hipStream_t)stream;
    h->cur_stream = s;
    GCA_TRY(frozen_setup(h, s));
    GCA_TRY(grad_setup(h, s));
    hipError_t e = precision == GCA_FP64 ? grad_device<double>(h, a, b, alpha, scale, dxyz, s)
                                         : grad_device<float>(h, a, b, alpha, scale, dxyz, s);
    if (e != hipSuccess) return set_error(GCA_EHIP, std::string("adjoint launch: ") + hipGetErrorString(e));
    return GCA_OK;
}

gca_status gca_basis_sizes(gca_h2 h, int64_t *n_pivots, int64_t *n_basis)
{
    clear_error();
    if (!h) return set_error(GCA_EINVAL, "handle is NULL");
    if (n_pivots) *n_pivots = h->n_piv;
    if (n_basis) *n_basis = h->n_v + h->n_e;
    return GCA_OK;
}

gca_status gca_basis_export(gca_h2 h, int32_t *ranks, int32_t *pivots, double *basis)
{
    clear_error();
    if (!h) return set_error(GCA_EINVAL, "handle is NULL");
    if (ranks) std::copy(h->rank.begin(), h->rank.end(), ranks);
    if (pivots)
        for (int64_t q = 0; q < h->n_piv; ++q) pivots[q] = h->tree.perm[h->pivots[q]];
    if (basis) {
        GCA_HIP_TRY(hipDeviceSynchronize());
        if (h->n_v) GCA_HIP_TRY(hipMemcpy(basis, h->d_V, h->n_v * 8, hipMemcpyDeviceToHost));
        if (h->n_e) GCA_HIP_TRY(hipMemcpy(basis + h->n_v, h->d_E, h->n_e * 8, hipMemcpyDeviceToHost));
    }
    return GCA_OK;
}

gca_status gca_stats(gca_h2 h, gca_stats_t *out)
{
    clear_error();
    if (!h || !out) return set_error(GCA_EINVAL, "NULL argument");
    *out = h->st;
    out->store_entries_far = h->n_far_store;
    out->store_entries_near = h->n_near_store;
    out->stored_mask = h->stored_mask;
    out->reserved_i = 0;
    out->basis_entries_leaf = h->n_v;
    out->basis_entries_transfer = h->n_e;
    if (h->events && h->timed) {
        const int slot = (int)((h->n_products - 1) % gca_h2_s::RING);
        GCA_HIP_TRY(hipEventSynchronize(h->ev_tot[slot][1]));
        GCA_TRY(phase_ms_of(h, slot, out->phase_ms));
    }
    return GCA_OK;
}

gca_status gca_phase_times(gca_h2 h, int64_t max_products, double *out, int64_t *count)
{
    clear_error();
    if (!h || !count) return set_error(GCA_EINVAL, "NULL argument");
    int64_t c = std::min<int64_t>({h->n_products, (int64_t)gca_h2_s::RING, std::max<int64_t>(max_products, 0)});
    *count = c;
    if (!c || !out) return GCA_OK;
    const int last = (int)((h->n_products - 1) % gca_h2_s::RING);
    GCA_HIP_TRY(hipEventSynchronize(h->ev_tot[last][1]));
    for (int64_t q = 0; q < c; ++q) {
        const int slot = (int)((h->n_products - c + q) % gca_h2_s::RING);
        GCA_TRY(phase_ms_of(h, slot, out + q * (GCA_NPHASE + 1)));
    }
    return GCA_OK;
}

void gca_destroy(gca_h2 h)
{
    if (!h) return;
    (void)hipDeviceSynchronize();
    free_all(h);
    delete h;
}

}  // extern "C"

namespace gca {

// Shared with the nodal-basis handle (lin_h2.cpp): the handle's device
// memory, the parameter checks and the level-wise basis construction.
gca_status handle_alloc(gca_h2_s *h, void **p, size_t bytes)
{
    char *q = nullptr;
    GCA_TRY(dalloc(h, &q, bytes));
    *p = q;
    return GCA_OK;
}
void handle_free_all(gca_h2_s *h) { free_all(h); }
gca_status params_check(const gca_params *p) { return check_params(p); }
gca_status basis_build(gca_h2_s *h, hipStream_t s) { return build_basis(h, s); }

gca_status energy_check(const gca_h2_s *h, const double *u, const double *e, const double *g, int32_t precision)
{
    if (!h) return set_error(GCA_EINVAL, "handle is NULL");
    if (!u) return set_error(GCA_EINVAL, "u is NULL");
    if (!e && !g) return set_error(GCA_EINVAL, "nothing to compute: e and g are both NULL");
    if (precision != GCA_FP64 && precision != GCA_MIXED) return set_error(GCA_EINVAL, "unknown precision");
    const int64_t n = h->n;
    if (g) {
        const char *ub = (const char *)u, *ue = (const char *)(u + n);
        const char *gb = (const char *)g, *ge = (const char *)(g + n);
        if (ub < ge && gb < ue) return set_error(GCA_EINVAL, "g and u overlap");
    }
    if (e && (const char *)e >= (const char *)u && (const char *)e < (const char *)(u + n))
        return set_error(GCA_EINVAL, "e lies inside u");
    return GCA_OK;
}

gca_status energy_run(gca_h2_s *h, const double *u, const double *scale, double *e, double *g, int32_t precision,
                      hipStream_t s, double *dotp, double *ews)
{
    const int64_t n = h->n;
    double *gu = g ? g : ews;
    hipError_t err = precision == GCA_FP64 ? matvec_one<double>(h, u, gu, false, true, s)
                                           : matvec_one<float>(h, u, gu, false, true, s);
    if (err == hipSuccess && e) err = launch_dot(u, gu, n, dotp, e, s, 0.5);
    if (err == hipSuccess && g && scale) err = launch_scale(scale, g, g, n, s);
    if (err != hipSuccess) return set_error(GCA_EHIP, std::string("energy launch: ") + hipGetErrorString(err));
    return GCA_OK;
}

bool tri_rule(int q, bool sym, TriRule &r)
{
    r = TriRule{};
    if (!sym) {
        if (q < 1 || q * q > 64) return false;
        double x[32], w[32];
        gauss_legendre01(q, x, w);
        for (int a = 0; a < q; ++a)
            for (int b = 0; b < q; ++b) {
                r.s1[r.np] = x[a];
                r.s2[r.np] = x[a] * x[b];
                r.w[r.np] = w[a] * w[b] * x[a];
                ++r.np;
            }
        return true;
    }
    // fully symmetric rules: orbits (a, a, 1 - 2a) of barycentric points with
    // barycentric weight w each; s1 = l1 + l2, s2 = l2, weight w / 2 on the
    // reference triangle.  Degree 2 (q = 2): a = 1/6, w = 1/3.  Degree 4
    // (q = 3, Strang-Fix / Dunavant): a = 0.445948490915965, w =
    // 0.223381589678011 and a = 0.091576213509771, w = 0.109951743655322.
    auto orbit = [&](double a, double w) {
        const double b = 1.0 - 2.0 * a;
        const double l[3][3] = {{b, a, a}, {a, b, a}, {a, a, b}};
        for (auto &k : l) {
            r.s1[r.np] = k[1] + k[2];
            r.s2[r.np] = k[2];
            r.w[r.np] = 0.5 * w;
            ++r.np;
        }
    };
    if (q == 2) {
        orbit(1.0 / 6.0, 1.0 / 3.0);
        return true;
    }
    if (q == 3) {
        orbit(0.445948490915965, 0.223381589678011);
        orbit(0.091576213509771, 0.109951743655322);
        return true;
    }
    return false;
}

}  // namespace gca
