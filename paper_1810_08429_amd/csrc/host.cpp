// Host side of libgca: mesh checks, adjacency, cluster tree, block tree and
// the per-case pair lists.  Compiled with -ffp-contract=off so that boxes,
// diameters and distances are rounded exactly as written (the admissibility
// test of Section 2 is a comparison of such values).
#include <algorithm>
#include <atomic>
#include <cmath>
#include <thread>
#include <cstring>
#include <numeric>
#include <utility>

#include "gca_internal.h"

namespace gca {

static thread_local std::string g_err;

gca_status set_error(gca_status s, const std::string &msg)
{
    g_err = msg;
    return s;
}

void clear_error() { g_err.clear(); }

const char *last_error_cstr() { return g_err.c_str(); }

// ------------------------------------------------------------------- mesh --

gca_status mesh_copy_validate(const gca_mesh *m, Mesh &out)
{
    if (!m) return set_error(GCA_EINVAL, "mesh is NULL");
    if (m->nt < 1 || m->nv < 3) return set_error(GCA_EINVAL, "mesh needs nt >= 1 and nv >= 3");
    if (m->nt > INT32_MAX / 4 || m->nv > INT32_MAX / 4)
        return set_error(GCA_EINVAL, "mesh too large for 32-bit indices");
    if (!m->xyz || !m->tri) return set_error(GCA_EINVAL, "mesh arrays are NULL");
    out.nv = m->nv;
    out.nt = m->nt;
    out.xyz.assign(m->xyz, m->xyz + 3 * m->nv);
    out.tri.assign(m->tri, m->tri + 3 * m->nt);
    for (double v : out.xyz)
        if (!std::isfinite(v)) return set_error(GCA_EINVAL, "non-finite vertex coordinate");
    for (int64_t t = 0; t < m->nt; ++t) {
        const int32_t *v = &out.tri[3 * t];
        for (int k = 0; k < 3; ++k)
            if (v[k] < 0 || v[k] >= m->nv)
                return set_error(GCA_EMESH, "triangle " + std::to_string(t) + ": vertex index out of range");
        if (v[0] == v[1] || v[1] == v[2] || v[0] == v[2])
            return set_error(GCA_EMESH, "triangle " + std::to_string(t) + ": repeated vertex");
        const double *a = &out.xyz[3 * v[0]], *b = &out.xyz[3 * v[1]], *c = &out.xyz[3 * v[2]];
        double e1[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
        double e2[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
        double cx = e1[1] * e2[2] - e1[2] * e2[1];
        double cy = e1[2] * e2[0] - e1[0] * e2[2];
        double cz = e1[0] * e2[1] - e1[1] * e2[0];
        if (!(cx * cx + cy * cy + cz * cz > 0.0))
            return set_error(GCA_EMESH, "triangle " + std::to_string(t) + ": zero area");
    }
    // duplicate triangles and non-manifold edges
    {
        std::vector<std::array<int32_t, 3>> s(m->nt);
        for (int64_t t = 0; t < m->nt; ++t) {
            std::array<int32_t, 3> k = {out.tri[3 * t], out.tri[3 * t + 1], out.tri[3 * t + 2]};
            std::sort(k.begin(), k.end());
            s[t] = k;
        }
        std::sort(s.begin(), s.end());
        for (size_t i = 1; i < s.size(); ++i)
            if (s[i] == s[i - 1]) return set_error(GCA_EMESH, "duplicate triangle");
        std::vector<std::pair<int32_t, int32_t>> e;
        e.reserve(3 * m->nt);
        for (int64_t t = 0; t < m->nt; ++t)
            for (int k = 0; k < 3; ++k) {
                int32_t a = out.tri[3 * t + k], b = out.tri[3 * t + (k + 1) % 3];
                e.emplace_back(std::min(a, b), std::max(a, b));
            }
        std::sort(e.begin(), e.end());
        size_t run = 1;
        for (size_t i = 1; i <= e.size(); ++i) {
            if (i < e.size() && e[i] == e[i - 1]) {
                if (++run > 2) return set_error(GCA_EMESH, "non-manifold edge (more than two triangles)");
            } else {
                run = 1;
            }
        }
    }
    return GCA_OK;
}

gca_status build_adjacency(const Mesh &m, Adjacency &adj)
{
    const int64_t nv = m.nv, nt = m.nt;
    adj.vt_ptr.assign(nv + 1, 0);
    for (int64_t t = 0; t < nt; ++t)
        for (int k = 0; k < 3; ++k) adj.vt_ptr[m.tri[3 * t + k] + 1]++;
    for (int64_t v = 0; v < nv; ++v) adj.vt_ptr[v + 1] += adj.vt_ptr[v];
    adj.vt.assign(adj.vt_ptr[nv], 0);
    {
        std::vector<int64_t> fill(adj.vt_ptr.begin(), adj.vt_ptr.end() - 1);
        for (int64_t t = 0; t < nt; ++t)
            for (int k = 0; k < 3; ++k) adj.vt[fill[m.tri[3 * t + k]]++] = (int32_t)t;
    }
    // vertex neighbours through edges
    std::vector<std::vector<int32_t>> nb(nv);
    for (int64_t t = 0; t < nt; ++t)
        for (int k = 0; k < 3; ++k) {
            int32_t a = m.tri[3 * t + k], b = m.tri[3 * t + (k + 1) % 3];
            nb[a].push_back(b);
            nb[b].push_back(a);
        }
    adj.vv_ptr.assign(nv + 1, 0);
    for (int64_t v = 0; v < nv; ++v) {
        auto &l = nb[v];
        std::sort(l.begin(), l.end());
        l.erase(std::unique(l.begin(), l.end()), l.end());
        adj.vv_ptr[v + 1] = adj.vv_ptr[v] + (int64_t)l.size();
    }
    adj.vv.resize(adj.vv_ptr[nv]);
    for (int64_t v = 0; v < nv; ++v) std::copy(nb[v].begin(), nb[v].end(), adj.vv.begin() + adj.vv_ptr[v]);
    return GCA_OK;
}

// ------------------------------------------------------------ cluster tree --

namespace {

struct TreeBuilder {
    const Mesh &m;
    int32_t leaf;
    gca_tree_s &t;
    std::vector<double> cent;   // nt x 3
    std::vector<int32_t> tmp;

    void box_of(int32_t b, int32_t e, Node &nd)
    {
        for (int d = 0; d < 3; ++d) {
            nd.lo[d] = INFINITY;
            nd.hi[d] = -INFINITY;
        }
        for (int32_t p = b; p < e; ++p) {
            int32_t tri = t.perm[p];
            for (int k = 0; k < 3; ++k) {
                const double *v = &m.xyz[3 * (int64_t)m.tri[3 * (int64_t)tri + k]];
                for (int d = 0; d < 3; ++d) {
                    nd.lo[d] = std::min(nd.lo[d], v[d]);
                    nd.hi[d] = std::max(nd.hi[d], v[d]);
                }
            }
        }
        double e0 = nd.hi[0] - nd.lo[0], e1 = nd.hi[1] - nd.lo[1], e2 = nd.hi[2] - nd.lo[2];
        nd.diam = std::sqrt((e0 * e0 + e1 * e1) + e2 * e2);
    }

    int32_t rec(int32_t b, int32_t e, int32_t level, int32_t parent)
    {
        int32_t me = (int32_t)t.nodes.size();
        t.nodes.push_back(Node{});
        {
            Node &nd = t.nodes[me];
            nd.begin = b;
            nd.end = e;
            nd.son[0] = nd.son[1] = -1;
            nd.parent = parent;
            nd.level = level;
        }
        t.depth = std::max(t.depth, level);
        if (e - b <= leaf) return me;
        double clo[3] = {INFINITY, INFINITY, INFINITY}, chi[3] = {-INFINITY, -INFINITY, -INFINITY};
        for (int32_t p = b; p < e; ++p)
            for (int d = 0; d < 3; ++d) {
                double c = cent[3 * (int64_t)t.perm[p] + d];
                clo[d] = std::min(clo[d], c);
                chi[d] = std::max(chi[d], c);
            }
        int axis = 0;
        double best = chi[0] - clo[0];
        for (int d = 1; d < 3; ++d)
            if (chi[d] - clo[d] > best) {
                best = chi[d] - clo[d];
                axis = d;
            }
        const double *cc = cent.data();
        auto less = [cc, axis](int32_t x, int32_t y) {
            double kx = cc[3 * (int64_t)x + axis], ky = cc[3 * (int64_t)y + axis];
            if (kx != ky) return kx < ky;
            return x < y;
        };
        // Same result as sorting the whole range by (coordinate, id) and cutting
        // at the median: the partition needs only nth_element; a son that is a
        // leaf keeps the sorted order, a son that is split sorts its own range.
        int32_t mid = b + (e - b) / 2;
        std::nth_element(t.perm.begin() + b, t.perm.begin() + mid, t.perm.begin() + e, less);
        if (mid - b <= leaf) std::sort(t.perm.begin() + b, t.perm.begin() + mid, less);
        if (e - mid <= leaf) std::sort(t.perm.begin() + mid, t.perm.begin() + e, less);
        int32_t s0 = rec(b, mid, level + 1, me);
        int32_t s1 = rec(mid, e, level + 1, me);
        t.nodes[me].son[0] = s0;
        t.nodes[me].son[1] = s1;
        return me;
    }
};

}  // namespace

gca_status tree_build(const Mesh &m, int32_t leaf, gca_tree_s &t)
{
    if (leaf < 1) return set_error(GCA_EINVAL, "leaf_size must be >= 1");
    t.nt = m.nt;
    t.nv = m.nv;
    t.leaf = leaf;
    t.perm.resize(m.nt);
    std::iota(t.perm.begin(), t.perm.end(), 0);
    t.nodes.clear();
    t.nodes.reserve(4 * (m.nt / std::max(1, leaf / 2) + 1));
    t.depth = 0;
    TreeBuilder tb{m, leaf, t, {}, {}};
    tb.cent.resize(3 * m.nt);
    for (int64_t i = 0; i < m.nt; ++i)
        for (int d = 0; d < 3; ++d) {
            double v0 = m.xyz[3 * (int64_t)m.tri[3 * i] + d];
            double v1 = m.xyz[3 * (int64_t)m.tri[3 * i + 1] + d];
            double v2 = m.xyz[3 * (int64_t)m.tri[3 * i + 2] + d];
            tb.cent[3 * i + d] = ((v0 + v1) + v2) / 3.0;
        }
    tb.rec(0, (int32_t)m.nt, 0, -1);
    // boxes of the supports: leaves from their vertices, parents as the union of
    // their sons' boxes (min / max are exact, so this equals a direct scan)
    for (int64_t c = (int64_t)t.nodes.size() - 1; c >= 0; --c) {
        Node &nd = t.nodes[c];
        if (nd.son[0] < 0) {
            tb.box_of(nd.begin, nd.end, nd);
        } else {
            const Node &a = t.nodes[nd.son[0]], &b = t.nodes[nd.son[1]];
            for (int d = 0; d < 3; ++d) {
                nd.lo[d] = std::min(a.lo[d], b.lo[d]);
                nd.hi[d] = std::max(a.hi[d], b.hi[d]);
            }
            double e0 = nd.hi[0] - nd.lo[0], e1 = nd.hi[1] - nd.lo[1], e2 = nd.hi[2] - nd.lo[2];
            nd.diam = std::sqrt((e0 * e0 + e1 * e1) + e2 * e2);
        }
    }
    t.mesh_xyz = m.xyz;
    t.mesh_tri = m.tri;
    return GCA_OK;
}

// -------------------------------------------------------------- block tree --

static double box_dist(const Node &a, const Node &b)
{
    double g[3];
    for (int d = 0; d < 3; ++d) g[d] = std::max(0.0, std::max(b.lo[d] - a.hi[d], a.lo[d] - b.hi[d]));
    return std::sqrt((g[0] * g[0] + g[1] * g[1]) + g[2] * g[2]);
}

void block_tree(const gca_tree_s &t, double eta, Blocks &out)
{
    out = Blocks{};
    // Only the half t <= s is visited: the partition of I x I is symmetric
    // because admissibility is symmetric and both sides use the same tree.
    // (t, s) with t < s stands for itself and its transpose.
    std::vector<std::pair<int32_t, int32_t>> stack;
    stack.emplace_back(0, 0);
    while (!stack.empty()) {
        auto [a, b] = stack.back();
        stack.pop_back();
        const Node &na = t.nodes[a], &nb = t.nodes[b];
        double d = box_dist(na, nb);
        if (d > 0.0 && std::max(na.diam, nb.diam) <= 2.0 * eta * d) {
            out.far_t.push_back(a);
            out.far_s.push_back(b);
            out.n_far_full += (a == b) ? 1 : 2;
            continue;
        }
        bool la = na.son[0] < 0, lb = nb.son[0] < 0;
        if (la && lb) {
            out.near_t.push_back(a);
            out.near_s.push_back(b);
            out.n_near_full += (a == b) ? 1 : 2;
            continue;
        }
        int32_t as[2] = {a, -1}, bs[2] = {b, -1};
        int na_ = 1, nb_ = 1;
        if (!la) { as[0] = na.son[0]; as[1] = na.son[1]; na_ = 2; }
        if (!lb) { bs[0] = nb.son[0]; bs[1] = nb.son[1]; nb_ = 2; }
        for (int i = 0; i < na_; ++i)
            for (int j = 0; j < nb_; ++j) {
                int32_t x = as[i], y = bs[j];
                if (a == b && x > y) continue;   // transposed copy of (y, x), visited once
                stack.emplace_back(std::min(x, y), std::max(x, y));
            }
    }
    // deterministic order: by (t, s)
    auto sort_pairs = [](std::vector<int32_t> &u, std::vector<int32_t> &v) {
        std::vector<std::pair<int32_t, int32_t>> p(u.size());
        for (size_t i = 0; i < u.size(); ++i) p[i] = {u[i], v[i]};
        std::sort(p.begin(), p.end());
        for (size_t i = 0; i < u.size(); ++i) {
            u[i] = p[i].first;
            v[i] = p[i].second;
        }
    };
    sort_pairs(out.far_t, out.far_s);
    sort_pairs(out.near_t, out.near_s);
}

// -------------------------------------------------------------- pair lists --

// Permutation codes: the vertex order (p0, p1, p2) of a triangle as local
// indices, code = index into this table.
static const int kPerm[6][3] = {{0, 1, 2}, {1, 2, 0}, {2, 0, 1}, {0, 2, 1}, {1, 0, 2}, {2, 1, 0}};

static int perm_code(int a, int b, int c)
{
    for (int k = 0; k < 6; ++k)
        if (kPerm[k][0] == a && kPerm[k][1] == b && kPerm[k][2] == c) return k;
    return 0;
}

// Class of the pair (i, j) of ORIGINAL triangle ids, i != j (the identical
// case is i == j): 1 common edge, 2 common vertex, 3 near-regular, 4 regular.
// For touching pairs `code` packs the vertex orders of t_i | t_j << 4 so that
// the shared vertices come first: common edge (a, b, third) with a < b by
// vertex id; common vertex (shared, then cyclic mesh order).
int classify_pair(const Mesh &m, const Adjacency &adj, int32_t i, int32_t j, int32_t *code)
{
    *code = 0;
    if (i == j) return 0;
    const int32_t *ti = &m.tri[3 * (int64_t)i], *tj = &m.tri[3 * (int64_t)j];
    int shared = 0, ka = -1, kb = -1;
    int sa[3], sb[3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            if (ti[a] == tj[b]) {
                sa[shared] = a;
                sb[shared] = b;
                ++shared;
                ka = a;
                kb = b;
            }
    if (shared == 3) return 0;
    if (shared == 2) {
        int lo_a = sa[0], hi_a = sa[1], lo_b = sb[0], hi_b = sb[1];
        if (ti[lo_a] > ti[hi_a]) {
            std::swap(lo_a, hi_a);
            std::swap(lo_b, hi_b);
        }
        int oa = 3 - lo_a - hi_a, ob = 3 - lo_b - hi_b;
        *code = perm_code(lo_a, hi_a, oa) | (perm_code(lo_b, hi_b, ob) << 4);
        return 1;
    }
    if (shared == 1) {
        *code = perm_code(ka, (ka + 1) % 3, (ka + 2) % 3) | (perm_code(kb, (kb + 1) % 3, (kb + 2) % 3) << 4);
        return 2;
    }
    for (int a = 0; a < 3; ++a)
        for (int64_t e = adj.vv_ptr[ti[a]]; e < adj.vv_ptr[ti[a] + 1]; ++e)
            for (int b = 0; b < 3; ++b)
                if (adj.vv[e] == tj[b]) return 3;
    return 4;
}

gca_status build_pair_lists(const Mesh &m, const Adjacency &adj, const gca_tree_s &t, bool with_nearreg,
                            PairLists &pl)
{
    const int64_t nt = m.nt;
    std::vector<int32_t> iperm(nt);
    for (int64_t p = 0; p < nt; ++p) iperm[t.perm[p]] = (int32_t)p;

    // per class: (first original id, second original id, code), first < second.
    // Triangles are processed in contiguous chunks on several threads; the
    // chunks are concatenated in order, so the lists do not depend on the
    // thread count.
    struct P { int32_t i, j, code; };
    const int nthr = (int)std::max<unsigned>(1, std::min<unsigned>(16, std::thread::hardware_concurrency()));
    const int nchunk = (int)std::min<int64_t>(nt, 4 * nthr);
    std::vector<std::array<std::vector<P>, 4>> part(nchunk);
    std::atomic<int> next{0};
    std::atomic<bool> dup{false};
    auto worker = [&]() {
        std::vector<int32_t> cand;
        for (;;) {
            const int c = next.fetch_add(1);
            if (c >= nchunk) break;
            const int64_t i0 = nt * c / nchunk, i1 = nt * (c + 1) / nchunk;
            auto &cls = part[c];
            for (int64_t i = i0; i < i1; ++i) {
                const int32_t *ti = &m.tri[3 * i];
                cls[0].push_back(P{(int32_t)i, (int32_t)i, 0});
                // candidates: triangles around the vertices of t_i and around
                // their edge neighbours (covers touching and near-regular pairs)
                cand.clear();
                for (int k = 0; k < 3; ++k) {
                    for (int64_t q = adj.vt_ptr[ti[k]]; q < adj.vt_ptr[ti[k] + 1]; ++q) cand.push_back(adj.vt[q]);
                    for (int64_t e = adj.vv_ptr[ti[k]]; e < adj.vv_ptr[ti[k] + 1]; ++e) {
                        int32_t v = adj.vv[e];
                        for (int64_t q = adj.vt_ptr[v]; q < adj.vt_ptr[v + 1]; ++q) cand.push_back(adj.vt[q]);
                    }
                }
                std::sort(cand.begin(), cand.end());
                cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
                for (int32_t j : cand) {
                    if (j <= i) continue;
                    int32_t code;
                    int k = classify_pair(m, adj, (int32_t)i, j, &code);
                    if (k == 0) dup = true;
                    if (k >= 1 && k <= 2) cls[k].push_back(P{(int32_t)i, j, code});
                    if (k == 3 && with_nearreg) cls[k].push_back(P{(int32_t)i, j, code});
                }
            }
        }
    };
    {
        std::vector<std::thread> th;
        for (int t = 1; t < nthr; ++t) th.emplace_back(worker);
        worker();
        for (auto &x : th) x.join();
    }
    if (dup) return set_error(GCA_EMESH, "duplicate triangle");
    std::vector<P> cls[4];
    for (int k = 0; k < 4; ++k) {
        size_t tot = 0;
        for (auto &pc : part) tot += pc[k].size();
        cls[k].reserve(tot);
        for (auto &pc : part) cls[k].insert(cls[k].end(), pc[k].begin(), pc[k].end());
    }
    pl.a.clear();
    pl.b.clear();
    pl.code.clear();
    pl.off[0] = 0;
    for (int c = 0; c < 4; ++c) {
        for (const P &p : cls[c]) {
            pl.a.push_back(iperm[p.i]);
            pl.b.push_back(iperm[p.j]);
            pl.code.push_back(p.code);
        }
        pl.off[c + 1] = (int64_t)pl.a.size();
    }
    // row CSR over positions (identical pairs once, others in both rows)
    const int64_t np = (int64_t)pl.a.size();
    pl.row_ptr.assign(nt + 1, 0);
    for (int64_t p = 0; p < np; ++p) {
        pl.row_ptr[pl.a[p] + 1]++;
        if (pl.a[p] != pl.b[p]) pl.row_ptr[pl.b[p] + 1]++;
    }
    for (int64_t i = 0; i < nt; ++i) pl.row_ptr[i + 1] += pl.row_ptr[i];
    pl.row_other.assign(pl.row_ptr[nt], 0);
    pl.row_pair.assign(pl.row_ptr[nt], 0);
    std::vector<int64_t> fill(pl.row_ptr.begin(), pl.row_ptr.end() - 1);
    for (int64_t p = 0; p < np; ++p) {
        int32_t a = pl.a[p], b = pl.b[p];
        pl.row_other[fill[a]] = b;
        pl.row_pair[fill[a]++] = (int32_t)p;
        if (a != b) {
            pl.row_other[fill[b]] = a;
            pl.row_pair[fill[b]++] = (int32_t)p;
        }
    }
    // value CSRs (touching, near-regular): row entries in pair order
    {
        const int64_t nts = pl.off[3];   // touching pairs are classes 0..2
        if (2 * np >= INT32_MAX) return set_error(GCA_EINVAL, "too many pairs for 32-bit slots");
        pl.t_ptr.assign(nt + 1, 0);
        pl.n_ptr.assign(nt + 1, 0);
        for (int64_t p = 0; p < np; ++p) {
            auto &ptr = p < nts ? pl.t_ptr : pl.n_ptr;
            ptr[pl.a[p] + 1]++;
            if (pl.a[p] != pl.b[p]) ptr[pl.b[p] + 1]++;
        }
        for (int64_t i = 0; i < nt; ++i) {
            pl.t_ptr[i + 1] += pl.t_ptr[i];
            pl.n_ptr[i + 1] += pl.n_ptr[i];
        }
        pl.t_other.assign(pl.t_ptr[nt], 0);
        pl.n_other.assign(pl.n_ptr[nt], 0);
        pl.slot_a.assign(np, -1);
        pl.slot_b.assign(np, -1);
        std::vector<int64_t> ft(pl.t_ptr.begin(), pl.t_ptr.end() - 1), fn(pl.n_ptr.begin(), pl.n_ptr.end() - 1);
        for (int64_t p = 0; p < np; ++p) {
            auto &f = p < nts ? ft : fn;
            auto &other = p < nts ? pl.t_other : pl.n_other;
            const int32_t a = pl.a[p], b = pl.b[p];
            pl.slot_a[p] = (int32_t)f[a];
            other[f[a]++] = b;
            if (a != b) {
                pl.slot_b[p] = (int32_t)f[b];
                other[f[b]++] = a;
            }
        }
    }
    // sort each row by the other position (the nearfield kernel builds masks from it)
    for (int64_t i = 0; i < nt; ++i) {
        int64_t b = pl.row_ptr[i], e = pl.row_ptr[i + 1];
        std::vector<std::pair<int32_t, int32_t>> tmp(e - b);
        for (int64_t k = b; k < e; ++k) tmp[k - b] = {pl.row_other[k], pl.row_pair[k]};
        std::sort(tmp.begin(), tmp.end());
        for (int64_t k = b; k < e; ++k) {
            pl.row_other[k] = tmp[k - b].first;
            pl.row_pair[k] = tmp[k - b].second;
        }
    }
    return GCA_OK;
}

// -------------------------------------------------------- Gauss-Legendre --

// Nodes: roots of P_q on [-1, 1] by Newton's method started from
// cos(pi (k - 1/4) / (q + 1/2)); P_q and P_q' by the three-term recurrence.
void gauss_legendre01(int q, double *x, double *w)
{
    const double pi = 3.141592653589793238462643383279502884;
    for (int k = 1; k <= q; ++k) {
        double t = std::cos(pi * (k - 0.25) / (q + 0.5));
        double pq = 0.0, dpq = 1.0;
        for (int it = 0; it < 100; ++it) {
            double pm = 1.0, p = t;
            for (int l = 2; l <= q; ++l) {
                double pn = ((2 * l - 1) * t * p - (l - 1) * pm) / l;
                pm = p;
                p = pn;
            }
            if (q == 1) { p = t; pm = 1.0; }
            pq = p;
            dpq = q * (pm - t * p) / (1.0 - t * t);
            double step = pq / dpq;
            t -= step;
            if (std::fabs(step) < 1e-17) break;
        }
        double pm = 1.0, p = t;
        for (int l = 2; l <= q; ++l) {
            double pn = ((2 * l - 1) * t * p - (l - 1) * pm) / l;
            pm = p;
            p = pn;
        }
        if (q == 1) { p = t; pm = 1.0; }
        dpq = q * (pm - t * p) / (1.0 - t * t);
        // k-th root counted from the largest; store ascending in x = (1 + t)/2
        x[q - k] = 0.5 * (1.0 + t);
        w[q - k] = 1.0 / ((1.0 - t * t) * dpq * dpq);
    }
}

}  // namespace gca
