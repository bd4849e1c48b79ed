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

gca_status mesh_copy_validate(const gca_mesh *m, Mesh &out, bool topology)
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
    std::atomic<bool> bad_xyz{false};
    parallel_for(3 * m->nv, [&](int64_t i0, int64_t i1) {
        for (int64_t i = i0; i < i1; ++i)
            if (!std::isfinite(out.xyz[i])) bad_xyz = true;
    });
    if (bad_xyz) return set_error(GCA_EINVAL, "non-finite vertex coordinate");
    // first failing triangle (lowest index) and its reason
    std::atomic<int64_t> first_bad{INT64_MAX};
    std::vector<int8_t> why((size_t)m->nt, 0);
    parallel_for(m->nt, [&](int64_t t0, int64_t t1) {
        for (int64_t t = t0; t < t1; ++t) {
            const int32_t *v = &out.tri[3 * t];
            int8_t r = 0;
            for (int k = 0; k < 3; ++k)
                if (v[k] < 0 || v[k] >= m->nv) r = 1;
            if (!r && (v[0] == v[1] || v[1] == v[2] || v[0] == v[2])) r = 2;
            if (!r) {
                const double *a = &out.xyz[3 * v[0]], *b = &out.xyz[3 * v[1]], *c = &out.xyz[3 * v[2]];
                double e1[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
                double e2[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
                double cx = e1[1] * e2[2] - e1[2] * e2[1];
                double cy = e1[2] * e2[0] - e1[0] * e2[2];
                double cz = e1[0] * e2[1] - e1[1] * e2[0];
                if (!(cx * cx + cy * cy + cz * cz > 0.0)) r = 3;
            }
            if (r) {
                why[t] = r;
                int64_t cur = first_bad.load();
                while (t < cur && !first_bad.compare_exchange_weak(cur, t)) {
                }
            }
        }
    });
    if (first_bad.load() != INT64_MAX) {
        const int64_t t = first_bad.load();
        const char *msg[4] = {"", ": vertex index out of range", ": repeated vertex", ": zero area"};
        return set_error(GCA_EMESH, "triangle " + std::to_string(t) + msg[why[t]]);
    }
    if (!topology) return GCA_OK;
    // duplicate triangles and non-manifold edges, through the triangles
    // around each vertex
    std::vector<int64_t> ptr(m->nv + 1, 0);
    for (int64_t i = 0; i < 3 * m->nt; ++i) ptr[out.tri[i] + 1]++;
    for (int64_t v = 0; v < m->nv; ++v) ptr[v + 1] += ptr[v];
    std::vector<int32_t> vt(ptr[m->nv]);
    {
        std::vector<int64_t> fill(ptr.begin(), ptr.end() - 1);
        for (int64_t t = 0; t < m->nt; ++t)
            for (int k = 0; k < 3; ++k) vt[fill[out.tri[3 * t + k]]++] = (int32_t)t;
    }
    std::atomic<bool> dup{false}, nonman{false};
    parallel_for(m->nt, [&](int64_t t0, int64_t t1) {
        for (int64_t t = t0; t < t1; ++t) {
            const int32_t *v = &out.tri[3 * t];
            std::array<int32_t, 3> key = {v[0], v[1], v[2]};
            std::sort(key.begin(), key.end());
            for (int k = 0; k < 3; ++k) {
                const int32_t a = v[k], b = v[(k + 1) % 3];
                int cnt = 0;
                for (int64_t q = ptr[a]; q < ptr[a + 1]; ++q) {
                    const int32_t *w = &out.tri[3 * (int64_t)vt[q]];
                    if (w[0] == b || w[1] == b || w[2] == b) ++cnt;
                    if (k == 0 && vt[q] != t) {
                        std::array<int32_t, 3> k2 = {w[0], w[1], w[2]};
                        std::sort(k2.begin(), k2.end());
                        if (k2 == key) dup = true;
                    }
                }
                if (cnt > 2) nonman = true;
            }
        }
    });
    if (dup) return set_error(GCA_EMESH, "duplicate triangle");
    if (nonman) return set_error(GCA_EMESH, "non-manifold edge (more than two triangles)");
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
    // vertex neighbours through edges: the other vertices of the triangles
    // around v, sorted and unique (parallel over vertices)
    std::vector<int32_t> cnt(nv, 0);
    std::vector<int32_t> tmp(2 * adj.vt_ptr[nv]);
    parallel_for(nv, [&](int64_t v0, int64_t v1) {
        for (int64_t v = v0; v < v1; ++v) {
            int32_t *l = tmp.data() + 2 * adj.vt_ptr[v];
            int n = 0;
            for (int64_t q = adj.vt_ptr[v]; q < adj.vt_ptr[v + 1]; ++q) {
                const int32_t *w = &m.tri[3 * (int64_t)adj.vt[q]];
                for (int k = 0; k < 3; ++k)
                    if (w[k] != v) l[n++] = w[k];
            }
            std::sort(l, l + n);
            cnt[v] = (int32_t)(std::unique(l, l + n) - l);
        }
    });
    adj.vv_ptr.assign(nv + 1, 0);
    for (int64_t v = 0; v < nv; ++v) adj.vv_ptr[v + 1] = adj.vv_ptr[v] + cnt[v];
    adj.vv.resize(adj.vv_ptr[nv]);
    parallel_for(nv, [&](int64_t v0, int64_t v1) {
        for (int64_t v = v0; v < v1; ++v)
            std::copy(tmp.begin() + 2 * adj.vt_ptr[v], tmp.begin() + 2 * adj.vt_ptr[v] + cnt[v],
                      adj.vv.begin() + adj.vv_ptr[v]);
    });
    return GCA_OK;
}

// ------------------------------------------------------------ cluster tree --

namespace {

// Items (triangles, or the vertices of the nodal basis) with a point each
// (cent, the splitting coordinate) and the box of their support (sup: lo,
// hi per item).
struct TreeBuilder {
    int32_t leaf;
    gca_tree_s &t;
    const std::vector<double> &cent;   // n x 3
    const std::vector<double> &sup;    // n x 6

    void box_of(int32_t b, int32_t e, Node &nd)
    {
        for (int d = 0; d < 3; ++d) {
            nd.lo[d] = INFINITY;
            nd.hi[d] = -INFINITY;
        }
        for (int32_t p = b; p < e; ++p) {
            const double *bx = &sup[6 * (int64_t)t.perm[p]];
            for (int d = 0; d < 3; ++d) {
                nd.lo[d] = std::min(nd.lo[d], bx[d]);
                nd.hi[d] = std::max(nd.hi[d], bx[3 + d]);
            }
        }
        double e0 = nd.hi[0] - nd.lo[0], e1 = nd.hi[1] - nd.lo[1], e2 = nd.hi[2] - nd.lo[2];
        nd.diam = std::sqrt((e0 * e0 + e1 * e1) + e2 * e2);
    }

    // Splits [b, e) and appends the subtree in pre-order to `out` (indices
    // local to `out`); the top `par` levels build their two sons on two
    // threads and append them afterwards, which gives the same numbering.
    int32_t rec(int32_t b, int32_t e, int32_t level, int32_t parent, int par, std::vector<Node> &out)
    {
        int32_t me = (int32_t)out.size();
        out.push_back(Node{});
        {
            Node &nd = out[me];
            nd.begin = b;
            nd.end = e;
            nd.son[0] = nd.son[1] = -1;
            nd.parent = parent;
            nd.level = level;
        }
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
        int32_t s0, s1;
        if (par > 0) {
            std::vector<Node> left, right;
            std::thread th([&]() { rec(b, mid, level + 1, -1, par - 1, left); });
            rec(mid, e, level + 1, -1, par - 1, right);
            th.join();
            s0 = append(out, left, me);
            s1 = append(out, right, me);
        } else {
            s0 = rec(b, mid, level + 1, me, 0, out);
            s1 = rec(mid, e, level + 1, me, 0, out);
        }
        out[me].son[0] = s0;
        out[me].son[1] = s1;
        return me;
    }

    // appends a subtree built with local indices; returns its root's index
    static int32_t append(std::vector<Node> &out, const std::vector<Node> &sub, int32_t parent)
    {
        const int32_t base = (int32_t)out.size();
        for (const Node &n0 : sub) {
            Node n = n0;
            n.parent = n.parent < 0 ? parent : n.parent + base;
            if (n.son[0] >= 0) n.son[0] += base;
            if (n.son[1] >= 0) n.son[1] += base;
            out.push_back(n);
        }
        return base;
    }
};

}  // namespace

// The tree over n items: median splits of the points, boxes of the supports
// (leaves from their items' boxes, parents as the union of their sons' boxes;
// min / max are exact, so this equals a direct scan).
static void build_items(const std::vector<double> &cent, const std::vector<double> &sup, int64_t n, int32_t leaf,
                        gca_tree_s &t)
{
    t.perm.resize(n);
    std::iota(t.perm.begin(), t.perm.end(), 0);
    t.nodes.clear();
    t.nodes.reserve(4 * (n / std::max(1, leaf / 2) + 1));
    t.depth = 0;
    TreeBuilder tb{leaf, t, cent, sup};
    int par = 0;
    while (par < 4 && (1 << (par + 1)) <= host_threads() && (n >> par) > 8 * (int64_t)leaf) ++par;
    tb.rec(0, (int32_t)n, 0, -1, par, t.nodes);
    for (const Node &nd : t.nodes) t.depth = std::max(t.depth, nd.level);
    parallel_for((int64_t)t.nodes.size(), [&](int64_t c0, int64_t c1) {
        for (int64_t c = c0; c < c1; ++c)
            if (t.nodes[c].son[0] < 0) tb.box_of(t.nodes[c].begin, t.nodes[c].end, t.nodes[c]);
    });
    for (int64_t c = (int64_t)t.nodes.size() - 1; c >= 0; --c) {
        Node &nd = t.nodes[c];
        if (nd.son[0] < 0) continue;
        const Node &a = t.nodes[nd.son[0]], &b = t.nodes[nd.son[1]];
        for (int d = 0; d < 3; ++d) {
            nd.lo[d] = std::min(a.lo[d], b.lo[d]);
            nd.hi[d] = std::max(a.hi[d], b.hi[d]);
        }
        double e0 = nd.hi[0] - nd.lo[0], e1 = nd.hi[1] - nd.lo[1], e2 = nd.hi[2] - nd.lo[2];
        nd.diam = std::sqrt((e0 * e0 + e1 * e1) + e2 * e2);
    }
}

gca_status tree_build(const Mesh &m, int32_t leaf, gca_tree_s &t)
{
    if (leaf < 1) return set_error(GCA_EINVAL, "leaf_size must be >= 1");
    t.nt = m.nt;
    t.nv = m.nv;
    t.leaf = leaf;
    // triangle centroids ((v0 + v1) + v2) / 3 and the boxes of the triangles
    std::vector<double> cent(3 * m.nt), sup(6 * m.nt);
    parallel_for(m.nt, [&](int64_t i0, int64_t i1) {
        for (int64_t i = i0; i < i1; ++i)
            for (int d = 0; d < 3; ++d) {
                double v0 = m.xyz[3 * (int64_t)m.tri[3 * i] + d];
                double v1 = m.xyz[3 * (int64_t)m.tri[3 * i + 1] + d];
                double v2 = m.xyz[3 * (int64_t)m.tri[3 * i + 2] + d];
                cent[3 * i + d] = ((v0 + v1) + v2) / 3.0;
                sup[6 * i + d] = std::min(v0, std::min(v1, v2));
                sup[6 * i + 3 + d] = std::max(v0, std::max(v1, v2));
            }
    });
    build_items(cent, sup, m.nt, leaf, t);
    t.mesh_xyz = m.xyz;
    t.mesh_tri = m.tri;
    return GCA_OK;
}

gca_status tree_build_vertices(const Mesh &m, const std::vector<int64_t> &vt_ptr, const std::vector<int32_t> &vt,
                               int32_t leaf, gca_tree_s &t)
{
    if (leaf < 1) return set_error(GCA_EINVAL, "leaf_size must be >= 1");
    t.nt = m.nt;
    t.nv = m.nv;
    t.leaf = leaf;
    // the vertex itself, and the box of every triangle of its support
    std::vector<double> sup(6 * m.nv);
    parallel_for(m.nv, [&](int64_t v0, int64_t v1) {
        for (int64_t v = v0; v < v1; ++v) {
            double *bx = &sup[6 * v];
            for (int d = 0; d < 3; ++d) {
                bx[d] = INFINITY;
                bx[3 + d] = -INFINITY;
            }
            for (int64_t q = vt_ptr[v]; q < vt_ptr[v + 1]; ++q)
                for (int k = 0; k < 3; ++k) {
                    const double *x = &m.xyz[3 * (int64_t)m.tri[3 * (int64_t)vt[q] + k]];
                    for (int d = 0; d < 3; ++d) {
                        bx[d] = std::min(bx[d], x[d]);
                        bx[3 + d] = std::max(bx[3 + d], x[d]);
                    }
                }
        }
    });
    build_items(m.xyz, sup, m.nv, leaf, t);
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
                            PairLists &pl, const std::function<bool(int32_t, int32_t)> &near_ok)
{
    const int64_t nt = m.nt;
    std::vector<int32_t> iperm(nt);
    parallel_for(nt, [&](int64_t p0, int64_t p1) {
        for (int64_t p = p0; p < p1; ++p) iperm[t.perm[p]] = (int32_t)p;
    });

    // Rows in position order, built in contiguous chunks of positions on
    // several threads.  The row of position r (triangle i = perm[r]) lists
    // every listed partner (touching, and near-regular if with_nearreg) by
    // its position, ascending.  A pair belongs to the row of its smaller
    // position; its class and order code are those of (lower original id,
    // higher original id).  Pair ids: class by class, and within a class in
    // the order of the owning rows, so nothing depends on the thread count.
    struct E {
        int32_t other;   // position of the partner
        int32_t cc;      // owned: class << 8 | code; else -1
    };
    const int nthr = host_threads();
    const int64_t nchunk = std::min<int64_t>(nt, 8 * nthr);
    std::vector<std::vector<E>> ent(nchunk);
    std::vector<std::array<int64_t, 4>> ccount(nchunk);
    std::vector<int32_t> rowlen(nt);
    std::atomic<bool> dup{false};
    parallel_for(nchunk, [&](int64_t c0, int64_t c1) {
        std::vector<int32_t> cand;
        std::vector<E> row;
        for (int64_t c = c0; c < c1; ++c) {
            const int64_t r0 = nt * c / nchunk, r1 = nt * (c + 1) / nchunk;
            auto &out = ent[c];
            auto &cnt = ccount[c];
            cnt = {0, 0, 0, 0};
            for (int64_t r = r0; r < r1; ++r) {
                const int32_t i = t.perm[r];
                const int32_t *ti = &m.tri[3 * (int64_t)i];
                // candidates: triangles around the vertices of t_i (touching
                // pairs) and, when near-regular pairs are listed, around their
                // edge neighbours too
                cand.clear();
                for (int k = 0; k < 3; ++k) {
                    for (int64_t q = adj.vt_ptr[ti[k]]; q < adj.vt_ptr[ti[k] + 1]; ++q) cand.push_back(adj.vt[q]);
                    if (!with_nearreg) continue;
                    for (int64_t e = adj.vv_ptr[ti[k]]; e < adj.vv_ptr[ti[k] + 1]; ++e) {
                        int32_t v = adj.vv[e];
                        for (int64_t q = adj.vt_ptr[v]; q < adj.vt_ptr[v + 1]; ++q) cand.push_back(adj.vt[q]);
                    }
                }
                std::sort(cand.begin(), cand.end());
                cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
                row.clear();
                for (int32_t j : cand) {
                    const int32_t pj = iperm[j];
                    int kls, code = 0;
                    if (j == i) {
                        kls = 0;
                    } else {
                        kls = classify_pair(m, adj, std::min(i, j), std::max(i, j), &code);
                        if (kls == 0) {
                            dup = true;
                            continue;
                        }
                        if (kls > 3 || (kls == 3 && !with_nearreg)) continue;
                        if (kls == 3 && near_ok && !near_ok((int32_t)r, pj)) continue;
                    }
                    const bool own = pj >= r;
                    row.push_back(E{pj, own ? (kls << 8 | code) : -1});
                    if (own) cnt[kls]++;
                }
                std::sort(row.begin(), row.end(), [](const E &x, const E &y) { return x.other < y.other; });
                out.insert(out.end(), row.begin(), row.end());
                rowlen[r] = (int32_t)row.size();
            }
        }
    }, 1);
    if (dup) return set_error(GCA_EMESH, "duplicate triangle");
    pl.row_ptr.assign(nt + 1, 0);
    for (int64_t r = 0; r < nt; ++r) pl.row_ptr[r + 1] = pl.row_ptr[r] + rowlen[r];
    // pair ids: class offsets, then per chunk
    pl.off[0] = 0;
    for (int k = 0; k < 4; ++k) {
        int64_t tot = 0;
        for (int64_t c = 0; c < nchunk; ++c) tot += ccount[c][k];
        pl.off[k + 1] = pl.off[k] + tot;
    }
    const int64_t np = pl.off[4];
    if (2 * np >= INT32_MAX) return set_error(GCA_EINVAL, "too many pairs for 32-bit slots");
    std::vector<std::array<int64_t, 4>> cbase(nchunk);
    {
        std::array<int64_t, 4> run = {pl.off[0], pl.off[1], pl.off[2], pl.off[3]};
        for (int64_t c = 0; c < nchunk; ++c)
            for (int k = 0; k < 4; ++k) {
                cbase[c][k] = run[k];
                run[k] += ccount[c][k];
            }
    }
    pl.a.assign(np, 0);
    pl.b.assign(np, 0);
    pl.code.assign(np, 0);
    pl.row_other.assign(pl.row_ptr[nt], 0);
    pl.row_pair.assign(pl.row_ptr[nt], -1);
    parallel_for(nchunk, [&](int64_t c0, int64_t c1) {
        for (int64_t c = c0; c < c1; ++c) {
            const int64_t r0 = nt * c / nchunk, r1 = nt * (c + 1) / nchunk;
            std::array<int64_t, 4> id = cbase[c];
            int64_t k = pl.row_ptr[r0];
            const E *e = ent[c].data();
            for (int64_t r = r0; r < r1; ++r)
                for (int64_t q = pl.row_ptr[r]; q < pl.row_ptr[r + 1]; ++q, ++k, ++e) {
                    pl.row_other[q] = e->other;
                    if (e->cc < 0) continue;
                    const int kls = e->cc >> 8;
                    const int64_t p = id[kls]++;
                    const int32_t i = t.perm[r], j = t.perm[e->other];
                    pl.a[p] = i < j ? (int32_t)r : e->other;
                    pl.b[p] = i < j ? e->other : (int32_t)r;
                    pl.code[p] = e->cc & 0xff;
                    pl.row_pair[q] = (int32_t)p;
                }
            std::vector<E>().swap(ent[c]);
        }
    }, 1);
    // entries owned by the other row: find this row in the partner's row
    parallel_for(nt, [&](int64_t r0, int64_t r1) {
        for (int64_t r = r0; r < r1; ++r)
            for (int64_t q = pl.row_ptr[r]; q < pl.row_ptr[r + 1]; ++q) {
                if (pl.row_pair[q] >= 0) continue;
                const int32_t o = pl.row_other[q];
                const int32_t *b0 = pl.row_other.data() + pl.row_ptr[o], *b1 = pl.row_other.data() + pl.row_ptr[o + 1];
                const int32_t *f = std::lower_bound(b0, b1, (int32_t)r);
                pl.row_pair[q] = pl.row_pair[pl.row_ptr[o] + (f - b0)];
            }
    });
    // value CSRs used by the product: the row CSR split into touching pairs
    // (classes 0-2) and near-regular pairs (class 3), same order; slot_a[p] /
    // slot_b[p] is the entry of pair p in the row of its first / second
    // triangle
    {
        const int64_t nts = pl.off[3];
        pl.t_ptr.assign(nt + 1, 0);
        pl.n_ptr.assign(nt + 1, 0);
        parallel_for(nt, [&](int64_t i0, int64_t i1) {
            for (int64_t i = i0; i < i1; ++i) {
                int64_t ct = 0;
                for (int64_t k = pl.row_ptr[i]; k < pl.row_ptr[i + 1]; ++k) ct += pl.row_pair[k] < nts;
                pl.t_ptr[i + 1] = ct;
                pl.n_ptr[i + 1] = (pl.row_ptr[i + 1] - pl.row_ptr[i]) - ct;
            }
        });
        for (int64_t i = 0; i < nt; ++i) {
            pl.t_ptr[i + 1] += pl.t_ptr[i];
            pl.n_ptr[i + 1] += pl.n_ptr[i];
        }
        pl.t_other.assign(pl.t_ptr[nt], 0);
        pl.n_other.assign(pl.n_ptr[nt], 0);
        pl.slot_a.assign(np, -1);
        pl.slot_b.assign(np, -1);
        parallel_for(nt, [&](int64_t i0, int64_t i1) {
            for (int64_t i = i0; i < i1; ++i) {
                int64_t ft = pl.t_ptr[i], fn = pl.n_ptr[i];
                for (int64_t k = pl.row_ptr[i]; k < pl.row_ptr[i + 1]; ++k) {
                    const int32_t p = pl.row_pair[k];
                    const bool touch = p < nts;
                    const int64_t q = touch ? ft++ : fn++;
                    (touch ? pl.t_other : pl.n_other)[q] = pl.row_other[k];
                    if (pl.a[p] == i)
                        pl.slot_a[p] = (int32_t)q;
                    else
                        pl.slot_b[p] = (int32_t)q;
                }
            }
        });
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
