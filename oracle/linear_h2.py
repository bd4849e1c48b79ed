"""Oracle for GCA-H^2 with the continuous piecewise-linear nodal basis
(Sections 2-5 with the index set of Section 5: one basis function per
vertex), step by step, and the dense matrix it approximates.

TEST INFRASTRUCTURE ONLY, like the rest of this package: the test-suite, the
smoke check and the bench's CPU baseline leg may use it; the product library
never does, and nothing here is shared with it.

* ``lin_dense``: the whole Galerkin matrix of the nodal basis, assembled
  triangle pair by triangle pair (Section 5): the nine moments of every pair
  (t, s) -- the regular rule on both triangles, or the Sauter-Schwab rules
  with the nodal weights when they share a vertex -- added into the entries
  of their corners' vertices.
* ``vertex_cluster_tree``: the binary tree of Section 4 over the vertices;
  the boxes of Section 2 enclose the supports (all triangles of T_i).
* ``lin_green_factor``: the factor A of Section 2 for vertex rows:
  a_{i nu} = sqrt(w_nu) int g(x, z_nu) phi_i(x) dx over the support of phi_i,
  and the normal-derivative columns, with the collapsed rule of order q_A on
  every triangle of T_i and the nodal weights.
* ``gca_lin_h2``: Green points, A, full-pivot ACA and the nested bases exactly
  as for the piecewise-constant basis (the same routines), the coupling
  matrices G|tau~ x sigma~ and the nearfield blocks read from the dense
  matrices of the two rules; ``h2_matvec`` and ``h2_dense`` of the package
  apply to the result.
"""
from __future__ import annotations

import math

import numpy as np

from . import Cluster, ClusterTree, Entries, aca_full, block_tree, green_points
from .linear import basis_weights, vertex_triangles


def lin_dense(verts, tris, q, sym=False, q_s=None):
    """n_v x n_v Galerkin matrix of the nodal basis: for every triangle pair
    (t, s) the moments M_ab = int_t lambda_a int_s g lambda_b are added to the
    entry (vertex of corner a of t, vertex of corner b of s)."""
    verts = np.asarray(verts, dtype=np.float64)
    tris = np.asarray(tris, dtype=np.int64)
    nv, nt = verts.shape[0], tris.shape[0]
    X, W = zip(*[basis_weights(verts[t], q, sym) for t in tris])
    X, W = np.stack(X), np.stack(W)                       # (nt, P, 3) each
    ent = Entries(verts, tris, q, q, q_s, sym=sym) if q_s is not None else None
    G = np.zeros((nv, nv))
    for t in range(nt):
        d = X[t][None, :, None, :] - X[:, None, :, :]     # (nt, P, P, 3)
        with np.errstate(divide="ignore"):
            g = 1.0 / np.sqrt((d * d).sum(axis=3))
        M = np.einsum("pa,spq,sqb->sab", W[t], g, W) / (4.0 * math.pi)
        touch = np.nonzero(np.isin(tris, tris[t]).any(axis=1))[0]
        for s in touch:
            if ent is None:
                raise ValueError("triangles %d and %d share a vertex: q_s is needed" % (t, s))
            M[s] = ent.lin_touch_moments(t, int(s))
        for a in range(3):
            for b in range(3):
                np.add.at(G, (np.full(nt, tris[t, a]), tris[:, b]), M[:, a, b])
    return G


def vertex_cluster_tree(verts, tris, leaf):
    """Binary cluster tree over the vertices (Section 4 splits a cluster into
    two disjoint sons).  Splitting rule as for the triangles, with the vertex
    positions as the points: the bounding box of the cluster's vertices is cut
    along its longest axis (lowest axis on ties), the vertices are sorted by
    that coordinate (ties by vertex id) and the first floor(#/2) form the
    first son; at most `leaf` vertices make a leaf.  The box of a cluster
    (Section 2) encloses the supports: every vertex of every triangle in T_i
    for the cluster's vertices i; diam is its diagonal.  Pre-order numbering."""
    verts = np.asarray(verts, dtype=np.float64)
    tris = np.asarray(tris, dtype=np.int64)
    n = verts.shape[0]
    T = vertex_triangles(tris, n)
    sup_lo = np.array([verts[tris[T[i]].ravel()].min(axis=0) for i in range(n)])
    sup_hi = np.array([verts[tris[T[i]].ravel()].max(axis=0) for i in range(n)])
    perm = np.arange(n, dtype=np.int64)
    nodes = []

    def rec(b, e, level):
        me = len(nodes)
        nodes.append(Cluster(b, e, level))
        idx = perm[b:e]
        nodes[me].lo = sup_lo[idx].min(axis=0)
        nodes[me].hi = sup_hi[idx].max(axis=0)
        ext = nodes[me].hi - nodes[me].lo
        nodes[me].diam = math.sqrt((ext[0] * ext[0] + ext[1] * ext[1]) + ext[2] * ext[2])
        if e - b <= leaf:
            return me
        c = verts[idx]
        cext = c.max(axis=0) - c.min(axis=0)
        axis = int(np.argmax(cext))
        order = np.lexsort((idx, c[:, axis]))
        perm[b:e] = idx[order]
        mid = b + (e - b) // 2
        s1 = rec(b, mid, level + 1)
        s2 = rec(mid, e, level + 1)
        nodes[me].sons = [s1, s2]
        return me

    rec(0, n, 0)
    return ClusterTree(perm, nodes)


def lin_green_factor(rows, verts, tris, T, q_A, z, wz, nz, diam):
    """A in R^{rows x 2k} (Section 2) for vertex rows:
        a_{i nu}     =  sqrt(w_nu) int g(x, z_nu) phi_i(x) dx
        a_{i, nu+k}  = -d_tau sqrt(w_nu) int dg/dn_z(x, z_nu) phi_i(x) dx,
    each integral the sum over t in T_i of the collapsed rule of order q_A
    with the weight w_p |J| lambda_{t,i}(x_p)."""
    k = z.shape[0]
    A = np.zeros((len(rows), 2 * k))
    sw = np.sqrt(wz)
    for r, i in enumerate(rows):
        pts, wts = [], []
        for t in T[int(i)]:
            x, W = basis_weights(verts[tris[t]], q_A)
            a = list(tris[t]).index(int(i))
            pts.append(x)
            wts.append(W[:, a])
        P, Wt = np.concatenate(pts), np.concatenate(wts)
        d = P[:, None, :] - z[None, :, :]
        rr = np.sqrt((d * d).sum(axis=2))
        g = 1.0 / (4.0 * math.pi * rr)
        dg = np.einsum("pkd,kd->pk", d, nz) / (4.0 * math.pi * rr ** 3)
        A[r, :k] = sw * (Wt @ g)
        A[r, k:] = -diam * sw * (Wt @ dg)
    return A


class LinH2:
    """The approximation: tree, blocks, pivots (vertex ids, pivot order),
    leaf bases V, transfers E; coupling matrices from the dense matrix of the
    coupling rule, nearfield blocks from that of the nearfield rules."""

    def __init__(self, tree, far, near, pivots, V, E, Gnear, Gcoup):
        self.tree, self.far, self.near = tree, far, near
        self.pivots, self.V, self.E = pivots, V, E
        self.Gnear, self.Gcoup = Gnear, Gcoup
        self.ent = None   # the entries come from the dense matrices

    def coupling(self, t, s):
        return self.Gcoup[np.ix_(self.pivots[t], self.pivots[s])]

    def nearblock(self, t, s):
        return self.Gnear[np.ix_(self.tree.indices(t), self.tree.indices(s))]


def gca_lin_h2(verts, tris, leaf=16, eta=2.0, m=3, eps=1e-6, q_A=3, q=3, q_s=4, q_c=None, sym=False,
               omega_scale=0.25, Gnear=None, Gcoup=None):
    """Build the GCA-H^2 approximation of the nodal-basis matrix step by step:
    the vertex tree, the block tree (Section 2 admissibility on the support
    boxes), Green points and A per cluster from the leaves up (a parent's
    rows are its sons' pivots), full-pivot ACA and the nested bases (Sections
    3-4).  q: regular rule of the nearfield pairs (q_s for the touching ones),
    q_c: that of the coupling entries (default q).  Gnear / Gcoup: the dense
    matrices of those rules if already assembled."""
    verts = np.asarray(verts, dtype=np.float64)
    tris = np.asarray(tris, dtype=np.int64)
    tree = vertex_cluster_tree(verts, tris, leaf)
    far, near = block_tree(tree, eta)
    T = vertex_triangles(tris, verts.shape[0])
    pivots, V, E = {}, {}, {}
    for c in reversed(range(len(tree.nodes))):
        nd = tree.nodes[c]
        z, wz, nz = green_points(nd, m, eta, omega_scale)
        rows = tree.indices(c) if not nd.sons else np.concatenate([pivots[s] for s in nd.sons])
        A = lin_green_factor(rows, verts, tris, T, q_A, z, wz, nz, nd.diam)
        I, _, Vh = aca_full(A, eps)
        pivots[c] = rows[I]
        if not nd.sons:
            V[c] = Vh
        else:
            o = 0
            for s in nd.sons:
                r = len(pivots[s])
                E[s] = Vh[o:o + r, :]
                o += r
    qc = q if q_c is None else q_c
    if Gnear is None:
        Gnear = lin_dense(verts, tris, q, sym, q_s)
    if Gcoup is None:
        Gcoup = Gnear if qc == q else lin_dense(verts, tris, qc, sym, q_s)
    return LinH2(tree, far, near, pivots, V, E, Gnear, Gcoup)
