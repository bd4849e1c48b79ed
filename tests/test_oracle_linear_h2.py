"""Pins of the GCA-H^2 oracle for the piecewise-linear nodal basis
(oracle/linear_h2.py; Sections 2-5 with one basis function per vertex).  CPU
only.

* The dense nodal matrix (triangle pair by pair) equals the entry-wise
  definition of oracle.linear.lin_block, pinned on its own, on sampled
  blocks; it is symmetric to the touching rules' asymmetry and positive
  definite.
* The vertex tree: a permutation, sons partition their parent, leaf sizes,
  boxes that contain every triangle of every support; the block tree tiles
  V x V once and no admissible block has a triangle pair with a common vertex.
* The Green factor with the nodal weights: G|tau x sigma ~ A B^T with B
  written out in this test (Section 2), the error decaying with the Green
  order.
* eta -> 0 reproduces the dense matrix exactly; the spectral error of the
  approximation follows eps; the nested bases interpolate (identity on the
  pivots).
"""
import math

import numpy as np
import pytest

import synth
from oracle import linear as L
from oracle import linear_h2 as LH


@pytest.fixture(scope="module")
def l2():
    m = synth.jitter(synth.icosphere(2), 0.005, seed=4)
    return m, LH.lin_dense(m.verts, m.tris, 3, False, 5)


def test_dense_equals_entrywise_definition(l2):
    m, G = l2
    T = L.vertex_triangles(m.tris, m.nv)
    rng = np.random.default_rng(0)
    for _ in range(3):
        rows = rng.choice(m.nv, 6, replace=False)
        cols = np.concatenate([rows[:2], rng.choice(m.nv, 5, replace=False)])
        B = L.lin_block(m.verts, m.tris, rows, cols, 3, False, T=T, q_s=5)
        assert np.abs(G[np.ix_(rows, cols)] - B).max() < 1e-13 * np.abs(B).max()
    assert np.abs(G - G.T).max() < 1e-7 * np.abs(G).max()
    assert np.linalg.eigvalsh(0.5 * (G + G.T)).min() > 0


def test_vertex_tree_and_blocks():
    m = synth.icosphere(3)
    tree = LH.vertex_cluster_tree(m.verts, m.tris, 16)
    assert sorted(tree.perm) == list(range(m.nv))
    T = L.vertex_triangles(m.tris, m.nv)
    for c, nd in enumerate(tree.nodes):
        if nd.sons:
            a, b = (tree.nodes[s] for s in nd.sons)
            assert (a.begin, a.end, b.begin, b.end) == (nd.begin, a.end, a.end, nd.end)
        else:
            assert nd.end - nd.begin <= 16
        sup = m.verts[m.tris[np.concatenate([T[i] for i in tree.indices(c)])].ravel()]
        assert (sup >= nd.lo - 1e-15).all() and (sup <= nd.hi + 1e-15).all()
        assert np.isclose(nd.diam, np.linalg.norm(nd.hi - nd.lo))
    import oracle
    far, near = oracle.block_tree(tree, 2.0)
    cover = np.zeros((m.nv, m.nv), dtype=np.int32)
    for (t, s) in far + near:
        cover[np.ix_(tree.indices(t), tree.indices(s))] += 1
    assert (cover == 1).all()
    for (t, s) in far:
        tt = set(np.concatenate([T[i] for i in tree.indices(t)]))
        ss = set(np.concatenate([T[i] for i in tree.indices(s)]))
        vt = set(m.tris[list(tt)].ravel())
        vs = set(m.tris[list(ss)].ravel())
        assert not (vt & vs), (t, s)


def test_green_factor_factorises_an_admissible_block():
    """G|tau x sigma ~ A B^T (Section 2) with
        b_{j nu} = sqrt(w) int dg/dn_z(z_nu, y) phi_j(y) dy,
        b_{j nu+k} = sqrt(w) / d_tau int g(z_nu, y) phi_j(y) dy,
    the nodal integrals by a rule of this test (the collapsed rule of order 6
    on every triangle of the support)."""
    import oracle
    m = synth.icosphere(3)
    tree = LH.vertex_cluster_tree(m.verts, m.tris, 16)
    far, _ = oracle.block_tree(tree, 2.0)
    t, s = next((t, s) for (t, s) in far if not tree.nodes[t].sons and not tree.nodes[s].sons)
    rows, cols = tree.indices(t), tree.indices(s)
    T = L.vertex_triangles(m.tris, m.nv)
    Gts = L.lin_block(m.verts, m.tris, rows, cols, 6, T=T)
    # the nodal integrals of the columns: points and weights per column vertex
    colp = []
    for j in cols:
        xs, ws = [], []
        for tri in T[int(j)]:
            P = m.verts[m.tris[tri]]
            x, w = np.polynomial.legendre.leggauss(6)
            x, w = (x + 1) / 2, w / 2
            u, v = np.meshgrid(x, x, indexing="ij")
            wu, wv = np.meshgrid(w, w, indexing="ij")
            c = list(m.tris[tri]).index(int(j))
            # Duffy map at corner c: the nodal function of c is 1 - u
            A0, B0, C0 = P[c], P[(c + 1) % 3], P[(c + 2) % 3]
            pts = A0 + u[..., None] * ((B0 - A0) + v[..., None] * (C0 - B0))
            area2 = np.linalg.norm(np.cross(B0 - A0, C0 - A0))
            xs.append(pts.reshape(-1, 3))
            ws.append((wu * wv * u * area2 * (1 - u)).reshape(-1))
        colp.append((np.concatenate(xs), np.concatenate(ws)))
    errs = []
    for mq in (2, 4, 6, 10):
        nd = tree.nodes[t]
        z, w, nrm = oracle.green_points(nd, mq, 2.0, omega_scale=0.25)
        A = LH.lin_green_factor(rows, m.verts, m.tris, T, 6, z, w, nrm, nd.diam)
        sw = np.sqrt(w)
        B = np.zeros((len(cols), 2 * len(w)))
        for jj, (P, W) in enumerate(colp):
            d = P[:, None, :] - z[None, :, :]
            r = np.linalg.norm(d, axis=-1)
            g = 1 / (4 * math.pi * r)
            dg = np.einsum("pkd,kd->pk", d, nrm) / (4 * math.pi * r ** 3)
            B[jj] = np.concatenate([sw * (W @ dg), sw / nd.diam * (W @ g)])
        errs.append(np.linalg.norm(Gts - A @ B.T) / np.linalg.norm(Gts))
    assert errs[-1] < 1e-3 * errs[0], errs
    assert errs[-1] < 1e-4, errs


def test_eta_zero_spectral_error_and_interpolation():
    import oracle
    m = synth.jitter(synth.icosphere(3), 0.002, seed=4)
    G = LH.lin_dense(m.verts, m.tris, 3, False, 5)
    h0 = LH.gca_lin_h2(m.verts, m.tris, leaf=16, eta=1e-9, eps=1e-2, Gnear=G)
    assert not h0.far and np.array_equal(oracle.h2_dense(h0), G)
    errs = []
    for eps in (1e-2, 1e-4):
        h = LH.gca_lin_h2(m.verts, m.tris, leaf=16, eta=2.0, m=3, eps=eps, q=3, q_s=5, Gnear=G)
        assert h.far
        Gt = oracle.h2_dense(h)
        errs.append(np.linalg.norm(Gt - G, 2) / np.linalg.norm(G, 2))
        assert errs[-1] < 10 * eps, (eps, errs)
        x = np.random.default_rng(1).standard_normal(m.nv)
        assert np.abs(oracle.h2_matvec(h, x) - Gt @ x).max() < 1e-12 * np.abs(Gt @ x).max()
        for c, V in h.V.items():
            rows = list(h.tree.indices(c))
            loc = [rows.index(p) for p in h.pivots[c]]
            assert np.array_equal(V[loc], np.eye(len(loc)))
    assert errs[1] < errs[0] / 100
