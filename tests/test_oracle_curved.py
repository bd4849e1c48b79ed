"""Pins of the curved-triangle oracle (Section 6: quadratic parametrisations
from the vertices and edge midpoints, Gramians, mapped nodal basis functions,
Sauter's rules on the reference coordinates; the double layer with the unit
normal n / gamma).  CPU only.

* Straight edge points reduce the quadratic map to the flat one: every class
  of the single- and double-layer entries and the nodal moments equal the
  flat oracle's (pinned on their own) to rounding.
* A surface the quadratic map reproduces exactly -- triangles on the graph
  of a quadratic z = f(x, y) over flat triangles in the plane -- against an
  independent quadrature over the plane triangles with the graph's area
  element sqrt(1 + |grad f|^2) and the plane barycentric coordinates: areas,
  nodal masses and the nine moments of a separated pair.
* Gauss' law on the closed curved surfaces (edges shared, so the pieces
  match): every row sum of the double-layer matrix equals -|t_i| / 2 with the
  curved area, to rounding as the orders grow.  A wrong normal, sign,
  Gramian or edge point breaks it.
* The potential of the unit density on the curved unit sphere converges to 1
  at fourth order in h (the flat sphere's at second): the quadratic
  geometry is what the convergence order checks.
* Homogeneity (lambda^3 single, lambda^2 double), translation invariance,
  symmetry of the single layer, the sign of a column when t_j is reversed.
"""
import math

import numpy as np
import pytest

import synth
from oracle import linear as L
from oracle.curved import DOUBLE, SINGLE, Curved


def _touching_pairs(mesh, t):
    sh = np.isin(mesh.tris, mesh.tris[t]).sum(axis=1)
    return [int(s) for s in np.nonzero(sh > 0)[0]]


def test_straight_edge_points_give_the_flat_entries(orc):
    m = synth.jitter(synth.icosphere(2), 0.01, seed=3)
    qf = synth.quadratic(m, "flat")
    C = Curved(qf.nodes, qf.tris, 3, 5)
    E = orc.Entries(m.verts, m.tris, 3, 3, 5)
    rng = np.random.default_rng(0)
    I = list(rng.integers(m.nt, size=150))
    J = list(rng.integers(m.nt, size=150))
    for t in (0, 41):
        nb = _touching_pairs(m, t)
        I += [t] * len(nb)
        J += nb
    I, J = np.array(I), np.array(J)
    # the flat oracle evaluates touching pairs as (min, max): the same order here
    lo, hi = np.minimum(I, J), np.maximum(I, J)
    cls = E.classify(lo, hi)
    assert set(cls) >= {orc.REG, orc.VERT, orc.EDGE, orc.IDENT}
    ec, ef = C.entries(lo, hi), E.entries(lo, hi)
    assert np.abs(ec - ef).max() < 1e-13 * np.abs(ef).max()
    dc, df = C.entries(I, J, DOUBLE), E.dl_entries(I, J)
    assert np.abs(dc - df).max() < 1e-13 * np.abs(df).max()
    # nodal moments: touching pairs against the flat nodal Sauter-Schwab rule,
    # separated pairs against the flat basis weights
    for t, s in [(0, nb[0]), (0, nb[-1]), (41, 41)] + [(int(a), int(b)) for a, b in zip(I[:5], J[:5])]:
        M = C.moments(t, s)[0]
        if E.classify(t, s)[0] in (orc.REG, orc.NEAR):
            xt, Wt = L.basis_weights(m.verts[m.tris[t]], 3)
            xs, Ws = L.basis_weights(m.verts[m.tris[s]], 3)
            d = xt[:, None, :] - xs[None, :, :]
            ref = Wt.T @ (1.0 / np.sqrt((d * d).sum(axis=2))) @ Ws / (4 * math.pi)
        else:
            ref = E.lin_touch_moments(t, s)
        assert np.abs(M - ref).max() < 1e-13 * np.abs(ref).max(), (t, s)


# ---- a quadratic graph surface -------------------------------------------

def _f(p):
    x, y = p[..., 0], p[..., 1]
    return 0.3 * x * x - 0.2 * x * y + 0.5 * y * y + 0.1 * x


def _grad_f(p):
    x, y = p[..., 0], p[..., 1]
    return np.stack([0.6 * x - 0.2 * y + 0.1, -0.2 * x + 1.0 * y], axis=-1)


def _graph_mesh(tris2d):
    """Curved triangles on z = f(x, y) over the given plane triangles."""
    nodes, t6 = [], []
    for A, B, Cc in tris2d:
        base = len(nodes)
        for p in (A, B, Cc, (A + B) / 2, (B + Cc) / 2, (Cc + A) / 2):
            nodes.append([p[0], p[1], _f(np.asarray(p))])
        t6.append(list(range(base, base + 6)))
    return np.array(nodes), np.array(t6, dtype=np.int32)


def _graph_rule(A, B, Cc, q):
    """Points, plane barycentric coordinates and weights (with the graph's area
    element) of a Duffy-collapsed Gauss rule at corner A of the plane triangle."""
    x, w = np.polynomial.legendre.leggauss(q)
    x, w = (x + 1) / 2, w / 2
    u, v = np.meshgrid(x, x, indexing="ij")
    wu, wv = np.meshgrid(w, w, indexing="ij")
    p = A + u[..., None] * ((B - A) + v[..., None] * (Cc - B))
    det = abs((B - A)[0] * (Cc - A)[1] - (B - A)[1] * (Cc - A)[0])
    g = _grad_f(p)
    wt = wu * wv * u * det * np.sqrt(1 + (g * g).sum(axis=-1))
    lb, lc = u * (1 - v), u * v          # barycentric weights of B and C
    lam = np.stack([1 - lb - lc, lb, lc], axis=-1)
    pts = np.concatenate([p, _f(p)[..., None]], axis=-1)
    return pts.reshape(-1, 3), lam.reshape(-1, 3), wt.reshape(-1)


TRIS2D = [(np.array([0.0, 0.0]), np.array([1.0, 0.0]), np.array([0.2, 0.9])),
          (np.array([2.5, 0.3]), np.array([3.4, 0.5]), np.array([2.8, 1.4]))]


def test_quadratic_graph_against_independent_quadrature():
    nodes, t6 = _graph_mesh(TRIS2D)
    C = Curved(nodes, t6, 10, 4)
    for k, tri in enumerate(TRIS2D):
        pts, lam, wt = _graph_rule(*tri, 24)
        ref = lam.T @ wt
        assert np.abs(C.mass(k, 16) - ref).max() < 1e-13 * ref.sum()
    # a separated pair: the nine moments
    P, la, wa = _graph_rule(*TRIS2D[0], 20)
    Q, lb, wb = _graph_rule(*TRIS2D[1], 20)
    d = P[:, None, :] - Q[None, :, :]
    G = 1.0 / (4 * math.pi * np.sqrt((d * d).sum(axis=2)))
    ref = (la * wa[:, None]).T @ G @ (lb * wb[:, None])
    M = C.moments(0, 1)[0]
    assert np.abs(M - ref).max() < 1e-12 * np.abs(ref).max()
    # the flat triangle through the same corners is measurably different
    flat = Curved(np.concatenate([nodes[:3], (nodes[[0, 1]].mean(0), nodes[[1, 2]].mean(0), nodes[[2, 0]].mean(0)),
                                  nodes[6:]]), t6, 10, 4)
    assert np.abs(flat.moments(0, 1)[0] - ref).max() > 1e-4 * np.abs(ref).max()
    # the double layer of the same pair: the graph's upward normal (-f_x, -f_y, 1)
    # is the orientation of counter-clockwise plane triangles
    g = _grad_f(Q[:, :2])
    nq = np.concatenate([-g, np.ones((g.shape[0], 1))], axis=1)
    nq /= np.linalg.norm(nq, axis=1, keepdims=True)
    K = (d * nq[None, :, :]).sum(axis=2) / (4 * math.pi * ((d * d).sum(axis=2)) ** 1.5)
    refk = (la * wa[:, None]).T @ K @ (lb * wb[:, None])
    Mk = C.moments(0, 1, DOUBLE)[0]
    assert np.abs(Mk - refk).max() < 1e-12 * np.abs(refk).max()


@pytest.mark.parametrize("surface", ["sphere", "ellipsoid"])
def test_gauss_law_on_closed_curved_surfaces(surface):
    axes = (1.0, 0.7, 0.4)
    m = synth.icosphere(1) if surface == "sphere" else synth.ellipsoid(1, axes)
    q = synth.quadratic(m, surface, axes)
    rows = [0, 7, m.nt // 2, m.nt - 1]
    errs = []
    for orders in ((3, 4), (5, 8), (8, 12), (12, 16)):
        C = Curved(q.nodes, q.tris, *orders)
        area = np.array([C.mass(t, 16).sum() for t in rows])
        K = C.block(rows, np.arange(m.nt), DOUBLE)
        errs.append(np.abs(K.sum(axis=1) / area + 0.5).max())
    assert all(a > b for a, b in zip(errs, errs[1:])), errs
    assert errs[-1] < (1e-13 if surface == "sphere" else 1e-9), errs
    # the flat-sided surface through the same vertices obeys it with its own
    # (flat) areas, but not with the curved ones
    C = Curved(q.nodes, q.tris, 8, 12)
    flat = Curved(synth.quadratic(m, "flat").nodes, q.tris, 8, 12)
    af = np.array([flat.mass(t, 4).sum() for t in rows])
    kf = flat.block(rows, np.arange(m.nt), DOUBLE).sum(axis=1)
    assert np.abs(kf / af + 0.5).max() < 1e-8
    area = np.array([C.mass(t, 16).sum() for t in rows])
    assert np.abs(kf / area + 0.5).max() > 1e-3


def test_sphere_potential_converges_at_fourth_order():
    devs, flat = [], []
    for level in (1, 2, 3):
        m = synth.icosphere(level)
        for surf, out in (("sphere", devs), ("flat", flat)):
            q = synth.quadratic(m, surf)
            C = Curved(q.nodes, q.tris, 4, 6)
            rows = [0, m.nt // 3, m.nt - 1]
            area = np.array([C.mass(t, 16).sum() for t in rows])
            out.append(np.abs(C.block(rows, np.arange(m.nt)).sum(axis=1) / area - 1).max())
    assert devs[-1] < 1e-5
    for a, b in zip(devs, devs[1:]):
        assert 12.0 < a / b < 20.0, devs
    for a, b in zip(flat, flat[1:]):
        assert 3.0 < a / b < 5.0, flat


def test_homogeneity_translation_symmetry_orientation():
    m = synth.icosphere(1)
    q = synth.quadratic(m)
    rows, cols = [0, 3, 17], [0, 1, 3, 9, 40, 77]
    C = Curved(q.nodes, q.tris, 3, 5)
    G, K = C.block(rows, cols), C.block(rows, cols, DOUBLE)
    C2 = Curved(2.5 * q.nodes, q.tris, 3, 5)
    assert np.abs(C2.block(rows, cols) - 2.5 ** 3 * G).max() < 1e-13 * np.abs(G).max() * 2.5 ** 3
    assert np.abs(C2.block(rows, cols, DOUBLE) - 2.5 ** 2 * K).max() < 1e-13 * np.abs(K).max() * 2.5 ** 2
    Ct = Curved(q.nodes + np.array([0.3, -1.0, 2.0]), q.tris, 3, 5)
    assert np.abs(Ct.block(rows, cols) - G).max() < 1e-12 * np.abs(G).max()
    assert np.abs(Ct.block(rows, cols, DOUBLE) - K).max() < 1e-12 * np.abs(K).max()
    # symmetry of the single layer: exact for separated pairs, to the Sauter-Schwab
    # rules' asymmetry for touching ones
    Gs = C.block(range(m.nt), range(m.nt))
    sep = np.array([[C.classify(i, j) == 0 for j in range(m.nt)] for i in range(m.nt)])
    assert np.abs((Gs - Gs.T)[sep]).max() < 1e-15 * np.abs(Gs).max()
    assert np.abs(Gs - Gs.T).max() < 1e-6 * np.abs(Gs).max()
    # reversing t_j (corners 1 and 2 swapped, edge points with their edges) flips
    # the double-layer column and leaves the single layer
    t6 = q.tris.copy()
    j = 9
    t6[j] = q.tris[j][[0, 2, 1, 5, 4, 3]]
    Cr = Curved(q.nodes, t6, 3, 5)
    kr = Cr.block(rows, [j], DOUBLE)[:, 0]
    assert np.abs(kr + K[:, cols.index(j)]).max() < 1e-12 * np.abs(K).max()
    assert np.abs(Cr.block(rows, [j])[:, 0] - G[:, cols.index(j)]).max() < 1e-6 * np.abs(G).max()
