"""Pins of the linear-basis oracle (Section 5) against what the paper and the
mathematics fix: the printed worked example of the merge, the set definitions
of T_i, exact moments of the nodal functions, an independent subdivision
quadrature, the partition of unity against the piecewise-constant oracle, and
the symmetry of the Galerkin form."""
import json
import math
import os

import numpy as np
import pytest

import oracle
from oracle import linear as L
import synth
from synth import icosphere

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "merge_example.json")


def _from_printed(r):
    return (r[0] - 1,) + tuple(-1 if x is None else x - 1 for x in r[1:])


def test_merge_worked_example():
    g = json.load(open(GOLDEN))
    tris = [[v - 1 for v in t] for t in g["triangles"]]
    T = L.vertex_triangles(tris, 7)
    sub = [v - 1 for v in g["subset"]]
    for loc, v in enumerate(sub):
        one = L.merge_triangle_lists(tris, T, [v])
        want = [_from_printed(r) for r in g["per_vertex"][str(v + 1)]]
        # a single-vertex subset has local index 0; the printed table carries loc + 1
        assert [(r[0],) + tuple(-1 if x < 0 else loc for x in r[1:]) for r in one] == want
    got = L.merge_triangle_lists(tris, T, sub)
    assert got == [_from_printed(r) for r in g["merged"]]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_merge_matches_set_definition(seed):
    m = icosphere(2)
    T = L.vertex_triangles(m.tris, m.nv)
    rng = np.random.default_rng(seed)
    sub = [int(v) for v in rng.choice(m.nv, size=17, replace=False)]
    rows = L.merge_triangle_lists(m.tris, T, sub)
    union = sorted(set(t for v in sub for t in T[v]))
    assert [r[0] for r in rows] == union
    pos = {v: k for k, v in enumerate(sub)}
    for r in rows:
        for c in range(3):
            v = int(m.tris[r[0]][c])
            assert r[1 + c] == pos.get(v, -1)


def test_vertex_triangles_degree():
    m = icosphere(2)
    T = L.vertex_triangles(m.tris, m.nv)
    deg = sorted(len(x) for x in T)
    # an icosphere has 12 vertices of degree 5, all others degree 6
    assert deg.count(5) == 12 and deg.count(6) == m.nv - 12
    assert sum(deg) == 3 * m.nt


@pytest.mark.parametrize("q,sym", [(2, False), (3, False), (4, False), (2, True), (3, True)])
def test_basis_weight_moments(q, sym):
    rng = np.random.default_rng(q + 10 * sym)
    P = rng.normal(size=(3, 3))
    x, W = L.basis_weights(P, q, sym)
    area = 0.5 * np.linalg.norm(np.cross(P[1] - P[0], P[2] - P[0]))
    for a in range(3):
        b, c = [k for k in range(3) if k != a]
        # integral of lambda_a over t is |t| / 3; its first moment is
        # |t| (2 v_a + v_b + v_c) / 12 (exact for rules of degree >= 2)
        assert abs(W[:, a].sum() - area / 3) < 1e-14 * area
        mom = W[:, a] @ x
        assert np.allclose(mom, area * (2 * P[a] + P[b] + P[c]) / 12, rtol=0, atol=1e-14 * area * 10)


def _subdivided(P, k):
    """Centroids, areas and barycentric coordinates of the 4^k congruent
    subtriangles of P (midpoint refinement)."""
    tri = [np.eye(3)]
    for _ in range(k):
        nxt = []
        for B in tri:
            m01, m12, m20 = (B[0] + B[1]) / 2, (B[1] + B[2]) / 2, (B[2] + B[0]) / 2
            nxt += [np.array([B[0], m01, m20]), np.array([m01, B[1], m12]),
                    np.array([m20, m12, B[2]]), np.array([m01, m12, m20])]
        tri = nxt
    bary = np.array([B.mean(axis=0) for B in tri])
    area = 0.5 * np.linalg.norm(np.cross(P[1] - P[0], P[2] - P[0])) / len(tri)
    return bary @ P, area, bary


def _pair_subdivision(P, Q, k):
    x, ax, lx = _subdivided(P, k)
    y, ay, ly = _subdivided(Q, k)
    d = x[:, None, :] - y[None, :, :]
    g = 1.0 / np.sqrt((d * d).sum(axis=2))
    return (lx.T @ g @ ly) * ax * ay / (4 * math.pi)


def test_two_triangle_block_vs_subdivision():
    # two separate triangles at a distance comparable to their size, so that
    # the nine vertex combinations differ well beyond the tolerance
    P = np.array([[0.0, 0.0, 0.0], [1.0, 0.1, 0.0], [0.2, 0.9, 0.1]])
    Q = np.array([[1.6, 0.3, 0.4], [2.4, 0.2, 0.1], [1.9, 1.1, 0.5]])
    verts = np.vstack([P, Q])
    tris = np.array([[0, 1, 2], [3, 4, 5]])
    got = L.lin_block(verts, tris, [0, 1, 2], [3, 4, 5], q=8)
    # midpoint rule on 4^k subtriangles is O(h^2); Richardson on k = 4, 5
    I4, I5 = _pair_subdivision(P, Q, 4), _pair_subdivision(P, Q, 5)
    ref = (4 * I5 - I4) / 3
    assert np.abs(got - ref).max() < 1e-6 * np.abs(ref).max()
    assert np.ptp(ref) > 0.2 * np.abs(ref).max()


@pytest.mark.parametrize("q,sym", [(2, False), (3, False), (2, True), (3, True)])
def test_partition_of_unity_vs_constant_oracle(q, sym):
    # two disjoint icosahedra: with every vertex of A as a row and every vertex
    # of B as a column the nodal functions sum to one on every triangle, so the
    # block sum equals the sum of the piecewise-constant entries over A x B
    A = icosphere(0)
    nvA, ntA = A.nv, A.nt
    verts = np.vstack([A.verts, A.verts + np.array([3.0, 0.5, -0.2])])
    tris = np.vstack([A.tris, A.tris + nvA]).astype(np.int32)
    lin = L.lin_block(verts, tris, list(range(nvA)), list(range(nvA, 2 * nvA)), q, sym)
    E = oracle.Entries(verts, tris, q_r=q, q_nr=q, q_s=4, sym=sym)
    const = E.block(np.arange(ntA), np.arange(ntA, 2 * ntA))
    assert abs(lin.sum() - const.sum()) < 1e-13 * abs(const.sum())


def test_symmetry_and_shared_vertex():
    m = icosphere(2)
    T = L.vertex_triangles(m.tris, m.nv)
    c = m.verts
    # two vertex patches on opposite sides of the sphere
    a = np.argsort(((c - c[0]) ** 2).sum(1))[:6]
    b = np.argsort(((c + c[0]) ** 2).sum(1))[:5]
    G = L.lin_block(m.verts, m.tris, a, b, 3, T=T)
    Gt = L.lin_block(m.verts, m.tris, b, a, 3, T=T)
    assert np.allclose(G, Gt.T, rtol=1e-13, atol=0)
    assert (G > 0).all()
    with pytest.raises(ValueError):
        L.lin_block(m.verts, m.tris, a[:2], a[2:4], 3, T=T)


def _touching_partners(orc, ent, t, nt):
    out = {}
    for s in range(nt):
        k = int(ent.classify(t, s)[0])
        if k in (orc.IDENT, orc.EDGE, orc.VERT):
            out.setdefault(k, s)
    return out


def test_touching_moments_rows_against_semianalytic(orc):
    """Sauter-Schwab with the nodal weights (Section 5's basis on touching
    pairs): the row sums sum_b M_ab = int_t lambda_a(x) int_s g(x, y) dy dx
    against the analytic inner potential and a graded outer rule weighted by
    lambda_a (tests/semianalytic.py), for the identical, common-edge and
    common-vertex case (1e-11); the column sums by the transposition
    M(s, t) = M(t, s)^T of the same integral with the roles swapped."""
    import math
    from tests import semianalytic as SA
    m = synth.jitter(synth.icosphere(2), 0.01, seed=2)
    ent = orc.Entries(m.verts, m.tris, 3, 3, 12)
    for t in (5, 77):
        parts = _touching_partners(orc, ent, t, m.nt)
        assert set(parts) == {orc.IDENT, orc.EDGE, orc.VERT}
        for k, s in parts.items():
            M = ent.lin_touch_moments(t, s)
            T, S = m.verts[m.tris[t]], m.verts[m.tris[s]]
            for a in range(3):
                ref = SA.pair_integral(T, S, corner=a) / (4 * math.pi)
                assert abs(M[a].sum() - ref) < 1e-11 * ref, (t, s, k, a)
            Mt = ent.lin_touch_moments(s, t)
            assert np.abs(Mt - M.T).max() < 1e-9 * np.abs(M).max(), (t, s, k)
            if k == orc.IDENT:
                assert np.abs(M - M.T).max() < 1e-13 * np.abs(M).max()


def test_touching_moments_partition_of_unity_and_nan_for_disjoint(orc):
    m = synth.icosphere(2)
    ent = orc.Entries(m.verts, m.tris, 3, 3, 5)
    for k, s in _touching_partners(orc, ent, 0, m.nt).items():
        M = ent.lin_touch_moments(0, s)
        g = ent.entries(0, s)[0]
        assert abs(M.sum() - g) < 1e-14 * g
        assert np.all(M > 0)
    far = next(s for s in range(m.nt) if ent.classify(0, s) == orc.REG)
    assert np.isnan(ent.lin_touch_moments(0, far)).all()


def test_lin_block_with_touching_pairs_partition_of_unity(orc):
    """All vertices against all vertices of one icosahedron (every pair of
    triangles touches or is near): the sum of the linear-basis block equals
    the sum of the piecewise-constant oracle's whole matrix with the same
    rules (the nodal functions sum to one on every triangle)."""
    m = synth.icosphere(0)
    T = L.vertex_triangles(m.tris, m.nv)
    B = L.lin_block(m.verts, m.tris, range(m.nv), range(m.nv), 3, False, T=T, q_s=6)
    G = orc.Entries(m.verts, m.tris, 3, 3, 6).dense()
    assert abs(B.sum() - G.sum()) < 1e-13 * G.sum()
    # symmetric up to the Sauter-Schwab quadrature error (the common-edge maps treat x and y differently)
    assert np.abs(B - B.T).max() < 1e-8 * np.abs(B).max()
    with pytest.raises(ValueError):
        L.lin_block(m.verts, m.tris, [0], [0], 3, False, T=T)
