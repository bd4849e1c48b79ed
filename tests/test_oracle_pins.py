"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Each test names the mathematical fact it uses.  Together they are meant to catch
a plausible mistake anywhere in the oracle: a wrong Gauss node, a Sauter-Schwab
region that overlaps or misses part of T x T, a dropped Jacobian factor, a wrong
sign or scale in the Green-quadrature factor, a wrong cross-approximation
update, a transposed transfer matrix or a missing matrix-vector phase.
"""
import json
import math
import os

import numpy as np
import pytest

import synth
from tests import semianalytic as sa

HERE = os.path.dirname(os.path.abspath(__file__))


def one_pair_mesh(T, S, shared):
    """Two-triangle mesh; `shared` lists which vertices of S are T's (index
    pairs (k_T, k_S))."""
    verts = [np.asarray(p, dtype=np.float64) for p in T]
    sidx = []
    for k in range(3):
        hit = [a for (a, b) in shared if b == k]
        if hit:
            sidx.append(hit[0])
        else:
            verts.append(np.asarray(S[k], dtype=np.float64))
            sidx.append(len(verts) - 1)
    return np.array(verts), np.array([[0, 1, 2], sidx], dtype=np.int32)


def tri_areas(mesh):
    T = mesh.verts[mesh.tris]
    return 0.5 * np.linalg.norm(np.cross(T[:, 1] - T[:, 0], T[:, 2] - T[:, 0]), axis=1)


# ---------------------------------------------------------------- quadrature --

@pytest.mark.parametrize("q", [1, 2, 3, 4, 5, 8, 13, 20])
def test_gauss_legendre_matches_library_and_is_exact(orc, q):
    x, w = orc.gauss01(q)
    xr, wr = np.polynomial.legendre.leggauss(q)
    np.testing.assert_allclose(x, 0.5 * (xr + 1.0), rtol=0, atol=1e-15)
    np.testing.assert_allclose(w, 0.5 * wr, rtol=0, atol=1e-15)
    for d in range(2 * q):
        assert abs(np.sum(w * x ** d) - 1.0 / (d + 1)) < 1e-14


def _tri_moment(a, b):
    # int_T s1^a s2^b over T = {0 <= s2 <= s1 <= 1}
    return 1.0 / ((b + 1) * (a + b + 2))


@pytest.mark.parametrize("q,sym", [(2, False), (3, False), (4, False), (2, True), (3, True)])
def test_triangle_rules_integrate_polynomials_of_their_degree(orc, q, sym):
    """Both rule families of the disjoint classes are exact for every
    polynomial in (s1, s2) of total degree <= 2q - 2 on the reference triangle
    (the collapsed rule: Gauss-Legendre exact to degree 2q - 1 in s1 after the
    factor s1 of the collapse; the symmetric rules by construction), and the
    symmetric ones are not exact one degree higher (so the degree is the
    stated one, not an accident of the test).  Exactness to rounding pins the
    printed orbit constants."""
    s1, s2, w = orc.tri_rule(q, sym)
    assert len(w) == (q * q if not sym else {2: 3, 3: 6}[q])
    assert np.all(w > 0)
    assert np.all((s2 >= 0) & (s2 <= s1) & (s1 <= 1))
    deg = 2 * q - 2
    for a in range(deg + 1):
        for b in range(deg + 1 - a):
            assert abs(np.sum(w * s1 ** a * s2 ** b) - _tri_moment(a, b)) < 2e-15, (a, b)
    if sym:
        worst = max(abs(np.sum(w * s1 ** a * s2 ** (deg + 1 - a)) - _tri_moment(a, deg + 1 - a))
                    for a in range(deg + 2))
        assert worst > 1e-6


def test_symmetric_rule_entries_are_invariant_under_vertex_rotation(orc):
    """The symmetric rules are invariant under the permutations of a
    triangle's vertices, so rotating the vertex order of every triangle leaves
    their regular entries unchanged (to rounding); the collapsed rule is not
    invariant (it distinguishes P0), which the same test shows."""
    m = synth.icosphere(2)
    rot = np.ascontiguousarray(m.tris[:, [1, 2, 0]])
    a = orc.Entries(m.verts, m.tris, 3, 3, 4, sym=True)
    b = orc.Entries(m.verts, rot, 3, 3, 4, sym=True)
    c0 = orc.Entries(m.verts, m.tris, 3, 3, 4)
    c1 = orc.Entries(m.verts, rot, 3, 3, 4)
    I = np.arange(m.nt)
    J = (I * 37 + 11) % m.nt
    reg = a.classify(I, J) == orc.REG
    I, J = I[reg], J[reg]
    ga, gb = a.entries(I, J), b.entries(I, J)
    np.testing.assert_allclose(ga, gb, rtol=1e-13, atol=0)
    assert np.max(np.abs(c0.entries(I, J) - c1.entries(I, J)) / np.abs(c0.entries(I, J))) > 1e-9


def test_symmetric_rule_converges_like_the_collapsed_rule(orc):
    """Disjoint pairs of the level-3 sphere: against an order-8 collapsed
    reference, the symmetric rule of degree 4 (6 points) is as accurate as
    the collapsed rule of the same degree (9 points) -- within a factor 3 --
    and far more accurate than the degree-2 rules; near-regular pairs use the
    same family."""
    m = synth.icosphere(3)
    ref = orc.Entries(m.verts, m.tris, 8, 8, 4)
    rng = np.random.default_rng(3)
    I = rng.integers(0, m.nt, 4000)
    J = rng.integers(0, m.nt, 4000)
    cls = ref.classify(I, J)
    sel = (cls == orc.REG) | (cls == orc.NEAR)
    I, J = I[sel], J[sel]
    g = ref.entries(I, J)
    err = {}
    for q in (2, 3):
        for sym in (False, True):
            e = orc.Entries(m.verts, m.tris, q, q, 4, sym=sym)
            err[q, sym] = np.linalg.norm(e.entries(I, J) - g) / np.linalg.norm(g)
    assert err[3, True] < 3 * err[3, False] and err[3, False] < 3 * err[3, True]
    assert err[3, True] < err[2, True] / 10 and err[3, True] < 1e-5
    with pytest.raises(ValueError):
        orc.Entries(m.verts, m.tris, 4, 4, 4, sym=True)


@pytest.mark.parametrize("kase", ["ident", "edge", "vert"])
def test_sauter_schwab_maps_tile_the_product_domain(orc, kase):
    """The regions' maps must cover T x T exactly once: every moment
    int_T int_T x1^a x2^b y1^c y2^d equals 1/((b+1)(a+b+2)) * 1/((d+1)(c+d+2))."""
    k = {"ident": orc.IDENT, "edge": orc.EDGE, "vert": orc.VERT}[kase]
    for a in range(3):
        for b in range(3):
            for c in range(3):
                for d in range(3):
                    exact = 1.0 / ((b + 1) * (a + b + 2)) / ((d + 1) * (c + d + 2))
                    got = orc.ss_moment(k, 8, a, b, c, d)
                    assert abs(got - exact) <= 1e-14 * max(1.0, exact), (a, b, c, d, got, exact)


IDENT_TRIS = {
    "equilateral": [[0, 0, 0], [1, 0, 0], [0.5, math.sqrt(3) / 2, 0]],
    "right": [[0, 0, 0], [1, 0, 0], [0, 1, 0]],
    "scalene_3d": [[0.1, -0.2, 0.3], [1.1, 0.1, 0.2], [0.3, 0.8, 0.05]],
    "obtuse": [[0, 0, 0], [1, 0, 0], [0.7, 0.35, 0.05]],
}


@pytest.mark.parametrize("name", list(IDENT_TRIS))
def test_identical_pair_matches_closed_form(orc, name):
    """P1: int_t int_t 1/|x-y| for a flat triangle in closed form."""
    T = np.array(IDENT_TRIS[name])
    e = orc.Entries(T, np.array([[0, 1, 2]], dtype=np.int32), 3, 3, 24)
    ref = sa.self_integral_closed_form(T) / (4 * math.pi)
    got = e.entries(0, 0)[0]
    assert abs(got / ref - 1) < 1e-11, (got, ref)


def test_identical_thin_triangle_converges_to_closed_form(orc):
    """A thin triangle makes the regularised integrand nearly singular; the rule
    still converges to the closed form, only more slowly."""
    T = np.array([[0, 0, 0], [1, 0, 0], [0.55, 0.12, 0.02]])
    ref = sa.self_integral_closed_form(T) / (4 * math.pi)
    errs = [abs(orc.Entries(T, np.array([[0, 1, 2]], dtype=np.int32), 3, 3, q).entries(0, 0)[0] / ref - 1)
            for q in (8, 20, 32)]
    assert errs[-1] < 1e-7 and errs[-1] < errs[0] * 1e-3, errs


EDGE_PAIRS = [
    ([[0, 0, 0], [1.0, 0.1, 0], [0.3, 0.8, 0.05]], [[0, 0, 0], [1.0, 0.1, 0], [0.6, -0.7, 0.3]]),
    ([[0, 0, 0], [1.0, 0, 0], [0.5, 0.9, 0]], [[0, 0, 0], [1.0, 0, 0], [0.4, -0.8, 0.0]]),  # coplanar
]
VERT_PAIRS = [
    ([[0, 0, 0], [1.0, 0.1, 0], [0.3, 0.8, 0.05]], [[0, 0, 0], [-0.9, 0.2, 0.1], [-0.4, -0.8, 0.2]]),
    ([[0, 0, 0], [1.0, 0, 0], [0.5, 0.9, 0]], [[0, 0, 0], [-0.7, -0.3, 0.0], [0.2, -0.9, 0.0]]),  # coplanar
]


@pytest.mark.parametrize("k", range(len(EDGE_PAIRS)))
def test_common_edge_pair_matches_semi_analytic(orc, k):
    """P2: inner integral in closed form, outer by graded Gauss (independent of
    the Sauter-Schwab maps)."""
    T, S = map(np.array, EDGE_PAIRS[k])
    verts, tris = one_pair_mesh(T, S, [(0, 0), (1, 1)])
    e = orc.Entries(verts, tris, 3, 3, 14)
    assert e.classify(0, 1)[0] == orc.EDGE
    ref = sa.pair_integral(T, S) / (4 * math.pi)
    got = e.entries(0, 1)[0]
    assert abs(got / ref - 1) < 1e-10, (got, ref)
    assert e.entries(1, 0)[0] == got


@pytest.mark.parametrize("k", range(len(VERT_PAIRS)))
def test_common_vertex_pair_matches_semi_analytic(orc, k):
    T, S = map(np.array, VERT_PAIRS[k])
    verts, tris = one_pair_mesh(T, S, [(0, 0)])
    e = orc.Entries(verts, tris, 3, 3, 14)
    assert e.classify(0, 1)[0] == orc.VERT
    ref = sa.pair_integral(T, S) / (4 * math.pi)
    got = e.entries(0, 1)[0]
    assert abs(got / ref - 1) < 1e-10, (got, ref)


def test_regular_pair_matches_semi_analytic(orc):
    """Disjoint pair at moderate distance: the tensor rule converges to the
    semi-analytic value."""
    T = np.array([[0, 0, 0], [1.0, 0.1, 0], [0.3, 0.8, 0.05]])
    S = T + np.array([1.4, 0.3, 0.5])
    verts = np.concatenate([T, S])
    tris = np.array([[0, 1, 2], [3, 4, 5]], dtype=np.int32)
    e = orc.Entries(verts, tris, 16, 16, 4)
    assert e.classify(0, 1)[0] == orc.REG
    ref = sa.pair_integral(T, S) / (4 * math.pi)
    got = e.entries(0, 1)[0]
    assert abs(got / ref - 1) < 1e-11


def test_orders_converge_for_every_pair_class(orc):
    """P15: the difference between successive orders decays for every class."""
    m = synth.icosphere(2)
    cls_pairs = {}
    e0 = orc.Entries(m.verts, m.tris)
    for j in range(m.nt):
        c = int(e0.classify(0, j)[0])
        cls_pairs.setdefault(c, j)
    assert set(cls_pairs) == {orc.REG, orc.NEAR, orc.VERT, orc.EDGE, orc.IDENT}
    for c, j in cls_pairs.items():
        vals = []
        for q in (2, 4, 6, 8, 10):
            e = orc.Entries(m.verts, m.tris, q, q, q)
            vals.append(e.entries(0, j)[0])
        d = np.abs(np.diff(vals))
        assert d[-1] < 1e-3 * d[0] + 1e-16, (c, d)
        assert d[-1] < 1e-8 * abs(vals[-1]), (c, d)


def test_pair_classes_brute_force(orc):
    """Classification from vertex ids only, checked by brute force on a small
    sphere: identical n, common edge 3n/2 unordered, common vertex and
    near-regular as counted from vertex sets and the edge set."""
    m = synth.icosphere(2)
    e = orc.Entries(m.verts, m.tris)
    edges = set()
    for t in m.tris:
        for a in range(3):
            u, v = int(t[a]), int(t[(a + 1) % 3])
            edges.add((min(u, v), max(u, v)))
    n = m.nt
    I, J = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    got = e.classify(I.ravel(), J.ravel()).reshape(n, n)
    for i in range(0, n, 7):
        for j in range(n):
            sh = len(set(m.tris[i]) & set(m.tris[j]))
            if sh == 3:
                exp = orc.IDENT
            elif sh == 2:
                exp = orc.EDGE
            elif sh == 1:
                exp = orc.VERT
            elif any((min(a, b), max(a, b)) in edges for a in m.tris[i] for b in m.tris[j]):
                exp = orc.NEAR
            else:
                exp = orc.REG
            assert got[i, j] == exp
    assert (got == orc.IDENT).sum() == n
    assert (got == orc.EDGE).sum() == 3 * n
    np.testing.assert_array_equal(got, got.T)


# ------------------------------------------------------------ dense matrix --

@pytest.fixture(scope="module")
def sphere3_dense(orc):
    m = synth.icosphere(3)
    e = orc.Entries(m.verts, m.tris)
    return m, e, e.dense()


def test_dense_symmetric_and_positive_definite(sphere3_dense):
    """P11: G = G^T exactly, and G is SPD (the single-layer operator is
    coercive), so Cholesky succeeds."""
    m, e, G = sphere3_dense
    assert np.array_equal(G, G.T)
    np.linalg.cholesky(G)
    assert np.all(np.diag(G) > 0)


def test_rows_and_entries_agree_with_dense(sphere3_dense):
    m, e, G = sphere3_dense
    rng = np.random.default_rng(3)
    rows = rng.choice(m.nt, 16, replace=False)
    x = synth.rhs_normal(m.nt, 1, seed=0)
    np.testing.assert_allclose(e.matvec_rows(rows, x), G[rows] @ x, rtol=1e-13, atol=1e-15)


def test_scaling_and_translation(orc, sphere3_dense):
    """P12: every rule lives on reference elements, so G(lambda X) =
    lambda^3 G(X); the dense G is translation invariant."""
    m, e, G = sphere3_dense
    rng = np.random.default_rng(5)
    I = rng.integers(0, m.nt, 400)
    J = rng.integers(0, m.nt, 400)
    I = np.concatenate([I, np.arange(20)])
    J = np.concatenate([J, np.arange(20)])
    e2 = orc.Entries(m.verts * 2.5, m.tris)
    np.testing.assert_allclose(e2.entries(I, J), 2.5 ** 3 * G[I, J], rtol=1e-12)
    e3 = orc.Entries(m.verts + np.array([0.3, -0.2, 0.7]), m.tris)
    np.testing.assert_allclose(e3.entries(I, J), G[I, J], rtol=1e-11)


def test_sphere_constant_potential_converges_at_second_order(orc):
    """P3: on the sphere of radius r the single-layer potential of the constant
    1 is r, so (G 1)_i / |t_i| -> r; the deviation falls ~4x per refinement."""
    devs = []
    for lev in (2, 3, 4):
        m = synth.icosphere(lev, radius=1.0)
        e = orc.Entries(m.verts, m.tris, 6, 8, 7)
        rows = np.arange(0, m.nt, max(1, m.nt // 48))
        y = e.matvec_rows(rows, np.ones(m.nt)) / tri_areas(m)[rows]
        devs.append(np.abs(y - 1.0).max())
    assert devs[-1] < 1e-3
    for a, b in zip(devs, devs[1:]):
        assert 3.6 < a / b < 4.4, devs


def test_sphere_energy_of_constant(orc, sphere3_dense):
    """P6: E(1) = 1/2 1^T G 1 -> 2 pi r^3, at second order in h."""
    m, e, G = sphere3_dense
    dev3 = abs(0.5 * G.sum() / (2 * math.pi) - 1)
    m2 = synth.icosphere(2)
    G2 = orc.Entries(m2.verts, m2.tris).dense()
    dev2 = abs(0.5 * G2.sum() / (2 * math.pi) - 1)
    assert dev3 < 1e-2
    assert 3.5 < dev2 / dev3 < 4.5, (dev2, dev3)


def test_ellipsoid_equilibrium_density(orc):
    """P5: the density Q/(4 pi abc) (x^2/a^4 + y^2/b^4 + z^2/c^4)^(-1/2) has the
    constant potential (Q / 8 pi) int_0^inf ds / sqrt((a^2+s)(b^2+s)(c^2+s))
    on the ellipsoid; the Galerkin rows divided by |t_i| approach it."""
    from scipy.integrate import quad
    ax = (1.0, 0.7, 0.4)
    f = lambda s: 1.0 / math.sqrt((ax[0] ** 2 + s) * (ax[1] ** 2 + s) * (ax[2] ** 2 + s))
    phi = (quad(f, 0, 1)[0] + quad(f, 1, np.inf)[0]) / (8 * math.pi)
    assert abs(phi - 0.115111869267) < 1e-11
    devs = []
    for lev in (2, 3, 4):
        m = synth.ellipsoid(lev, ax)
        T = m.verts[m.tris]
        c = T.mean(axis=1)
        sig = 1.0 / (4 * math.pi * ax[0] * ax[1] * ax[2]) / np.sqrt(
            c[:, 0] ** 2 / ax[0] ** 4 + c[:, 1] ** 2 / ax[1] ** 4 + c[:, 2] ** 2 / ax[2] ** 4)
        e = orc.Entries(m.verts, m.tris, 5, 7, 6)
        rows = np.arange(0, m.nt, max(1, m.nt // 48))
        y = e.matvec_rows(rows, sig) / tri_areas(m)[rows]
        devs.append(np.abs(y / phi - 1).max())
    assert devs[-1] < 1e-3
    for a, b in zip(devs, devs[1:]):
        assert 3.3 < a / b < 4.6, devs


def test_dense_storage_figure():
    """P16: the full matrix of the n = 32768 sphere in FP64 needs 8192 MB."""
    g = json.load(open(os.path.join(HERE, "golden", "dense_storage.json")))
    assert g["n"] * g["n"] * 8 / 2 ** 20 == g["MiB"]


# ------------------------------------------------ Green quadrature factor --

def test_green_rule_reproduces_gauss_flux(orc):
    """P7: sum_nu w_nu dg/dn_z(x, z_nu) approximates int_{d omega} dg/dn_z(x,z) dz,
    which is -1 for x inside omega and 0 outside (Gauss' law with the outward
    normal)."""
    tree = orc.cluster_tree(*_mesh3(), 32)
    nd = tree.nodes[3]
    errs = []
    for mq in (4, 8, 16):
        z, w, nrm = orc.green_points(nd, mq, 2.0)
        x_in = 0.5 * (nd.lo + nd.hi)
        out = nd.hi + 2.0 * (nd.hi - nd.lo) + 0.5
        d_in = x_in[None, :] - z
        d_out = out[None, :] - z
        f_in = np.sum(w * np.einsum("kd,kd->k", nrm, d_in) / (4 * math.pi * np.linalg.norm(d_in, axis=1) ** 3))
        f_out = np.sum(w * np.einsum("kd,kd->k", nrm, d_out) / (4 * math.pi * np.linalg.norm(d_out, axis=1) ** 3))
        errs.append((abs(f_in + 1.0), abs(f_out)))
    assert errs[-1][0] < 1e-6 and errs[-1][1] < 1e-8
    assert errs[-1][0] < errs[0][0]


def _mesh3():
    m = synth.icosphere(3)
    return m.verts, m.tris


def test_green_quadrature_approximates_kernel(orc):
    """Eq. quadrature_apx: sum_nu w_nu [g(x,z) dg/dn_z(z,y) - dg/dn_z(x,z) g(z,y)]
    -> g(x, y) for x in tau, y outside omega, exponentially in the order."""
    tree = orc.cluster_tree(*_mesh3(), 32)
    nd = tree.nodes[5]
    x = nd.lo + 0.3 * (nd.hi - nd.lo)
    y = nd.hi + 1.5 * (nd.hi - nd.lo)
    gxy = 1 / (4 * math.pi * np.linalg.norm(x - y))
    errs = []
    for mq in (2, 4, 6, 8):
        z, w, nrm = orc.green_points(nd, mq, 2.0, omega_scale=0.5)
        dx = x[None, :] - z
        dy = y[None, :] - z
        rx = np.linalg.norm(dx, axis=1)
        ry = np.linalg.norm(dy, axis=1)
        gxz = 1 / (4 * math.pi * rx)
        gzy = 1 / (4 * math.pi * ry)
        dn_xz = np.einsum("kd,kd->k", nrm, dx) / (4 * math.pi * rx ** 3)
        dn_zy = np.einsum("kd,kd->k", nrm, dy) / (4 * math.pi * ry ** 3)
        errs.append(abs(np.sum(w * (gxz * dn_zy - dn_xz * gzy)) - gxy) / gxy)
    assert errs[-1] < 1e-4
    assert errs[-1] < 1e-2 * errs[0]


def test_green_factorisation_approximates_admissible_block(orc):
    """P8 (Section 2): G|tau x sigma ~ A B^T with B written out in this test,
        b_{j nu} = sqrt(w) int dg/dn_z(z_nu, y) phi_j,
        b_{j nu+k} = sqrt(w)/d_tau int g(z_nu, y) phi_j,
    and the error decays with the Green order.  A wrong sign or d_tau scale in
    the oracle's A breaks the factorisation."""
    verts, tris = _mesh3()
    tree = orc.cluster_tree(verts, tris, 32)
    far, _ = orc.block_tree(tree, 2.0)
    t, s = next((t, s) for (t, s) in far if not tree.nodes[t].sons and not tree.nodes[s].sons)
    ent = orc.Entries(verts, tris, 6, 8, 6)
    tp, tw = ent.triangle_points(6)
    rows, cols = tree.indices(t), tree.indices(s)
    Gts = ent.block(rows, cols)
    errs = []
    for mq in (2, 4, 6, 10):
        nd = tree.nodes[t]
        z, w, nrm = orc.green_points(nd, mq, 2.0, omega_scale=0.25)
        A = orc.green_factor_A(rows, tp, tw, z, w, nrm, nd.diam)
        P, W = tp[cols], tw[cols]
        d = P[:, :, None, :] - z[None, None, :, :]          # y - z
        r = np.linalg.norm(d, axis=-1)
        g = 1 / (4 * math.pi * r)
        dg = np.einsum("jpkd,kd->jpk", d, nrm) / (4 * math.pi * r ** 3)
        sw = np.sqrt(w)
        B = np.concatenate([sw * np.einsum("jp,jpk->jk", W, dg),
                            sw / nd.diam * np.einsum("jp,jpk->jk", W, g)], axis=1)
        errs.append(np.linalg.norm(Gts - A @ B.T) / np.linalg.norm(Gts))
    assert errs[-1] < 1e-3 * errs[0], errs
    assert errs[-1] < 1e-4, errs


# ------------------------------------------------------ cross approximation --

def test_aca_recovers_exact_low_rank(orc):
    rng = np.random.default_rng(0)
    A = rng.standard_normal((40, 7)) @ rng.standard_normal((7, 108))
    I, J, V = orc.aca_full(A, 1e-12)
    assert len(I) == 7
    np.testing.assert_allclose(V @ A[I], A, atol=1e-10 * np.abs(A).max())
    np.testing.assert_array_equal(V[I], np.eye(7))


def test_aca_first_pivot_is_global_max_and_stop_rule(orc):
    rng = np.random.default_rng(1)
    U = rng.standard_normal((30, 108)) * np.exp(-0.5 * np.arange(108))[None, :]
    I, J, V = orc.aca_full(U, 1e-4)
    p, q = np.unravel_index(np.argmax(np.abs(U)), U.shape)
    assert (I[0], J[0]) == (p, q)
    assert len(I) <= min(U.shape)
    res = np.linalg.norm(U - V @ U[I])
    assert res <= 1e-4 * np.linalg.norm(U) * (1 + 1e-8)
    # one step fewer would not have met the criterion
    I2, J2, V2 = orc.aca_full(U, 1e-4)
    assert np.array_equal(I, I2)


# ------------------------------------------------------ trees and H^2 ------

def test_cluster_tree_invariants(orc):
    verts, tris = _mesh3()
    tree = orc.cluster_tree(verts, tris, 32)
    assert sorted(tree.perm.tolist()) == list(range(len(tris)))
    for nd in tree.nodes:
        idx = tree.perm[nd.begin:nd.end]
        vv = verts[tris[idx].ravel()]
        assert np.all(vv >= nd.lo) and np.all(vv <= nd.hi)
        if nd.sons:
            a, b = (tree.nodes[s] for s in nd.sons)
            assert a.begin == nd.begin and a.end == b.begin and b.end == nd.end
            assert a.end - a.begin == (nd.end - nd.begin) // 2
        else:
            assert nd.end - nd.begin <= 32


# Hand-built boxes whose diameters and distance are exact in binary floating
# point (sides 3, 4, 0 give a diagonal of exactly 5).  Each case is
# (lo_a, hi_a, lo_b, hi_b, eta, admissible?) for Section 2's condition
# max{diam tau, diam sigma} <= 2 eta dist(tau, sigma), dist the Euclidean
# distance of the boxes, diam the length of a box's diagonal; equality is
# admissible, overlapping or touching boxes never are.
ADMISSIBILITY_CASES = [
    # gap 1.25 along x, both diameters 5: 2 eta dist = 5 at eta = 2 (equality)
    ((0, 0, 0), (3, 4, 0), (4.25, 0, 0), (7.25, 4, 0), 2.0, True),
    ((0, 0, 0), (3, 4, 0), (4.25, 0, 0), (7.25, 4, 0), 1.96875, False),
    ((0, 0, 0), (3, 4, 0), (4.25, 0, 0), (7.25, 4, 0), 1.0, False),
    # diagonal gaps (0.75, 1, 0): Euclidean 1.25, Chebyshev 1, Manhattan 1.75
    ((0, 0, 0), (3, 4, 0), (3.75, 5, 0), (6.75, 9, 0), 2.0, True),
    ((0, 0, 0), (3, 4, 0), (3.75, 5, 0), (6.75, 9, 0), 1.875, False),
    # gaps along y and z only, (0, 0.75, 1): Euclidean 1.25
    ((0, 0, 0), (3, 4, 0), (0, 4.75, 1), (3, 8.75, 1), 2.0, True),
    ((0, 0, 0), (3, 4, 0), (0, 4.75, 1), (3, 8.75, 1), 1.9375, False),
    # sigma smaller (diagonal 1): the larger diameter decides
    ((0, 0, 0), (3, 4, 0), (4.25, 0, 0), (4.85, 0.8, 0), 2.0, True),
    ((0, 0, 0), (3, 4, 0), (4.25, 0, 0), (4.85, 0.8, 0), 1.0, False),
    ((4.25, 0, 0), (4.85, 0.8, 0), (0, 0, 0), (3, 4, 0), 1.0, False),
    # touching faces and overlapping boxes: distance zero
    ((0, 0, 0), (3, 4, 0), (3, 0, 0), (6, 4, 0), 1e9, False),
    ((0, 0, 0), (3, 4, 0), (1, 1, 0), (4, 5, 0), 1e9, False),
    # far apart: gap 20 along z, eta 1/8 gives 2 eta dist = 5
    ((0, 0, 0), (3, 4, 0), (0, 0, 20), (3, 4, 20), 0.125, True),
    ((0, 0, 0), (3, 4, 0), (0, 0, 20), (3, 4, 20), 0.12, False),
]


def _box(orc, lo, hi):
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    e = hi - lo
    return orc.Cluster(0, 1, 0, lo=lo, hi=hi, diam=math.sqrt((e[0] * e[0] + e[1] * e[1]) + e[2] * e[2]))


def _admissibility_failures(orc, admissible):
    bad = []
    for k, (la, ha, lb, hb, eta, want) in enumerate(ADMISSIBILITY_CASES):
        if bool(admissible(_box(orc, la, ha), _box(orc, lb, hb), eta)) != want:
            bad.append(k)
    return bad


def test_admissibility_condition_on_boxes_with_exact_distances(orc):
    """Section 2's admissibility condition on hand-built boxes: the flip
    happens exactly at max{diam} = 2 eta dist, with equality admissible, dist
    Euclidean, the larger diameter deciding, boxes at distance zero never
    admissible."""
    assert _box(orc, (0, 0, 0), (3, 4, 0)).diam == 5.0
    assert orc.box_dist(_box(orc, (0, 0, 0), (3, 4, 0)), _box(orc, (3.75, 5, 0), (6.75, 9, 0))) == 1.25
    assert orc.box_dist(_box(orc, (0, 0, 0), (3, 4, 0)), _box(orc, (1, 1, 0), (4, 5, 0))) == 0.0
    assert _admissibility_failures(orc, orc.admissible) == []


def test_admissibility_cases_reject_plausible_misreadings(orc):
    """The cases above are strong enough: a factor eta instead of 2 eta, a
    strict inequality, the smaller diameter, or a Chebyshev or Manhattan box
    distance each fail at least one of them."""
    def gaps(a, b):
        return [max(0.0, max(b.lo[d] - a.hi[d], a.lo[d] - b.hi[d])) for d in range(3)]

    eucl = lambda a, b: math.sqrt(sum(g * g for g in gaps(a, b)))
    mutants = {
        "eta": lambda a, b, eta: eucl(a, b) > 0 and max(a.diam, b.diam) <= eta * eucl(a, b),
        "strict": lambda a, b, eta: eucl(a, b) > 0 and max(a.diam, b.diam) < 2 * eta * eucl(a, b),
        "min_diam": lambda a, b, eta: eucl(a, b) > 0 and min(a.diam, b.diam) <= 2 * eta * eucl(a, b),
        "chebyshev": lambda a, b, eta: max(gaps(a, b)) > 0 and max(a.diam, b.diam) <= 2 * eta * max(gaps(a, b)),
        "manhattan": lambda a, b, eta: sum(gaps(a, b)) > 0 and max(a.diam, b.diam) <= 2 * eta * sum(gaps(a, b)),
        "4eta": lambda a, b, eta: eucl(a, b) > 0 and max(a.diam, b.diam) <= 4 * eta * eucl(a, b),
    }
    for name, fn in mutants.items():
        assert _admissibility_failures(orc, fn), name


@pytest.mark.parametrize("level,leaf", [(3, 32), (5, 64)])
def test_admissible_blocks_keep_sigma_outside_omega(orc, level, leaf):
    """Section 2 needs every admissible sigma outside the closure of omega:
    with the default margin delta = diam(tau) / (4 eta) per side,
    sqrt(3) delta < diam / (2 eta) <= dist(tau, sigma), so the box of sigma
    keeps a positive distance from omega_tau (and omega_sigma from tau)."""
    m = synth.icosphere(level)
    tree = orc.cluster_tree(m.verts, m.tris, leaf)
    eta = 2.0
    far, _ = orc.block_tree(tree, eta)
    assert far
    for (t, s) in far:
        a, b = tree.nodes[t], tree.nodes[s]
        assert max(a.diam, b.diam) <= 2 * eta * orc.box_dist(a, b)
        for u, v in ((a, b), (b, a)):
            d = 0.25 * u.diam / eta
            om = orc.Cluster(0, 1, 0, lo=u.lo - d, hi=u.hi + d, diam=0.0)
            assert orc.box_dist(om, v) > 0, (t, s)
            # the points of omega's faces (the Green points) stay away from sigma
            z, _, _ = orc.green_points(u, 3, eta, omega_scale=0.25)
            inside = np.all((z >= v.lo) & (z <= v.hi), axis=1)
            assert not inside.any()


def test_cluster_diameter_is_the_box_diagonal(orc):
    """Reading s5: d_tau is the Euclidean length of the bounding box's
    diagonal (the same value the admissibility condition uses)."""
    verts, tris = _mesh3()
    tree = orc.cluster_tree(verts, tris, 32)
    for nd in tree.nodes:
        assert nd.diam == pytest.approx(float(np.linalg.norm(nd.hi - nd.lo)), rel=1e-15)


def test_block_tree_tiles_index_square_once(orc):
    """P10: admissible and near blocks cover I x I exactly once; no admissible
    block holds a touching or near-regular pair."""
    verts, tris = _mesh3()
    tree = orc.cluster_tree(verts, tris, 32)
    far, near = orc.block_tree(tree, 2.0)
    n = len(tris)
    cover = np.zeros((n, n), dtype=np.int32)
    for (t, s) in far + near:
        cover[np.ix_(tree.indices(t), tree.indices(s))] += 1
    assert np.all(cover == 1)
    ent = orc.Entries(verts, tris)
    for (t, s) in far:
        I, J = np.meshgrid(tree.indices(t), tree.indices(s), indexing="ij")
        assert np.all(ent.classify(I.ravel(), J.ravel()) == orc.REG)
    assert (set(far) == {(s, t) for (t, s) in far}) and (set(near) == {(s, t) for (t, s) in near})


def test_h2_without_admissible_blocks_is_exact(orc, sphere3_dense):
    """P14: with eta -> 0 nothing is admissible and G~ = G."""
    m, e, G = sphere3_dense
    h = orc.gca_h2(m.verts, m.tris, leaf=32, eta=1e-6, eps=1e-6, ent=e)
    assert not h.far
    x = synth.rhs_normal(m.nt, 1, seed=0)
    np.testing.assert_allclose(orc.h2_matvec(h, x), G @ x, rtol=1e-12, atol=1e-14)


def test_h2_error_follows_tolerance(orc, sphere3_dense):
    """GCA-H^2 converges as eps decreases (Section 4 reports exponential
    convergence); the relative spectral error (power iteration, Section 2)
    tracks eps, the bases satisfy rank <= min(#rows, 2k), and the four-phase
    matrix-vector product agrees with the explicitly assembled H^2 matrix."""
    m, e, G = sphere3_dense
    prev = None
    nG = orc.spectral_norm_sym(lambda v: G @ v, m.nt)
    for eps in (1e-2, 1e-4, 1e-6):
        h = orc.gca_h2(m.verts, m.tris, leaf=32, eta=2.0, eps=eps, ent=e)
        Gt = orc.h2_dense(h)
        D = Gt - G
        err = orc.spectral_norm_sym(lambda v: D @ v, m.nt) / nG
        assert err < 10 * eps, (eps, err)
        if prev is not None:
            assert err < prev / 5
        prev = err
        for c, V in h.V.items():
            assert V.shape[1] <= min(V.shape[0], 108)
        x = synth.rhs_normal(m.nt, 1, seed=0)
        np.testing.assert_allclose(orc.h2_matvec(h, x), Gt @ x, rtol=1e-11, atol=1e-13)
    assert h.far


def test_coupling_rule_order_changes_only_admissible_blocks(orc, sphere3_dense):
    """The coupling matrices G|t~ x s~ (Section 4) are Galerkin entries of
    well-separated pairs; evaluating them with a lower regular order q_c = 2
    changes the assembled matrix on admissible blocks only, by no more than the
    quadrature error of such pairs, and q_c equal to the regular order is the
    default build."""
    m, e, G = sphere3_dense
    h3 = orc.gca_h2(m.verts, m.tris, leaf=32, eta=2.0, eps=1e-6, ent=e)
    hs = orc.gca_h2(m.verts, m.tris, leaf=32, eta=2.0, eps=1e-6, ent=e, q_c=3)
    h2 = orc.gca_h2(m.verts, m.tris, leaf=32, eta=2.0, eps=1e-6, ent=e, q_c=2)
    D3, D2 = orc.h2_dense(h3), orc.h2_dense(h2)
    assert np.array_equal(orc.h2_dense(hs), D3)
    tree = h3.tree
    for (t, s) in h3.near:
        ix = np.ix_(tree.indices(t), tree.indices(s))
        assert np.array_equal(D3[ix], D2[ix])
    changed = 0.0
    for (t, s) in h3.far:
        ix = np.ix_(tree.indices(t), tree.indices(s))
        # an order-6 rule stands in for the exact integral of a separated pair
        changed = max(changed, np.abs(D3[ix] - D2[ix]).max())
    assert changed > 0
    e6 = orc.Entries(m.verts, m.tris, 6, 5, 4)
    t, s = h3.far[0]
    Pt, Ps = h2.pivots[t], h2.pivots[s]
    Bx = e6.block(Pt, Ps)
    assert np.abs(h2.coupling(t, s) - Bx).max() < 1e-3 * np.abs(Bx).max()
    assert np.abs(h3.coupling(t, s) - Bx).max() < np.abs(h2.coupling(t, s) - Bx).max()
    nG = np.linalg.norm(G)
    assert np.linalg.norm(D2 - G) < 1e-3 * nG


def test_h2_nested_basis_matches_direct_interpolation(orc, sphere3_dense):
    """Section 4: V_tau = diag(V_tau1, V_tau2) V^_tau, so the expanded basis is
    the identity on the pivot rows tau~ and V_tau G|tau~ x sigma^ approximates
    G|tau^ x sigma^ on the cluster's admissible columns."""
    m, e, G = sphere3_dense
    h = orc.gca_h2(m.verts, m.tris, leaf=32, eta=2.0, eps=1e-6, ent=e)
    tree = h.tree
    c = next(t for (t, s) in h.far if tree.nodes[t].sons)
    Vc = orc.expanded_basis(h, c)
    idx = tree.indices(c)
    pos = {int(t): k for k, t in enumerate(idx)}
    piv_rows = [pos[int(t)] for t in h.pivots[c]]
    np.testing.assert_allclose(Vc[piv_rows], np.eye(len(piv_rows)), atol=1e-9)
    cols = np.concatenate([tree.indices(s) for (t, s) in h.far if t == c])
    Gb = G[np.ix_(idx, cols)]
    approx = Vc @ G[np.ix_(h.pivots[c], cols)]
    assert np.linalg.norm(Gb - approx) < 1e-4 * np.linalg.norm(Gb)


def test_mesh_generator_counts():
    for lev in range(4):
        m = synth.icosphere(lev)
        assert m.nt == 20 * 4 ** lev and m.nv == 10 * 4 ** lev + 2
        T = m.verts[m.tris]
        s = np.einsum("ij,ij->i", np.cross(T[:, 1] - T[:, 0], T[:, 2] - T[:, 0]), T[:, 0])
        assert np.all(s > 0)
        edges = {tuple(sorted((int(t[a]), int(t[(a + 1) % 3])))) for t in m.tris for a in range(3)}
        assert m.nv - len(edges) + m.nt == 2


# ------------------------------------------------------------- gradients --

def test_entry_gradients_match_central_differences(orc):
    """The analytic pair derivatives (chain rule through the fixed reference
    points and the surface elements) against central differences of the
    oracle's own entries, for every pair class."""
    m = synth.jitter(synth.icosphere(2), 0.01, seed=3)
    e0 = orc.Entries(m.verts, m.tris, 3, 4, 4)
    found = {}
    for j in range(m.nt):
        found.setdefault(int(e0.classify(5, j)[0]), j)
    assert set(found) == {orc.REG, orc.NEAR, orc.VERT, orc.EDGE, orc.IDENT}
    h = 1e-6
    for cls, j in found.items():
        g = e0.entry_grad(5, j)
        scale = np.abs(g).max()
        tris = [5] if j == 5 else [5, j]
        for t in tris:
            for k in range(3):
                v = m.tris[t][k]
                for d in range(3):
                    vp, vm = m.verts.copy(), m.verts.copy()
                    vp[v, d] += h
                    vm[v, d] -= h
                    fd = (orc.Entries(vp, m.tris, 3, 4, 4).entries(5, j)[0]
                          - orc.Entries(vm, m.tris, 3, 4, 4).entries(5, j)[0]) / (2 * h)
                    an = sum(g[side, kk, d] for side, tt in enumerate([5, j]) if not (j == 5 and side == 1)
                             for kk in range(3) if m.tris[tt][kk] == v)
                    assert abs(fd - an) <= 1e-7 * scale, (cls, t, k, d, fd, an)


def test_energy_gradient_invariants(orc):
    """P13 for the dense energy E = 1/2 u^T G u: translation invariance
    (sum of gradients 0), Euler homogeneity of degree 3 (sum X.grad = 3E) and
    rotation invariance (sum X x grad = 0)."""
    m = synth.jitter(synth.icosphere(2), 0.01, seed=4)
    e = orc.Entries(m.verts, m.tris, 3, 4, 4)
    u = synth.rhs_normal(m.nt, 1, seed=2)
    grad = e.energy_grad_vertices(u, np.arange(m.nv))
    E = 0.5 * u @ (e.dense() @ u)
    scale = np.abs(grad).sum() * np.abs(m.verts).max()
    assert np.abs(grad.sum(axis=0)).max() < 1e-12 * np.abs(grad).sum()
    assert abs(np.sum(m.verts * grad) - 3 * E) < 1e-12 * scale
    assert np.abs(np.cross(m.verts, grad).sum(axis=0)).max() < 1e-12 * scale
