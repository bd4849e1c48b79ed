"""Pins of the collocation oracle (Section 6, collocation with the
piecewise-linear nodal basis and a Duffy-regularised single integral).
CPU only.

* The Duffy rule at a corner against closed forms: in polar coordinates
  around the corner A of t = (A, B, C), the integral of 1/r over t is the
  integral over the angle of the distance R(phi) = d sec(phi) to the opposite
  edge (d: distance from A to the line BC, phi measured from the foot of the
  perpendicular), and a barycentric weight that is linear along each ray
  integrates to R/2 times its value on BC.  With sec and sec tan integrated
  in closed form (asinh(tan phi) and sec phi) this gives every corner moment
  exactly; the 4D-free Duffy rule must converge to it.
* The regular rule against brute force: 4^k congruent subtriangles with the
  centroid rule, Richardson-extrapolated over two levels (independent of the
  oracle's triangle rules).
* The sphere potential: the nodal functions sum to one, so the row sums of
  the collocation matrix are the potential of the uniform unit density on
  the polyhedral sphere at its vertices, which tends to r = 1 (a uniform
  shell of radius 1 has potential 1 on its surface) at second order in h.
* Homogeneity g(lambda X) = lambda g(X), translation invariance, and the
  singular case decided by vertex ids.
"""
import math

import numpy as np
import pytest

import synth
from oracle import collocation as C
from oracle.linear import vertex_triangles


def closed_moments(A, B, Cc):
    """(M_A, M_B, M_C) = int_t g(A, y) lambda_c(y) dy by the polar closed form."""
    A, B, Cc = (np.asarray(p, dtype=np.float64) for p in (A, B, Cc))
    L = np.linalg.norm(Cc - B)
    e = (Cc - B) / L
    F = B + np.dot(A - B, e) * e
    d = np.linalg.norm(A - F)
    tB, tC = np.dot(B - F, e), np.dot(Cc - F, e)
    ash = math.asinh(tC / d) - math.asinh(tB / d)
    sec = math.sqrt(1 + (tC / d) ** 2) - math.sqrt(1 + (tB / d) ** 2)
    total = d * ash / (4 * math.pi)
    mb = (tC * d * ash - d * d * sec) / (8 * math.pi * L)
    mc = (-tB * d * ash + d * d * sec) / (8 * math.pi * L)
    return np.array([total / 2, mb, mc])


# (corner A, B, C), Gauss order at which the Duffy rule meets the closed form to 1e-10
TRIANGLES = [
    ([[0, 0, 0], [1, 0, 0], [0, 1, 0]], 16),                     # right angle at the singular corner
    ([[0.1, 0.2, 0.3], [1.3, 0.1, 0.2], [0.4, 1.7, -0.3]], 16),   # scalene, off the axes
    ([[0, 0, 0], [2, 0, 0], [1.9, 0.3, 0.1]], 16),               # thin, acute at A
    # obtuse at A: A lies close to the line BC, so 1/|d(v)| is sharply peaked in v
    # and the Gauss rule converges slowly (1e-3 at order 16)
    ([[0, 0, 0], [1, 0, 0], [-0.8, 0.3, 0]], 64),
]


@pytest.mark.parametrize("tri,q", TRIANGLES)
def test_duffy_moments_equal_the_closed_form(tri, q):
    ref = closed_moments(*tri)
    # the weight of the singular corner is 1 - r/R along each ray: half of the total
    assert abs(ref[1] + ref[2] - ref[0]) < 1e-14 * ref[0]
    m = C.duffy_moments(*tri, q)
    assert np.abs(m - ref).max() < 1e-10 * np.abs(ref).max()
    # a weight placed on the wrong corner is far off
    assert np.abs(m[[1, 2, 0]] - ref).max() > 1e-3 * np.abs(ref).max()
    errs = [np.abs(C.duffy_moments(*tri, k) - ref).max() for k in (2, 4, 8)]
    assert errs[0] > errs[1] > errs[2] or errs[2] < 1e-14


def brute_force_moments(x, p0, p1, p2, k):
    """Centroid rule on 4^k congruent subtriangles (corner moments)."""
    x, p0, p1, p2 = (np.asarray(p, dtype=np.float64) for p in (x, p0, p1, p2))
    n = 2 ** k
    area = 0.5 * np.linalg.norm(np.cross(p1 - p0, p2 - p0)) / (n * n)
    m = np.zeros(3)
    # barycentric grid: upright and inverted subtriangles
    for i in range(n):
        for j in range(n - i):
            for cen in ([(i + 1 / 3) / n, (j + 1 / 3) / n], [(i + 2 / 3) / n, (j + 2 / 3) / n]):
                a, b = cen
                if a + b > 1 + 1e-12:
                    continue
                lam = np.array([1 - a - b, a, b])
                y = lam[0] * p0 + lam[1] * p1 + lam[2] * p2
                m += area * lam / (4 * math.pi * np.linalg.norm(x - y))
    return m


@pytest.mark.parametrize("x", [[0.3, 0.3, 0.4], [2.0, -1.0, 0.5], [0.5, 0.5, 0.15]])
def test_regular_moments_against_subdivision(x):
    p = [[0.0, 0.0, 0.0], [1.0, 0.1, 0.0], [0.2, 0.9, 0.1]]
    i5, i6 = brute_force_moments(x, *p, 5), brute_force_moments(x, *p, 6)
    ref = (4 * i6 - i5) / 3
    near = x[2] < 0.2
    # the near point (0.1 from the plane, over the triangle) needs a high order
    m = C.regular_moments(x, *p, 20 if near else 12)
    assert np.abs(m - ref).max() < (1e-4 if near else 1e-7) * np.abs(ref).max()
    # a permuted weight is far off
    assert np.abs(m[[1, 2, 0]] - ref).max() > 1e-3 * np.abs(ref).max()
    # both rule families converge to the same integral as the order grows
    err = lambda q, sym: np.abs(C.regular_moments(x, *p, q, sym=sym) - ref).max()
    assert err(2, False) > err(4, False) > err(8, False)
    assert err(2, True) > err(3, True)


def test_sphere_potential_at_the_vertices_converges_to_one():
    devs = []
    for level in (1, 2, 3):
        m = synth.icosphere(level)
        rows = [0, m.nv // 3, m.nv - 1]
        dev = 0.0
        for i in rows:
            s = sum(C.point_triangle_moments(m.verts, t, i, 4, 8).sum() for t in m.tris)
            dev = max(dev, abs(s - 1.0))
        devs.append(dev)
    assert devs[-1] < 1e-2
    for a, b in zip(devs, devs[1:]):
        assert 3.0 < a / b < 5.0, devs


def test_row_sums_are_the_sums_of_the_entries():
    m = synth.icosphere(1)
    T = vertex_triangles(m.tris, m.nv)
    G = C.coll_block(m.verts, m.tris, T, range(m.nv), range(m.nv), 3, 6)
    for i in (0, 7):
        s = sum(C.point_triangle_moments(m.verts, t, i, 3, 6).sum() for t in m.tris)
        assert abs(G[i].sum() - s) < 1e-14 * s
    # not symmetric (collocation), positive entries
    assert np.all(G > 0) and np.abs(G - G.T).max() > 1e-6


def test_homogeneity_translation_and_singular_class():
    m = synth.icosphere(1)
    T = vertex_triangles(m.tris, m.nv)
    rows, cols = [0, 3, 5], [0, 1, 3, 9]
    G = C.coll_block(m.verts, m.tris, T, rows, cols, 3, 6)
    G2 = C.coll_block(2.5 * m.verts, m.tris, T, rows, cols, 3, 6)
    Gt = C.coll_block(m.verts + np.array([0.3, -1.0, 2.0]), m.tris, T, rows, cols, 3, 6)
    assert np.abs(G2 - 2.5 * G).max() < 1e-13 * np.abs(G).max()
    assert np.abs(Gt - G).max() < 1e-12 * np.abs(G).max()
    # a triangle with the point as a corner is integrated with the Duffy rule
    t = m.tris[T[0][0]]
    k = list(t).index(0)
    md = C.duffy_moments(m.verts[t[k]], m.verts[t[(k + 1) % 3]], m.verts[t[(k + 2) % 3]], 6)
    assert np.isclose(C.point_triangle_moments(m.verts, t, 0, 3, 6)[k], md[0], rtol=1e-15)
