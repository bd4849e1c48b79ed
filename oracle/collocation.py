"""Oracle for collocation with the continuous piecewise-linear nodal basis on
flat triangles (Section 6, the collocation paragraph).

TEST INFRASTRUCTURE ONLY, like the rest of this package: the test-suite, the
smoke check and the bench's CPU baseline leg may use it; the product library
never does, and nothing here is shared with it.

The collocation matrix has one row per collocation point x_i, a vertex of the
mesh, and one column per nodal basis function phi_j:

    g_ij = int_Gamma g(x_i, y) phi_j(y) dy,   g(x, y) = 1 / (4 pi |x - y|),

a single integral, summed here over the triangles t of the support of phi_j
(the sets T_j of Section 5), with phi_j = lambda_{t,j} (the barycentric
coordinate of corner j) on t.

* A triangle that has x_i as a corner: the integrand is singular at that
  corner, and the Duffy transformation that collapses the unit square onto
  the triangle at x_i,  y(u, v) = x_i + u ((a - x_i) + v (b - a)),  dy = 2|t| u
  du dv, cancels the 1 / |x_i - y| = 1 / (u |(a - x_i) + v (b - a)|); the
  resulting smooth integrand is integrated by the tensor Gauss-Legendre rule
  of order q_s in (u, v).  a, b are the other two corners, in the cyclic mesh
  order after x_i.
* Any other triangle: the regular triangle rule of order q (the collapsed
  Gauss rule of Section 1, or the symmetric rule of the same degree), with
  lambda_{t,j} at the rule's points.

The class of a (point, triangle) pair is decided from vertex ids alone.
"""
from __future__ import annotations

import math

import numpy as np

from . import gauss01, tri_rule

INV4PI = 1.0 / (4.0 * math.pi)


def duffy_moments(x, a, b, q_s):
    """int_t g(x, y) lambda_c(y) dy over t = (x, a, b) for its corners
    c = x, a, b (x a corner of t), by the Duffy transformation at x and the
    q_s x q_s tensor Gauss rule on the unit square."""
    x, a, b = (np.asarray(p, dtype=np.float64) for p in (x, a, b))
    area2 = np.linalg.norm(np.cross(a - x, b - x))   # 2 |t|
    g, w = gauss01(q_s)
    m = np.zeros(3)
    for u, wu in zip(g, w):
        for v, wv in zip(g, w):
            d = (a - x) + v * (b - a)
            y = x + u * d
            r = np.linalg.norm(y - x)
            # barycentric coordinates of y: lambda_x = 1 - u, lambda_a = u (1 - v), lambda_b = u v
            lam = np.array([1.0 - u, u * (1.0 - v), u * v])
            jac = area2 * u
            m += wu * wv * jac * INV4PI / r * lam
    return m


def regular_moments(x, p0, p1, p2, q, sym=False):
    """int_t g(x, y) lambda_c(y) dy, c = 0, 1, 2 (corners p0, p1, p2), by the
    regular rule of order q on t = (p0, p1, p2): chi(s) = p0 + s1 (p1 - p0) +
    s2 (p2 - p1), lambda = (1 - s1, s1 - s2, s2), |J| = 2 |t|."""
    x, p0, p1, p2 = (np.asarray(p, dtype=np.float64) for p in (x, p0, p1, p2))
    area2 = np.linalg.norm(np.cross(p1 - p0, p2 - p0))
    s1, s2, w = tri_rule(q, sym)
    m = np.zeros(3)
    for a, b, wk in zip(s1, s2, w):
        y = p0 + a * (p1 - p0) + b * (p2 - p1)
        lam = np.array([1.0 - a, a - b, b])
        m += wk * area2 * INV4PI / np.linalg.norm(x - y) * lam
    return m


def point_triangle_moments(verts, tri, i, q, q_s, sym=False):
    """The three corner moments of triangle `tri` (vertex ids, mesh order) at
    the collocation point x_i, in the corner order of `tri`."""
    tri = [int(v) for v in tri]
    P = [verts[v] for v in tri]
    if i in tri:
        k = tri.index(i)
        a, b = (k + 1) % 3, (k + 2) % 3
        md = duffy_moments(P[k], P[a], P[b], q_s)
        m = np.zeros(3)
        m[k], m[a], m[b] = md
        return m
    return regular_moments(verts[i], P[0], P[1], P[2], q, sym)


def coll_entry(verts, tris, T, i, j, q=3, q_s=4, sym=False):
    """g_ij by its definition: the sum over t in T_j (ascending) of the
    moment of corner j of t at x_i.  T: the sets T_j (vertex_triangles)."""
    verts = np.asarray(verts, dtype=np.float64)
    s = 0.0
    for t in T[j]:
        tri = [int(v) for v in tris[t]]
        s += point_triangle_moments(verts, tri, i, q, q_s, sym)[tri.index(j)]
    return s


def coll_block(verts, tris, T, rows, cols, q=3, q_s=4, sym=False):
    """Dense block g(rows[k], cols[l]) of the collocation matrix."""
    out = np.zeros((len(rows), len(cols)))
    for a, i in enumerate(rows):
        for b, j in enumerate(cols):
            out[a, b] = coll_entry(verts, tris, T, int(i), int(j), q, q_s, sym)
    return out
