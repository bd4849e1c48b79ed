"""Oracle for the continuous piecewise-linear basis on flat triangles (Section 5).

TEST INFRASTRUCTURE ONLY, like the rest of this package: the test-suite, the
smoke check and the bench's CPU baseline leg may use it; the product library
never does, and nothing here is shared with it.

* ``vertex_triangles``: the sets T_i of triangles in the support of the nodal
  basis function of vertex i.
* ``merge_triangle_lists``: the mergesort of Section 5 that unites the sets T_i
  of a vertex subset into one list of triangles, each row carrying, per
  triangle corner, the local index of that corner's vertex in the subset, or
  "bottom" (here -1) when the vertex is not in the subset.  Local indices are
  0-based positions in the subset (the worked example counts from 1).
* ``basis_weights``: the quadrature points of one triangle with the weights
  w_p |J| lambda_a(x_p) of its three nodal functions.
* ``lin_block``: Galerkin entries of the linear nodal basis by their plain
  definition (Section 5): for rows i and columns j, the sum over t in T_i and
  s in T_j of the integral over t of phi_i times the integral over s of
  g(x, y) phi_j(y), with the regular rule of Section 1 on both triangles, and
  for a pair with a common vertex the Sauter-Schwab rules with the nodal
  weights (the C oracle's ``orc_lin_touch_moments``).
"""
from __future__ import annotations

import math

import numpy as np

from . import tri_rule

BOTTOM = -1


def vertex_triangles(tris, nv):
    """T_i for every vertex: sorted triangle ids whose corners include i."""
    T = [[] for _ in range(nv)]
    for t, (a, b, c) in enumerate(np.asarray(tris)):
        for v in {int(a), int(b), int(c)}:
            T[v].append(t)
    return [sorted(x) for x in T]


def _combine(r, s):
    """Two rows of the same triangle: a corner takes the index that is not
    bottom (Section 5)."""
    return (r[0],) + tuple(a if a != BOTTOM else b for a, b in zip(r[1:], s[1:]))


def _merge(left, right):
    out, i, j = [], 0, 0
    while i < len(left) and j < len(right):
        if left[i][0] < right[j][0]:
            out.append(left[i]); i += 1
        elif right[j][0] < left[i][0]:
            out.append(right[j]); j += 1
        else:
            out.append(_combine(left[i], right[j])); i += 1; j += 1
    return out + left[i:] + right[j:]


def _mergesort(lists):
    if not lists:
        return []
    if len(lists) == 1:
        return lists[0]
    h = len(lists) // 2
    return _merge(_mergesort(lists[:h]), _mergesort(lists[h:]))


def merge_triangle_lists(tris, T, subset):
    """Rows (t, l0, l1, l2) sorted by triangle id, one per triangle of the
    union of T_i over the subset: l_c is the position in `subset` of corner c's
    vertex, or -1.  Each vertex starts as its own sorted row list (Section 5,
    worked example), and the lists are merged pairwise, combining the rows of
    a triangle met twice."""
    tris = np.asarray(tris)
    lists = []
    for loc, v in enumerate(subset):
        rows = []
        for t in T[int(v)]:
            rows.append((t,) + tuple(loc if int(tris[t][c]) == int(v) else BOTTOM for c in range(3)))
        lists.append(rows)
    return _mergesort(lists)


def basis_weights(P, q, sym=False):
    """Points x_p of the regular rule on triangle P (3 x 3 vertex rows) and
    W[p, a] = w_p |J| lambda_a(x_p), so that sum_p W[p, a] f(x_p) approximates
    the integral of lambda_a f over the triangle.  The rule lives on the
    reference triangle {0 <= s2 <= s1 <= 1}, x = P0 + s1 (P1 - P0) + s2 (P2 - P1),
    where the barycentric coordinates are (1 - s1, s1 - s2, s2) and |J| is
    twice the area."""
    P = np.asarray(P, dtype=np.float64)
    s1, s2, w = tri_rule(q, sym)
    J = np.linalg.norm(np.cross(P[1] - P[0], P[2] - P[1]))
    lam = np.stack([1.0 - s1, s1 - s2, s2], axis=1)
    x = P[0][None, :] + s1[:, None] * (P[1] - P[0])[None, :] + s2[:, None] * (P[2] - P[1])[None, :]
    return x, (w * J)[:, None] * lam


def lin_block(verts, tris, rows, cols, q, sym=False, T=None, q_s=None):
    """Dense block (len(rows) x len(cols)) of the linear-basis Galerkin matrix
    by the plain definition.  A triangle pair with a common vertex (identical,
    common edge, common vertex) takes the Sauter-Schwab rules of order q_s with
    the nodal weights (``Entries.lin_touch_moments``); without q_s such a pair
    raises ValueError."""
    verts = np.asarray(verts, dtype=np.float64)
    tris = np.asarray(tris)
    if T is None:
        T = vertex_triangles(tris, verts.shape[0])
    cache = {}
    ss = {}

    def touch(t, s):
        if "e" not in ss:
            from . import Entries
            ss["e"] = Entries(verts, tris, q, q, q_s, sym=sym)
        if (t, s) not in ss:
            ss[(t, s)] = ss["e"].lin_touch_moments(t, s)
        return ss[(t, s)]

    def bw(t):
        if t not in cache:
            cache[t] = basis_weights(verts[tris[t]], q, sym)
        return cache[t]

    out = np.zeros((len(rows), len(cols)))
    for ii, i in enumerate(rows):
        for jj, j in enumerate(cols):
            acc = 0.0
            for t in T[int(i)]:
                a = list(tris[t]).index(int(i))
                x, Wt = bw(t)
                for s in T[int(j)]:
                    b = list(tris[s]).index(int(j))
                    if set(map(int, tris[t])) & set(map(int, tris[s])):
                        if q_s is None:
                            raise ValueError("triangles %d and %d share a vertex" % (t, s))
                        acc += 4.0 * math.pi * touch(int(t), int(s))[a, b]
                        continue
                    y, Ws = bw(s)
                    d = x[:, None, :] - y[None, :, :]
                    g = 1.0 / np.sqrt((d * d).sum(axis=2))
                    acc += Wt[:, a] @ g @ Ws[:, b]
            out[ii, jj] = acc / (4.0 * math.pi)
    return out
