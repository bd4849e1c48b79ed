"""Oracle for curved (quadratic) triangles (Section 6): Galerkin moments of
the single- and double-layer kernels with the mapped nodal basis functions,
by the definition written out in gca_oracle.c (orc_curved_*).

TEST INFRASTRUCTURE ONLY, like the rest of this package: the test-suite, the
smoke check and the bench's CPU baseline leg may use it; the product library
never does, and nothing here is shared with it.

A triangle is given by six nodes: its corners X0, X1, X2 and one point per
edge X0-X1, X1-X2, X2-X0, interpolated at the edge midpoints by the
quadratic map Phi_t of the reference triangle; gamma_t = |dPhi/ds1 x
dPhi/ds2| is the Gramian.  The moments of a pair (t, s),

    M[a][b] = int int l_a(x) k(Phi_t(x), Phi_s(y)) l_b(y) gamma_t gamma_s,

with l_a the barycentric coordinates of the reference point (the mapped
nodal functions), a and b the corners in mesh order, k = g (op 0) or the
double-layer kernel n_s(y) . (x - y) / (4 pi |x - y|^3) with the unit normal
of the mesh orientation (op 1).  The piecewise-constant entry is the sum of
the nine.  Touching pairs (shared corners) take the Sauter-Schwab maps with
q_s Gauss points per variable, the others the regular triangle rule of order
q_r (collapsed, or the symmetric rules with sym).
"""
from __future__ import annotations

import numpy as np

from . import _load, _ptr

SINGLE, DOUBLE = 0, 1


class Curved:
    def __init__(self, nodes, tris6, q_r, q_s, sym=False):
        self.lib = _load()
        self.nodes = np.ascontiguousarray(nodes, dtype=np.float64)
        self.tris = np.ascontiguousarray(tris6, dtype=np.int32)
        assert self.tris.ndim == 2 and self.tris.shape[1] == 6
        self.nt = self.tris.shape[0]
        self.h = self.lib.orc_curved_create(self.nodes.shape[0], self.nt, _ptr(self.nodes), _ptr(self.tris),
                                            int(q_r), int(q_s), int(bool(sym)))
        if not self.h:
            raise ValueError("unsupported rule orders")

    def __del__(self):
        if getattr(self, "h", None):
            self.lib.orc_curved_destroy(self.h)
            self.h = None

    def classify(self, t, s):
        return int(self.lib.orc_curved_classify(self.h, int(t), int(s)))

    def moments(self, I, J, op=SINGLE):
        """(m, 3, 3) moments of the pairs (I[k], J[k])."""
        I = np.ascontiguousarray(np.atleast_1d(I), dtype=np.int64)
        J = np.ascontiguousarray(np.atleast_1d(J), dtype=np.int64)
        out = np.zeros((I.size, 9))
        self.lib.orc_curved_moments_many(self.h, int(op), I.size, _ptr(I), _ptr(J), _ptr(out))
        return out.reshape(-1, 3, 3)

    def entries(self, I, J, op=SINGLE):
        """Piecewise-constant entries: the sums of the moments."""
        return self.moments(I, J, op).sum(axis=(1, 2))

    def block(self, rows, cols, op=SINGLE):
        rows = np.asarray(rows, dtype=np.int64)
        cols = np.asarray(cols, dtype=np.int64)
        return self.entries(np.repeat(rows, cols.size), np.tile(cols, rows.size), op).reshape(rows.size, cols.size)

    def mass(self, t, q=8):
        """int_t phi_a for the three corners of t (their sum: the area of t)."""
        m = np.zeros(3)
        self.lib.orc_curved_mass(self.h, int(t), int(q), _ptr(m))
        return m
