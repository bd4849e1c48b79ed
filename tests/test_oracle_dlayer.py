"""Pins of the double-layer oracle (Section 1's second-kind formulation with
the normal derivative of g at y; unit normals of the flat triangles):
k_ij = int_{t_i} int_{t_j} n_j . (x - y) / (4 pi |x - y|^3) dy dx.  CPU only.

* Gauss' law: for a closed polyhedron with outward normals the double-layer
  potential of the unit density is -1/2 at every point inside a face (the
  face itself contributes nothing, and the solid angle the rest subtends is
  the half space's), so every row sum equals -|t_i| / 2 exactly, up to the
  quadrature error alone; checked on a sphere and an ellipsoid, converging to
  rounding as the orders grow.  A wrong sign, a missing 1/(4 pi), the normal
  of the other triangle or the wrong power of |x - y| all break it.
* Coplanar pairs are 0 (identical pairs, and every pair of a flat patch).
* Homogeneity k(lambda X) = lambda^2 k(X), translation invariance, and the sign
  change of column j when t_j's orientation is reversed.
"""
import numpy as np
import pytest

import synth


def areas(m):
    T = m.verts[m.tris]
    return 0.5 * np.linalg.norm(np.cross(T[:, 1] - T[:, 0], T[:, 2] - T[:, 0]), axis=1)


@pytest.mark.parametrize("mesh", ["sphere", "ellipsoid"])
def test_gauss_law_row_sums(orc, mesh):
    m = synth.icosphere(2) if mesh == "sphere" else synth.ellipsoid(2)
    a = areas(m)
    rows = [0, 7, m.nt // 2, m.nt - 1]
    errs = []
    for q in ((3, 3, 4), (5, 5, 8), (16, 16, 24)):
        e = orc.Entries(m.verts, m.tris, *q)
        K = e.dl_block(rows, np.arange(m.nt))
        errs.append(np.abs(K.sum(axis=1) / a[rows] + 0.5).max())
    assert errs[0] < 1e-4 and errs[-1] < 1e-12
    assert errs[0] > errs[1] > errs[2]


def test_identical_and_coplanar_pairs_are_zero(orc):
    # a flat patch: a 5 x 5 grid of squares in the plane z = 0.3, two triangles each
    g = np.stack(np.meshgrid(np.arange(6.0), np.arange(6.0), indexing="ij"), -1).reshape(-1, 2) * 0.2
    verts = np.column_stack([g, np.full(len(g), 0.3)])
    tris = []
    for i in range(5):
        for j in range(5):
            a, b, c, d = 6 * i + j, 6 * (i + 1) + j, 6 * (i + 1) + j + 1, 6 * i + j + 1
            tris += [[a, b, c], [a, c, d]]
    tris = np.array(tris)
    e = orc.Entries(verts, tris, 3, 3, 4)
    K = e.dl_block(np.arange(len(tris)), np.arange(len(tris)))
    assert np.abs(K).max() < 1e-16
    m = synth.icosphere(2)
    e2 = orc.Entries(m.verts, m.tris, 3, 3, 4)
    assert np.all(e2.dl_entries(np.arange(m.nt), np.arange(m.nt)) == 0.0)


def test_homogeneity_translation_and_orientation(orc):
    m = synth.jitter(synth.icosphere(2), 0.01, seed=3)
    rows, cols = np.arange(0, m.nt, 17), np.arange(0, m.nt, 13)
    K = orc.Entries(m.verts, m.tris, 3, 3, 4).dl_block(rows, cols)
    K2 = orc.Entries(1.7 * m.verts, m.tris, 3, 3, 4).dl_block(rows, cols)
    Kt = orc.Entries(m.verts + np.array([2.0, -1.0, 0.5]), m.tris, 3, 3, 4).dl_block(rows, cols)
    scale = np.abs(K).max()
    assert np.abs(K2 - 1.7 ** 2 * K).max() < 1e-13 * scale
    assert np.abs(Kt - K).max() < 1e-12 * scale
    # reversing the orientation of t_j (swapping two of its vertices) negates n_j: the
    # regular entries of column j change sign exactly
    j = int(cols[3])
    flipped = m.tris.copy()
    flipped[j] = flipped[j][[0, 2, 1]]
    e, ef = orc.Entries(m.verts, m.tris, 3, 3, 4), orc.Entries(m.verts, flipped, 3, 3, 4)
    far = [i for i in rows if e.classify(i, j) == orc.REG]
    assert len(far) > 5
    a, b = e.dl_entries(far, j), ef.dl_entries(far, j)
    assert np.abs(a + b).max() < 1e-13 * np.abs(a).max()
