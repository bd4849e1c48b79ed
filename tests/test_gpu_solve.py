"""Conjugate gradients on the mixed-precision H^2 product inside FP64
iterative refinement (gca_solve_refined), checked against the oracle."""
import math

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


@pytest.fixture(scope="module")
def gca():
    import paper_1810_08429_amd as g
    g.lib()
    return g


def areas_centroids(m):
    T = m.verts[m.tris]
    area = 0.5 * np.linalg.norm(np.cross(T[:, 1] - T[:, 0], T[:, 2] - T[:, 0]), axis=1)
    return area, T.mean(axis=1)


def test_solve_matches_dense_cholesky(torch, gca, orc):
    """n = 1280: the refined solve reaches 1e-8 against its own FP64 operator
    and agrees with the oracle's dense Cholesky solution to the compression
    error amplified by the condition number."""
    m = synth.icosphere(3)
    p = gca.Params(eta=2.0, eps=1e-6)
    H = gca.H2(m.verts, m.tris, gca.Tree(m.verts, m.tris, 32), p)
    area, c = areas_centroids(m)
    f = area * c[:, 2]                      # int_{t_i} x_3 dx, exact for a linear function
    u, outer, inner, rel = H.solve(torch.tensor(f, device="cuda"), rtol=1e-8)
    assert rel <= 1e-8 and outer >= 1 and inner >= 1
    G = orc.Entries(m.verts, m.tris, p.q_r, p.q_nr, p.q_s).dense()
    L = np.linalg.cholesky(G)
    ud = np.linalg.solve(L.T, np.linalg.solve(L, f))
    uu = u.cpu().numpy()
    assert np.linalg.norm(uu - ud) / np.linalg.norm(ud) < 1e-4
    # residual against the dense matrix: H^2 error only
    assert np.linalg.norm(G @ uu - f) / np.linalg.norm(f) < 1e-5


def test_solve_recovers_sphere_harmonic(torch, gca):
    """P4: on the unit sphere V x_3 = x_3 / 3, so u_i -> 3 (c_i)_3 at first
    order in h (error falls ~2x per refinement level)."""
    errs = []
    for lev in (3, 4, 5):
        m = synth.icosphere(lev)
        H = gca.H2(m.verts, m.tris, gca.Tree(m.verts, m.tris, 64 if lev > 3 else 32),
                   gca.Params(eta=2.0, eps=1e-6))
        area, c = areas_centroids(m)
        u, outer, inner, rel = H.solve(torch.tensor(area * c[:, 2], device="cuda"), rtol=1e-8)
        assert rel <= 1e-8
        uu = u.cpu().numpy()
        exact = 3.0 * c[:, 2]
        errs.append(math.sqrt(np.sum(area * (uu - exact) ** 2) / np.sum(area * exact ** 2)))
        H.close()
    assert errs[-1] < 0.05
    for a, b in zip(errs, errs[1:]):
        assert 1.5 < a / b < 4.5, errs


def test_solve_zero_rhs_and_bad_arguments(torch, gca):
    m = synth.icosphere(3)
    H = gca.H2(m.verts, m.tris, gca.Tree(m.verts, m.tris, 32), gca.Params(eps=1e-6))
    u, outer, inner, rel = H.solve(torch.zeros(m.nt, dtype=torch.float64, device="cuda"))
    assert outer == 0 and rel == 0.0 and torch.count_nonzero(u) == 0
    with pytest.raises(gca.Error) as e:
        H.solve(torch.ones(m.nt, dtype=torch.float64, device="cuda"), rtol=0.0)
    assert e.value.code == -1
    # an iteration budget that cannot reach the tolerance reports GCA_ENOCONV
    with pytest.raises(gca.Error) as e:
        H.solve(torch.ones(m.nt, dtype=torch.float64, device="cuda"), rtol=1e-12, max_outer=1, max_inner=2)
    assert e.value.code == -6
