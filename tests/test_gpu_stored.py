"""Stored-block mode (gca_store_blocks): the coupling and nearfield block
rows computed once and read by the product, against the recomputing product
and the dense oracle."""
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


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("params", [dict(eta=2.0, eps=1e-6), dict(eta=2.0, eps=1e-6, q_nr=4),
                                    dict(eta=1e-3, eps=1e-6)])
def test_stored_product_equals_recomputed_and_dense(torch, gca, orc, params):
    """Level-3 sphere (n = 1280, leaf 32; several blocks per row, ragged
    ranks): the stored product equals the recomputing one to rounding in
    both precisions and the dense oracle to the compression tolerance; the
    third case has no admissible blocks, the second a near-regular list."""
    m = synth.icosphere(3)
    p = gca.Params(**params)
    H = gca.H2(m.verts, m.tris, gca.Tree(m.verts, m.tris, 32), p)
    X = torch.tensor(synth.rhs_normal(m.nt, 2, seed=3), device="cuda")
    y64 = H.matvec(X, gca.FP64).cpu().numpy()
    y32 = H.matvec(X, gca.MIXED).cpu().numpy()
    H.store_blocks(fp64=True, mixed=True)
    st = H.stats()
    assert st["stored_mask"] == 3 and st["store_entries_near"] > 0
    s64 = H.matvec(X, gca.FP64).cpu().numpy()
    s32 = H.matvec(X, gca.MIXED).cpu().numpy()
    assert rel(s64, y64) < 1e-13
    assert rel(s32, y32) < 1e-6
    G = orc.Entries(m.verts, m.tris, p.q_r, p.q_nr, p.q_s).dense()
    ref = G @ X.cpu().numpy()
    assert rel(s64, ref) < 10 * p.eps + 1e-12
    assert rel(s32, ref) < 10 * p.eps + 1e-5
    # release: back to recomputation, same result bitwise
    H.store_blocks(False, False)
    assert H.stats()["stored_mask"] == 0
    assert np.array_equal(H.matvec(X, gca.FP64).cpu().numpy(), y64)


def test_stored_single_precision_and_geometry_update(torch, gca):
    """Only the mixed copy stored: FP64 products keep recomputing; after a
    geometry update the stored entries follow the new vertices."""
    base = synth.icosphere(3)
    m = synth.jitter(base, 0.02 * synth.mean_edge_length(base), seed=4)
    H = gca.H2(m.verts, m.tris, gca.Tree(m.verts, m.tris, 32), gca.Params(eta=2.0, eps=1e-6))
    x = torch.tensor(synth.rhs_normal(m.nt, 1, seed=5), device="cuda")
    y64 = H.matvec(x, gca.FP64).cpu().numpy()
    H.store_blocks(fp64=False, mixed=True)
    assert H.stats()["stored_mask"] == 2
    assert np.array_equal(H.matvec(x, gca.FP64).cpu().numpy(), y64)
    moved = m.verts * 1.01 + np.array([0.0, 2e-3, -1e-3])
    H.update_geometry(moved)
    s32 = H.matvec(x, gca.MIXED).cpu().numpy()
    H.store_blocks(False, False)
    r32 = H.matvec(x, gca.MIXED).cpu().numpy()
    assert rel(s32, r32) < 1e-6


def test_store_rejects_unknown_bits(torch, gca):
    m = synth.icosphere(2)
    H = gca.H2(m.verts, m.tris, gca.Tree(m.verts, m.tris, 16), gca.Params(eps=1e-6))
    with pytest.raises(gca.Error) as e:
        gca._check(gca.lib().gca_store_blocks(H.h, 4, None))
    assert e.value.code == -1
    assert H.stats()["stored_mask"] == 0
