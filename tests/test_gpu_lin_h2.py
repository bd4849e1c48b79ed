"""GPU parity of the nodal-basis GCA-H^2 handle (gca_lin_build /
gca_lin_matvec; Sections 2-5 over the vertices) against the step-by-step
oracle (oracle/linear_h2.py): the vertex tree, the ranks and the pivots of
every cluster exactly, the product to 1e-10; with eta -> 0 the product of the
dense nodal matrix (touching pairs by Sauter-Schwab) to 1e-12; the
approximation error against the dense matrix; bit equality between
products; coupling blocks applied in several column pieces (level 5)."""
import numpy as np
import pytest

import synth
import oracle
from oracle import linear_h2 as LH

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_1810_08429_amd as g
    g.lib()
    return g, torch


@pytest.fixture(scope="module")
def l3():
    m = synth.jitter(synth.icosphere(3), 0.002, seed=4)
    return m, LH.lin_dense(m.verts, m.tris, 3, False, 5)


def _params(g, **kw):
    base = dict(eta=2.0, eps=1e-4, green_m=3, q_A=3, q_r=3, q_nr=3, q_s=5, q_c=3)
    base.update(kw)
    return g.Params(**base)


@pytest.mark.parametrize("eps", [1e-2, 1e-4])
def test_lin_h2_equals_oracle(env, l3, eps):
    g, torch = env
    m, G = l3
    H = g.LinH2(m.verts, m.tris, leaf=16, params=_params(g, eps=eps))
    ref = LH.gca_lin_h2(m.verts, m.tris, leaf=16, eta=2.0, m=3, eps=eps, q_A=3, q=3, q_s=5, Gnear=G)
    perm, ranks, piv = H.export()
    assert np.array_equal(perm, ref.tree.perm)
    assert len(ranks) == len(ref.tree.nodes)
    for c in range(len(ranks)):
        assert np.array_equal(piv[c], ref.pivots[c]), c
    inf = H.info()
    assert inf["far_blocks"] == 2 * len([b for b in ref.far if b[0] < b[1]]) and inf["far_blocks"] == len(ref.far)
    assert inf["near_blocks"] == len(ref.near)
    x = synth.rhs_normal(m.nv, seed=3)
    y = H.matvec(torch.as_tensor(x).cuda()).cpu().numpy()
    yo = oracle.h2_matvec(ref, x)
    assert np.abs(y - yo).max() <= 1e-10 * np.abs(yo).max()
    err = np.abs(y - G @ x).max() / np.abs(G @ x).max()
    assert err < 10 * eps, err
    y2 = H.matvec(torch.as_tensor(x).cuda()).cpu().numpy()
    assert np.array_equal(y, y2)


def test_lin_h2_eta_zero_is_the_dense_matrix(env, l3):
    g, torch = env
    m, G = l3
    H = g.LinH2(m.verts, m.tris, leaf=16, params=_params(g, eta=1e-9))
    assert H.info()["far_blocks"] == 0
    for seed in (0, 1):
        x = synth.rhs_normal(m.nv, seed=seed)
        y = H.matvec(torch.as_tensor(x).cuda()).cpu().numpy()
        assert np.abs(y - G @ x).max() <= 1e-12 * np.abs(G @ x).max()
    # the smooth vectors too: the all-ones vector
    y = H.matvec(torch.ones(m.nv, dtype=torch.float64).cuda()).cpu().numpy()
    assert np.abs(y - G.sum(axis=1)).max() <= 1e-12 * np.abs(G.sum(axis=1)).max()


def test_lin_h2_symmetric_rules_and_coupling_order(env):
    g, torch = env
    m = synth.jitter(synth.icosphere(2), 0.004, seed=9)
    Gn = LH.lin_dense(m.verts, m.tris, 3, True, 4)
    Gc = LH.lin_dense(m.verts, m.tris, 2, True, 4)
    H = g.LinH2(m.verts, m.tris, leaf=8, params=_params(g, q_s=4, q_c=2, sym_rules=1, eps=1e-6))
    ref = LH.gca_lin_h2(m.verts, m.tris, leaf=8, eta=2.0, m=3, eps=1e-6, q_A=3, q=3, q_s=4, q_c=2, sym=True,
                        Gnear=Gn, Gcoup=Gc)
    assert H.info()["far_blocks"] > 0
    x = synth.rhs_normal(m.nv, seed=5)
    y = H.matvec(torch.as_tensor(x).cuda()).cpu().numpy()
    yo = oracle.h2_matvec(ref, x)
    assert np.abs(y - yo).max() <= 1e-10 * np.abs(yo).max()


def test_lin_h2_large_coupling_blocks_in_pieces(env):
    """Level-5 sphere (10,242 vertices) with the measured workload's settings
    (leaf 32, Green order 4, eps 1e-5, q_A 2, symmetric rules, coupling
    order 2): some coupling blocks exceed 4,096 entries and are applied in
    several column pieces.  The product equals that of the same handle with
    eta -> 0 (every block stored dense, pinned to the oracle at level 3) to
    the compression tolerance, and is bit-equal on a second call."""
    g, torch = env
    m = synth.icosphere(5)
    kw = dict(eps=1e-5, green_m=4, q_A=2, q_r=3, q_nr=3, q_s=4, q_c=2, sym_rules=1)
    H = g.LinH2(m.verts, m.tris, leaf=32, params=_params(g, **kw))
    perm, ranks, _ = H.export()
    tree = LH.vertex_cluster_tree(m.verts, m.tris, 32)
    assert np.array_equal(perm, tree.perm)
    far, _ = oracle.block_tree(tree, 2.0)
    assert max(int(ranks[t]) * int(ranks[s]) for t, s in far) > 4096
    H0 = g.LinH2(m.verts, m.tris, leaf=32, params=_params(g, eta=1e-9, **kw))
    assert H0.info()["far_blocks"] == 0
    for x in (torch.as_tensor(synth.rhs_normal(m.nv, seed=6)).cuda(), torch.ones(m.nv, dtype=torch.float64).cuda()):
        y, y0 = H.matvec(x), H0.matvec(x)
        err = float((y - y0).abs().max() / y0.abs().max())
        print(f"[lin-h2 pieces] rel err {err:.2e}", flush=True)
        assert err < 5e-4, err
        assert torch.equal(y, H.matvec(x))
