"""GPU parity of the double-layer entries (gca_dl_entries) through the C-ABI
against the oracle's (same rules per Sauter case): every class, both orders
of a pair (the operator is not symmetric), FP64 to 1e-12 of the class's
largest entry; identical pairs exactly 0; the row sums of the GPU entries
reproduce Gauss' law (-|t_i|/2) as the oracle's do."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_1810_08429_amd as g
    g.lib()
    return g, torch


def build(g, m, **kw):
    return g.H2(m.verts, m.tris, g.Tree(m.verts, m.tris, 32), g.Params(eta=2.0, eps=1e-6, **kw))


@pytest.mark.parametrize("kw", [dict(), dict(sym_rules=1), dict(q_nr=5, q_s=6)])
def test_dl_entries_equal_oracle_every_class(env, orc, kw):
    g, torch = env
    m = synth.jitter(synth.ellipsoid(3), 0.002, seed=4)
    H = build(g, m, **kw)
    p = H.params
    ent = orc.Entries(m.verts, m.tris, p.q_r, p.q_nr, p.q_s, sym=bool(p.sym_rules))
    rng = np.random.default_rng(9)
    I = rng.integers(0, m.nt, 40000)
    J = rng.integers(0, m.nt, 40000)
    # all touching pairs of some rows, in both orders
    rows = rng.choice(m.nt, 60, replace=False)
    ri = np.repeat(rows, m.nt)
    cj = np.tile(np.arange(m.nt), len(rows))
    keep = ent.classify(ri, cj) != orc.REG
    ri, cj = ri[keep], cj[keep]
    I = np.concatenate([I, ri, cj, np.arange(50)])
    J = np.concatenate([J, cj, ri, np.arange(50)])
    cls = ent.classify(I, J)
    got = H.dl_entries(I, J).cpu().numpy()
    ref = ent.dl_entries(I, J)
    for k in (orc.REG, orc.NEAR, orc.VERT, orc.EDGE, orc.IDENT):
        sel = cls == k
        if k == orc.NEAR and kw.get("q_nr") is None:
            assert sel.sum() > 0
        if not sel.any():
            continue
        if k == orc.IDENT:
            assert np.all(got[sel] == 0.0)
            continue
        scale = np.abs(ref[sel]).max()
        assert np.abs(got[sel] - ref[sel]).max() <= 1e-12 * scale, k
    H.close()


def test_dl_row_sums_gauss_law(env, orc):
    g, torch = env
    m = synth.icosphere(3)
    H = build(g, m)
    T = m.verts[m.tris]
    area = 0.5 * np.linalg.norm(np.cross(T[:, 1] - T[:, 0], T[:, 2] - T[:, 0]), axis=1)
    rows = [0, 100, 777, m.nt - 1]
    I = np.repeat(rows, m.nt)
    J = np.tile(np.arange(m.nt), len(rows))
    K = H.dl_entries(I, J).cpu().numpy().reshape(len(rows), m.nt)
    p = H.params
    Ko = orc.Entries(m.verts, m.tris, p.q_r, p.q_nr, p.q_s).dl_block(rows, np.arange(m.nt))
    assert np.abs(K.sum(1) - Ko.sum(1)).max() < 1e-12 * np.abs(Ko.sum(1)).max()
    assert np.abs(K.sum(1) / area[rows] + 0.5).max() < 1e-4
    H.close()
