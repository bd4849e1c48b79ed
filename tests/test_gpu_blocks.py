"""Element-wise parity of the block-row kernels at the parameters of the
level-8 bench workload (leaf 64, Green order 5, omega margin 1.5, eps 1e-5,
coupling rule order 2, symmetric triangle rules for the disjoint pairs), on a
jittered level-4 sphere (n = 5120), where ranks reach the 60s and block rows
span several column chunks.

The stored-block mode runs the same kernels as the recomputing product
(k_far_rows / k_near_rows with the store switch) and gca_block_entries hands
every stored entry back with its triangle ids:
  - coupling entries G|t~ x s~ against the oracle's entries with the coupling
    rule (FP64 1e-12 relative, mixed 1e-5);
  - nearfield entries G|t^ x s^ against the oracle's entries (same bars);
    every unordered pair of the inadmissible leaf blocks is either stored
    once (non-zero) or owned by a touching list (stored as 0);
  - the FP64 product equals the oracle's step-by-step GCA-H^2 (same pivots,
    ranks and bases) to 1e-10, and with eta -> 0 at leaf 64 the mixed product
    equals the oracle's dense matrix to 1e-5.
"""
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


@pytest.fixture(scope="module")
def case(torch, gca, orc):
    _, prm = synth.workload("sphere_l8")
    base = synth.icosphere(4)
    m = synth.jitter(base, 0.02 * synth.mean_edge_length(base), seed=11)
    p = gca.Params(eta=prm["eta"], eps=prm["eps"], green_m=prm["green_m"], omega_scale=prm["omega_scale"],
                   q_c=prm["q_c"], sym_rules=prm["sym_rules"])
    tree = gca.Tree(m.verts, m.tris, prm["leaf"])
    H = gca.H2(m.verts, m.tris, tree, p)
    H.tree_perm = tree.export()[0]
    H.store_blocks(fp64=True, mixed=True)
    print(f"[blocks] jittered level-4 sphere n {m.nt}, leaf {prm['leaf']}, rank max {H.stats()['rank_max']}",
          flush=True)
    yield m, p, prm, H
    H.close()


def test_bench_shape_is_exercised(case):
    """The case has what the level-8 block rows have: ranks above 32 (two
    tile rows per wavefront), block rows wider than one column chunk, more
    than one nearfield block per leaf."""
    m, p, prm, H = case
    st = H.stats()
    assert st["rank_max"] > 32 and st["n_far_sym"] > 0
    assert st["n_near_sym"] > 2 * st["n_leaves"]
    r, c, _ = H.block_entries(0, kind=0)
    _, counts = np.unique(r, return_counts=True)
    assert counts.max() > 256   # a row pivot with more than one chunk of columns


@pytest.mark.parametrize("prec,tol", [(0, 1e-12), (1, 1e-5)])
def test_coupling_entries_equal_oracle(case, orc, gca, prec, tol):
    m, p, prm, H = case
    r, c, v = H.block_entries(prec, kind=0)
    st = H.stats()
    assert r.size == st["coupling_entries"] == st["store_entries_far"]
    ent_c = orc.Entries(m.verts, m.tris, p.q_c, p.q_c, p.q_s, sym=bool(p.sym_rules))
    # admissible blocks hold regular pairs only, so the coupling rule applies to every entry
    assert np.all(ent_c.classify(r, c) == orc.REG)
    ref = ent_c.entries(r, c)
    rel = np.abs(v - ref) / np.abs(ref)
    assert rel.max() < tol, (prec, rel.max())


@pytest.mark.parametrize("prec,tol", [(0, 1e-12), (1, 1e-5)])
def test_nearfield_entries_equal_oracle_and_cover_each_pair_once(case, orc, gca, prec, tol):
    m, p, prm, H = case
    r, c, v = H.block_entries(prec, kind=1)
    st = H.stats()
    assert r.size == st["store_entries_near"]
    ent = orc.Entries(m.verts, m.tris, p.q_r, p.q_nr, p.q_s, sym=bool(p.sym_rules))
    nz = v != 0
    assert nz.sum() == st["near_regular_pairs"]
    cls = ent.classify(r, c)
    # zeros: touching pairs (the lists own them) or the mirrored half of a
    # diagonal block (the same leaf, each unordered pair once)
    perm = H.tree_perm
    pos = np.empty(m.nt, dtype=np.int64)
    pos[perm] = np.arange(m.nt)
    touching = np.isin(cls, [orc.IDENT, orc.EDGE, orc.VERT])
    assert not np.any(touching & nz)
    lower = pos[c] <= pos[r]
    assert np.all(touching[~nz] | lower[~nz])
    assert np.all(cls[nz] != orc.IDENT)
    # each unordered non-touching pair once
    key = np.minimum(r[nz], c[nz]).astype(np.int64) * m.nt + np.maximum(r[nz], c[nz])
    assert np.unique(key).size == key.size
    ref = ent.entries(r[nz], c[nz])
    rel = np.abs(v[nz] - ref) / np.abs(ref)
    assert rel.max() < tol, (prec, rel.max())


def test_product_equals_oracle_step_by_step_at_bench_parameters(case, orc, gca, torch):
    m, p, prm, H = case
    ent = orc.Entries(m.verts, m.tris, p.q_r, p.q_nr, p.q_s, sym=bool(p.sym_rules))
    ho = orc.gca_h2(m.verts, m.tris, leaf=prm["leaf"], eta=p.eta, m=p.green_m, eps=p.eps, ent=ent,
                    q=(p.q_r, p.q_nr, p.q_s), omega_scale=p.omega_scale, q_c=p.q_c)
    ranks, piv, _ = H.basis()
    o = 0
    for cl in range(len(ho.tree.nodes)):
        assert ranks[cl] == len(ho.pivots[cl]), cl
        assert np.array_equal(piv[o:o + ranks[cl]], ho.pivots[cl]), cl
        o += ranks[cl]
    x = synth.rhs_normal(m.nt, 1, seed=4)
    yo = orc.h2_matvec(ho, x)
    xt = torch.tensor(x, device="cuda")
    H.store_blocks(False, False)
    y = H.matvec(xt).cpu().numpy()
    assert np.linalg.norm(y - yo) / np.linalg.norm(yo) < 1e-10
    ym = H.matvec(xt, precision=gca.MIXED).cpu().numpy()
    assert np.linalg.norm(ym - yo) / np.linalg.norm(yo) < 1e-5
    H.store_blocks(True, True)


def test_nearfield_only_mixed_product_at_leaf_64_equals_dense(case, orc, gca, torch):
    """eta -> 0: every block is a nearfield block of leaf size 64; the mixed
    product (FP32 block kernels, FP64 touching pairs) equals the oracle's
    dense matrix with the same rules to 1e-5, the FP64 one to 1e-12."""
    m, p, prm, H = case
    ent = orc.Entries(m.verts, m.tris, p.q_r, p.q_nr, p.q_s, sym=bool(p.sym_rules))
    G = ent.dense()
    p0 = gca.Params(eta=1e-6, eps=p.eps, green_m=3, q_c=p.q_c, sym_rules=p.sym_rules)
    H0 = gca.H2(m.verts, m.tris, gca.Tree(m.verts, m.tris, prm["leaf"]), p0)
    assert H0.stats()["n_far_sym"] == 0
    X = synth.rhs_normal(m.nt, 2, seed=6)
    ref = G @ X
    x = torch.tensor(X, device="cuda")
    scale = np.abs(ref).max()
    assert np.abs(H0.matvec(x).cpu().numpy() - ref).max() < 1e-12 * scale
    assert np.abs(H0.matvec(x, precision=gca.MIXED).cpu().numpy() - ref).max() < 1e-5 * scale
    H0.close()
