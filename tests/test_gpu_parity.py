"""Parity of the HIP path with the CPU oracle (runs on an MI355X).

Tolerances (FP64 path): entries and the nearfield-only operator to 1e-12
relative (same rules, only rounding order differs); the H^2 product to the
compression tolerance against the dense matrix and to 1e-10 against the
oracle's step-by-step GCA-H^2 when both select the same pivots.
Mixed path: FP32 regular-pair quadrature with cluster-local coordinates,
tolerance 1e-5 relative (FP32 rounding of a sum of O(100) terms).
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


def orders(gca):
    p = gca.Params()
    return (p.q_r, p.q_nr, p.q_s)


@pytest.fixture(scope="module")
def c1(orc, gca):
    m = synth.icosphere(3)
    ent = orc.Entries(m.verts, m.tris, *orders(gca))
    G = ent.dense()
    return m, ent, G


def build(gca, m, leaf, **kw):
    tree = gca.Tree(m.verts, m.tris, leaf)
    return gca.H2(m.verts, m.tris, tree, gca.Params(**kw))


def class_samples(orc, ent, n, rng, per_class=1500):
    I = rng.integers(0, n, 60000)
    J = rng.integers(0, n, 60000)
    I = np.concatenate([I, np.arange(n)])
    J = np.concatenate([J, np.arange(n)])
    c = ent.classify(I, J)
    out = {}
    for k in range(5):
        sel = np.nonzero(c == k)[0][:per_class]
        out[k] = (I[sel], J[sel])
    # all touching pairs of a few rows, both orders
    rows = rng.choice(n, 40, replace=False)
    for r in rows:
        cc = ent.classify(np.full(n, r), np.arange(n))
        for k in (orc.EDGE, orc.VERT):
            js = np.nonzero(cc == k)[0]
            out[k] = (np.concatenate([out[k][0], np.full(js.size, r), js]),
                      np.concatenate([out[k][1], js, np.full(js.size, r)]))
    return out


def test_entries_fp64_match_oracle_per_class(torch, gca, orc, c1):
    m, ent, G = c1
    H = build(gca, m, 32, eta=2.0, eps=1e-6)
    rng = np.random.default_rng(0)
    for k, (I, J) in class_samples(orc, ent, m.nt, rng).items():
        assert I.size > 0, k
        got = H.entries(I, J).cpu().numpy()
        ref = G[I, J]
        err = np.max(np.abs(got - ref) / np.abs(ref))
        assert err < 1e-12, (k, err)


def test_entries_mixed_match_oracle(torch, gca, orc, c1):
    m, ent, G = c1
    H = build(gca, m, 32, eta=2.0, eps=1e-6)
    rng = np.random.default_rng(1)
    for k, (I, J) in class_samples(orc, ent, m.nt, rng).items():
        got = H.entries(I, J, precision=gca.MIXED).cpu().numpy()
        ref = G[I, J]
        err = np.max(np.abs(got - ref) / np.abs(ref))
        # mixed: touching pairs stay FP64 (Sauter-Schwab), the disjoint classes
        # run in FP32
        tol = 1e-12 if k in (orc.IDENT, orc.EDGE, orc.VERT) else 2e-6
        assert err < tol, (k, err)


def test_entries_mixed_fp32_sauter_schwab_loops(torch, gca, orc, c1):
    """ss_fp32 = 1 (opt-in): the mixed product's Sauter-Schwab Gauss loops run
    in FP32 on FP64 edge vectors; sums of at most 128 positive terms give a
    relative rounding below 128 x 2^-24 ~ 8e-6.  The FP64 precision is not
    affected by the flag."""
    m, ent, G = c1
    H = build(gca, m, 32, eta=2.0, eps=1e-6, ss_fp32=1)
    rng = np.random.default_rng(1)
    for k, (I, J) in class_samples(orc, ent, m.nt, rng).items():
        if k not in (orc.IDENT, orc.EDGE, orc.VERT):
            continue
        ref = G[I, J]
        got = H.entries(I, J, precision=gca.MIXED).cpu().numpy()
        err = np.max(np.abs(got - ref) / np.abs(ref))
        assert 1e-12 < err < 1e-5, (k, err)
        got64 = H.entries(I, J, precision=gca.FP64).cpu().numpy()
        assert np.max(np.abs(got64 - ref) / np.abs(ref)) < 1e-12, k


def test_nearfield_only_operator_equals_dense(torch, gca, c1):
    """eta -> 0: no admissible block, the H^2 operator is the plain Galerkin
    matrix assembled by the block kernel and the per-case lists."""
    m, ent, G = c1
    H = build(gca, m, 32, eta=1e-6, eps=1e-6)
    st = H.stats()
    assert st["n_far_sym"] == 0
    X = synth.rhs_normal(m.nt, 3, seed=0)
    ref = G @ X
    x = torch.tensor(X, device="cuda")
    y = H.matvec(x).cpu().numpy()
    scale = np.abs(ref).max()
    assert np.abs(y - ref).max() < 1e-12 * scale
    ym = H.matvec(x, precision=gca.MIXED).cpu().numpy()
    assert np.abs(ym - ref).max() < 1e-5 * scale


def test_h2_fp64_matches_dense_within_tolerance(torch, gca, orc, c1):
    m, ent, G = c1
    for eps in (1e-4, 1e-6):
        H = build(gca, m, 32, eta=2.0, eps=eps)
        assert H.stats()["n_far_sym"] > 0
        x = synth.rhs_normal(m.nt, 1, seed=0)
        ref = G @ x
        y = H.matvec(torch.tensor(x, device="cuda")).cpu().numpy()
        rel = np.linalg.norm(y - ref) / np.linalg.norm(ref)
        assert rel < 10 * eps, (eps, rel)
        ym = H.matvec(torch.tensor(x, device="cuda"), precision=gca.MIXED).cpu().numpy()
        relm = np.linalg.norm(ym - ref) / np.linalg.norm(ref)
        assert relm < 10 * eps + 1e-5, (eps, relm)


def test_h2_matches_oracle_step_by_step_on_jittered_mesh(torch, gca, orc):
    """Off the symmetric sphere the pivot choice is unique: the GPU pivots,
    ranks and bases equal the oracle's, and so does the product."""
    base = synth.icosphere(3)
    m = synth.jitter(base, 0.02 * synth.mean_edge_length(base), seed=7)
    ent = orc.Entries(m.verts, m.tris, *orders(gca))
    ho = orc.gca_h2(m.verts, m.tris, leaf=32, eta=2.0, m=3, eps=1e-5, ent=ent)
    H = build(gca, m, 32, eta=2.0, eps=1e-5)
    ranks, piv, basis = H.basis()
    nc = len(ho.tree.nodes)
    assert ranks.shape[0] == nc
    o = 0
    for c in range(nc):
        r = ranks[c]
        assert r == len(ho.pivots[c]), c
        assert np.array_equal(piv[o:o + r], ho.pivots[c]), c
        o += r
    x = synth.rhs_normal(m.nt, 1, seed=0)
    yo = orc.h2_matvec(ho, x)
    y = H.matvec(torch.tensor(x, device="cuda")).cpu().numpy()
    assert np.linalg.norm(y - yo) / np.linalg.norm(yo) < 1e-10
    # leaf bases and transfers
    nv_ = 0
    for c in range(nc):
        nd = ho.tree.nodes[c]
        if not nd.sons:
            V = basis[nv_:nv_ + (nd.end - nd.begin) * ranks[c]].reshape(nd.end - nd.begin, ranks[c])
            np.testing.assert_allclose(V, ho.V[c], rtol=0, atol=1e-9 * max(1.0, np.abs(ho.V[c]).max()))
            nv_ += V.size


def test_matvec_is_deterministic_and_multi_rhs_consistent(torch, gca, c1):
    """Repeated products are bit-equal; the batched product of 4 right-hand
    sides (matrix-core transfers and block products) equals the single
    products column by column up to the rounding of the different
    summation order."""
    m, ent, G = c1
    H = build(gca, m, 32, eta=2.0, eps=1e-6)
    X = torch.tensor(synth.rhs_normal(m.nt, 4, seed=3), device="cuda")
    for prec, tol in ((gca.FP64, 1e-13), (gca.MIXED, 2e-6)):
        Y1 = H.matvec(X, precision=prec)
        Y2 = H.matvec(X, precision=prec)
        assert torch.equal(Y1, Y2)
        for k in range(4):
            yk = H.matvec(X[:, k].contiguous(), precision=prec)
            assert torch.equal(yk, H.matvec(X[:, k].contiguous(), precision=prec))
            assert float((yk - Y1[:, k]).abs().max()) <= tol * float(yk.abs().max()), (prec, k)


def test_sphere_constant_potential_on_gpu(torch, gca, orc):
    """P3 through the whole H^2 product: (G~ 1)_i / |t_i| -> r = 1."""
    m = synth.icosphere(4)
    H = build(gca, m, 32, eta=2.0, eps=1e-6)
    T = m.verts[m.tris]
    area = 0.5 * np.linalg.norm(np.cross(T[:, 1] - T[:, 0], T[:, 2] - T[:, 0]), axis=1)
    y = H.matvec(torch.ones(m.nt, dtype=torch.float64, device="cuda")).cpu().numpy() / area
    assert np.abs(y - 1).max() < 2e-3
    ent = orc.Entries(m.verts, m.tris, *orders(gca))
    rows = np.arange(0, m.nt, 97)
    ref = ent.matvec_rows(rows, np.ones(m.nt)) / area[rows]
    assert np.abs(y[rows] - ref).max() < 1e-5


def test_larger_sphere_sampled_rows(torch, gca, orc):
    """n = 20480 (leaf 64, eps 1e-5, 16 right-hand sides): sampled rows of
    the H^2 product against the oracle's dense rows."""
    m = synth.icosphere(5)
    H = build(gca, m, 64, eta=2.0, eps=1e-5)
    X = synth.rhs_normal(m.nt, 16, seed=0)
    Y = H.matvec(torch.tensor(X, device="cuda")).cpu().numpy()
    ent = orc.Entries(m.verts, m.tris, *orders(gca))
    rows = np.random.default_rng(2).choice(m.nt, 48, replace=False)
    ref = ent.matvec_rows(rows, X)
    rel = np.linalg.norm(Y[rows] - ref) / np.linalg.norm(ref)
    assert rel < 1e-4, rel
    Ym = H.matvec(torch.tensor(X, device="cuda"), precision=gca.MIXED).cpu().numpy()
    relm = np.linalg.norm(Ym[rows] - ref) / np.linalg.norm(ref)
    assert relm < 1e-4, relm


def test_coupling_rule_order_matches_oracle(torch, gca, orc):
    """A lower-order regular rule for the coupling entries G|t~ x s~ only
    (q_c = 2): the GPU product equals the oracle's GCA-H^2 built with the same
    coupling rule, and stays within the compression tolerance of the dense
    matrix on this mesh."""
    base = synth.icosphere(3)
    m = synth.jitter(base, 0.02 * synth.mean_edge_length(base), seed=7)
    ent = orc.Entries(m.verts, m.tris, *orders(gca))
    ho = orc.gca_h2(m.verts, m.tris, leaf=32, eta=2.0, m=3, eps=1e-5, ent=ent,
                    q=orders(gca), q_c=2)
    x = synth.rhs_normal(m.nt, 1, seed=3)
    yo = orc.h2_matvec(ho, x)
    for qc in (2,):
        H = build(gca, m, 32, eta=2.0, eps=1e-5, q_c=qc)
        y = H.matvec(torch.tensor(x, device="cuda")).cpu().numpy()
        assert np.linalg.norm(y - yo) / np.linalg.norm(yo) < 1e-10
        ym = H.matvec(torch.tensor(x, device="cuda"), precision=gca.MIXED).cpu().numpy()
        assert np.linalg.norm(ym - yo) / np.linalg.norm(yo) < 2e-5
    yd = ent.dense() @ x
    assert np.linalg.norm(yo - yd) / np.linalg.norm(yd) < 1e-3
    # q_c = 0 means "the regular order": identical to the default build
    H0 = build(gca, m, 32, eta=2.0, eps=1e-5, q_c=0)
    H3 = build(gca, m, 32, eta=2.0, eps=1e-5, q_c=orders(gca)[0])
    xt = torch.tensor(x, device="cuda")
    assert torch.equal(H0.matvec(xt), H3.matvec(xt))


@pytest.fixture(scope="module")
def c1_sym(orc, gca):
    m = synth.icosphere(3)
    ent = orc.Entries(m.verts, m.tris, 3, 3, 4, sym=True)
    return m, ent, ent.dense()


def test_symmetric_rule_entries_and_nearfield_match_oracle(torch, gca, orc, c1_sym):
    """sym_rules = 1 (6-point symmetric rule for the disjoint classes): every
    class through gca_entries equals the oracle with the same rules (FP64
    1e-12; mixed 2e-6 for the disjoint classes), and with eta -> 0 the
    product is the oracle's dense matrix times x."""
    m, ent, G = c1_sym
    H = build(gca, m, 32, eta=2.0, eps=1e-6, sym_rules=1)
    rng = np.random.default_rng(5)
    for k, (I, J) in class_samples(orc, ent, m.nt, rng, per_class=600).items():
        ref = G[I, J]
        got = H.entries(I, J).cpu().numpy()
        assert np.max(np.abs(got - ref) / np.abs(ref)) < 1e-12, k
        gm = H.entries(I, J, precision=gca.MIXED).cpu().numpy()
        tol = 1e-12 if k in (orc.IDENT, orc.EDGE, orc.VERT) else 2e-6   # FP64 Sauter-Schwab
        assert np.max(np.abs(gm - ref) / np.abs(ref)) < tol, k
    H0 = build(gca, m, 32, eta=1e-6, eps=1e-6, sym_rules=1)
    X = synth.rhs_normal(m.nt, 2, seed=1)
    ref = G @ X
    x = torch.tensor(X, device="cuda")
    scale = np.abs(ref).max()
    assert np.abs(H0.matvec(x).cpu().numpy() - ref).max() < 1e-12 * scale
    assert np.abs(H0.matvec(x, precision=gca.MIXED).cpu().numpy() - ref).max() < 1e-5 * scale


def test_symmetric_rule_h2_matches_oracle_step_by_step(torch, gca, orc):
    """Jittered level-3 sphere, symmetric rules for the regular pairs (6
    points) and for the coupling entries (q_c = 2: 3 points): the GPU product
    equals the oracle's GCA-H^2 built with the same rules, and stays within
    the compression tolerance of the dense matrix of the collapsed rules."""
    base = synth.icosphere(3)
    m = synth.jitter(base, 0.02 * synth.mean_edge_length(base), seed=7)
    ent = orc.Entries(m.verts, m.tris, 3, 3, 4, sym=True)
    ho = orc.gca_h2(m.verts, m.tris, leaf=32, eta=2.0, m=3, eps=1e-5, ent=ent, q=(3, 3, 4), q_c=2)
    x = synth.rhs_normal(m.nt, 1, seed=3)
    yo = orc.h2_matvec(ho, x)
    H = build(gca, m, 32, eta=2.0, eps=1e-5, sym_rules=1, q_c=2)
    xt = torch.tensor(x, device="cuda")
    y = H.matvec(xt).cpu().numpy()
    assert np.linalg.norm(y - yo) / np.linalg.norm(yo) < 1e-10
    ym = H.matvec(xt, precision=gca.MIXED).cpu().numpy()
    assert np.linalg.norm(ym - yo) / np.linalg.norm(yo) < 2e-5
    yd = orc.Entries(m.verts, m.tris, *orders(gca)).dense() @ x
    assert np.linalg.norm(yo - yd) / np.linalg.norm(yd) < 1e-3
    # stored blocks give the recomputed product
    H.store_blocks(fp64=True, mixed=True)
    ys = H.matvec(xt).cpu().numpy()
    assert np.linalg.norm(ys - y) / np.linalg.norm(y) < 1e-13


def test_side_stream_orders_products_and_geometry_updates(torch, gca):
    """The touching values run on the handle's side stream, forked from and
    joined back into the caller's stream: products and a geometry update
    queued back to back on a non-default stream equal, bit for bit, the same
    calls separated by device synchronisations."""
    base = synth.icosphere(3)
    m = synth.jitter(base, 0.02 * synth.mean_edge_length(base), seed=8)
    moved = m.verts * 1.02 + np.array([1e-3, 0.0, -2e-3])
    x = torch.tensor(synth.rhs_normal(m.nt, 1, seed=9), device="cuda")
    torch.cuda.synchronize()
    res = []
    for asynchronous in (True, False):
        H = build(gca, m, 32, eta=2.0, eps=1e-6)
        s = torch.cuda.Stream() if asynchronous else torch.cuda.current_stream()
        sync = (lambda: None) if asynchronous else torch.cuda.synchronize
        ys = []
        with torch.cuda.stream(s):
            for prec in (gca.MIXED, gca.FP64, gca.MIXED):
                ys.append(H.matvec(x, precision=prec))
                sync()
            H.update_geometry(moved)
            sync()
            for prec in (gca.MIXED, gca.FP64):
                ys.append(H.matvec(x, precision=prec))
                sync()
        torch.cuda.synchronize()
        res.append([y.cpu().numpy() for y in ys])
    for a, b in zip(*res):
        assert np.array_equal(a, b)
    assert np.array_equal(res[0][0], res[0][2])
    assert not np.array_equal(res[0][0], res[0][3])


def test_near_regular_pairs_of_admissible_blocks_stay_in_those_blocks(torch, gca, orc):
    """With a near-regular order of its own (q_nr = 5 != q_r = 3), a pair whose
    vertices are joined by a mesh edge can lie in an admissible block (boxes
    apart, the edge bridging them): it is then represented by that block like
    every other pair of it, and only the near-regular pairs of nearfield
    blocks are listed.  Jittered level-3 sphere, leaf 16, eta 2: the build
    succeeds, the product equals the oracle's step-by-step GCA-H^2 to 1e-10
    and the dense matrix to the compression tolerance."""
    base = synth.icosphere(3)
    m = synth.jitter(base, 0.02 * synth.mean_edge_length(base), seed=7)
    q = (3, 5, 4)
    ent = orc.Entries(m.verts, m.tris, *q)
    tree = orc.cluster_tree(m.verts, m.tris, 16)
    far, _ = orc.block_tree(tree, 2.0)
    bridged = 0
    for t, s in far:
        I, J = np.meshgrid(tree.indices(t), tree.indices(s), indexing="ij")
        bridged += int((ent.classify(I.ravel(), J.ravel()) == orc.NEAR).sum())
    assert bridged > 0
    H = build(gca, m, 16, eta=2.0, eps=1e-8, q_nr=5)
    ho = orc.gca_h2(m.verts, m.tris, leaf=16, eta=2.0, m=3, eps=1e-8, ent=ent, q=q)
    x = synth.rhs_normal(m.nt, 1, seed=2)
    yo = orc.h2_matvec(ho, x)
    xt = torch.tensor(x, device="cuda")
    y = H.matvec(xt).cpu().numpy()
    assert np.linalg.norm(y - yo) / np.linalg.norm(yo) < 1e-10
    yd = ent.dense() @ x
    assert np.linalg.norm(y - yd) / np.linalg.norm(yd) < 1e-6
    ym = H.matvec(xt, precision=gca.MIXED).cpu().numpy()
    assert np.linalg.norm(ym - yo) / np.linalg.norm(yo) < 1e-5
    H.close()


def test_serial_and_overlapped_products_are_bit_equal(torch, gca):
    """The overlapped product (touching values and transform chain on the
    handle's side streams) and the serial one (every phase on the caller's
    stream) run the same kernels on the same data with one writer per
    partial: bit-equal results, both precisions, several right-hand sides;
    every phase time is recorded."""
    m = synth.icosphere(4)
    tree = gca.Tree(m.verts, m.tris, 32)
    Ho = gca.H2(m.verts, m.tris, tree, gca.Params(eta=2.0, eps=1e-6))
    Hs = gca.H2(m.verts, m.tris, tree, gca.Params(eta=2.0, eps=1e-6, serial=1))
    x = torch.tensor(synth.rhs_normal(m.nt, 3, seed=9), device="cuda")
    for prec in (gca.FP64, gca.MIXED):
        yo = Ho.matvec(x, precision=prec)
        ys = Hs.matvec(x, precision=prec)
        assert torch.equal(yo, ys), prec
    for H in (Ho, Hs):
        ph = H.phase_times(4)
        assert ph.shape[1] == len(gca.PHASES) and np.all(np.isfinite(ph)) and np.all(ph >= 0)
        assert np.all(ph[:, -1] > 0)
    Ho.close()
    Hs.close()
