"""The batched product (h2_matvec with nrhs > 1): right-hand sides 16 at a
time, every block entry evaluated once per 16, and the transfer, coupling
and nearfield products of the 16 columns as 16 x 16 matrix-core tiles.

Against the single products column by column (FP64 1e-13, mixed 2e-6 of the
column's max norm: only the summation order differs), against the oracle's
step-by-step GCA-H^2 (FP64 1e-10), for 3, 16 and 20 columns (one partial and
two passes), a mesh size that is not a multiple of 64, ld > n, FP32 vectors,
ranks above 64 (several row blocks in the coupling kernel and several tiles
per transfer), the collapsed and the symmetric rules; serial and overlapped
phases bit-equal; the stored-block mode (column by column) agrees."""
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


def jittered(level, seed):
    base = synth.icosphere(level)
    return synth.jitter(base, 0.02 * synth.mean_edge_length(base), seed=seed)


def columns_match(torch, H, X, Y, prec, tol):
    for k in range(X.shape[1]):
        yk = H.matvec(X[:, k].contiguous(), precision=prec)
        err = float((yk - Y[:, k]).abs().max()) / float(yk.abs().max())
        assert err <= tol, (prec, k, err)


@pytest.mark.parametrize("nrhs", [3, 16, 20])
@pytest.mark.parametrize("sym", [0, 1])
def test_batched_equals_single_products(torch, gca, nrhs, sym):
    m = jittered(4, seed=21)
    H = gca.H2(m.verts, m.tris, gca.Tree(m.verts, m.tris, 64),
               gca.Params(eta=2.0, eps=1e-6, sym_rules=sym, q_c=2 if sym else 0))
    X = torch.tensor(synth.rhs_normal(m.nt, nrhs, seed=nrhs), device="cuda")
    print(f"[multi-rhs] n {m.nt} nrhs {nrhs} sym {sym}", flush=True)
    for prec, tol in ((gca.FP64, 1e-13), (gca.MIXED, 2e-6)):
        Y = H.matvec(X, precision=prec)
        assert torch.equal(Y, H.matvec(X, precision=prec))
        columns_match(torch, H, X, Y, prec, tol)
    H.close()


def test_batched_ragged_patch(torch, gca):
    """An open patch of n = 1243 triangles (the level-3 sphere without its
    last 37): the last 64-id group of the input permutation and the last
    leaves are partial."""
    base = synth.icosphere(3)
    tris = np.ascontiguousarray(base.tris[:1243])
    H = gca.H2(base.verts, tris, gca.Tree(base.verts, tris, 64), gca.Params(eta=2.0, eps=1e-6))
    X = torch.tensor(synth.rhs_normal(1243, 16, seed=31), device="cuda")
    print("[multi-rhs] ragged n 1243", flush=True)
    for prec, tol in ((gca.FP64, 1e-13), (gca.MIXED, 2e-6)):
        Y = H.matvec(X, precision=prec)
        columns_match(torch, H, X, Y, prec, tol)
    H.close()


def test_batched_with_ranks_above_64_and_strided_fp32_vectors(torch, gca):
    """Green order 5 and eps 1e-9 on the jittered level-4 sphere: ranks above
    64, so the coupling rows of a cluster span two row blocks and transfers
    several 16-column tiles; x and y FP32 with ld = n + 3."""
    m = jittered(4, seed=22)
    H = gca.H2(m.verts, m.tris, gca.Tree(m.verts, m.tris, 64), gca.Params(eta=2.0, eps=1e-9, green_m=5))
    assert H.stats()["rank_max"] > 64
    n, k, ld = m.nt, 16, m.nt + 3
    X = synth.rhs_normal(n, k, seed=5)
    x32 = torch.zeros((k, ld), dtype=torch.float32, device="cuda")
    x32[:, :n] = torch.tensor(X.T, dtype=torch.float32, device="cuda")
    xs = torch.as_strided(x32, (n, k), (1, ld))
    y32 = torch.as_strided(torch.full((k, ld), 5.0, dtype=torch.float32, device="cuda"), (n, k), (1, ld))
    for prec, tol in ((gca.FP64, 1e-6), (gca.MIXED, 3e-6)):
        H.matvec_into(xs, y32, precision=prec)
        Y64 = H.matvec(xs.double(), precision=prec)
        assert torch.equal(y32, Y64.float())
        base = torch.as_strided(y32, (k, ld), (ld, 1))
        assert torch.all(base[:, n:] == 5.0)
        columns_match(torch, H, xs.double(), Y64, prec, 1e-13 if prec == gca.FP64 else 2e-6)
    H.close()


def test_batched_equals_oracle_step_by_step(torch, gca, orc):
    m = jittered(3, seed=7)
    p = gca.Params(eta=2.0, eps=1e-5)
    ent = orc.Entries(m.verts, m.tris, p.q_r, p.q_nr, p.q_s)
    ho = orc.gca_h2(m.verts, m.tris, leaf=32, eta=2.0, m=3, eps=1e-5, ent=ent, q=(p.q_r, p.q_nr, p.q_s))
    H = gca.H2(m.verts, m.tris, gca.Tree(m.verts, m.tris, 32), p)
    X = synth.rhs_normal(m.nt, 16, seed=12)
    Y = H.matvec(torch.tensor(X, device="cuda")).cpu().numpy()
    Ym = H.matvec(torch.tensor(X, device="cuda"), precision=gca.MIXED).cpu().numpy()
    for k in (0, 5, 15):
        yo = orc.h2_matvec(ho, X[:, k])
        assert np.linalg.norm(Y[:, k] - yo) / np.linalg.norm(yo) < 1e-10
        assert np.linalg.norm(Ym[:, k] - yo) / np.linalg.norm(yo) < 1e-5
    H.close()


def test_batched_serial_overlapped_and_stored(torch, gca):
    m = jittered(4, seed=23)
    tree = gca.Tree(m.verts, m.tris, 64)
    Ho = gca.H2(m.verts, m.tris, tree, gca.Params(eta=2.0, eps=1e-6))
    Hs = gca.H2(m.verts, m.tris, tree, gca.Params(eta=2.0, eps=1e-6, serial=1))
    X = torch.tensor(synth.rhs_normal(m.nt, 16, seed=3), device="cuda")
    for prec in (gca.FP64, gca.MIXED):
        assert torch.equal(Ho.matvec(X, precision=prec), Hs.matvec(X, precision=prec))
    Y = Ho.matvec(X)
    Ho.store_blocks(fp64=True, mixed=False)
    Ys = Ho.matvec(X)
    assert float((Ys - Y).abs().max()) <= 1e-13 * float(Y.abs().max())
    Ho.close()
    Hs.close()
