"""GPU parity of collocation with the linear nodal basis (Section 6) through
the C-ABI: dense blocks g(x_i, phi_j) (x_i the row subset's vertices, phi_j
the column subset's nodal functions over its merged triangle list) against
the oracle's plain definition (oracle/collocation.py), FP64 1e-12 relative.

Blocks of ragged sizes, rows and columns from the same patch (collocation
points that are corners of column triangles: the Duffy rule) and from
patches far apart (regular rule only), collapsed and symmetric rules, several
Duffy orders; run-to-run bit equality and the limit status."""
import numpy as np
import pytest

import synth
from oracle import collocation as C
from oracle import linear as L

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_1810_08429_amd as g
    g.lib()
    return g, torch


def _device(g, torch, m):
    off, lst = g.lin_vertex_triangles(m.tris, m.nv)
    d = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt).cuda()
    return d(m.verts, torch.float64), d(m.tris, torch.int32), d(off, torch.int32), d(lst, torch.int32)


def _run(g, torch, m, sets, pairs, q, sym, q_s, ld=64 * 64):
    xyz, tri, off, lst = _device(g, torch, m)
    so = torch.as_tensor(np.concatenate([[0], np.cumsum([len(s) for s in sets])]).astype(np.int32)).cuda()
    sv = torch.as_tensor(np.concatenate([np.asarray(s, dtype=np.int32) for s in sets])).cuda()
    merged = g.lin_merge(off, lst, tri, so, sv, 192)
    assert (merged[2].cpu().numpy() >= 0).all()
    br = torch.tensor([p[0] for p in pairs], dtype=torch.int32).cuda()
    bc = torch.tensor([p[1] for p in pairs], dtype=torch.int32).cuda()
    out, st = g.coll_blocks(xyz, tri, sv, merged, so, br, bc, ld, q, sym, q_s)
    torch.cuda.synchronize()
    return out, st


def _patch(verts, centre, k, pool, rng):
    near = np.argsort(((verts - verts[centre]) ** 2).sum(1))[:pool]
    return rng.choice(near, size=k, replace=False)


@pytest.mark.parametrize("q,sym,q_s", [(2, False, 4), (3, False, 8), (1, False, 2), (4, False, 8),
                                       (2, True, 6), (3, True, 12)])
def test_collocation_blocks_equal_oracle(env, q, sym, q_s):
    g, torch = env
    m = synth.icosphere(3)
    T = L.vertex_triangles(m.tris, m.nv)
    rng = np.random.default_rng(q + 10 * sym + 100 * q_s)
    sets, pairs = [], []
    for n_r, n_c, pool, same in [(1, 1, 1, True), (7, 13, 40, True), (32, 32, 40, True), (64, 29, 64, False),
                                 (5, 64, 64, True), (64, 64, 72, False)]:
        a = int(rng.integers(m.nv))
        if same:
            b = a
        else:
            while True:
                b = int(rng.integers(m.nv))
                if np.linalg.norm(m.verts[a] - m.verts[b]) > 1.5:
                    break
        sets.append(_patch(m.verts, a, n_r, pool, rng))
        sets.append(_patch(m.verts, b, n_c, pool, rng))
        pairs.append((len(sets) - 2, len(sets) - 1))
    out, st = _run(g, torch, m, sets, pairs, q, sym, q_s)
    out, st = out.cpu().numpy(), st.cpu().numpy()
    assert (st == 0).all()
    singular = 0
    for b, (r, c) in enumerate(pairs):
        want = C.coll_block(m.verts, m.tris, T, sets[r], sets[c], q, q_s, sym)
        got = out[b, :want.size].reshape(want.shape)
        assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max(), (b, q, sym, q_s)
        # count the entries whose support holds the collocation point (the Duffy case)
        singular += sum(1 for i in sets[r] for j in sets[c] if any(int(i) in m.tris[t] for t in T[int(j)]))
    assert singular > 0


def test_collocation_deterministic_and_status(env):
    g, torch = env
    m = synth.icosphere(3)
    rng = np.random.default_rng(4)
    a = _patch(m.verts, 0, 30, 40, rng)
    big = _patch(m.verts, 5, 65, 65, rng)
    sets = [a, big]
    pairs = [(0, 0), (0, 1), (1, 0)]
    out1, st1 = _run(g, torch, m, sets, pairs, 3, False, 8, ld=65 * 64)
    out2, st2 = _run(g, torch, m, sets, pairs, 3, False, 8, ld=65 * 64)
    assert list(st1.cpu().numpy()) == [0, 2, 2]
    assert torch.equal(out1[0, :900], out2[0, :900])
    assert (out1[1, :30 * 65] == 0).all()


def test_collocation_row_sums_on_the_sphere(env):
    """All vertices of the level-2 sphere against all nodal functions in
    16 x 16 blocks: each row sums to the potential of the uniform density on
    the polyhedral sphere at the vertex, within 3e-2 of the sphere's 1 (1.4e-2
    at the vertices the oracle's pin samples)."""
    g, torch = env
    m = synth.icosphere(2)
    sets = [np.arange(k, min(k + 16, m.nv)) for k in range(0, m.nv, 16)]
    pairs = [(r, c) for r in range(len(sets)) for c in range(len(sets))]
    out, st = _run(g, torch, m, sets, pairs, 4, False, 16, ld=256)
    out, st = out.cpu().numpy(), st.cpu().numpy()
    assert (st == 0).all()
    rows = np.zeros(m.nv)
    for b, (r, c) in enumerate(pairs):
        n, k = len(sets[r]), len(sets[c])
        rows[sets[r]] += out[b, :n * k].reshape(n, k).sum(axis=1)
    assert np.abs(rows - 1).max() < 3e-2
    ref = sum(C.point_triangle_moments(m.verts, t, 0, 4, 16).sum() for t in m.tris)
    assert abs(rows[0] - ref) < 1e-12 * ref
