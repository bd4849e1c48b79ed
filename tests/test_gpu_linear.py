"""GPU parity of the piecewise-linear nodal basis (Section 5) through the C-ABI:
merged triangle lists bit for bit against the oracle's mergesort (and the
paper's printed example), dense blocks of the linear-basis Galerkin matrix
against the oracle's plain definition."""
import json
import os

import numpy as np
import pytest

import synth
from oracle import linear as L

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "merge_example.json")


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_1810_08429_amd as g
    g.lib()
    return g, torch


def _numpy_T(tris, nv):
    # test-local sets T_i (numpy), for the oracle
    t = np.repeat(np.arange(len(tris)), 3)
    v = np.asarray(tris).reshape(-1)
    order = np.lexsort((t, v))
    T = [[] for _ in range(nv)]
    for k in order:
        T[v[k]].append(int(t[k]))
    return T


def _device_mesh(g, torch, verts, tris):
    off, lst = g.lin_vertex_triangles(tris, len(verts))
    d = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt).cuda()
    return (d(verts, torch.float64), d(tris, torch.int32), d(off, torch.int32), d(lst, torch.int32))


def _subsets(torch, sets):
    off = np.concatenate([[0], np.cumsum([len(s) for s in sets])]).astype(np.int32)
    vtx = np.concatenate([np.asarray(s, dtype=np.int32) for s in sets] + [np.zeros(1, np.int32)])
    return torch.as_tensor(off).cuda(), torch.as_tensor(vtx).cuda()


def _merge(g, torch, dm, sets, cap):
    xyz, tri, off, lst = dm
    so, sv = _subsets(torch, sets)
    mt, ml, mc = g.lin_merge(off, lst, tri, so, sv, cap)
    torch.cuda.synchronize()
    return so, (mt, ml, mc)


def test_merge_worked_example(env):
    g, torch = env
    ex = json.load(open(GOLDEN))
    tris = np.array(ex["triangles"]) - 1
    verts = np.random.default_rng(0).normal(size=(7, 3))
    dm = _device_mesh(g, torch, verts, tris)
    sub = [v - 1 for v in ex["subset"]]
    _, (mt, ml, mc) = _merge(g, torch, dm, [sub, [sub[0]], [], [sub[2]]], cap=8)
    mt, ml, mc = mt.cpu().numpy(), ml.cpu().numpy(), mc.cpu().numpy()
    want = [(r[0] - 1,) + tuple(-1 if x is None else x - 1 for x in r[1:]) for r in ex["merged"]]
    got = [(int(mt[0, r]),) + tuple(int(x) for x in ml[0, r]) for r in range(mc[0])]
    assert got == want
    assert mc[2] == 0
    one = [(int(mt[1, r]),) + tuple(int(x) for x in ml[1, r]) for r in range(mc[1])]
    assert one == [(t, a, b, c) for (t, a, b, c) in
                   [(r[0] - 1,) + tuple(-1 if x is None else x - 1 for x in r[1:]) for r in ex["per_vertex"]["1"]]]


@pytest.mark.parametrize("level,sizes,seed", [(3, [1, 2, 17, 64, 100, 255, 300], 0), (4, [5, 33, 257, 340], 1)])
def test_merge_equals_oracle(env, level, sizes, seed):
    g, torch = env
    m = synth.icosphere(level)
    dm = _device_mesh(g, torch, m.verts, m.tris)
    rng = np.random.default_rng(seed)
    sets = [rng.choice(m.nv, size=s, replace=False) for s in sizes]
    # a contiguous patch too: many triangles shared by several subset vertices
    c = m.verts[int(rng.integers(m.nv))]
    sets.append(np.argsort(((m.verts - c) ** 2).sum(1))[:150])
    cap = 2048
    _, (mt, ml, mc) = _merge(g, torch, dm, sets, cap)
    mt, ml, mc = mt.cpu().numpy(), ml.cpu().numpy(), mc.cpu().numpy()
    T = _numpy_T(m.tris, m.nv)
    for k, s in enumerate(sets):
        want = L.merge_triangle_lists(m.tris, T, [int(v) for v in s])
        got = [(int(mt[k, r]),) + tuple(int(x) for x in ml[k, r]) for r in range(mc[k])]
        assert got == want, k


def test_merge_limits(env):
    g, torch = env
    m = synth.icosphere(4)
    dm = _device_mesh(g, torch, m.verts, m.tris)
    rng = np.random.default_rng(3)
    big = rng.choice(m.nv, size=400, replace=False)      # sum |T_i| > 2048
    huge = rng.choice(m.nv, size=1100, replace=False)    # more than 1024 vertices
    small = rng.choice(m.nv, size=20, replace=False)     # ~120 rows > cap 64
    tiny = rng.choice(m.nv, size=2, replace=False)
    _, (mt, ml, mc) = _merge(g, torch, dm, [big, huge, small, tiny], cap=64)
    mc = mc.cpu().numpy()
    assert list(mc[:3]) == [-1, -1, -1]
    T = _numpy_T(m.tris, m.nv)
    assert mc[3] == len(L.merge_triangle_lists(m.tris, T, [int(v) for v in tiny]))


def _patch(verts, centre, k, pool, rng):
    near = np.argsort(((verts - verts[centre]) ** 2).sum(1))[:pool]
    return rng.choice(near, size=k, replace=False)


@pytest.mark.parametrize("q,sym", [(2, False), (3, False), (1, False), (4, False), (2, True), (3, True)])
def test_blocks_equal_oracle(env, q, sym):
    g, torch = env
    m = synth.icosphere(3)
    dm = _device_mesh(g, torch, m.verts, m.tris)
    rng = np.random.default_rng(q + 7 * sym)
    T = _numpy_T(m.tris, m.nv)
    sets, pairs = [], []
    # ragged sizes: contiguous patches and scattered subsets of a neighbourhood
    for n_r, n_c, pool in [(1, 1, 1), (7, 13, 40), (32, 32, 32), (64, 29, 64), (5, 64, 64), (64, 64, 72)]:
        while True:
            a, b = rng.integers(m.nv, size=2)
            if np.linalg.norm(m.verts[a] - m.verts[b]) > 1.75:
                break
        sets.append(_patch(m.verts, a, n_r, pool, rng))
        sets.append(_patch(m.verts, b, n_c, pool, rng))
        pairs.append((len(sets) - 2, len(sets) - 1))
        pairs.append((len(sets) - 1, len(sets) - 2))
    assert max(len(L.merge_triangle_lists(m.tris, T, [int(v) for v in x])) for x in sets) <= g.LIN_MAX_TRIS
    so, merged = _merge(g, torch, dm, sets, cap=192)
    assert (merged[2].cpu().numpy() >= 0).all()
    br = torch.tensor([p[0] for p in pairs], dtype=torch.int32).cuda()
    bc = torch.tensor([p[1] for p in pairs], dtype=torch.int32).cuda()
    ld = 64 * 64
    out, st = g.lin_blocks(dm[0], dm[1], merged, so, br, bc, ld, q, sym)
    out, st = out.cpu().numpy(), st.cpu().numpy()
    assert (st == 0).all()
    for b in range(0, len(pairs), 2):
        r, c = pairs[b]
        # the reversed block is the transpose (symmetry of the oracle is pinned on the CPU)
        want = L.lin_block(m.verts, m.tris, sets[r], sets[c], q, sym, T=T)
        for got in (out[b, :want.size].reshape(want.shape), out[b + 1, :want.size].reshape(want.T.shape).T):
            assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max(), (b, q, sym)


def test_blocks_deterministic_and_status(env):
    g, torch = env
    m = synth.icosphere(3)
    dm = _device_mesh(g, torch, m.verts, m.tris)
    rng = np.random.default_rng(11)
    a = _patch(m.verts, 0, 30, 60, rng)
    far = int(np.argmax(((m.verts - m.verts[0]) ** 2).sum(1)))
    b = _patch(m.verts, far, 30, 60, rng)
    a2 = _patch(m.verts, 0, 10, 10, rng)                 # touches a
    big = _patch(m.verts, far, 65, 65, rng)              # more than 64 vertices
    sets = [a, b, a2, big]
    so, merged = _merge(g, torch, dm, sets, cap=512)
    br = torch.tensor([0, 0, 0, 3], dtype=torch.int32).cuda()
    bc = torch.tensor([1, 2, 1, 0], dtype=torch.int32).cuda()
    out1, st1 = g.lin_blocks(dm[0], dm[1], merged, so, br, bc, 65 * 64, 3, False)
    out2, st2 = g.lin_blocks(dm[0], dm[1], merged, so, br, bc, 65 * 64, 3, False)
    torch.cuda.synchronize()
    assert list(st1.cpu().numpy()) == [0, 1, 0, 2]
    assert torch.equal(out1[0, :900], out2[0, :900]) and torch.equal(out1[0, :900], out1[2, :900])
    assert (out1[1, :300] == 0).all() and (out1[3, :65 * 30] == 0).all()


def test_blocks_sphere_l8_sample(env):
    # the bench workload's block shape on the level-8 sphere: rows and columns
    # 32 vertices drawn from the 256 nearest to a random centre
    g, torch = env
    m = synth.icosphere(8)
    dm = _device_mesh(g, torch, m.verts, m.tris)
    rng = np.random.default_rng(5)
    from scipy.spatial import cKDTree
    kd = cKDTree(m.verts)
    sets, pairs = [], []
    for _ in range(4):
        while True:
            a, b = rng.integers(m.nv, size=2)
            if np.linalg.norm(m.verts[a] - m.verts[b]) > 0.2:
                break
        for c in (a, b):
            _, nb = kd.query(m.verts[c], k=256)
            sets.append(rng.choice(nb, size=32, replace=False))
        pairs.append((len(sets) - 2, len(sets) - 1))
    so, merged = _merge(g, torch, dm, sets, cap=192)
    br = torch.tensor([p[0] for p in pairs], dtype=torch.int32).cuda()
    bc = torch.tensor([p[1] for p in pairs], dtype=torch.int32).cuda()
    out, st = g.lin_blocks(dm[0], dm[1], merged, so, br, bc, 1024, 2, True)
    out, st = out.cpu().numpy(), st.cpu().numpy()
    assert (st == 0).all()
    # the oracle's sets T_i for the vertices involved only
    need = sorted(set(int(v) for s in sets for v in s))
    hit = np.isin(m.tris, need).any(axis=1)
    T = {}
    for t in np.nonzero(hit)[0]:
        for v in m.tris[t]:
            T.setdefault(int(v), []).append(int(t))
    T = [sorted(T.get(v, [])) if v in T else [] for v in range(m.nv)]
    for b, (r, c) in enumerate(pairs):
        want = L.lin_block(m.verts, m.tris, sets[r], sets[c], 2, True, T=T)
        assert np.abs(out[b].reshape(32, 32) - want).max() <= 1e-12 * np.abs(want).max()


@pytest.mark.parametrize("q,sym,q_s", [(3, False, 5), (2, True, 4), (1, False, 3)])
def test_touching_blocks_equal_oracle(env, q, sym, q_s):
    # blocks whose row and column triangles share vertices (identical, common
    # edge, common vertex): the Sauter-Schwab rules with the nodal weights
    g, torch = env
    m = synth.icosphere(2)
    dm = _device_mesh(g, torch, m.verts, m.tris)
    rng = np.random.default_rng(50 + q + 7 * sym)
    T = _numpy_T(m.tris, m.nv)
    c = int(rng.integers(m.nv))
    far = int(np.argmax(((m.verts - m.verts[c]) ** 2).sum(1)))
    sets = [_patch(m.verts, c, 24, 24, rng),          # contiguous patch
            _patch(m.verts, c, 17, 60, rng),          # scattered over a wider neighbourhood
            np.array([c]),
            _patch(m.verts, far, 9, 9, rng)]          # far away: regular pairs only
    pairs = [(0, 0), (0, 1), (1, 0), (2, 2), (2, 0), (1, 1), (0, 3)]
    so, merged = _merge(g, torch, dm, sets, cap=192)
    br = torch.tensor([p[0] for p in pairs], dtype=torch.int32).cuda()
    bc = torch.tensor([p[1] for p in pairs], dtype=torch.int32).cuda()
    out, st = g.lin_blocks(dm[0], dm[1], merged, so, br, bc, 64 * 64, q, sym, q_s=q_s)
    out2, _ = g.lin_blocks(dm[0], dm[1], merged, so, br, bc, 64 * 64, q, sym, q_s=q_s)
    out, out2, st = out.cpu().numpy(), out2.cpu().numpy(), st.cpu().numpy()
    assert (st == 0).all()
    for k, (r, c_) in enumerate(pairs):
        want = L.lin_block(m.verts, m.tris, sets[r], sets[c_], q, sym, T=T, q_s=q_s)
        got = out[k, :want.size].reshape(want.shape)
        assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max(), (k, q, sym, q_s)
        # the stride beyond n m is not written; the block is the same bit for bit
        assert np.array_equal(out[k, :want.size], out2[k, :want.size])


def test_touching_full_matrix_level1(env):
    # the whole linear-basis Galerkin matrix of the level-1 sphere as one block:
    # equal to the oracle, symmetric up to the rules' asymmetry, positive definite
    g, torch = env
    m = synth.icosphere(1)
    dm = _device_mesh(g, torch, m.verts, m.tris)
    T = _numpy_T(m.tris, m.nv)
    sets = [np.arange(m.nv)]
    so, merged = _merge(g, torch, dm, sets, cap=192)
    z = torch.zeros(1, dtype=torch.int32).cuda()
    out, st = g.lin_blocks(dm[0], dm[1], merged, so, z, z, 64 * 64, 3, False, q_s=6)
    G = out.cpu().numpy()[0, :m.nv * m.nv].reshape(m.nv, m.nv)
    assert st.cpu().numpy()[0] == 0
    want = L.lin_block(m.verts, m.tris, range(m.nv), range(m.nv), 3, False, T=T, q_s=6)
    assert np.abs(G - want).max() <= 1e-12 * np.abs(want).max()
    assert np.abs(G - G.T).max() <= 1e-6 * np.abs(G).max()
    assert np.linalg.eigvalsh(0.5 * (G + G.T)).min() > 0
    # without q_s the same block is refused (status 1, zeros)
    out0, st0 = g.lin_blocks(dm[0], dm[1], merged, so, z, z, 64 * 64, 3, False)
    assert st0.cpu().numpy()[0] == 1 and (out0[0, :m.nv * m.nv] == 0).all()
