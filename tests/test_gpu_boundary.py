"""The C-ABI conventions of include/gca.h on the GPU: vector element types,
the device-memory callbacks, and the energy call.  Every call goes through
libgca (ctypes); the references are other calls of the same library, or the
dense oracle."""
import ctypes

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no HIP device")
    return t


@pytest.fixture(scope="module")
def gca(torch):
    import paper_1810_08429_amd as g
    g.lib()
    return g


@pytest.fixture(scope="module")
def mesh():
    return synth.jitter(synth.icosphere(3), 1e-3 * 0.15, seed=3)


def build(gca, m, leaf=32, **kw):
    tree = gca.Tree(m.verts, m.tris, leaf)
    return gca.H2(m.verts, m.tris, tree, gca.Params(eta=2.0, eps=1e-6, **kw))


@pytest.mark.parametrize("prec", [0, 1])
def test_fp32_vectors_are_widened_and_rounded(torch, gca, mesh, prec):
    """dtype GCA_F32: x is widened on entry and y rounded on exit, so the
    result equals the FP64-vector product of the same (FP32-representable) x,
    rounded to FP32, bit for bit; several right-hand sides with ld > n too."""
    H = build(gca, mesh)
    n = mesh.nt
    X = synth.rhs_normal(n, 3, seed=4)
    ld = n + 5
    x32 = torch.zeros((3, ld), dtype=torch.float32, device="cuda")
    x32[:, :n] = torch.tensor(X.T, dtype=torch.float32, device="cuda")
    xs = torch.as_strided(x32, (n, 3), (1, ld))
    y32 = torch.as_strided(torch.full((3, ld), 7.0, dtype=torch.float32, device="cuda"), (n, 3), (1, ld))
    H.matvec_into(xs, y32, precision=prec)
    y64 = H.matvec(xs.double(), precision=prec)
    assert torch.equal(y32, y64.float())
    # the padding between columns is not written
    base = torch.as_strided(y32, (3, ld), (ld, 1))
    assert torch.all(base[:, n:] == 7.0)


def test_fp32_vectors_rejected_when_overlapping(torch, gca, mesh):
    H = build(gca, mesh)
    n = mesh.nt
    buf = torch.zeros(2 * n, dtype=torch.float32, device="cuda")
    L = gca.lib()
    s = gca._stream_ptr(None)
    # y starts inside x's n FP32 elements
    rc = L.h2_matvec(H.h, ctypes.c_void_p(buf.data_ptr()), ctypes.c_void_p(buf.data_ptr() + 4 * (n - 1)), 1, n,
                     gca.F32, 0, s)
    assert rc == -1
    rc = L.h2_matvec(H.h, ctypes.c_void_p(buf.data_ptr()), ctypes.c_void_p(buf.data_ptr() + 4 * n), 1, n,
                     gca.F32, 0, s)
    assert rc == 0
    assert L.h2_matvec(H.h, ctypes.c_void_p(buf.data_ptr()), ctypes.c_void_p(buf.data_ptr() + 4 * n), 1, n,
                       2, 0, s) == -1


def test_torch_allocator_callbacks(torch, gca, mesh):
    """Built with torch's caching allocator the handle's memory shows up in
    torch's accounting and goes back to it at close; products are bit for bit
    those of a handle built on hipMalloc."""
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    Ht = build(gca, mesh, allocator="torch")
    during = torch.cuda.memory_allocated()
    st = Ht.stats()
    assert during - before >= st["basis_bytes_fp64"]
    Hh = build(gca, mesh, allocator=None)
    assert torch.cuda.memory_allocated() == during
    x = torch.tensor(synth.rhs_normal(mesh.nt, 1, seed=2), device="cuda")
    for prec in (gca.FP64, gca.MIXED):
        assert torch.equal(Ht.matvec(x, prec), Hh.matvec(x, prec))
    # calls that allocate lazily (entries, energy, solve, gradient) use it too
    Ht.entries(np.arange(10), np.arange(10) + 3)
    Ht.energy(x)
    Ht.bilinear_grad(x, x, 0.5)
    torch.cuda.synchronize()
    del x
    grown = torch.cuda.memory_allocated()
    assert grown > during
    Ht.close()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == before
    Hh.close()


def test_allocator_failure_is_enomem(torch, gca, mesh):
    """An alloc callback that returns NULL makes gca_build fail with
    GCA_ENOMEM and leaves no handle."""
    calls = []

    def alloc(nbytes, stream, ctx):
        calls.append(nbytes)
        return None

    def free(ptr, stream, ctx):
        raise AssertionError("nothing was allocated")

    fa, ff = gca._ALLOC_FN(alloc), gca._FREE_FN(free)
    tree = gca.Tree(mesh.verts, mesh.tris, 32)
    p = gca.Params(allocator=None)._c()
    p.alloc, p.free = fa, ff
    h = ctypes.c_void_p()
    m = gca._MeshArrays(mesh.verts, mesh.tris)
    rc = gca.lib().gca_build(ctypes.byref(m.c), tree.h, ctypes.byref(p), None, ctypes.byref(h))
    assert rc == -2 and not h.value and calls


@pytest.mark.parametrize("prec", [0, 1])
def test_energy_call(torch, gca, orc, mesh, prec):
    """gca_energy: E = 1/2 u^T G~ u with G~ u the library's product (FP64 dot
    in a fixed order), g = scale * G~ u bit for bit; against the dense oracle
    within the compression tolerance."""
    H = build(gca, mesh)
    u = torch.tensor(synth.rhs_normal(mesh.nt, 1, seed=6), device="cuda")
    e, g = H.energy(u, prec, want_g=True)
    gu = H.matvec(u, prec)
    assert torch.equal(g, gu)
    ref = 0.5 * float(torch.dot(u, gu))
    assert abs(float(e) - ref) <= 1e-13 * abs(ref)
    sc = torch.tensor(-2.5, dtype=torch.float64, device="cuda")
    _, g2 = H.energy(u, prec, scale=sc, want_e=False, want_g=True)
    assert torch.equal(g2, -2.5 * gu)
    G = orc.Entries(mesh.verts, mesh.tris, 3, 3, 4).dense()
    uh = u.cpu().numpy()
    ed = 0.5 * uh @ (G @ uh)
    assert abs(float(e) - ed) <= 1e-5 * abs(ed)


def test_energy_arguments(torch, gca, mesh):
    H = build(gca, mesh)
    L = gca.lib()
    u = torch.zeros(mesh.nt, dtype=torch.float64, device="cuda")
    s = gca._stream_ptr(None)
    vp = lambda t: ctypes.c_void_p(t.data_ptr())
    assert L.gca_energy(H.h, vp(u), None, None, None, 0, s) == -1          # nothing requested
    assert L.gca_energy(H.h, None, None, vp(u), None, 0, s) == -1          # u NULL
    assert L.gca_energy(H.h, vp(u), None, None, vp(u), 0, s) == -1        # g aliases u
    e = torch.zeros((), dtype=torch.float64, device="cuda")
    assert L.gca_energy(H.h, vp(u), None, vp(e), None, 5, s) == -1        # precision
    assert L.gca_energy(H.h, vp(u), None, vp(e), None, 0, s) == 0
    assert float(e) == 0.0


def test_bilinear_grad_device_scale(torch, gca, mesh):
    """The device-scalar factor of h2_bilinear_grad multiplies the gradient
    exactly as the host factor does."""
    H = build(gca, mesh)
    u = torch.tensor(synth.rhs_normal(mesh.nt, 1, seed=8), device="cuda")
    d1 = H.bilinear_grad(u, u, 0.5 * 3.0)
    d2 = H.bilinear_grad(u, u, 0.5, scale=torch.tensor(3.0, dtype=torch.float64, device="cuda"))
    assert torch.allclose(d1, d2, rtol=1e-15, atol=0)
