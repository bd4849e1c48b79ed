"""gca_energy_noalloc (the energy call whose workspace is the library's fixed
device array) against gca_energy through the C-ABI: two calls in a row, the
second on a smaller mesh, E alone and E with g = scale * G~ u, both
precisions; bit-equal results (the same kernels in the same order), and the
size limit when g is NULL."""
import ctypes

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


def _handle(gca, level, leaf):
    m = synth.icosphere(level)
    return m, gca.H2(m.verts, m.tris, gca.Tree(m.verts, m.tris, leaf), gca.Params(eta=2.0, eps=1e-6))


def _raw_call(gca, torch, H, u, e, g, prec, fn):
    """The entry point called through ctypes with raw device pointers."""
    L = gca.lib()
    vp = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else None
    sp = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return getattr(L, fn)(H.h, vp(u), None, vp(e), vp(g), int(prec), sp)


@pytest.mark.parametrize("prec", [0, 1])
def test_noalloc_energy_equals_energy_on_two_calls_second_smaller(torch, gca, prec):
    cases = [(4, 32), (2, 16)]   # n = 5120, then n = 320
    for level, leaf in cases:
        m, H = _handle(gca, level, leaf)
        print(f"[no-alloc] level {level} n {m.nt} precision {prec}", flush=True)
        u = torch.tensor(synth.rhs_normal(m.nt, 1, seed=level), device="cuda")
        sc = torch.tensor(0.75, dtype=torch.float64, device="cuda")
        # E alone: the product G~ u lives in the fixed workspace
        e_ref = torch.empty((), dtype=torch.float64, device="cuda")
        e_new = torch.full((), float("nan"), dtype=torch.float64, device="cuda")
        assert _raw_call(gca, torch, H, u, e_ref, None, prec, "gca_energy") == 0
        assert _raw_call(gca, torch, H, u, e_new, None, prec, "gca_energy_noalloc") == 0, \
            gca.lib().gca_last_error()
        torch.cuda.synchronize()
        assert float(e_new) == float(e_ref) and np.isfinite(float(e_ref))
        # E and g = scale * G~ u through the binding
        e1, g1 = H.energy(u, prec, scale=sc, want_e=True, want_g=True)
        e2, g2 = H.energy_noalloc(u, prec, scale=sc, want_e=True, want_g=True)
        torch.cuda.synchronize()
        assert float(e1) == float(e2) == float(e_ref)
        assert torch.equal(g1, g2)
        # the energy is 1/2 u^T G~ u of the product (FP64 dot, fixed order)
        y = H.matvec(u, precision=prec)
        assert abs(float(e_ref) - 0.5 * float(torch.dot(u, y))) <= 1e-12 * abs(float(e_ref))
        H.close()


def test_noalloc_energy_rejects_n_beyond_the_limit_without_g(torch, gca):
    m, H = _handle(gca, 6, 64)   # n = 81920 > GCA_NOALLOC_MAX_N = 65536
    u = torch.tensor(synth.rhs_normal(m.nt, 1, seed=0), device="cuda")
    e = torch.empty((), dtype=torch.float64, device="cuda")
    assert _raw_call(gca, torch, H, u, e, None, 0, "gca_energy_noalloc") == -1
    assert b"GCA_NOALLOC_MAX_N" in gca.lib().gca_last_error()
    # with g given any n is accepted (the workspace is the dot partials only)
    g = torch.empty_like(u)
    e2 = torch.empty((), dtype=torch.float64, device="cuda")
    assert _raw_call(gca, torch, H, u, e2, g, 0, "gca_energy_noalloc") == 0
    assert _raw_call(gca, torch, H, u, e, None, 0, "gca_energy") == 0
    torch.cuda.synchronize()
    assert float(e2) == float(e)
    H.close()
