"""torch.autograd glue of the binding: the vector-Jacobian products of
y = G~ x and of E = 1/2 u^T G~ u with respect to the vector and to the vertex
coordinates (frozen structure), checked against the library calls they route
to and against central differences (runs on an MI355X)."""
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
def setup(torch, gca):
    base = synth.icosphere(3)
    m = synth.jitter(base, 0.02 * synth.mean_edge_length(base), seed=21)
    H = gca.H2(m.verts, m.tris, gca.Tree(m.verts, m.tris, 32), gca.Params(eta=2.0, eps=1e-6))
    return m, H


def test_matvec_vjp_routes_to_the_symmetric_product_and_the_adjoint(torch, gca, setup):
    m, H = setup
    x = torch.tensor(synth.rhs_normal(m.nt, 1, seed=1), device="cuda", requires_grad=True)
    w = torch.tensor(synth.rhs_normal(m.nt, 1, seed=2), device="cuda")
    X = torch.tensor(m.verts, device="cuda", requires_grad=True)
    y = gca.matvec(H, x, X)
    assert torch.equal(y.detach(), H.matvec(x.detach()))
    (w * y).sum().backward()
    # G~ is symmetric: the VJP w.r.t. x is G~ w
    assert torch.equal(x.grad, H.matvec(w))
    ref = H.bilinear_grad(w, x.detach())
    assert torch.equal(X.grad, ref)
    # symmetry itself: w^T G~ x == x^T G~ w to rounding
    a = float(torch.dot(w, H.matvec(x.detach())))
    b = float(torch.dot(x.detach(), H.matvec(w)))
    assert abs(a - b) <= 1e-12 * abs(a)


def test_matvec_vjp_multiple_right_hand_sides(torch, gca, setup):
    m, H = setup
    xs = torch.tensor(synth.rhs_normal(m.nt, 3, seed=4), device="cuda")
    ws = torch.tensor(synth.rhs_normal(m.nt, 3, seed=5), device="cuda")
    X = torch.tensor(m.verts, device="cuda", requires_grad=True)
    (ws * gca.matvec(H, xs, X)).sum().backward()
    ref = sum(H.bilinear_grad(ws[:, k].contiguous(), xs[:, k].contiguous()) for k in range(3))
    assert torch.allclose(X.grad, ref, rtol=1e-12, atol=1e-14 * float(ref.abs().max()))


def test_energy_gradient_matches_central_differences(torch, gca, setup):
    """dE/du = G~ u exactly; dE/dX along a random direction d against the
    central difference of E(X +- h d) with the frozen structure (h = 1e-6)."""
    m, H = setup
    u = torch.tensor(synth.rhs_normal(m.nt, 1, seed=6), device="cuda", requires_grad=True)
    X = torch.tensor(m.verts, device="cuda", requires_grad=True)
    E = gca.energy(H, u, X)
    E.backward()
    assert torch.equal(u.grad, H.matvec(u.detach()))
    d = np.random.default_rng(8).standard_normal(m.verts.shape)
    dirderiv = float((X.grad.cpu() * torch.tensor(d)).sum())
    h = 1e-6
    ud = u.detach()
    vals = []
    for sgn in (1.0, -1.0):
        H.update_geometry(m.verts + sgn * h * d)
        vals.append(float(gca.energy(H, ud)))
    H.update_geometry(m.verts)
    fd = (vals[0] - vals[1]) / (2 * h)
    assert abs(fd - dirderiv) <= 1e-6 * abs(dirderiv), (fd, dirderiv)


def test_mixed_precision_gradient_is_close_to_fp64(torch, gca, setup):
    m, H = setup
    u = torch.tensor(synth.rhs_normal(m.nt, 1, seed=9), device="cuda")
    X64 = torch.tensor(m.verts, device="cuda", requires_grad=True)
    gca.energy(H, u, X64, precision=gca.FP64).backward()
    X32 = torch.tensor(m.verts, device="cuda", requires_grad=True)
    gca.energy(H, u, X32, precision=gca.MIXED).backward()
    err = float((X32.grad - X64.grad).norm() / X64.grad.norm())
    assert err < 1e-4, err
