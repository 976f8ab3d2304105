"""The differentiable imaging operator (degrid forward, grid adjoint backward)
against the oracle, the dot-product adjoint test, gradcheck and finite
differences."""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import synth  # noqa: E402
from oracle import wstack as o  # noqa: E402
import paper_2301_06061_amd as ws  # noqa: E402
from paper_2301_06061_amd.autograd import imaging_op  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _setup(precision, n=32, m=400, seed=5, nw=4, weights=True):
    wl = synth.random_case(seed, n=n, nw=nw, support=7, m=m,
                           precision=1 if precision == "fp64" else 0,
                           weights=weights)
    plan = ws.WStackPlan.from_workload(wl)
    uvw = torch.from_numpy(wl.uvw).to(DEV)
    wt = None if wl.weight is None else torch.from_numpy(wl.weight).to(DEV)
    vis = torch.from_numpy(wl.vis).to(DEV)
    return wl, plan, uvw, wt, vis


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_dot_product_adjoint(precision, tol):
    wl, plan, uvw, wt, vis = _setup(precision, n=64, m=3000)
    rng = np.random.default_rng(1)
    x = (rng.standard_normal((64, 64)) + 1j * rng.standard_normal((64, 64)))
    xt = torch.from_numpy(x).to(DEV).to(plan.cdtype)
    ax = plan.degrid(xt, uvw, wt)
    ahv = plan.dirty_image(uvw, vis, wt)
    lhs = torch.vdot(vis.to(torch.complex128), ax.to(torch.complex128))
    rhs = torch.vdot(ahv.to(torch.complex128).reshape(-1),
                     xt.to(torch.complex128).reshape(-1))
    scale = (torch.linalg.vector_norm(ax.to(torch.complex128)) *
             torch.linalg.vector_norm(vis.to(torch.complex128)))
    assert float(abs(lhs - rhs) / scale) <= tol


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_loss_gradient_matches_oracle(precision, tol):
    """grad ||A x - V||^2 = 2 Re(A^H (A x - V)), checked against the oracle."""
    wl, plan, uvw, wt, vis = _setup(precision, n=64, m=3000, seed=8)
    p = o.Params.of(wl)
    rng = np.random.default_rng(2)
    x = np.zeros((64, 64))
    idx = rng.choice(64 * 64, 40, replace=False)
    x.flat[idx] = rng.standard_normal(40)
    xt = torch.from_numpy(x).to(DEV).to(plan.rdtype).requires_grad_(True)
    y = imaging_op(xt, plan, uvw, wt)
    loss = (y - vis).abs().pow(2).sum()
    loss.backward()
    ax = o.degrid(p, x, wl.uvw, wl.weight)
    r = ax - wl.vis.astype(np.complex128)
    g_ref = 2 * o.image(p, wl.uvw, r, wl.weight).real
    g = xt.grad.detach().cpu().numpy()
    err = np.linalg.norm(g - g_ref) / np.linalg.norm(g_ref)
    assert err <= tol, err
    lref = float(np.sum(np.abs(r) ** 2))
    assert float(loss.item()) == pytest.approx(lref, rel=tol * 10)


def test_gradcheck_fp64():
    wl, plan, uvw, wt, vis = _setup("fp64", n=16, m=40, nw=2)
    x = torch.randn(16, 16, dtype=torch.float64, device=DEV,
                    requires_grad=True)
    assert torch.autograd.gradcheck(
        lambda t: imaging_op(t, plan, uvw, wt), (x,), eps=1e-6, atol=1e-8,
        rtol=1e-6)
    xc = torch.randn(16, 16, dtype=torch.complex128, device=DEV,
                     requires_grad=True)
    assert torch.autograd.gradcheck(
        lambda t: imaging_op(t, plan, uvw, wt), (xc,), eps=1e-6, atol=1e-8,
        rtol=1e-6)


def test_finite_differences_fp32():
    """Central differences of the FP32 loss along random directions."""
    wl, plan, uvw, wt, vis = _setup("fp32", n=64, m=3000, seed=3)
    rng = np.random.default_rng(4)
    x0 = torch.from_numpy(rng.standard_normal((64, 64)).astype(np.float32)
                          ).to(DEV)
    x = x0.clone().requires_grad_(True)
    loss = (imaging_op(x, plan, uvw, wt) - vis).abs().pow(2).sum()
    loss.backward()
    g = x.grad.detach().double()

    def f(t):
        with torch.no_grad():
            return float((imaging_op(t, plan, uvw, wt) - vis).abs().pow(2)
                         .double().sum())

    for k in range(3):
        d = torch.from_numpy(rng.standard_normal((64, 64)).astype(np.float32)
                             ).to(DEV)
        eps = 1e-2
        fd = (f(x0 + eps * d) - f(x0 - eps * d)) / (2 * eps)
        an = float((g * d.double()).sum())
        assert fd == pytest.approx(an, rel=2e-3), (k, fd, an)


def test_config5_scaled_gradient():
    """Config-5 recipe at reduced size: sparse real sky, 2e5 visibilities."""
    wl, x = synth.config5(m=200_000, n=512, nsrc=100)
    p = o.Params.of(wl)
    plan = ws.WStackPlan.from_workload(wl)
    uvw = torch.from_numpy(wl.uvw).to(DEV)
    wt = torch.from_numpy(wl.weight).to(DEV)
    vis = torch.from_numpy(wl.vis).to(DEV)
    xt = torch.from_numpy(x).to(DEV).requires_grad_(True)
    loss = (imaging_op(xt, plan, uvw, wt) - vis).abs().pow(2).sum()
    loss.backward()
    ax = o.degrid(p, x.astype(np.float64), wl.uvw, wl.weight)
    r = ax - wl.vis.astype(np.complex128)
    g_ref = 2 * o.image(p, wl.uvw, r, wl.weight).real
    g = xt.grad.detach().cpu().numpy()
    err = np.linalg.norm(g - g_ref) / np.linalg.norm(g_ref)
    assert err <= 1e-5, err
