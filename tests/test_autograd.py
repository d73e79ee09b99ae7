"""Autograd adjoint pairs over the HIP projector and backprojector, checked by
central finite differences (exact for the quadratic losses used here, up to
rounding), by the adjoint identity and against the FP64 oracle's gradient."""
import math

import numpy as np
import pytest
import torch

import oracle
import synth
import paper_1306_1392_amd as ph
from paper_1306_1392_amd import autograd as ag

pytestmark = pytest.mark.gpu


def setup(N=64, K=48, s=1.0, shifts=True):
    ang = synth.uniform_angles(K)
    sh = np.random.default_rng(5).normal(0, 0.5, K) if shifts else None
    nb = int(math.ceil(N * s)) + 6
    g = ph.Geometry(N, N, nb, ang, (nb - 1) / 2 + 0.7, sh, pixel_size=s)
    og = oracle.Geom(N, N, nb, ang, (nb - 1) / 2 + 0.7, sh, pixel_size=s)
    return g, og, ph.Plan(g)


def fd_check(fn, x, v, eps):
    """directional derivative of a quadratic: autograd vs central difference (exact for any
    step up to rounding, so a large step keeps FP32 rounding of the residual negligible)"""
    x = x.clone().requires_grad_(True)
    loss = fn(x)
    (gr,) = torch.autograd.grad(loss, x)
    ana = float((gr.double() * v.double()).sum())
    with torch.no_grad():
        num = (float(fn(x + eps * v).double()) - float(fn(x - eps * v).double())) / (2 * eps)
    return ana, num


@pytest.mark.parametrize("s", [1.0, 0.75])
def test_project_finite_differences(dev, s):
    g, og, plan = setup(s=s)
    gen = torch.Generator(device="cpu").manual_seed(1)
    x = torch.rand((1, 64, 64), generator=gen).to(dev)
    y = torch.rand((1, g.n_angles, g.n_det), generator=gen).to(dev)
    v = torch.randn((1, 64, 64), generator=gen).to(dev)
    ana, num = fd_check(lambda z: ((ag.project(z, plan) - y).double() ** 2).sum(), x, v, 0.5)
    assert abs(ana - num) <= 2e-4 * abs(ana)


def test_backproject_finite_differences(dev):
    g, og, plan = setup()
    gen = torch.Generator(device="cpu").manual_seed(2)
    q = torch.rand((1, g.n_angles, g.n_det), generator=gen).to(dev)
    t = torch.rand((1, 64, 64), generator=gen).to(dev)
    v = torch.randn((1, g.n_angles, g.n_det), generator=gen).to(dev)
    ana, num = fd_check(lambda z: ((ag.backproject(z, plan) - t).double() ** 2).sum(), q, v, 0.5)
    assert abs(ana - num) <= 2e-4 * abs(ana)


def test_fbp_finite_differences(dev):
    g, og, plan = setup(shifts=False)
    gen = torch.Generator(device="cpu").manual_seed(3)
    p = torch.rand((1, g.n_angles, g.n_det), generator=gen).to(dev)
    t = torch.rand((1, 64, 64), generator=gen).to(dev)
    v = torch.randn((1, g.n_angles, g.n_det), generator=gen).to(dev)
    ana, num = fd_check(lambda z: ((ag.fbp(z, plan) - t).double() ** 2).sum(), p, v, 0.5)
    assert abs(ana - num) <= 2e-4 * abs(ana)


def test_project_gradient_matches_oracle(dev):
    """d/dx 1/2|A x - y|^2 = A^T (A x - y), with A^T from the FP64 oracle (s^2 B)."""
    g, og, plan = setup(s=0.9)
    rng = np.random.default_rng(4)
    x = rng.random((64, 64)).astype(np.float32)
    y = rng.random((g.n_angles, g.n_det)).astype(np.float32)
    xt = torch.from_numpy(x)[None].to(dev).requires_grad_(True)
    loss = 0.5 * ((ag.project(xt, plan) - torch.from_numpy(y)[None].to(dev)) ** 2).sum()
    loss.backward()
    r = oracle.forward_project(x, og) - y
    ref = og.pixel_size ** 2 * oracle.backproject(r, og)
    got = xt.grad[0].double().cpu().numpy()
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) <= 1e-5


@pytest.mark.parametrize("s", [1.0, 0.75])
def test_backproject_and_fbp_gradients_match_oracle(dev, s):
    """BackProject.backward = B^T g = A g / s^2 and FBP.backward = F^T B^T g = F (A g / s^2), each with A,
    B and F from the FP64 oracle (the backward passes run entirely in the library: forward_project with
    alpha = 1/s^2, then fbp_filter)."""
    g, og, plan = setup(s=s, shifts=False)
    rng = np.random.default_rng(9)
    q = rng.random((g.n_angles, g.n_det)).astype(np.float32)
    t = rng.random((64, 64)).astype(np.float32)
    qt = torch.from_numpy(q)[None].to(dev).requires_grad_(True)
    loss = 0.5 * ((ag.backproject(qt, plan) - torch.from_numpy(t)[None].to(dev)) ** 2).sum()
    loss.backward()
    r = oracle.backproject(q, og) - t
    ref = oracle.forward_project(r, og) / s ** 2
    assert np.linalg.norm(qt.grad[0].double().cpu().numpy() - ref) / np.linalg.norm(ref) <= 1e-5
    pt = torch.from_numpy(q)[None].to(dev).requires_grad_(True)
    loss = 0.5 * ((ag.fbp(pt, plan) - torch.from_numpy(t)[None].to(dev)) ** 2).sum()
    loss.backward()
    r = oracle.fbp(q, og) - t
    ref = oracle.fbp_filter(oracle.forward_project(r, og) / s ** 2, og)[0]
    assert np.linalg.norm(pt.grad[0].double().cpu().numpy() - ref) / np.linalg.norm(ref) <= 1e-5


def test_gradient_descent_through_projector_reduces_residual(dev):
    """Least-squares fitting through Project (the physics in the autograd graph)."""
    g, og, plan = setup(shifts=False)
    truth = synth.ellipse_raster(synth.disc_params(0.4, 1.0, 0.1, 0.0), 64).float()[None].to(dev)
    y = ph.forward_project(plan, truth.contiguous())
    x = torch.zeros_like(truth, requires_grad=True)
    opt = torch.optim.SGD([x], lr=1e-4)
    first = None
    for _ in range(50):
        opt.zero_grad()
        loss = 0.5 * ((ag.project(x, plan) - y) ** 2).sum()
        loss.backward()
        opt.step()
        first = first or float(loss)
    assert float(loss) < 0.2 * first
