"""Choice of beta (section 3.1): the cross-validation and decoherence estimators on the GPU against
the oracle, and the estimator curves of a beta sweep on a noisy sparse-angle phantom."""
import numpy as np
import pytest
import torch

import oracle
import synth
import paper_1306_1392_amd as ph
from paper_1306_1392_amd.beta import select_beta

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("kind", [ph.FP_AUTO, ph.FP_BLOCKS, ph.FP_STAGED, ph.FP_LINES])
def test_cv_error_parity(dev, kind):
    N, K, nb = 40, 24, 50
    rng = synth.rng_for(8, 0, 0)
    ang = synth.uniform_angles(K) + rng.uniform(-0.3, 0.3, K) * np.pi / K   # jittered, still covering 180 deg
    sh = rng.normal(0, 0.5, K)
    g = ph.Geometry(N, N, nb, ang, 24.3, axis_shift=sh, pixel_size=1.1)
    og = oracle.Geom(N, N, nb, ang, 24.3, shifts=sh, pixel_size=1.1)
    x = rng.standard_normal((2, N, N)).astype(np.float32)
    y = (oracle.forward_project(x, og) * 0.9 + 0.3 * rng.standard_normal((2, K, nb))).astype(np.float32)
    plan = ph.Plan(g, n_slices=2)
    plan.set_fp_kernel(kind)
    xt, yt = torch.from_numpy(x).to(dev), torch.from_numpy(y).to(dev)
    for k in (0, 7, K - 1):
        got = ph.cv_error(plan, xt, yt, k).cpu().numpy()
        ref = [oracle.cv_error(x[s], y[s], og, k) for s in range(2)]
        np.testing.assert_allclose(got, ref, rtol=1e-4)
    with pytest.raises(ph.PyhstError):
        ph.cv_error(plan, xt, yt, K)
    # the average over excluded projections, accumulated in the library with weight 1/count
    ks = (0, 7, K - 1)
    acc = torch.empty(2, device=dev, dtype=torch.float32)
    for n, k in enumerate(ks):
        ph.cv_error(plan, xt, yt, k, out=acc, weight=1.0 / len(ks), accumulate=n > 0)
    ref = [np.mean([oracle.cv_error(x[s], y[s], og, k) for k in ks]) for s in range(2)]
    np.testing.assert_allclose(acc.cpu().numpy(), ref, rtol=1e-4)


def test_decoherence_parity(dev):
    rng = synth.rng_for(8, 1, 0)
    a = rng.standard_normal((3, 33, 47)).astype(np.float32)
    b = (a + 0.3 * rng.standard_normal(a.shape)).astype(np.float32)
    g = ph.Geometry(47, 33, 60, synth.uniform_angles(10), 29.5)
    plan = ph.Plan(g, n_slices=3)
    got = ph.decoherence(plan, torch.from_numpy(a).to(dev), torch.from_numpy(b).to(dev)).cpu().numpy()
    ref = [oracle.e_cohe(a[s], b[s]) for s in range(3)]
    np.testing.assert_allclose(got, ref, rtol=1e-5, atol=1e-7)


def test_beta_sweep_estimators(dev):
    """96^2 phantom, 40 projections, 3 % Gaussian noise, FISTA: the cross-validation minimum lies within a
    factor 3 of the beta that minimises the error to the ground truth, and |E_cohe| grows past the optimum
    (the distortion region the paper describes)."""
    N, K = 96, 40
    ell = synth.random_ellipses(synth.rng_for(7, 0, 0), 8)
    ang = synth.uniform_angles(K)
    axis = (N - 1) / 2
    y0 = synth.ellipse_sinogram(ell, ang, N, axis, N).numpy()
    y = y0 + np.random.default_rng(1).standard_normal(y0.shape) * 0.03 * y0.max()
    truth = torch.from_numpy(synth.ellipse_raster(ell, N).numpy()).float().to(dev)
    g = ph.Geometry(N, N, N, ang, axis)
    betas = np.geomspace(0.3, 300, 10)
    r = select_beta(g, torch.from_numpy(y).float()[None].contiguous().to(dev), betas, n_iter=200, n_inner=10)
    rmse = torch.sqrt(((r["x"][:, 0] - truth) ** 2).mean(dim=(1, 2))).cpu().numpy()
    b_opt = betas[np.argmin(rmse)]
    b_cv = betas[np.argmin(r["cv"][:, 0])]
    assert b_opt / 3 <= b_cv <= 3 * b_opt, (b_cv, b_opt, r["cv"][:, 0], rmse)
    e = np.abs(r["e_cohe"][:, 0])
    assert e[-1] > 2 * e[np.argmin(rmse)], (e, rmse)
