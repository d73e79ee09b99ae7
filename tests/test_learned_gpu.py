"""The learned corrector, trained by the library's own kernels on phantoms the
method itself generates, improves on plain FBP; its data-consistency check
sends inconsistent data to the TV mode."""
import numpy as np
import pytest
import torch

import synth
import paper_1306_1392_amd as ph
from paper_1306_1392_amd.cnn import UNet, init_params
from paper_1306_1392_amd.corrector import Corrector

pytestmark = pytest.mark.gpu


def make(indices, stream, N, K, B, plan_hi, plan_b, dev):
    ys, xs, ts = [], [], []
    for i0 in range(0, len(indices), B):
        y, tr, _, _ = synth.configs.cfg_learned(list(indices[i0:i0 + B]), stream,
                                                lambda t: ph.forward_project(plan_hi, t), N=N, K=K, device=dev)
        xs.append(ph.reconstruct_slices(plan_b, sino=y.contiguous(), method=ph.FBP).clone())
        ys.append(y)
        ts.append(tr)
    return torch.cat(xs), torch.cat(ts), torch.cat(ys)


def test_trained_corrector_beats_fbp_and_falls_back(dev):
    N, K, B, SCALE = 128, 30, 16, 10.0
    ang = np.arange(K) * (np.pi / K)
    geo = ph.Geometry(N, N, N, ang, (N - 1) / 2)
    plan_b = ph.Plan(geo, n_slices=B)
    plan_hi = ph.Plan(ph.Geometry(2 * N, 2 * N, N, ang, (N - 1) / 2, pixel_size=0.5))
    xtr, ttr, _ = make(np.arange(512), 0, N, K, B, plan_hi, plan_b, dev)
    xte, tte, yte = make(np.arange(32), 1, N, K, B, plan_hi, plan_b, dev)
    net = UNet(B, N, N, 16, 3)
    net.set_params(init_params(16, 3, 0))
    rng = np.random.default_rng(0)
    steps = 400
    for st in range(steps):
        idx = torch.as_tensor(rng.choice(xtr.shape[0], B, replace=False), device=dev)
        lr = 2e-3 * 0.5 * (1 + np.cos(np.pi * st / steps))
        net.train_step((xtr[idx] * SCALE).contiguous(), (ttr[idx] * SCALE).contiguous(), lr)
    out = torch.cat([net.forward((xte[i:i + B] * SCALE).contiguous()) / SCALE for i in range(0, 32, B)])
    rmse_fbp = float(torch.sqrt(((xte - tte) ** 2).mean()))
    rmse_cnn = float(torch.sqrt(((out - tte) ** 2).mean()))
    assert rmse_cnn < 0.85 * rmse_fbp, (rmse_cnn, rmse_fbp)

    # data-consistency fallback: consistent test data pass, corrupted data go to TV
    params = net.get_params()
    corr = Corrector(geo, B, params, base=16, levels=3, tv_lambda=1e-3, tv_iters=30)
    corr.net = net      # same weights; the corrector applies the network to SCALE-free FBP input
    y = yte[:B].contiguous()
    _, r = corr.correct(y * 1.0)
    corr.dc_threshold = 1.5 * float(r.max())
    bad = y.clone()
    bad[: B // 2] += 0.5 * float(y.max()) * torch.randn_like(bad[: B // 2])
    x, fell = corr.reconstruct(bad)
    assert fell[: B // 2].all() and not fell[B // 2:].any()
    assert torch.isfinite(x).all()
