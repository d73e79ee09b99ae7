"""Parity at the full workload sizes, in the launch configuration bench.py times.

* Batched FBP from raw: 64 slices of 2048^2, 1800 projections, raw uint16 with two
  flats and a dark, one HIP graph per step.  The oracle recomputes two of the 64 slices
  at 3000 random pixels each (normalise, direct Ram-Lak filter of all 1800 rows,
  backprojection at those pixels).
* TV-CP at 1024^2 / 128 projections / Poisson 1e4: iterate 10 against the oracle's
  (with the same step bound L, a constant above |[A; grad]|).
"""
import numpy as np
import pytest
import torch

import oracle
import synth
import paper_1306_1392_amd as ph

pytestmark = pytest.mark.gpu


def test_fbp_2048_batch_sampled(dev):
    R, N, K = 64, 2048, 1800
    cfg = synth.cfg_batched_raw(R=R, N=N, K=K, device=dev)
    plan = ph.Plan(ph.Geometry(N, N, N, cfg["angles"], cfg["axis"]), n_slices=R)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        out = ph.reconstruct_slices(plan, raw=cfg["raw"], flats=cfg["flats"], flat_pos=cfg["flat_pos"],
                                    dark=cfg["dark"], method=ph.FBP, use_graph=True, stream=side)
    side.synchronize()
    g = oracle.Geom(N, N, N, cfg["angles"], cfg["axis"])
    rng = np.random.default_rng(2048)
    for r in (0, 37):
        raw = cfg["raw"][:, r:r + 1, :].cpu().numpy().astype(np.float64)
        sino = oracle.normalize(raw, cfg["flats"][:, r:r + 1, :].cpu().numpy(), cfg["flat_pos"],
                                cfg["dark"][r:r + 1].cpu().numpy())
        filt = oracle.fbp_filter(sino, g)[0]
        ix = rng.integers(0, N, 3000)
        iy = rng.integers(0, N, 3000)
        ref = oracle.backproject_points(filt, g, ix, iy)
        got = out[r].cpu().numpy()[iy, ix].astype(np.float64)
        rel = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        assert rel <= 1e-4, (r, rel)


def test_tv_cp_1024_iterates(dev):
    d = synth.cfg_tv_sparse(N=1024, K=128)
    g = ph.Geometry(1024, 1024, 1024, d["angles"], d["axis"])
    og = oracle.Geom(1024, 1024, 1024, d["angles"], d["axis"])
    L = 400.0     # above |[A; grad]| (about 361 for this geometry): CP converges for any L >= |K|
    y = d["y"][None].contiguous().to(dev)
    x = ph.reconstruct_slices(ph.Plan(g), sino=y, method=ph.TV_CP, lam=0.01, n_iter=10, op_norm=L)
    ref = oracle.cp_tv(d["y"].numpy(), og, 0.01, 10, L)
    rel = float(np.linalg.norm(x[0].double().cpu().numpy() - ref) / np.linalg.norm(ref))
    assert rel <= 1e-4, rel


def test_cp_300_iterations_small(dev):
    d = synth.cfg_tv_sparse(N=192, K=48, index=4)
    g = ph.Geometry(192, 192, 192, d["angles"], d["axis"])
    og = oracle.Geom(192, 192, 192, d["angles"], d["axis"])
    Lk = oracle.opnorm(og, synth.rng_for(3, 9, 1).standard_normal((192, 192)), 200)
    x = ph.reconstruct_slices(ph.Plan(g), sino=d["y"][None].contiguous().to(dev), method=ph.TV_CP, lam=0.01,
                              n_iter=300, op_norm=Lk)
    ref = oracle.cp_tv(d["y"].numpy(), og, 0.01, 300, Lk)
    rel = float(np.linalg.norm(x[0].double().cpu().numpy() - ref) / np.linalg.norm(ref))
    assert rel <= 1e-4, rel


def test_autotune_and_residual(dev):
    gen = np.random.default_rng(3)
    g = ph.Geometry(200, 200, 210, synth.uniform_angles(150), 104.2)
    plan = ph.Plan(g, n_slices=3)
    filt = torch.from_numpy(gen.standard_normal((3, 150, 210)).astype(np.float32)).to(dev)
    before = ph.backproject(plan, filt, 1)
    img = torch.empty_like(before)
    ms = plan.autotune(filt, img, reps=2)
    assert ms > 0
    after = ph.backproject(plan, filt, 1)
    assert float((after - before).norm() / before.norm()) < 1e-6
    y = torch.from_numpy(gen.random((3, 150, 210)).astype(np.float32)).to(dev)
    ax = y * torch.tensor([1.0, 1.1, 0.5], device=dev)[:, None, None]
    r = ph.slice_residual(plan, ax.contiguous(), y).cpu().numpy()
    np.testing.assert_allclose(r, [0.0, 0.1, 0.5], atol=1e-6)
