"""Parity at the full workload sizes, in the launch configuration bench.py times.

* Batched FBP from raw: 64 slices of 2048^2, 1800 projections, raw uint16 with two
  flats and a dark, one HIP graph per step.  The oracle recomputes two of the 64 slices
  at 3000 random pixels each (normalise, direct Ram-Lak filter of all 1800 rows,
  backprojection at those pixels).
* TV-CP at 1024^2 / 128 projections / Poisson 1e4 (eq. (3), section 3.1): iterates 1, 10,
  100 and 300 and the 300-step energy trace against the oracle's, with the oracle's |K|;
  the same with the gradient block scaled by mu = |A| / |grad|.
* Uneven persistent batch at real size: 2048^2 slices with up to 3600 projections, half
  of them 360 degree half-acquisition scans with the axis near a detector edge and
  per-projection axis shifts (section 2.1), plus smaller slices, in one persistent
  launch captured in a graph; 3000 oracle pixels per slice.
"""
import math

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


@pytest.fixture(scope="module")
def tv1024():
    """cfg: 1024^2, 1024 bins, 128 projections, Poisson 1e4, and the oracle's operator norms (x 1.02, so
    tau sigma |K|^2 < 1), computed once."""
    d = synth.cfg_tv_sparse(N=1024, K=128)
    og = oracle.Geom(1024, 1024, 1024, d["angles"], d["axis"])
    x0 = synth.rng_for(3, 9, 3).standard_normal((1024, 1024))
    norm_a = oracle.opnorm(og, x0, 60, with_grad=False)
    mu = norm_a / (2.0 * math.sqrt(2.0))
    return dict(d=d, og=og, Lk=1.02 * oracle.opnorm(og, x0, 60), mu=mu,
                Lk_mu=1.02 * oracle.opnorm(og, x0, 60, mu=mu),
                plan=ph.Plan(ph.Geometry(1024, 1024, 1024, d["angles"], d["axis"])))


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("k", [1, 10, 100])
def test_tv_cp_1024_iterates(dev, tv1024, k):
    d, og, Lk = tv1024["d"], tv1024["og"], tv1024["Lk"]
    y = d["y"][None].contiguous().to(dev)
    x = ph.reconstruct_slices(tv1024["plan"], sino=y, method=ph.TV_CP, lam=0.01, n_iter=k, op_norm=Lk)
    ref = oracle.cp_tv(d["y"].numpy(), og, 0.01, k, Lk)
    assert _rel(x[0].double().cpu().numpy(), ref) <= 1e-4, (k, _rel(x[0].double().cpu().numpy(), ref))


@pytest.mark.parametrize("balanced", [False, True])
def test_tv_cp_1024_300_iterations_and_energy(dev, tv1024, balanced):
    """300 iterations at full size, plain (mu = 1) and with the balanced gradient block, in one captured
    graph with the energy written on the device; iterate and the whole energy trace against the
    oracle's.  The balanced run ends at a lower energy of eq. (3)."""
    d, og = tv1024["d"], tv1024["og"]
    mu = tv1024["mu"] if balanced else 1.0
    Lk = tv1024["Lk_mu"] if balanced else tv1024["Lk"]
    y = d["y"][None].contiguous().to(dev)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        x, E = ph.reconstruct_slices(tv1024["plan"], sino=y, method=ph.TV_CP, lam=0.01, n_iter=300, op_norm=Lk,
                                     tv_mu=mu, energy=True, use_graph=True, stream=side)
    side.synchronize()
    ref, Er = oracle.cp_tv(d["y"].numpy(), og, 0.01, 300, Lk, energy=True, mu=mu)
    assert _rel(x[0].double().cpu().numpy(), ref) <= 1e-4, _rel(x[0].double().cpu().numpy(), ref)
    np.testing.assert_allclose(E, Er, rtol=1e-4)
    tv1024.setdefault("E300", {})[balanced] = float(Er[-1])
    if len(tv1024["E300"]) == 2:
        assert tv1024["E300"][True] < tv1024["E300"][False]


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


def test_uneven_realsize_sampled(dev):
    """Uneven batch at the sizes of the uneven workload: four 2048^2 slices with 3400-3600 projections (two
    of them 360 degree half-acquisition scans, axis 16-64 bins from an edge) and two smaller slices, every
    projection with its own axis shift, reconstructed by one persistent backprojection launch in a HIP
    graph; 3000 random pixels of each slice against the oracle (direct filter, point-wise backprojection)."""
    big = synth.cfg_uneven(n_slices=4, index=7, sizes=(2048,), k_range=(3400, 3600))
    small = synth.cfg_uneven(n_slices=2, index=8, sizes=(512, 1024), k_range=(90, 3600))
    specs, sinos = big["specs"] + small["specs"], big["sinos"] + small["sinos"]
    assert any(s["scan"] == ph.SCAN_360_HALF and s["N"] == 2048 for s in specs)
    geos = [ph.Geometry(s["N"], s["N"], s["nb"], s["angles"], s["axis"], axis_shift=s["shifts"], scan=s["scan"])
            for s in specs]
    plan = ph.Plan(geos, slice_geom=list(range(len(geos))))
    plan.set_tiles(-1, True)
    packed = torch.cat([t.reshape(-1) for t in sinos]).to(dev)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        out = ph.reconstruct_slices(plan, sino=packed, method=ph.FBP, use_graph=True, stream=side)
    side.synchronize()
    rng = np.random.default_rng(5005)
    for i, s in enumerate(specs):
        info = plan.slice_info(i)
        N = s["N"]
        og = oracle.Geom(N, N, s["nb"], s["angles"], s["axis"], s["shifts"], scan=s["scan"])
        filt = oracle.fbp_filter(sinos[i].numpy()[None], og)[0]
        ix, iy = rng.integers(0, N, 3000), rng.integers(0, N, 3000)
        ref = oracle.backproject_points(filt, og, ix, iy, extended=True)
        img = out[info.img_offset:info.img_offset + N * N].reshape(N, N)
        got = img.cpu().numpy()[iy, ix].astype(np.float64)
        assert _rel(got, ref) <= 1e-4, (i, s["N"], s["K"], s["scan"], _rel(got, ref))
