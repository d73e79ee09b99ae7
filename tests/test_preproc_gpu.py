"""Preprocessing extras of section 2.3 on the GPU against the oracle: the hot-spot median filter on
flat-field-corrected radiographs, the ring-artifact filter (with and without the thresholded object),
and both inside reconstruct_slices (FBP and Chambolle-Pock)."""
import numpy as np
import pytest
import torch

import oracle
import synth
import paper_1306_1392_amd as ph

pytestmark = pytest.mark.gpu
TOL_OP = 1e-5
TOL_PIPE = 1e-4


def rel(a, b):
    a = a.detach().double().cpu().numpy() if torch.is_tensor(a) else np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def raw_with_spikes(R, N, K, seed):
    """Raw radiographs of ellipse phantoms with 2 flats and a dark, plus hot pixels (+40 % counts)."""
    ang = synth.uniform_angles(K)
    axis = (N - 1) / 2 + 1.5
    p = torch.stack([synth.ellipse_sinogram(synth.random_ellipses(synth.rng_for(10, seed, r), 6), ang, N, axis, N)
                     for r in range(R)])
    raw, flats, flat_pos, dark, _ = synth.raw_acquisition(p, seed=seed)
    rng = synth.rng_for(10, seed, 999)
    r16 = raw.numpy().astype(np.float64)
    n_hot = K * R * N // 50
    kk, rr, jj = rng.integers(0, K, n_hot), rng.integers(0, R, n_hot), rng.integers(0, N, n_hot)
    r16[kk, rr, jj] = np.minimum(r16[kk, rr, jj] * 1.4, 65535)
    raw = torch.from_numpy(r16.round().astype(np.uint16))
    return raw, flats, flat_pos, dark, ang, axis


# With these seeds every pixel's |t - median - threshold| is at least 2.7e-5 (checked in FP64), far
# beyond FP32 rounding, so both sides take the same replacement decisions.
def test_hotspot_normalize_parity(dev):
    R, N, K = 5, 64, 40
    raw, flats, flat_pos, dark, ang, axis = raw_with_spikes(R, N, K, 1)
    plan = ph.Plan(ph.Geometry(N, N, N, ang, axis), n_slices=R)
    got = ph.normalize_hotspot(plan, raw.to(dev), flats.to(dev), flat_pos, dark.to(dev), 0.1)
    ref = oracle.normalize_hotspot(raw.numpy(), flats.numpy(), flat_pos, dark.numpy(), 0.1)
    assert rel(got, ref) <= TOL_OP
    plain = oracle.normalize(raw.numpy(), flats.numpy(), flat_pos, dark.numpy())
    assert rel(plain, ref) > 1e-2                       # the spikes were there and were removed


def test_hotspot_chunks_with_halo_equal_whole_volume(dev):
    """Chunks of rows given one halo row per side (raw, flats and dark of rows r0-1 .. r1) reproduce the
    whole-volume hot-spot filtering bit for bit, and match the oracle's whole volume."""
    R, N, K = 6, 64, 40
    raw, flats, flat_pos, dark, ang, axis = raw_with_spikes(R, N, K, 1)
    geo = ph.Geometry(N, N, N, ang, axis)
    whole = ph.normalize_hotspot(ph.Plan(geo, n_slices=R), raw.to(dev), flats.to(dev), flat_pos, dark.to(dev), 0.1)
    ref = oracle.normalize_hotspot(raw.numpy(), flats.numpy(), flat_pos, dark.numpy(), 0.1)
    for r0, r1 in ((0, 2), (2, 4), (4, 6)):
        lo, hi = max(r0 - 1, 0), min(r1 + 1, R)
        halo = (r0 - lo, hi - r1)
        part = ph.normalize_hotspot(ph.Plan(geo, n_slices=r1 - r0), raw[:, lo:hi].contiguous().to(dev),
                                    flats[:, lo:hi].contiguous().to(dev), flat_pos, dark[lo:hi].contiguous().to(dev),
                                    0.1, halo=halo)
        assert torch.equal(part, whole[r0:r1]), (r0, r1)
        assert rel(part, ref[r0:r1]) <= TOL_OP
        plan = ph.Plan(geo, n_slices=r1 - r0)
        x = ph.reconstruct_slices(plan, raw=raw[:, lo:hi].contiguous().to(dev), flats=flats[:, lo:hi].contiguous().to(dev),
                                  flat_pos=flat_pos, dark=dark[lo:hi].contiguous().to(dev), hot_threshold=0.1,
                                  halo=halo)
        xw = ph.reconstruct_slices(plan, sino=whole[r0:r1].contiguous())
        assert torch.equal(x, xw), (r0, r1)


def test_ring_filter_parity(dev):
    R, N, K = 3, 96, 60
    g = ph.Geometry(N, N, N, synth.uniform_angles(K), (N - 1) / 2)
    og = oracle.Geom(N, N, N, g.angles, g.axis_pos)
    rng = synth.rng_for(10, 2, 0)
    sino = np.stack([synth.ellipse_sinogram(synth.random_ellipses(synth.rng_for(10, 2, r), 5), g.angles, N,
                                            g.axis_pos, N).numpy() for r in range(R)])
    sino = (sino + 0.3 * rng.standard_normal((R, 1, N))).astype(np.float32)
    plan = ph.Plan(g, n_slices=R)
    for width in (0, 3, 20):
        got = ph.ring_filter(plan, torch.from_numpy(sino).to(dev), width)
        assert rel(got, oracle.ring_filter(sino, width)) <= TOL_OP, width
    obj = np.stack([oracle.ring_object(sino[r], og, 0.3) for r in range(R)]).astype(np.float32)
    got = ph.ring_filter(plan, torch.from_numpy(sino).to(dev), 12, obj=torch.from_numpy(obj).to(dev))
    assert rel(got, oracle.ring_filter(sino, 12, obj=obj)) <= TOL_OP


@pytest.fixture(scope="module")
def ringed_raw():
    R, N, K = 3, 64, 90
    raw, flats, flat_pos, dark, ang, axis = raw_with_spikes(R, N, K, 3)
    # detector gain errors: the same per-bin factor in every projection -> rings
    gain = 1 + 0.02 * synth.rng_for(10, 3, 7).standard_normal((1, R, N))
    raw = torch.from_numpy(np.clip(np.round(raw.numpy() * gain), 0, 65535).astype(np.uint16))
    return raw, flats, flat_pos, dark, ang, axis, R, N


@pytest.mark.parametrize("hot,width,obj_thr", [(None, 0, None), (0.1, 0, None), (None, 6, None), (None, 6, 0.02),
                                               (0.1, 6, 0.02)])
def test_fbp_with_preprocessing_parity(dev, ringed_raw, hot, width, obj_thr):
    raw, flats, flat_pos, dark, ang, axis, R, N = ringed_raw
    g = ph.Geometry(N, N, N, ang, axis)
    og = oracle.Geom(N, N, N, ang, axis)
    plan = ph.Plan(g, n_slices=R)
    args = dict(raw=raw.to(dev), flats=flats.to(dev), flat_pos=flat_pos, dark=dark.to(dev), method=ph.FBP)
    x = ph.reconstruct_slices(plan, hot_threshold=hot, ring_width=width, ring_object_threshold=obj_thr, **args)
    if hot is None:
        y = oracle.normalize(raw.numpy(), flats.numpy(), flat_pos, dark.numpy())
    else:
        y = oracle.normalize_hotspot(raw.numpy(), flats.numpy(), flat_pos, dark.numpy(), hot)
    ys = []
    for r in range(R):
        yr = y[r]
        if width:
            obj = None if obj_thr is None else oracle.ring_object(yr, og, obj_thr)
            yr = oracle.ring_filter(yr, width, obj=obj)
        ys.append(yr)
    ref = oracle.fbp(np.stack(ys), og)
    assert ref.shape == (R, N, N)
    # the same steps through the separate entry points
    if hot is None:
        yg = ph.normalize(plan, args["raw"], args["flats"], flat_pos, args["dark"])
    else:
        yg = ph.normalize_hotspot(plan, args["raw"], args["flats"], flat_pos, args["dark"], hot)
    assert rel(yg, y) <= TOL_OP
    if width:
        objg = None
        if obj_thr is not None:
            x0 = ph.reconstruct_slices(plan, sino=yg.clone(), method=ph.FBP)
            objg = ph.forward_project(plan, torch.where(x0 > obj_thr, x0, torch.zeros_like(x0)).contiguous())
        ph.ring_filter(plan, yg, width, obj=objg)
    xs = ph.reconstruct_slices(plan, sino=yg, method=ph.FBP)
    assert rel(xs, ref) <= TOL_PIPE, ("separate entry points", rel(xs, ref))
    assert rel(x, ref) <= TOL_PIPE, ("reconstruct_slices", rel(x, ref), rel(x, xs))


def test_cp_with_ring_filter_parity(dev):
    N, K = 64, 48
    g = ph.Geometry(N, N, N, synth.uniform_angles(K), (N - 1) / 2)
    og = oracle.Geom(N, N, N, g.angles, g.axis_pos)
    y = synth.ellipse_sinogram(synth.random_ellipses(synth.rng_for(10, 4, 0), 5), g.angles, N, g.axis_pos, N).numpy()
    y = (y + 0.2 * synth.rng_for(10, 4, 1).standard_normal((1, N))).astype(np.float32)
    Lk = oracle.opnorm(og, synth.rng_for(10, 4, 2).standard_normal((N, N)), 200)
    plan = ph.Plan(g)
    yt = torch.from_numpy(y)[None].contiguous().to(dev)
    x = ph.reconstruct_slices(plan, sino=yt, method=ph.TV_CP, lam=0.05, n_iter=10, op_norm=Lk, ring_width=5)
    ref = oracle.cp_tv(oracle.ring_filter(y, 5), og, 0.05, 10, Lk)
    assert rel(x[0], ref) <= TOL_PIPE
    assert torch.equal(yt[0].cpu(), torch.from_numpy(y))   # input not modified
