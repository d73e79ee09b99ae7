"""GPU parity: every HIP kernel against the FP64 oracle on the same seeded inputs.

Tolerances (relative L2, ||gpu - oracle|| / ||oracle||): 1e-5 for the projector,
backprojector, ramp filter and normalisation; 1e-4 for full FBP and TV iterates.
"""
import math

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
    return float(np.linalg.norm(a.ravel() - b.ravel()) / np.linalg.norm(b.ravel()))


def pair(nx, ny, nb, K, axis, shifts=None, s=1.0, scan=ph.SCAN_180, span=None, overlap=0.0, jitter=0.0, seed=0):
    span = span if span is not None else (math.pi if scan == ph.SCAN_180 else 2 * math.pi)
    ang = synth.uniform_angles(K, span)
    if jitter:
        ang = ang + np.random.default_rng(seed).uniform(-jitter, jitter, K) * span / K
    sh = None if shifts is None else np.random.default_rng(seed + 1).normal(0, shifts, K)
    return (ph.Geometry(nx, ny, nb, ang, axis, sh, scan, s, overlap),
            oracle.Geom(nx, ny, nb, ang, axis, sh, scan, s, overlap))


CASES = {
    "cfg1_256": dict(nx=256, ny=256, nb=256, K=180, axis=127.5),
    "odd_shift": dict(nx=77, ny=53, nb=101, K=61, axis=49.3, shifts=0.5, jitter=0.3),
    "wide_det": dict(nx=96, ny=96, nb=160, K=45, axis=81.25, shifts=0.5),
    "pix_0p7": dict(nx=70, ny=70, nb=64, K=50, axis=30.8, s=0.7),
    "pix_1p6": dict(nx=40, ny=50, nb=100, K=33, axis=50.0, s=1.6),
    "pix_0p4": dict(nx=60, ny=48, nb=50, K=37, axis=24.6, s=0.4, shifts=0.3),   # > 6 candidates per line
    # wider than the 224-position staged segment of six candidates: interior blocks take 16-byte reads
    "pix_0p7_wide": dict(nx=288, ny=264, nb=210, K=40, axis=104.5, s=0.7, shifts=0.3),
    "tiny": dict(nx=5, ny=3, nb=7, K=4, axis=3.0),
    "scan360": dict(nx=64, ny=64, nb=72, K=100, axis=36.4, scan=ph.SCAN_360),
}


@pytest.fixture(scope="module")
def gen():
    return np.random.default_rng(1234)


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("tile,persistent", [(-1, False), (0, False), (3, True), (1, False), (2, True), (5, False),
                                             (5, True), (4, False)])
def test_backproject_parity(dev, gen, case, tile, persistent):
    g, og = pair(**CASES[case])
    plan = ph.Plan(g, n_slices=2)
    plan.set_tiles(tile, persistent)
    y = gen.standard_normal((2, g.n_angles, g.n_det)).astype(np.float32)
    out = ph.backproject(plan, torch.from_numpy(y).to(dev))
    ref = oracle.backproject(y, og)
    assert rel(out, ref) <= TOL_OP, (case, tile, persistent, rel(out, ref))


@pytest.mark.parametrize("case", ["odd_shift", "pix_0p7", "pix_1p6", "tiny", "scan360"])
@pytest.mark.parametrize("tile", [0, 1, 2, 3, 4])
def test_bp_two_slices_equal_one_slice_kernel(dev, gen, case, tile):
    """Two slices per backprojector workgroup (the automatic choice on uniform plans) against one
    slice per workgroup with the same tile: equal bit for bit, with an odd slice count (the last
    slice runs as a pair with itself) and an accumulating beta."""
    g, og = pair(**CASES[case])
    plan = ph.Plan(g, n_slices=3)
    y = torch.from_numpy(gen.standard_normal((3, g.n_angles, g.n_det)).astype(np.float32)).to(dev)
    base = torch.from_numpy(gen.standard_normal((3, g.n_y, g.n_x)).astype(np.float32)).to(dev)
    outs = []
    for per in (1, 2):
        plan.set_tiles(tile, False)
        plan.set_bp_slices(per)
        o = base.clone()
        ph.backproject(plan, y, out=o, alpha=0.75, beta=0.5)
        outs.append(o)
    torch.cuda.synchronize()
    assert torch.equal(outs[0], outs[1]), (case, tile, float((outs[0] - outs[1]).abs().max()))
    ref = 0.75 * oracle.backproject(y.cpu().numpy(), og) + 0.5 * base.double().cpu().numpy()
    assert rel(outs[1], ref) <= TOL_OP, (case, tile, rel(outs[1], ref))


FP_KINDS = {"auto": ph.FP_AUTO, "blocks": ph.FP_BLOCKS, "staged": ph.FP_STAGED, "lines": ph.FP_LINES}


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("kind", list(FP_KINDS))
def test_forward_project_parity(dev, gen, case, kind):
    g, og = pair(**CASES[case])
    plan = ph.Plan(g, n_slices=2)
    plan.set_fp_kernel(FP_KINDS[kind])
    assert plan.get_fp_kernel() == FP_KINDS[kind]
    x = gen.standard_normal((2, g.n_y, g.n_x)).astype(np.float32)
    out = ph.forward_project(plan, torch.from_numpy(x).to(dev))
    ref = oracle.forward_project(x, og)
    assert rel(out, ref) <= TOL_OP, (case, kind, rel(out, ref))


@pytest.mark.parametrize("case", ["odd_shift", "pix_0p7", "pix_1p6", "pix_0p4"])
@pytest.mark.parametrize("kind", list(FP_KINDS))
def test_adjoint_identity_gpu(dev, gen, case, kind):
    g, _ = pair(**CASES[case])
    plan = ph.Plan(g)
    plan.set_fp_kernel(FP_KINDS[kind])
    x = torch.from_numpy(gen.standard_normal((1, g.n_y, g.n_x)).astype(np.float32)).to(dev)
    y = torch.from_numpy(gen.standard_normal((1, g.n_angles, g.n_det)).astype(np.float32)).to(dev)
    ax = ph.forward_project(plan, x).double()
    lhs = float((ax * y.double()).sum())
    rhs = g.pixel_size ** 2 * float((x.double() * ph.backproject(plan, y).double()).sum())
    # rounding in <Ax, y> is bounded by |Ax| |y| (Cauchy-Schwarz), not by |<Ax, y>|, which a random draw
    # can make arbitrarily small through cancellation
    scale = float(ax.norm() * y.double().norm())
    assert abs(lhs - rhs) <= 1e-5 * scale, (case, kind, lhs, rhs, scale)


def test_fp_kernel_override_rejects_bad_kind(dev):
    g, _ = pair(**CASES["tiny"])
    plan = ph.Plan(g)
    with pytest.raises(ph.PyhstError):
        plan.set_fp_kernel(4)
    assert plan.get_fp_kernel() == ph.FP_AUTO


FILTER_CASES = {
    "cfg1": dict(nx=256, ny=256, nb=256, K=180, axis=127.5),
    "odd": dict(nx=40, ny=40, nb=37, K=31, axis=17.5, jitter=0.4),
    "scan360": dict(nx=64, ny=64, nb=72, K=100, axis=36.4, scan=ph.SCAN_360),
    "half_right": dict(nx=96, ny=96, nb=59, K=180, axis=48.0, scan=ph.SCAN_360_HALF),
    "half_left": dict(nx=96, ny=96, nb=59, K=180, axis=10.0, scan=ph.SCAN_360_HALF, overlap=6.0),
    "long_rows": dict(nx=16, ny=16, nb=2500, K=4, axis=1249.5),
    # FFT length 4096 (the register-FFT filter): full rows, shorter rows, extended half-acquisition rows
    # on either side, odd projection counts (the last row pair has one row)
    "rows_2048_oddK": dict(nx=16, ny=16, nb=2048, K=5, axis=1023.5),
    "rows_1500": dict(nx=16, ny=16, nb=1500, K=4, axis=749.5, jitter=0.1),
    "half_right_p4096": dict(nx=32, ny=32, nb=600, K=7, axis=590.0, scan=ph.SCAN_360_HALF),
    "half_left_p4096": dict(nx=32, ny=32, nb=600, K=6, axis=9.0, scan=ph.SCAN_360_HALF, overlap=5.0),
}


DEGENERATE = {
    "one_pixel": dict(nx=1, ny=1, nb=1, K=2, axis=0.0),        # one pixel, one bin, two projections
    "one_row": dict(nx=9, ny=1, nb=5, K=3, axis=2.0),
    "one_col": dict(nx=1, ny=7, nb=4, K=3, axis=1.5),
    "two_angles": dict(nx=16, ny=16, nb=16, K=2, axis=7.5),    # the fewest projections a plan accepts
}


@pytest.mark.parametrize("case", list(DEGENERATE))
def test_degenerate_geometries(dev, gen, case):
    """The smallest plans the boundary accepts: backprojection (every tile shape, direct and persistent),
    projection (every projector kernel), ramp filter and the whole FBP against the oracle."""
    g, og = pair(**DEGENERATE[case])
    plan = ph.Plan(g, n_slices=2)
    y = gen.standard_normal((2, g.n_angles, g.n_det)).astype(np.float32)
    x = gen.standard_normal((2, g.n_y, g.n_x)).astype(np.float32)
    yt, xt = torch.from_numpy(y).to(dev), torch.from_numpy(x).to(dev)
    ref_bp, ref_fp = oracle.backproject(y, og), oracle.forward_project(x, og)
    for tile, pers in [(-1, False), (0, False), (3, True), (4, False), (5, False), (5, True)]:
        plan.set_tiles(tile, pers)
        assert rel(ph.backproject(plan, yt), ref_bp) <= TOL_OP, (case, tile, pers)
    plan.set_tiles(-1, False)
    for kind in FP_KINDS.values():
        plan.set_fp_kernel(kind)
        assert rel(ph.forward_project(plan, xt), ref_fp) <= TOL_OP, (case, kind)
    plan.set_fp_kernel(ph.FP_AUTO)
    assert rel(ph.fbp_filter(plan, yt), oracle.fbp_filter(y, og)) <= TOL_OP, case
    assert rel(ph.reconstruct_slices(plan, sino=yt, method=ph.FBP), oracle.fbp(y, og)) <= TOL_PIPE, case


@pytest.mark.parametrize("case", list(FILTER_CASES))
def test_fbp_filter_parity(dev, gen, case):
    g, og = pair(**FILTER_CASES[case])
    plan = ph.Plan(g, n_slices=2)
    p = gen.random((2, g.n_angles, g.n_det)).astype(np.float32)
    out = ph.fbp_filter(plan, torch.from_numpy(p).to(dev))
    ref = oracle.fbp_filter(p, og)
    assert out.shape == ref.shape
    assert rel(out, ref) <= TOL_OP, (case, rel(out, ref))


def test_fbp_filter_in_place(dev, gen):
    g, og = pair(**FILTER_CASES["odd"])
    plan = ph.Plan(g)
    p = gen.random((1, g.n_angles, g.n_det)).astype(np.float32)
    t = torch.from_numpy(p).to(dev)
    ph.fbp_filter(plan, t, out=t)
    assert rel(t, oracle.fbp_filter(p, og)) <= TOL_OP


def raw_case(R=3, N=96, K=90, nb=None, axis_offset=3.5, seed=7, n_flats=2):
    nb = nb or N
    ang = synth.uniform_angles(K)
    axis = (nb - 1) / 2 + axis_offset
    p = torch.stack([synth.ellipse_sinogram(synth.random_ellipses(synth.rng_for(9, 0, r), 8), ang, nb, axis, N)
                     for r in range(R)])
    raw, flats, fpos, dark, kap = synth.raw_acquisition(p, seed=seed)
    if n_flats == 3:   # a third flat acquired mid-scan
        flats = torch.cat([flats[:1], 0.5 * (flats[:1] + flats[1:]) * 1.01, flats[1:]])
        fpos = np.array([0.0, K / 2 + 0.5, K - 1.0])
    return ang, axis, raw, flats, fpos, dark


@pytest.mark.parametrize("n_flats", [2, 3])
def test_normalize_parity(dev, n_flats):
    ang, axis, raw, flats, fpos, dark = raw_case(n_flats=n_flats)
    g = ph.Geometry(96, 96, 96, ang, axis)
    plan = ph.Plan(g, n_slices=3)
    out = ph.normalize(plan, raw.to(dev), flats.to(dev), fpos, dark.to(dev))
    ref = oracle.normalize(raw.numpy().astype(np.float64), flats.numpy(), fpos, dark.numpy())
    assert rel(out, ref) <= TOL_OP


@pytest.mark.parametrize("graph", [False, True])
def test_fbp_from_raw_parity(dev, graph):
    ang, axis, raw, flats, fpos, dark = raw_case()
    g = ph.Geometry(96, 96, 96, ang, axis)
    og = oracle.Geom(96, 96, 96, ang, axis)
    plan = ph.Plan(g, n_slices=3)
    args = dict(raw=raw.to(dev), flats=flats.to(dev), flat_pos=fpos, dark=dark.to(dev), method=ph.FBP)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        out = ph.reconstruct_slices(plan, use_graph=graph, **args)
    side.synchronize()
    ref = oracle.fbp_raw(raw.numpy().astype(np.float64), flats.numpy(), fpos, dark.numpy(), og)
    assert rel(out, ref) <= TOL_PIPE
    if graph:   # replays of the captured graph give the eager result every time
        eager = ph.reconstruct_slices(plan, use_graph=False, **args).clone()
        torch.cuda.synchronize()
        for _ in range(3):
            with torch.cuda.stream(side):
                again = ph.reconstruct_slices(plan, use_graph=True, **args)
            side.synchronize()
            assert torch.equal(again, eager)
            eager.add_(0.0)     # eager work between replays


def test_fbp_from_raw_parity_p4096(dev):
    """2048-bin rows from raw (normalisation fused into the register-FFT filter, FFT length 4096), an odd
    number of projections, two slices."""
    ang, axis, raw, flats, fpos, dark = raw_case(R=2, N=32, K=7, nb=2048)
    g = ph.Geometry(32, 32, 2048, ang, axis)
    og = oracle.Geom(32, 32, 2048, ang, axis)
    plan = ph.Plan(g, n_slices=2)
    out = ph.reconstruct_slices(plan, raw=raw.to(dev), flats=flats.to(dev), flat_pos=fpos, dark=dark.to(dev),
                                method=ph.FBP)
    ref = oracle.fbp_raw(raw.numpy().astype(np.float64), flats.numpy(), fpos, dark.numpy(), og)
    assert rel(out, ref) <= TOL_PIPE


def test_fbp_batch_equals_single(dev, gen):
    g, _ = pair(**CASES["odd_shift"])
    plan4 = ph.Plan(g, n_slices=4)
    plan1 = ph.Plan(g, n_slices=1)
    y = torch.from_numpy(gen.random((4, g.n_angles, g.n_det)).astype(np.float32)).to(dev)
    batch = ph.reconstruct_slices(plan4, sino=y, method=ph.FBP)
    for i in range(4):
        single = ph.reconstruct_slices(plan1, sino=y[i:i + 1].contiguous(), method=ph.FBP)
        assert torch.equal(batch[i], single[0])


@pytest.mark.parametrize("persistent", [False, True])
def test_uniform_plan_shared_by_two_streams(dev, gen, persistent):
    """A uniform plan may serve two streams at once when each call has its own buffers: FBP and TV-CP
    interleaved on two streams (graph and direct launches) equal the same calls made one at a time, also
    with the persistent backprojector (its work counter belongs to the stream)."""
    g, _ = pair(**CASES["odd_shift"])
    plan = ph.Plan(g, n_slices=2)
    plan.set_tiles(-1, persistent)
    y = [torch.from_numpy(gen.standard_normal((2, g.n_angles, g.n_det)).astype(np.float32)).to(dev) for _ in range(2)]
    kw = [dict(method=ph.FBP), dict(method=ph.TV_CP, lam=0.02, n_iter=15, op_norm=200.0)]   # 200 > |K| here
    ref = [ph.reconstruct_slices(plan, sino=y[i], **kw[i]) for i in range(2)]
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    for st in streams:
        st.wait_stream(torch.cuda.current_stream())
    outs = []
    for rep in range(4):
        for i, st in enumerate(streams):
            with torch.cuda.stream(st):
                outs.append((i, ph.reconstruct_slices(plan, sino=y[i], use_graph=(rep + i) % 2 == 0, stream=st,
                                                      **kw[i])))
    torch.cuda.synchronize()
    for i, o in outs:
        assert torch.equal(o, ref[i]), i


def test_graph_cache_bound(dev, gen):
    """More distinct graph calls than the plan caches (64): the surplus run as plain launches, same result."""
    g, _ = pair(**CASES["tiny"])
    plan = ph.Plan(g)
    y = torch.from_numpy(gen.standard_normal((1, g.n_angles, g.n_det)).astype(np.float32)).to(dev)
    ref = ph.reconstruct_slices(plan, sino=y, method=ph.FBP)
    outs = [torch.empty_like(ref) for _ in range(70)]
    side = torch.cuda.Stream()   # graphs are captured on a created stream (the null stream cannot be)
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        for _ in range(2):
            for o in outs:
                ph.reconstruct_slices(plan, sino=y, method=ph.FBP, out=o, use_graph=True, stream=side)
    torch.cuda.synchronize()
    assert all(torch.equal(o, ref) for o in outs)


def test_uniform_plan_on_a_later_geometry(dev, gen):
    """A plan whose slices all use geometry 1 of two behaves as a plan of that geometry alone: the packed
    shapes, FBP, the projector and TV-CP use its sizes, not those of geometry 0."""
    g0, _ = pair(**CASES["wide_det"])
    g1, og1 = pair(**CASES["odd_shift"])
    both = ph.Plan([g0, g1], slice_geom=[1, 1])
    only = ph.Plan(g1, n_slices=2)
    assert both.uniform and both.sino_shape() == only.sino_shape() and both.img_shape() == only.img_shape()
    y = torch.from_numpy(gen.random((2, g1.n_angles, g1.n_det)).astype(np.float32)).to(dev)
    for kw in (dict(method=ph.FBP), dict(method=ph.TV_CP, lam=0.02, n_iter=5, op_norm=200.0)):
        assert torch.equal(ph.reconstruct_slices(both, sino=y, **kw), ph.reconstruct_slices(only, sino=y, **kw))
    x = ph.reconstruct_slices(only, sino=y, method=ph.FBP)
    assert torch.equal(ph.forward_project(both, x), ph.forward_project(only, x))
    assert rel(ph.reconstruct_slices(both, sino=y, method=ph.FBP)[1], oracle.fbp(y[1:].cpu().numpy(), og1)[0]) <= TOL_PIPE


def test_uneven_plan_matches_oracle(dev, gen):
    """One plan, slices of different sizes, angle counts and scan types (packed buffers)."""
    specs = [dict(nx=64, ny=64, nb=64, K=90, axis=31.5),
             dict(nx=96, ny=96, nb=59, K=180, axis=48.0, scan=ph.SCAN_360_HALF, shifts=0.5),
             dict(nx=48, ny=40, nb=70, K=31, axis=33.2, jitter=0.3)]
    pairs_ = [pair(**s, seed=i) for i, s in enumerate(specs)]
    sg = [0, 1, 2, 1, 0]
    plan = ph.Plan([p[0] for p in pairs_], slice_geom=sg)
    sinos = [gen.random((pairs_[i][0].n_angles, pairs_[i][0].n_det)).astype(np.float32) for i in sg]
    packed = torch.from_numpy(np.concatenate([s.ravel() for s in sinos])).to(dev)
    for persistent in (False, True):
        plan.set_tiles(-1, persistent)
        out = ph.reconstruct_slices(plan, sino=packed, method=ph.FBP).cpu().numpy()
        for i, gi in enumerate(sg):
            info = plan.slice_info(i)
            og = pairs_[gi][1]
            got = out[info.img_offset:info.img_offset + og.n_x * og.n_y].reshape(og.n_y, og.n_x)
            ref = oracle.fbp(sinos[i][None], og)[0]
            assert rel(got, ref) <= TOL_PIPE, (i, persistent, rel(got, ref))


@pytest.mark.parametrize("lam,n_inner", [(0.05, 40), (0.3, 100)])
def test_tv_prox_parity(dev, gen, lam, n_inner):
    g0 = (gen.standard_normal((2, 45, 61)) * 0.2 + 1.0).astype(np.float32)
    out = ph.tv_prox(torch.from_numpy(g0).to(dev), lam, n_inner)
    ref = oracle.tv_prox(g0, lam, n_inner)
    assert rel(out, ref) <= TOL_PIPE


def test_tv_prox_in_place_and_identity(dev, gen):
    g0 = gen.standard_normal((1, 20, 20)).astype(np.float32)
    t = torch.from_numpy(g0).to(dev)
    assert torch.equal(ph.tv_prox(t, 0.0, 10), t)
    ph.tv_prox(t, 0.1, 30, out=t)
    assert rel(t, oracle.tv_prox(g0, 0.1, 30)) <= TOL_PIPE


@pytest.fixture(scope="module")
def cp_problem():
    N, K = 128, 32
    d = synth.cfg_tv_sparse(N=N, K=K, index=3)
    g = ph.Geometry(N, N, N, d["angles"], d["axis"])
    og = oracle.Geom(N, N, N, d["angles"], d["axis"])
    Lk = oracle.opnorm(og, synth.rng_for(3, 9, 0).standard_normal((N, N)), 200)
    return d, g, og, Lk


@pytest.mark.parametrize("k", [1, 10, 100])
def test_cp_iterates_parity(dev, cp_problem, k):
    d, g, og, Lk = cp_problem
    plan = ph.Plan(g)
    y = d["y"][None].contiguous().to(dev)
    x = ph.reconstruct_slices(plan, sino=y, method=ph.TV_CP, lam=0.01, n_iter=k, op_norm=Lk)
    ref = oracle.cp_tv(d["y"].numpy(), og, 0.01, k, Lk)
    assert rel(x[0], ref) <= TOL_PIPE, (k, rel(x[0], ref))


@pytest.mark.parametrize("kind", ["blocks", "staged", "lines"])
def test_cp_iterates_every_fp_kernel(dev, cp_problem, kind):
    d, g, og, Lk = cp_problem
    plan = ph.Plan(g)
    plan.set_fp_kernel(FP_KINDS[kind])
    y = d["y"][None].contiguous().to(dev)
    x = ph.reconstruct_slices(plan, sino=y, method=ph.TV_CP, lam=0.01, n_iter=10, op_norm=Lk)
    ref = oracle.cp_tv(d["y"].numpy(), og, 0.01, 10, Lk)
    assert rel(x[0], ref) <= TOL_PIPE, (kind, rel(x[0], ref))


def test_cp_energy_and_graph(dev, cp_problem):
    d, g, og, Lk = cp_problem
    plan = ph.Plan(g)
    y = d["y"][None].contiguous().to(dev)
    x, E = ph.reconstruct_slices(plan, sino=y, method=ph.TV_CP, lam=0.01, n_iter=20, op_norm=Lk, energy=True)
    xr, Er = oracle.cp_tv(d["y"].numpy(), og, 0.01, 20, Lk, energy=True)
    np.testing.assert_allclose(E, Er, rtol=1e-4)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    for _ in range(2):
        with torch.cuda.stream(side):
            xg = ph.reconstruct_slices(plan, sino=y, method=ph.TV_CP, lam=0.01, n_iter=20, op_norm=Lk,
                                       use_graph=True)
        side.synchronize()
        assert torch.equal(xg, x)


def test_cp_opnorm_estimate(dev, cp_problem):
    """op_norm <= 0: the GPU power iteration gives 1.02 |K| (a 2 % safety margin)."""
    d, g, og, Lk = cp_problem
    plan = ph.Plan(g)
    y = d["y"][None].contiguous().to(dev)
    x = ph.reconstruct_slices(plan, sino=y, method=ph.TV_CP, lam=0.01, n_iter=50, op_norm=0.0)
    ref = oracle.cp_tv(d["y"].numpy(), og, 0.01, 50, 1.02 * Lk)
    assert rel(x[0], ref) < 2e-3


def test_cp_identity_limit_matches_prox(dev, gen):
    """TV-CP on a full-angle noise-free disc recovers it (eq. (3) with small beta)."""
    N = 64
    g = ph.Geometry(N, N, N, synth.uniform_angles(96), (N - 1) / 2)
    og = oracle.Geom(N, N, N, g.angles, g.axis_pos)
    y = synth.ellipse_sinogram(synth.disc_params(0.5, 1.0), g.angles, N, g.axis_pos, N).float()
    Lk = oracle.opnorm(og, gen.standard_normal((N, N)), 100)
    x = ph.reconstruct_slices(ph.Plan(g), sino=y[None].contiguous().to(dev), method=ph.TV_CP, lam=0.02,
                              n_iter=300, op_norm=Lk)[0].cpu().numpy()
    yy, xx = np.mgrid[0:N, 0:N]
    inside = (xx - (N - 1) / 2) ** 2 + (yy - (N - 1) / 2) ** 2 < (0.4 * N / 2) ** 2
    assert abs(x[inside].mean() - 1.0) < 0.03


# --------------------------------------------------------------------------- ISTA / FISTA (section 3.1)
@pytest.fixture(scope="module")
def fista_problem(cp_problem):
    d, g, og, _ = cp_problem
    La = oracle.opnorm(og, synth.rng_for(3, 9, 2).standard_normal((og.n_y, og.n_x)), 200, with_grad=False) ** 2
    return d, g, og, La


@pytest.mark.parametrize("method", ["ista", "fista"])
@pytest.mark.parametrize("k,lam", [(1, 1.0), (10, 1.0), (100, 1.0), (100, 0.01)])
def test_fista_iterates_parity(dev, fista_problem, method, k, lam):
    d, g, og, La = fista_problem
    fast = method == "fista"
    y = d["y"][None].contiguous().to(dev)
    x = ph.reconstruct_slices(ph.Plan(g), sino=y, method=ph.FISTA if fast else ph.ISTA, lam=lam, n_iter=k,
                              op_norm=math.sqrt(La), n_inner=20)
    ref = oracle.fista_tv(d["y"].numpy(), og, lam, k, La, 20, fast=fast)
    assert rel(x[0], ref) <= TOL_PIPE, (method, k, lam, rel(x[0], ref))


@pytest.mark.parametrize("kind", ["blocks", "staged", "lines"])
def test_fista_iterates_every_fp_kernel(dev, fista_problem, kind):
    d, g, og, La = fista_problem
    plan = ph.Plan(g)
    plan.set_fp_kernel(FP_KINDS[kind])
    y = d["y"][None].contiguous().to(dev)
    x = ph.reconstruct_slices(plan, sino=y, method=ph.FISTA, lam=1.0, n_iter=10, op_norm=math.sqrt(La), n_inner=20)
    ref = oracle.fista_tv(d["y"].numpy(), og, 1.0, 10, La, 20, fast=True)
    assert rel(x[0], ref) <= TOL_PIPE, (kind, rel(x[0], ref))


def test_fista_energy_graph_and_opnorm(dev, fista_problem):
    d, g, og, La = fista_problem
    plan = ph.Plan(g)
    y = d["y"][None].contiguous().to(dev)
    x, E = ph.reconstruct_slices(plan, sino=y, method=ph.FISTA, lam=1.0, n_iter=30, op_norm=math.sqrt(La),
                                 n_inner=10, energy=True)
    xr, Er = oracle.fista_tv(d["y"].numpy(), og, 1.0, 30, La, 10, fast=True, energy=True)
    np.testing.assert_allclose(E, Er, rtol=1e-4)
    assert rel(x[0], xr) <= TOL_PIPE
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    for _ in range(3):
        with torch.cuda.stream(side):
            xg = ph.reconstruct_slices(plan, sino=y, method=ph.FISTA, lam=1.0, n_iter=30, op_norm=math.sqrt(La),
                                       n_inner=10, use_graph=True)
        side.synchronize()
        assert torch.equal(xg, x)
    # op_norm <= 0: 1.02 |A| from the GPU power iteration on A^T A
    ph.reconstruct_slices(plan, sino=y, method=ph.ISTA, lam=1.0, n_iter=1, op_norm=0.0, n_inner=10)
    assert abs(plan.last_op_norm / (1.02 * math.sqrt(La)) - 1) < 1e-3


def test_fista_beats_ista_and_recovers_disc(dev):
    """The paper's claim (section 3.1): FISTA converges faster than ISTA; both reach the disc."""
    N = 64
    g = ph.Geometry(N, N, N, synth.uniform_angles(48), (N - 1) / 2)
    y = synth.ellipse_sinogram(synth.disc_params(0.5, 1.0), g.angles, N, g.axis_pos, N).float()
    y = y[None].contiguous().to(dev)
    plan = ph.Plan(g)
    xf, Ef = ph.reconstruct_slices(plan, sino=y, method=ph.FISTA, lam=0.5, n_iter=150, n_inner=10, energy=True)
    xi, Ei = ph.reconstruct_slices(plan, sino=y, method=ph.ISTA, lam=0.5, n_iter=150, n_inner=10, energy=True)
    assert Ef[-1] < Ei[-1] and Ef[30] < Ei[30]
    yy, xx = np.mgrid[0:N, 0:N]
    inside = (xx - (N - 1) / 2) ** 2 + (yy - (N - 1) / 2) ** 2 < (0.4 * N / 2) ** 2
    assert abs(xf[0].cpu().numpy()[inside].mean() - 1.0) < 0.03


@pytest.mark.parametrize("S", [7, 11])
def test_fp_slice_pairs_equal_one_slice_kernel(dev, gen, S):
    """The automatic projector choice on a uniform plan of several slices takes two (7 slices of 256^2 x
    720) or four (11 slices) slices per workgroup (one staged segment and one set of hat weights for all);
    every value equals the one-slice staged kernel's bit for bit: a slice count that the group size does
    not divide (the last workgroup holds fewer), groups of up to four projections, the plain projection,
    the Chambolle-Pock dual update and the FISTA residual in the projector's epilogue."""
    N, K = 256, 720
    g, og = pair(nx=N, ny=N, nb=N, K=K, axis=128.2, shifts=0.3)
    x = torch.from_numpy(gen.standard_normal((S, N, N)).astype(np.float32)).to(dev)
    y = torch.from_numpy(gen.standard_normal((S, K, N)).astype(np.float32)).to(dev)
    res = {}
    for kind in (ph.FP_AUTO, ph.FP_STAGED):
        plan = ph.Plan(g, n_slices=S)
        plan.set_fp_kernel(kind)
        fp = ph.forward_project(plan, x)
        cp = ph.reconstruct_slices(plan, sino=y, method=ph.TV_CP, lam=0.01, n_iter=2, op_norm=400.0)
        fi = ph.reconstruct_slices(plan, sino=y, method=ph.FISTA, lam=0.5, n_iter=2, op_norm=400.0, n_inner=4)
        torch.cuda.synchronize()
        res[kind] = (fp, cp, fi)
    for a, b in zip(res[ph.FP_AUTO], res[ph.FP_STAGED]):
        assert torch.equal(a, b)


def test_fp_groups_of_four_parity(dev, gen):
    """A plan big enough for the staged projector's groups of four (8 slices x 256^2 x 720 angles with
    axis shifts: about 5800 workgroups, at least 16 per CU): the plain projection of every slice, and
    two Chambolle-Pock iterations (dual update fused into the projector) and two FISTA iterations
    (residual in the projector's epilogue) of the first two slices, against the oracle."""
    import test_kernel_index_replay as rp
    N, K, S = 256, 720, 8
    g, og = pair(nx=N, ny=N, nb=N, K=K, axis=128.2, shifts=0.3)
    # the plan's grouping rule, replayed: groups of up to four and enough workgroups to keep them
    P = [rp._proj(k, th, 1.0, N, N, og.axis, og.shifts[k]) for k, th in enumerate(og.angles)]
    groups = rp.staged_groups(P, N, N, N, 3, cap=4)
    assert max(len(q) for q in groups) == 4 and S * (N // 64) * len(groups) >= 16 * 256
    plan = ph.Plan(g, n_slices=S)
    x = gen.standard_normal((S, N, N)).astype(np.float32)
    out = ph.forward_project(plan, torch.from_numpy(x).to(dev))
    assert rel(out, oracle.forward_project(x, og)) <= TOL_OP
    y = gen.standard_normal((S, K, N)).astype(np.float32)
    xs = ph.reconstruct_slices(plan, sino=torch.from_numpy(y).to(dev), method=ph.TV_CP, lam=0.01, n_iter=2,
                               op_norm=400.0)
    for s in range(2):
        assert rel(xs[s], oracle.cp_tv(y[s], og, 0.01, 2, 400.0)) <= TOL_PIPE, s
    # FISTA: the residual A x - y computed in the projector's epilogue
    xf = ph.reconstruct_slices(plan, sino=torch.from_numpy(y).to(dev), method=ph.FISTA, lam=0.5, n_iter=2,
                               op_norm=400.0, n_inner=4)
    for s in range(2):
        assert rel(xf[s], oracle.fista_tv(y[s], og, 0.5, 2, 400.0 ** 2, 4, fast=True)) <= TOL_PIPE, s
