"""Pins of the FP64 oracle against facts that do not come from the oracle itself:
closed forms, exact identities, textbook special cases and brute force.

Each test names the passage it checks.  A plausible mistake in the oracle (a
wrong sign or centre in the geometry, a dropped term in the filter, a wrong
boundary in the TV operators, a wrong step in the solvers) fails at least one.
"""
import math

import numpy as np
import pytest
import torch

import oracle
from oracle import Geom, SCAN_180, SCAN_360, SCAN_360_HALF
import synth


def rel(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


# ------------------------------------------------------------------ projector geometry (section 2.3)

def lerp_matrix(g: Geom) -> np.ndarray:
    """Brute force: explicit (K*nb) x (n_y*n_x) matrix of linear detector interpolation,
    entries written from the geometry with a floor/fraction split (not the hat form)."""
    M = np.zeros((g.K * g.n_det, g.n_y * g.n_x))
    cx, cy = (g.n_x - 1) / 2.0, (g.n_y - 1) / 2.0
    for k in range(g.K):
        c, s_ = math.cos(g.angles[k]), math.sin(g.angles[k])
        sh = 0.0 if g.shifts is None else g.shifts[k]
        for iy in range(g.n_y):
            for ix in range(g.n_x):
                t = g.pixel_size * ((ix - cx) * c + (iy - cy) * s_) + g.axis + sh
                j0 = math.floor(t)
                f = t - j0
                col = iy * g.n_x + ix
                if 0 <= j0 < g.n_det:
                    M[k * g.n_det + j0, col] += 1.0 - f
                if 0 <= j0 + 1 < g.n_det:
                    M[k * g.n_det + j0 + 1, col] += f
    return M


@pytest.mark.parametrize("K,nb,axis,shift,s", [
    (5, 12, 5.5, False, 1.0), (7, 14, 6.25, True, 1.0), (4, 10, 4.0, True, 0.7), (6, 20, 9.3, False, 1.6)])
def test_bruteforce_8x8(K, nb, axis, shift, s):
    rng = np.random.default_rng(K * 100 + nb)
    ang = np.sort(rng.uniform(0, math.pi, K))
    g = Geom(8, 8, nb, ang, axis, rng.normal(0, 0.5, K) if shift else None, pixel_size=s)
    M = lerp_matrix(g)
    x = rng.standard_normal((8, 8))
    y = rng.standard_normal((K, nb))
    np.testing.assert_allclose(oracle.forward_project(x, g).ravel(), s * s * (M @ x.ravel()), rtol=0, atol=1e-12)
    np.testing.assert_allclose(oracle.backproject(y, g).ravel(), M.T @ y.ravel(), rtol=0, atol=1e-12)


@pytest.mark.parametrize("K,nb,axis,shift,s", [(5, 12, 5.5, False, 1.0), (7, 14, 6.25, True, 1.0), (6, 20, 9.3, True, 1.6)])
def test_backproject_points_bruteforce(K, nb, axis, shift, s):
    """The point-wise backprojection (used to check full-size images pixel by pixel) is the column of the
    explicit interpolation matrix at each requested pixel, for every pixel of an 8x8 image in a shuffled
    order with repeats."""
    rng = np.random.default_rng(K * 10 + nb)
    g = Geom(8, 8, nb, np.sort(rng.uniform(0, math.pi, K)), axis, rng.normal(0, 0.5, K) if shift else None,
             pixel_size=s)
    M = lerp_matrix(g)
    y = rng.standard_normal((K, nb))
    pix = np.concatenate([rng.permutation(64), rng.integers(0, 64, 20)])
    iy, ix = pix // 8, pix % 8
    ref = (M.T @ y.ravel())[pix]
    np.testing.assert_allclose(oracle.backproject_points(y, g, ix, iy), ref, rtol=0, atol=1e-12)


def test_backproject_points_equals_backproject_and_half_layout():
    """At random pixels of a larger, uneven image the point-wise form equals the whole-image form, also on
    the extended rows of a half-acquisition scan (the layout the FBP filter writes)."""
    rng = np.random.default_rng(5)
    g = Geom(61, 47, 70, np.sort(rng.uniform(0, math.pi, 33)), 33.2, rng.normal(0, 0.5, 33), pixel_size=0.8)
    y = rng.standard_normal((33, 70))
    full = oracle.backproject(y, g)
    ix, iy = rng.integers(0, 61, 300), rng.integers(0, 47, 300)
    np.testing.assert_allclose(oracle.backproject_points(y, g, ix, iy), full[iy, ix], rtol=0, atol=1e-12)
    h = Geom(40, 40, 30, synth.uniform_angles(50, 2 * math.pi), 25.0, scan=SCAN_360_HALF)
    lay = oracle.half_acq_layout(h)
    ye = rng.standard_normal((50, lay["L"]))
    full = oracle.backproject(ye, h, extended=True)
    ix, iy = rng.integers(0, 40, 200), rng.integers(0, 40, 200)
    np.testing.assert_allclose(oracle.backproject_points(ye, h, ix, iy, extended=True), full[iy, ix], rtol=0,
                               atol=1e-12)


def test_adjoint_identity():
    rng = np.random.default_rng(3)
    g = Geom(37, 29, 50, np.sort(rng.uniform(0, math.pi, 23)), 24.3, rng.normal(0, 0.5, 23), pixel_size=0.9)
    x = rng.standard_normal((29, 37))
    y = rng.standard_normal((23, 50))
    lhs = float((oracle.forward_project(x, g) * y).sum())
    rhs = g.pixel_size ** 2 * float((x * oracle.backproject(y, g)).sum())
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_mass_conservation():
    """Hats form a partition of unity: sum_j (A x)[k][j] = s^2 sum x when every pixel lands inside."""
    rng = np.random.default_rng(4)
    g = Geom(16, 16, 40, np.linspace(0, math.pi, 13, endpoint=False), 19.5, rng.normal(0, 0.3, 13), pixel_size=1.2)
    x = rng.random((16, 16))
    sums = oracle.forward_project(x, g).sum(axis=1)
    np.testing.assert_allclose(sums, g.pixel_size ** 2 * x.sum(), rtol=1e-13)


def test_projection_matches_analytic_radon():
    """With pixels much smaller than bins, A(raster) tends to the exact Radon transform
    (Kak & Slaney ch. 3) seen through the unit hat of linear interpolation."""
    ell = np.array([[0.35, -0.2, 0.3, 0.15, 0.6, 1.0], [-0.3, 0.25, 0.2, 0.35, 2.0, 0.5]])
    nb, K, sub = 64, 12, 32
    ang = synth.uniform_angles(K)
    axis = (nb - 1) / 2.0 + 0.3
    errs = []
    for s in (0.5, 0.25, 0.125):
        N = int(round(nb / s))
        g = Geom(N, N, nb, ang, axis, pixel_size=s)
        num = oracle.forward_project(synth.ellipse_raster(ell, N, sub=4).numpy(), g)
        # analytic projection on a fine grid x_i = -1 + (i + 1/2)/sub, then averaged against hat(x - j)
        fine = synth.ellipse_sinogram(ell, ang, (nb + 2) * sub, (axis + 1) * sub - 0.5, N,
                                      pixel_size=s * sub).numpy() / sub
        x = -1.0 + (np.arange((nb + 2) * sub) + 0.5) / sub
        hat = np.clip(1.0 - np.abs(x[None, :] - np.arange(nb)[:, None]), 0.0, None)   # [nb][fine]
        ref = fine @ hat.T / sub
        errs.append(rel(num, ref))
    assert errs[2] < errs[1] < errs[0] and errs[2] < 4e-3, errs


def test_projection_orientation():
    """An off-centre disc projects to t = c + (N/2)(x0 cos th + y0 sin th) (sign and axis of x, y)."""
    N = 128
    x0, y0 = 0.45, -0.3
    ell = synth.disc_params(0.06, 1.0, x0, y0)
    ang = np.array([0.0, math.pi / 2, math.pi / 4, 2.3])
    g = Geom(N, N, N, ang, 60.0, np.array([0.0, 1.5, -2.0, 0.5]))
    sino = oracle.forward_project(synth.ellipse_raster(ell, N, sub=8).numpy(), g)
    j = np.arange(N)
    for k, th in enumerate(ang):
        centroid = (sino[k] * j).sum() / sino[k].sum()
        expect = g.axis + g.shifts[k] + (N / 2) * (x0 * math.cos(th) + y0 * math.sin(th))
        assert abs(centroid - expect) < 0.05, (k, centroid, expect)


# ------------------------------------------------------------------ ramp filter

def test_ramlak_frequency_response():
    """The Ram-Lak kernel samples the band-limited ramp: its DTFT is |w|/(2 pi) on [-pi, pi]."""
    L = 4001
    imp = np.zeros(L)
    imp[L // 2] = 1.0
    h = oracle.ramp_filter(imp[None], 1.0)[0]          # h[n - L//2]
    n = np.arange(L) - L // 2
    for w in (0.05, 0.4, 1.0, 2.0, 3.0):
        H = float(np.sum(h * np.cos(w * n)))
        assert abs(H - w / (2 * math.pi)) < 2e-4, (w, H)
    # zero DC gain in the limit, approached from above like 1/(pi^2 M)
    dc = float(h.sum())
    assert 0.0 < dc < 1.05 / (math.pi ** 2 * (L // 2))


def test_disc_filtered_projection_closed_form():
    """The ramp-filtered projection of a disc is rho/pi inside and
    (rho/pi)(1 - |u|/sqrt(u^2 - R^2)) outside (dtheta weight 1)."""
    L, R, rho = 1024, 150.0, 0.7
    u = np.arange(L) - 511.5
    p = 2 * rho * np.sqrt(np.clip(R * R - u * u, 0, None))
    q = oracle.ramp_filter(p[None], 1.0)[0]
    inside = np.abs(u) < R - 20
    assert np.max(np.abs(q[inside] * math.pi / rho - 1.0)) < 3e-3
    out = (np.abs(u) > R + 20) & (np.abs(u) < 400)
    ref = (rho / math.pi) * (1 - np.abs(u[out]) / np.sqrt(u[out] ** 2 - R * R))
    assert np.max(np.abs(q[out] - ref)) < 2e-3 * rho


def test_filter_fft_equals_direct():
    """Zero-padded FFT convolution with P >= 2L-1 gives the same linear convolution."""
    rng = np.random.default_rng(7)
    L = 93
    p = rng.standard_normal((3, L))
    q = oracle.ramp_filter(p, 1.0)
    P = 256
    lag = np.arange(P)
    lag = np.where(lag < P // 2, lag, lag - P).astype(float)
    odd = (np.abs(lag) % 2) == 1
    hc = np.where(lag == 0, 0.25, np.where(odd, -1.0 / (math.pi ** 2 * np.maximum(lag * lag, 1.0)), 0.0))
    hc = np.where(np.abs(lag) < L, hc, 0.0)
    H = np.fft.fft(hc)
    assert np.max(np.abs(H.imag)) < 1e-12          # even kernel: real spectrum (two rows per complex FFT)
    pad = np.zeros((3, P))
    pad[:, :L] = p
    ref = np.fft.ifft(np.fft.fft(pad) * H.real).real[:, :L]
    np.testing.assert_allclose(q, ref, atol=1e-12)


# ------------------------------------------------------------------ FBP

@pytest.mark.parametrize("scan,s,K", [(SCAN_180, 1.0, 180), (SCAN_180, 0.5, 120), (SCAN_360, 1.0, 240)])
def test_fbp_disc_interior(scan, s, K):
    """FBP of an analytic disc returns rho inside it."""
    N, rho = 96, 0.8
    span = math.pi if scan == SCAN_180 else 2 * math.pi
    ang = synth.uniform_angles(K, span)
    nb = int(math.ceil(N * s)) + 8
    axis = (nb - 1) / 2.0 + 1.25
    shifts = np.random.default_rng(1).normal(0, 0.5, K)
    g = Geom(N, N, nb, ang, axis, shifts, scan=scan, pixel_size=s)
    sino = synth.ellipse_sinogram(synth.disc_params(0.6, rho, 0.1, -0.05), ang, nb, axis, N, pixel_size=s,
                                  shifts=shifts).numpy()
    r = oracle.fbp(sino[None], g)[0]
    yy, xx = np.mgrid[0:N, 0:N]
    xn = (xx - (N - 1) / 2) * 2 / N - 0.1
    yn = (yy - (N - 1) / 2) * 2 / N + 0.05
    inside = xn ** 2 + yn ** 2 < 0.45 ** 2
    assert abs(r[inside].mean() / rho - 1) < 5e-3
    assert np.max(np.abs(r[inside] / rho - 1)) < 0.03


def test_fbp_ellipses_converges():
    """FBP of the ellipse phantom approaches the phantom as N and K grow."""
    errs = []
    for N in (64, 128):
        d = synth.cfg_single_slice(index=5, N=N, K=2 * N, noise_frac=0.0)
        g = Geom(N, N, N, d["angles"], d["axis"])
        r = oracle.fbp(d["sino"].double().numpy()[None], g)[0]
        errs.append(rel(r, d["truth"].numpy()))
    assert errs[1] < errs[0] < 0.5, errs


# ------------------------------------------------------------------ normalisation (section 2.3)

def test_normalize_noise_free_identity():
    rng = np.random.default_rng(9)
    R, K, nb = 3, 11, 17
    p = torch.as_tensor(rng.random((R, K, nb)) * 2.0)
    raw, flats, fpos, dark, kap = synth.raw_acquisition(p, seed=5, noise=False, rounding=False)
    out = oracle.normalize(raw, flats, fpos, dark)
    np.testing.assert_allclose(out, kap[:, None, None] * p.numpy(), rtol=0, atol=1e-12)


def test_normalize_flat_interpolation_and_clamp():
    """Flats interpolate linearly between acquisition positions; I <= D clamps to -ln(eps)."""
    K, R, nb = 9, 1, 2
    dark = np.array([[10.0, 10.0]])
    flats = np.array([[[110.0, 210.0]], [[130.0, 250.0]], [[90.0, 90.0]]])
    pos = np.array([2.0, 6.0, 8.0])
    raw = np.zeros((K, R, nb))
    raw[:, 0, 0] = 60.0
    raw[:, 0, 1] = 5.0
    out = oracle.normalize(raw, flats, pos, dark)
    f = np.array([110, 110, 110, 115, 120, 125, 130, 110, 90.0])
    np.testing.assert_allclose(out[0, :, 0], -np.log(50.0 / (f - 10.0)), rtol=1e-14)
    np.testing.assert_allclose(out[0, :, 1], -math.log(1e-6), rtol=1e-14)


# ------------------------------------------------------------------ angle weights / half acquisition (section 2.1)

def test_angle_weights_uniform_and_jittered():
    K = 36
    for scan, span, expect in ((SCAN_180, math.pi, math.pi / K), (SCAN_360, 2 * math.pi, math.pi / K),
                               (SCAN_360_HALF, 2 * math.pi, 2 * math.pi / K)):
        g = Geom(8, 8, 8, synth.uniform_angles(K, span), 3.5, scan=scan)
        np.testing.assert_allclose(oracle.angle_weights(g), expect, rtol=1e-14)
    rng = np.random.default_rng(2)
    ang = synth.uniform_angles(K) + rng.uniform(-0.02, 0.02, K)
    perm = rng.permutation(K)
    w = oracle.angle_weights(Geom(8, 8, 8, ang[perm], 3.5))
    assert abs(w.sum() - math.pi) < 1e-14 and np.all(w > 0)


@pytest.mark.parametrize("right", [True, False])
def test_half_acq_weights_sum_to_one(right):
    nb = 40
    axis = 33.0 if right else 6.0
    g = Geom(8, 8, nb, synth.uniform_angles(8, 2 * math.pi), axis, scan=SCAN_360_HALF)
    lay = oracle.half_acq_layout(g)
    w, c = lay["weights"], lay["axis"]
    j = np.arange(lay["L"])
    for jj in j:
        mirror = 2 * c - jj
        if abs(mirror - round(mirror)) < 1e-12 and 0 <= mirror < lay["L"]:
            assert abs(w[jj] + w[int(round(mirror))] - 1.0) < 1e-14
    lo, hi = lay["offset"], lay["offset"] + nb
    assert np.all(w[:lo] == 0) if not right else True
    assert np.all(w[hi:] == 0)


@pytest.mark.parametrize("right,delta", [(True, 10.0), (False, 10.0), (True, 20.5), (False, 20.5)])
def test_half_acq_mirror_consistency(right, delta):
    """A 360 degree half-acquisition (usable detector width doubled, section 2.1) of noise-free
    data reconstructs exactly what a 180 degree full-detector scan with the same bin
    alignment does: the lines at (theta, u) and (theta + pi, -u) coincide and their
    weights sum to one, so the identity holds to rounding when 2c is an integer."""
    N = 96
    ell = np.array([[0.2, 0.1, 0.35, 0.25, 0.3, 1.0], [-0.4, -0.2, 0.2, 0.15, 1.1, 0.6]])
    nb = N // 2 + int(delta) + 1
    axis = (nb - 1 - delta) if right else delta
    full = Geom(N, N, 2 * N, synth.uniform_angles(180), axis + N / 2)
    ref = oracle.fbp(synth.ellipse_sinogram(ell, full.angles, 2 * N, full.axis, N).numpy()[None], full)[0]
    half = Geom(N, N, nb, synth.uniform_angles(360, 2 * math.pi), axis, scan=SCAN_360_HALF)
    sino = synth.ellipse_sinogram(ell, half.angles, nb, axis, N).numpy()
    r = oracle.fbp(sino[None], half)[0]
    yy, xx = np.mgrid[0:N, 0:N]
    fov = (xx - (N - 1) / 2) ** 2 + (yy - (N - 1) / 2) ** 2 < (0.48 * N) ** 2     # common field of view
    assert rel(r[fov], ref[fov]) < 1e-12
    truth = synth.ellipse_raster(ell, N).numpy()
    assert rel(r[fov], truth[fov]) < 0.08


# ------------------------------------------------------------------ TV (eq. 2, Chambolle 2004)

def test_grad_div_adjoint():
    rng = np.random.default_rng(11)
    for ny, nx in ((13, 17), (1, 9), (7, 1)):
        x = rng.standard_normal((ny, nx))
        q1, q2 = rng.standard_normal((ny, nx)), rng.standard_normal((ny, nx))
        g1, g2 = oracle.grad(x)
        lhs = float((g1 * q1 + g2 * q2).sum())
        rhs = -float((x * oracle.div(q1, q2)).sum())
        assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs))


def test_tv_values():
    n, h = 12, 2.5
    step = np.zeros((n, n))
    step[:, 5:] = h
    assert abs(oracle.tv(step) - n * h) < 1e-12
    assert oracle.tv(np.full((n, n), 3.0)) == 0.0
    diag = np.zeros((4, 4))
    diag[1, 1] = 1.0     # isotropic: one pixel gives sqrt(2) at itself plus 1 + 1 at its neighbours
    assert abs(oracle.tv(diag) - (math.sqrt(2) + 2.0)) < 1e-12


def test_tv_prox_step_closed_form():
    """1-D ROF of a step of height J with plateaus a, b: the plateaus move by lambda/a and lambda/b."""
    ny, a, b, J, lam = 4, 9, 15, 1.0, 1.2
    g = np.zeros((ny, a + b))
    g[:, :a] = J
    u = oracle.tv_prox(g, lam, 6000)
    np.testing.assert_allclose(u[:, :a], J - lam / a, atol=1e-6)
    np.testing.assert_allclose(u[:, a:], lam / b, atol=1e-6)


def test_tv_prox_special_cases():
    rng = np.random.default_rng(12)
    g = rng.standard_normal((10, 14))
    np.testing.assert_array_equal(oracle.tv_prox(g, 0.0, 50), g)
    np.testing.assert_allclose(oracle.tv_prox(np.full((6, 7), 2.0), 0.5, 100), 2.0, atol=1e-14)
    u = oracle.tv_prox(g, 1e4, 20000)          # lambda -> infinity gives the mean
    np.testing.assert_allclose(u, g.mean(), atol=2e-3)
    u = oracle.tv_prox(g, 0.3, 200)
    assert oracle.tv(u) < oracle.tv(g)
    assert abs(u.mean() - g.mean()) < 1e-12      # div has zero mean: the prox keeps the mean


# ------------------------------------------------------------------ Chambolle-Pock (eq. 3)

def explicit_grad(ny, nx):
    n = ny * nx
    G = np.zeros((2 * n, n))
    for i in range(ny):
        for j in range(nx):
            o = i * nx + j
            if j + 1 < nx:
                G[o, o + 1], G[o, o] = 1.0, -1.0
            if i + 1 < ny:
                G[n + o, o + nx], G[n + o, o] = 1.0, -1.0
    return G


def test_opnorm_matches_svd():
    g = Geom(8, 8, 14, synth.uniform_angles(10), 6.7, pixel_size=1.0)
    Kmat = np.vstack([lerp_matrix(g), explicit_grad(8, 8)])
    ref = np.linalg.norm(Kmat, 2)
    x0 = np.random.default_rng(0).standard_normal((8, 8))
    assert abs(oracle.opnorm(g, x0, 400) / ref - 1) < 1e-8


def test_cp_identity_equals_rof():
    """With A = I, eq. (3) is the ROF problem: CP and Chambolle's projection reach the same minimiser."""
    rng = np.random.default_rng(13)
    y = rng.standard_normal((12, 12)) * 0.3 + np.kron(np.eye(2), np.ones((6, 6)))
    lam = 0.2
    Lk = math.sqrt(1 + 8)
    x = oracle.cp_tv(y, None, lam, 4000, Lk, identity_shape=(12, 12))
    u = oracle.tv_prox(y, lam, 20000)
    assert rel(x, u) < 1e-4


def test_opnorm_with_scaled_gradient_matches_svd():
    """|[A; mu grad]| (the balanced Chambolle-Pock operator) from the explicit matrices."""
    g = Geom(8, 8, 14, synth.uniform_angles(10), 6.7, pixel_size=1.0)
    for mu in (0.5, 3.7):
        ref = np.linalg.norm(np.vstack([lerp_matrix(g), mu * explicit_grad(8, 8)]), 2)
        x0 = np.random.default_rng(0).standard_normal((8, 8))
        assert abs(oracle.opnorm(g, x0, 600, mu=mu) / ref - 1) < 1e-8, mu


def test_cp_scaled_gradient_identity_equals_rof():
    """With A = I and a gradient block scaled by mu, CP still solves the ROF problem (lambda TV(x) =
    (lambda/mu) sum |mu grad x|): its limit is Chambolle's projection's."""
    rng = np.random.default_rng(13)
    y = rng.standard_normal((12, 12)) * 0.3 + np.kron(np.eye(2), np.ones((6, 6)))
    lam, mu = 0.2, 0.35
    Lk = math.sqrt(1 + 8 * mu * mu)
    x = oracle.cp_tv(y, None, lam, 6000, Lk, identity_shape=(12, 12), mu=mu)
    u = oracle.tv_prox(y, lam, 20000)
    assert rel(x, u) < 1e-4


def test_cp_balanced_reaches_the_fista_minimiser_in_300_iterations():
    """eq. (3) on a sparse-angle noisy problem.  With K = [A; grad] and tau = sigma = 1/|K|, |A| >> |grad|
    leaves the TV dual far from its bound after 300 iterations, so the iterate barely depends on lambda.
    Scaling the gradient block by mu = |A|/|grad| (same minimiser) brings the 300th iterate to the
    minimiser that FISTA, a separate code path, reaches, and the iterate then changes with lambda."""
    N, K = 24, 16
    g = Geom(N, N, N, synth.uniform_angles(K), (N - 1) / 2)
    ell = synth.random_ellipses(synth.rng_for(3, 5, 0), 5)
    y = synth.ellipse_sinogram(ell, g.angles, N, g.axis, N).numpy()
    y = y + 0.02 * y.max() * np.random.default_rng(0).standard_normal(y.shape)
    x0 = np.random.default_rng(1).standard_normal((N, N))
    nA = oracle.opnorm(g, x0, 300, with_grad=False)
    mu = nA / math.sqrt(8.0)
    xs = {}
    for lam in (0.3, 3.0):
        xf = oracle.fista_tv(y, g, lam, 1500, nA ** 2 * 1.0001, 60, fast=True)
        plain = oracle.cp_tv(y, g, lam, 300, 1.01 * oracle.opnorm(g, x0, 300))
        xs[lam] = oracle.cp_tv(y, g, lam, 300, 1.01 * oracle.opnorm(g, x0, 300, mu=mu), mu=mu)
        assert rel(xs[lam], xf) < 5e-3, lam
        assert rel(plain, xf) > 4 * rel(xs[lam], xf), lam
    assert rel(xs[0.3], xs[3.0]) > 0.1


def test_cp_lambda0_is_least_squares():
    """With beta = 0, eq. (3) is plain least squares: CP reaches numpy's lstsq solution."""
    g = Geom(6, 6, 12, synth.uniform_angles(40), 5.7)
    A = lerp_matrix(g)
    rng = np.random.default_rng(14)
    y = A @ rng.random(36) + 0.01 * rng.standard_normal(A.shape[0])
    ref = np.linalg.lstsq(A, y, rcond=None)[0]
    Lk = np.linalg.norm(np.vstack([A, explicit_grad(6, 6)]), 2)
    x, E = oracle.cp_tv(y.reshape(g.K, g.n_det), g, 0.0, 5000, Lk, energy=True)
    assert rel(x.ravel(), ref) < 1e-8
    assert E[-1] <= E[100] <= E[0]
    assert abs(E[-1] - 0.5 * np.sum((A @ ref - y) ** 2)) < 1e-12


def test_cp_energy_decreases_and_recovers_disc():
    N = 48
    g = Geom(N, N, N, synth.uniform_angles(60), (N - 1) / 2)
    y = synth.ellipse_sinogram(synth.disc_params(0.5, 1.0), g.angles, N, g.axis, N).numpy()
    Lk = oracle.opnorm(g, np.random.default_rng(0).standard_normal((N, N)), 100) * 1.01
    x, E = oracle.cp_tv(y, g, 0.05, 300, Lk, energy=True)
    assert E[-1] < E[50] < E[5]
    yy, xx = np.mgrid[0:N, 0:N]
    inside = ((xx - (N - 1) / 2) ** 2 + (yy - (N - 1) / 2) ** 2) < (0.4 * N / 2) ** 2     # disc radius 0.5 N/2
    assert abs(x[inside].mean() - 1.0) < 0.03


# --------------------------------------------------------------------------- ISTA / FISTA (section 3.1)
def test_opnorm_of_A_alone_matches_svd():
    g = Geom(8, 8, 14, synth.uniform_angles(10), 6.7, pixel_size=0.9)
    ref = np.linalg.norm(lerp_matrix(g) * 0.81, 2)          # A = s^2 B^T
    x0 = np.random.default_rng(1).standard_normal((8, 8))
    assert abs(oracle.opnorm(g, x0, 400, with_grad=False) / ref - 1) < 1e-8


def test_ista_identity_one_step_is_rof():
    """A = I, step 1 (|I|^2 = 1), x_0 = 0: the first ISTA/FISTA iterate is prox_{lambda TV}(y)."""
    rng = np.random.default_rng(21)
    y = rng.standard_normal((10, 12))
    for fast in (False, True):
        x = oracle.fista_tv(y, None, 0.3, 1, 1.0, 50, fast=fast, identity_shape=(10, 12))
        assert rel(x, oracle.tv_prox(y, 0.3, 50)) < 1e-14


def test_ista_lambda0_is_landweber_closed_form():
    """beta = 0: ISTA is the Landweber iteration x_k = sum_{j<k} (I - A^T A/La)^j A^T y / La, whose closed
    form in the eigenbasis of A^T A (eigenvalues e) is V diag((1 - (1 - e/La)^k) / e) V^T A^T y."""
    g = Geom(6, 6, 11, synth.uniform_angles(9), 5.2, shifts=np.linspace(-0.3, 0.4, 9))
    A = lerp_matrix(g)
    rng = np.random.default_rng(22)
    y = rng.standard_normal(A.shape[0])
    e, V = np.linalg.eigh(A.T @ A)
    La = 1.1 * e[-1]
    b = V.T @ (A.T @ y)
    for k in (1, 2, 7, 40):
        fac = np.where(e > 1e-12 * e[-1], (1 - (1 - e / La) ** k) / np.maximum(e, 1e-300), k / La)
        ref = V @ (fac * b)
        x = oracle.fista_tv(y.reshape(g.K, g.n_det), g, 0.0, k, La, 5, fast=False)
        assert rel(x.ravel(), ref) < 1e-12, k


def test_fista_rate_bound_and_limit():
    """beta = 0 (exact prox): Beck & Teboulle's bounds F(x_k) - F* <= 2 La |x* - x_0|^2 / (k+1)^2 for FISTA
    and La |x* - x_0|^2 / (2k) for ISTA hold at every k, FISTA ends far below ISTA, and both tend to the
    least-squares solution (numpy lstsq)."""
    g = Geom(8, 8, 12, synth.uniform_angles(6), 5.6)
    A = lerp_matrix(g)
    rng = np.random.default_rng(23)
    y = A @ rng.random(64) + 0.01 * rng.standard_normal(A.shape[0])
    xs = np.linalg.lstsq(A, y, rcond=None)[0]
    Fs = 0.5 * np.sum((A @ xs - y) ** 2)
    La = np.linalg.norm(A, 2) ** 2
    n = 400
    _, Ef = oracle.fista_tv(y.reshape(g.K, g.n_det), g, 0.0, n, La, 1, fast=True, energy=True)
    _, Ei = oracle.fista_tv(y.reshape(g.K, g.n_det), g, 0.0, n, La, 1, fast=False, energy=True)
    k = np.arange(1, n + 1)
    R2 = np.sum(xs ** 2)
    assert np.all(Ef - Fs <= 2 * La * R2 / (k + 1) ** 2 * (1 + 1e-9) + 1e-12)
    assert np.all(Ei - Fs <= La * R2 / (2 * k) * (1 + 1e-9) + 1e-12)
    assert np.all(np.diff(Ei) <= 1e-12)                  # ISTA is monotone
    assert Ef[-1] - Fs < 0.5 * (Ei[-1] - Fs)
    # the iterates themselves approach lstsq (condition number ~5e3 here)
    g = Geom(6, 6, 12, synth.uniform_angles(40), 5.7)
    A = lerp_matrix(g)
    y = A @ rng.random(36) + 0.01 * rng.standard_normal(A.shape[0])
    xs = np.linalg.lstsq(A, y, rcond=None)[0]
    La = np.linalg.norm(A, 2) ** 2
    xf = oracle.fista_tv(y.reshape(g.K, g.n_det), g, 0.0, 3000, La, 1, fast=True)
    xi = oracle.fista_tv(y.reshape(g.K, g.n_det), g, 0.0, 3000, La, 1, fast=False)
    assert rel(xf.ravel(), xs) < 2e-3
    assert rel(xf.ravel(), xs) < 0.05 * rel(xi.ravel(), xs)


def test_fista_and_ista_reach_the_cp_minimiser():
    """beta > 0 on a sparse-angle problem: FISTA, ISTA (accurate inner prox) and Chambolle-Pock, three
    iterations written independently, reach the same energy; FISTA gets there much faster than ISTA."""
    N = 12
    g = Geom(N, N, 16, synth.uniform_angles(8), 7.4)
    A = lerp_matrix(g)
    rng = np.random.default_rng(24)
    img = np.kron(np.array([[1.0, 0.2], [0.5, 0.0]]), np.ones((N // 2, N // 2)))
    y = (A @ img.ravel() + 0.02 * rng.standard_normal(A.shape[0])).reshape(g.K, g.n_det)
    lam = 0.05
    La = np.linalg.norm(A, 2) ** 2
    Lk = np.linalg.norm(np.vstack([A, explicit_grad(N, N)]), 2)
    _, Ec = oracle.cp_tv(y, g, lam, 20000, Lk, energy=True)
    _, Ef = oracle.fista_tv(y, g, lam, 1500, La, 300, fast=True, energy=True)
    _, Ei = oracle.fista_tv(y, g, lam, 60, La, 300, fast=False, energy=True)
    Fs = min(Ec[-1], Ef.min())
    assert abs(Ef[-1] - Ec[-1]) < 1e-6 * Ec[-1]
    assert Ef[59] - Fs < 0.5 * (Ei[59] - Fs)              # the accelerated scheme converges faster
    assert np.all(np.diff(Ei) <= 1e-9 * Ei[0])           # ISTA decreases the energy monotonically


def test_fista_third_iterate_by_hand():
    """A = I, beta = 0, step 1/2 (La = 2): the gradient step is v = (z + y)/2, so x_1 = y/2, z_2 = x_1
    (t_1 = 1 gives no momentum), x_2 = 3y/4, z_3 = x_2 + m_2 (x_2 - x_1), x_3 = (z_3 + y)/2 = y (7 + m_2)/8,
    with t_2 = (1 + sqrt 5)/2, t_3 = (1 + sqrt(1 + 4 t_2^2))/2 = 2.1935270..., m_2 = (t_2 - 1)/t_3 = 0.2817535...
    ISTA gives x_3 = 7y/8."""
    y = np.random.default_rng(25).standard_normal((5, 7))
    x3 = oracle.fista_tv(y, None, 0.0, 3, 2.0, 1, fast=True, identity_shape=(5, 7))
    assert rel(x3, y * (7 + 0.2817535251) / 8) < 1e-8
    x3i = oracle.fista_tv(y, None, 0.0, 3, 2.0, 1, fast=False, identity_shape=(5, 7))
    assert rel(x3i, y * 7 / 8) < 1e-15


def test_fista_lyapunov_function_decreases():
    """Beck & Teboulle's proof: with t_k of FISTA, t_k^2 (F(x_k) - F*) + La/2 |t_k x_k - (t_k - 1) x_{k-1} - x*|^2
    does not increase (beta = 0, exact prox; iterates x_k from separate runs of k iterations)."""
    g = Geom(6, 6, 10, synth.uniform_angles(5), 4.6)
    A = lerp_matrix(g)
    rng = np.random.default_rng(26)
    y = A @ rng.random(36) + 0.01 * rng.standard_normal(A.shape[0])
    xs = np.linalg.lstsq(A, y, rcond=None)[0]
    Fs = 0.5 * np.sum((A @ xs - y) ** 2)
    La = np.linalg.norm(A, 2) ** 2
    X = [np.zeros(36)] + [oracle.fista_tv(y.reshape(g.K, g.n_det), g, 0.0, k, La, 1).ravel() for k in range(1, 61)]
    t, V = 1.0, []
    for k in range(1, 61):
        u = t * X[k] - (t - 1) * X[k - 1] - xs
        V.append(t * t * (0.5 * np.sum((A @ X[k] - y) ** 2) - Fs) + 0.5 * La * np.sum(u * u))
        t = 0.5 * (1 + math.sqrt(1 + 4 * t * t))
    assert np.all(np.diff(V) <= 1e-10 * V[0])


# --------------------------------------------------------------------------- beta selection (section 3.1)
def test_cv_error_is_the_excluded_row_of_the_projection_matrix():
    """|(A x)_k - y_k|^2 with (A x)_k from the explicit interpolation matrix's rows of projection k."""
    g = Geom(8, 8, 13, synth.uniform_angles(7), 6.1, shifts=np.linspace(-0.4, 0.2, 7), pixel_size=0.8)
    A = lerp_matrix(g) * 0.64
    rng = np.random.default_rng(31)
    x = rng.standard_normal(64)
    y = rng.standard_normal((g.K, g.n_det))
    for k in (0, 3, 6):
        ref = np.sum((A[k * g.n_det:(k + 1) * g.n_det] @ x - y[k]) ** 2)
        assert abs(oracle.cv_error(x.reshape(8, 8), y, g, k) / ref - 1) < 1e-12
    gd = oracle.drop_angle(g, 3)
    assert gd.K == 6 and not np.any(gd.angles == g.angles[3]) and np.all(gd.shifts == np.delete(g.shifts, 3))


def test_cv_error_vanishes_on_consistent_data():
    """Data that the image explains exactly (y = A x): zero cross-validation error at every angle."""
    g = Geom(10, 10, 16, synth.uniform_angles(9), 7.3)
    x = np.random.default_rng(32).random((10, 10))
    y = oracle.forward_project(x, g)
    assert max(oracle.cv_error(x, y, g, k) for k in range(g.K)) < 1e-24


def test_e_cohe_values():
    """cos(I(beta) - I(0+), I(beta)): 1 when I(0+) = 0; 0 when the removed part is orthogonal to I(beta);
    -1 when I(0+) = 2 I(beta); -1/sqrt(2) for I(beta) = e1 + e2, I(0+) = e1 + 2 e2; invariant to a common
    positive scale."""
    e1, e2 = np.eye(4)[0], np.eye(4)[1]
    assert abs(oracle.e_cohe(e1 + e2, np.zeros(4)) - 1) < 1e-15
    assert abs(oracle.e_cohe(e1, e1 + e2)) < 1e-15
    assert abs(oracle.e_cohe(e1, 2 * e1) + 1) < 1e-15
    assert abs(oracle.e_cohe(e1 + e2, e1 + 2 * e2) + 1 / math.sqrt(2)) < 1e-15
    rng = np.random.default_rng(33)
    a, b = rng.standard_normal((2, 6, 6))
    assert abs(oracle.e_cohe(3 * a, 3 * b) - oracle.e_cohe(a, b)) < 1e-14


# --------------------------------------------------------------------------- preprocessing extras (section 2.3)
def _flat_setup(K, R, nb, trans):
    """Counts that give exactly the transmission trans [K][R][nb] with dark 100 and flat 30100."""
    dark = np.full((R, nb), 100.0)
    flats = np.full((1, R, nb), 30100.0)
    raw = 100.0 + 30000.0 * trans
    return raw, flats, np.array([0.0]), dark


def test_hotspot_replaces_a_spike_by_the_neighbour_median():
    K, R, nb = 2, 5, 6
    jj, rr = np.meshgrid(np.arange(nb), np.arange(R))
    base = 0.5 + 0.01 * jj + 0.02 * rr                        # linear ramp: 8-neighbour median = centre
    trans = np.repeat(base[None], K, 0)
    trans[1, 2, 3] += 0.3                                      # hot pixel
    trans[0, 1, 1] -= 0.2                                      # cold pixel: the rule is one-sided
    raw, flats, fp, dark = _flat_setup(K, R, nb, trans)
    out = oracle.normalize_hotspot(raw, flats, fp, dark, thr=0.1)
    want = -np.log(np.repeat(base[None], K, 0))
    want[0, 1, 1] = -math.log(base[1, 1] - 0.2)
    # out is [R][K][nb]
    np.testing.assert_allclose(out.transpose(1, 0, 2), want, rtol=0, atol=1e-13)
    # a threshold above the spike keeps it; an infinite threshold is plain normalisation
    out2 = oracle.normalize_hotspot(raw, flats, fp, dark, thr=0.31)
    assert abs(out2[2, 1, 3] + math.log(base[2, 3] + 0.3)) < 1e-13
    np.testing.assert_array_equal(oracle.normalize_hotspot(raw, flats, fp, dark, thr=np.inf),
                                  oracle.normalize(raw, flats, fp, dark))


def test_hotspot_chunks_with_one_row_halo_equal_the_whole_volume():
    """The hot-spot filter's neighbourhood is 3 x 3, so rows r0..r1 of a volume are reproduced exactly by
    filtering only rows r0-1..r1+1 (one halo row per side) and dropping the halo: chunked reconstruction
    equals the whole volume.  Without the halo the chunk's edge rows differ (fewer neighbours)."""
    rng = np.random.default_rng(40)
    K, R, nb = 3, 9, 11
    trans = 0.3 + 0.4 * rng.random((K, R, nb))
    trans[rng.random((K, R, nb)) < 0.08] += 0.4                       # scattered hot pixels
    raw, flats, fp, dark = _flat_setup(K, R, nb, trans)
    whole = oracle.normalize_hotspot(raw, flats, fp, dark, thr=0.15)
    for r0, r1 in ((0, 3), (3, 6), (6, 9)):
        lo, hi = max(r0 - 1, 0), min(r1 + 1, R)
        part = oracle.normalize_hotspot(raw[:, lo:hi], flats[:, lo:hi], fp, dark[lo:hi], thr=0.15)
        np.testing.assert_array_equal(part[r0 - lo:r0 - lo + (r1 - r0)], whole[r0:r1])
    bare = oracle.normalize_hotspot(raw[:, 3:6], flats[:, 3:6], fp, dark[3:6], thr=0.15)
    assert not np.array_equal(bare, whole[3:6])


def test_hotspot_even_neighbour_count_and_edges():
    """Corner pixel: 3 neighbours (odd median); edge pixel: 5; interior: 8 (mean of the middle two)."""
    trans = np.full((1, 3, 3), 0.5)
    trans[0, 0, 0] = 0.9                                       # corner spike, neighbours 0.5 -> median 0.5
    trans[0, 1, 1] = 0.95                                      # centre spike: neighbours 0.9 + seven 0.5
    raw, flats, fp, dark = _flat_setup(1, 3, 3, trans)
    out = oracle.normalize_hotspot(raw, flats, fp, dark, thr=0.1)
    assert abs(out[0, 0, 0] + math.log(0.5)) < 1e-13
    assert abs(out[1, 0, 1] + math.log(0.5)) < 1e-13          # median of {0.9, 0.5 x 7} = 0.5
    trans[0, 0, 1] = trans[0, 0, 2] = trans[0, 1, 0] = 0.9     # now 4 of 8 neighbours are 0.9
    raw, flats, fp, dark = _flat_setup(1, 3, 3, trans)
    out = oracle.normalize_hotspot(raw, flats, fp, dark, thr=0.1)
    assert abs(out[1, 0, 1] + math.log(0.7)) < 1e-13          # (0.5 + 0.9) / 2


def test_ring_filter_closed_forms():
    K, L, w = 7, 40, 3
    rng = np.random.default_rng(41)
    # a constant-in-j signal has no high frequencies: unchanged
    p = np.tile(rng.standard_normal((K, 1)), (1, L))
    np.testing.assert_allclose(oracle.ring_filter(p, w), p, atol=1e-14)
    # linear in j: unchanged wherever the whole window exists
    p = np.tile(0.3 * np.arange(L), (K, 1)) + rng.standard_normal((K, 1))
    q = oracle.ring_filter(p, w)
    np.testing.assert_allclose(q[:, w:L - w], p[:, w:L - w], atol=1e-12)
    # a stripe of height h in bin j0: residue h/(2w+1) at j0, +h/(2w+1) in the w bins on each side
    h, j0 = 2.0, 17
    p = np.zeros((K, L))
    p[:, j0] = h
    q = oracle.ring_filter(p, w)
    want = np.zeros(L)
    want[j0 - w:j0 + w + 1] = h / (2 * w + 1)
    np.testing.assert_allclose(q, np.tile(want, (K, 1)), atol=1e-14)
    # with obj = p the data are left exactly as they are
    p = rng.standard_normal((K, L))
    np.testing.assert_allclose(oracle.ring_filter(p, w, obj=p), p, atol=1e-14)


def test_ring_filter_on_an_ellipse_sinogram_and_object_subtraction():
    """Per-bin offsets (rings) on an ellipse object.  A narrow window removes most of the stripe energy;
    a wide one lets the object's own angle-averaged profile into the high-pass part and adds new errors
    larger than the stripes (the failure the paper shows at a bone); subtracting the projection of the
    thresholded first reconstruction before the average removes that leak."""
    N, K = 64, 90
    g = Geom(N, N, N, synth.uniform_angles(K), (N - 1) / 2)
    clean = synth.ellipse_sinogram(synth.random_ellipses(synth.rng_for(9, 0, 0), 5), g.angles, N, g.axis, N).numpy()
    stripes = 0.05 * np.random.default_rng(42).standard_normal(N) * clean.max()
    ref = np.linalg.norm(np.tile(stripes, (K, 1)))
    data = clean + stripes[None]
    assert np.linalg.norm(oracle.ring_filter(data, 2) - clean) < 0.45 * ref
    assert np.linalg.norm(oracle.ring_filter(data, 16) - clean) > 1.5 * ref
    obj = oracle.ring_object(data, g, 0.3)
    assert np.linalg.norm(oracle.ring_filter(data, 16, obj=obj) - clean) < 0.5 * ref
