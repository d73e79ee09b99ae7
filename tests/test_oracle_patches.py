"""Pins of the overlapping-patch prior oracle (section 3.2, eqs. (4)-(9)) against hand-worked core maps,
finite differences of the functional, and closed-form minimisers."""
import numpy as np
import pytest

import oracle
import synth
from oracle import Geom
from oracle.patches import PatchGrid, PatchProblem, fista, soft
from synth import dct_dictionary


def test_core_map_by_hand():
    """8 x 8 image, 4 x 4 patches, stride 2: corners 0, 2, 4, centres 1.5, 3.5, 5.5; along one axis the
    L1-nearest centre of pixels 0..7 is 0, 0, 0, 1, 1, 2, 2, 2 (pixel 3 is 0.5 from 3.5), and with L1
    distance the 2-D core is the pair of 1-D cores (patch index = 3 a_row + a_col)."""
    g = PatchGrid(8, 8, 4, 2)
    a = np.array([0, 0, 0, 1, 1, 2, 2, 2])
    np.testing.assert_array_equal(g.core, 3 * a[:, None] + a[None, :])
    assert g.n_p == 9 and np.all(g.r[4] == [2, 2])


def test_core_ties_and_partition():
    """m = 5, stride 3 on 11 x 13 pixels: the cores partition the image, each core lies inside its patch,
    every pixel is covered; an exact L1 tie goes to the lower patch index."""
    g = PatchGrid(11, 13, 5, 3)
    assert set(np.unique(g.core)) == set(range(g.n_p))
    for p, (ry, rx) in enumerate(g.r):
        iy, ix = np.nonzero(g.core == p)
        assert iy.min() >= ry and iy.max() < ry + 5 and ix.min() >= rx and ix.max() < rx + 5
    cover = g.scatter_add(np.ones((g.n_p, 25)))
    assert cover.min() >= 1
    h = PatchGrid(4, 7, 4, 3)          # column corners 0, 3; centres 1.5, 4.5; pixel 3 is 1.5 from both
    assert np.all(h.core[:, 3] == 0)   # lowest patch index wins


def test_assemble_scatter_patches_adjoint():
    rng = np.random.default_rng(1)
    g = PatchGrid(12, 10, 4, 2)
    x = rng.standard_normal((12, 10))
    P = rng.standard_normal((g.n_p, 16))
    assert abs(np.sum(g.patches(x) * P) - np.sum(x * g.scatter_add(P))) < 1e-12
    # core_patches is the adjoint of assemble
    assert abs(np.sum(g.assemble(P) * x) - np.sum(P * g.core_patches(x))) < 1e-12


@pytest.mark.parametrize("tomo", [False, True])
def test_gradient_matches_finite_differences(tomo):
    """eq. (9) against central differences of eq. (8)'s smooth part (FP64)."""
    rng = np.random.default_rng(2)
    N, m, st = 10, 4, 3
    g = PatchGrid(N, N, m, st)
    D = dct_dictionary(m, extra=8, seed=3)
    if tomo:
        geo = Geom(N, N, 14, synth.uniform_angles(7), 6.4)
        y = rng.standard_normal((7, 14))
        prob = PatchProblem(g, D, y, rho=0.7, beta=0.1, project=lambda x: oracle.forward_project(x, geo),
                            backproject=lambda r: oracle.backproject(r, geo))
    else:
        prob = PatchProblem(g, D, rng.standard_normal((N, N)), rho=0.7, beta=0.1)
    W = rng.standard_normal((g.n_p, D.shape[0]))
    G = prob.grad(W)
    h = 1e-5
    for _ in range(12):
        p, k = rng.integers(g.n_p), rng.integers(D.shape[0])
        E = np.zeros_like(W)
        E[p, k] = h
        fd = (prob.smooth(W + E) - prob.smooth(W - E)) / (2 * h)
        assert abs(fd - G[p, k]) <= 1e-6 * max(1.0, abs(fd)), (p, k, fd, G[p, k])


def test_single_patch_identity_is_soft_threshold():
    """One patch covering the image, D = identity, Pi = I: eq. (8) is |y - w|^2 + beta |w|_1 (the rho
    term vanishes), whose minimiser is the soft threshold of y at beta/2."""
    rng = np.random.default_rng(4)
    m = 6
    g = PatchGrid(m, m, m, m)
    y = rng.standard_normal((m, m))
    prob = PatchProblem(g, np.eye(m * m), y, rho=3.0, beta=0.8)
    W, x = fista(prob, 200, L=2.0)
    np.testing.assert_allclose(x, soft(y, 0.4), atol=1e-12)
    assert abs(prob.lipschitz(50) - 2.0) < 1e-9


def test_ista_decreases_and_fista_is_faster():
    rng = np.random.default_rng(5)
    N = 16
    g = PatchGrid(N, N, 4, 2)
    D = dct_dictionary(4, extra=16, seed=6)
    geo = Geom(N, N, 22, synth.uniform_angles(10), 10.3)
    img = np.kron(np.array([[1.0, 0.0], [0.3, 0.6]]), np.ones((N // 2, N // 2)))
    y = oracle.forward_project(img, geo) + 0.05 * rng.standard_normal((10, 22))
    prob = PatchProblem(g, D, y, rho=0.5, beta=0.05, project=lambda x: oracle.forward_project(x, geo),
                        backproject=lambda r: oracle.backproject(r, geo))
    L = prob.lipschitz(100) * 1.01
    _, _, Ei = fista(prob, 60, L, fast=False, energy=True)
    _, _, Ef = fista(prob, 60, L, fast=True, energy=True)
    assert np.all(np.diff(Ei) <= 1e-9 * Ei[0])
    assert Ef[-1] < Ei[-1]
