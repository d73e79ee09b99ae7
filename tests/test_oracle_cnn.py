"""Pins of the CNN oracle: finite differences of its hand-derived backward pass
(FP64), its convolutions against explicit loops, BF16 rounding values, and the
first Adam step's closed form."""
import math

import numpy as np
import pytest

from oracle.cnn import UNetOracle, to_bf16, layers


def rand_params(base, levels, seed, scale=1.0):
    lay, n = layers(base, levels)
    rng = np.random.default_rng(seed)
    p = np.zeros(n)
    for d in lay.values():
        fan = {"conv": 9 * d["cin"], "up": d["cin"], "head": d["cin"]}[d["kind"]]
        p[d["w"]:d["b"]] = rng.standard_normal(d["b"] - d["w"]) * scale * math.sqrt(2.0 / fan)
        nb = d["cout"] if d["kind"] != "head" else 1
        p[d["b"]:d["b"] + nb] = rng.uniform(0.0, 0.1, nb)
    return p


@pytest.mark.parametrize("levels", [2, 3])
def test_backward_matches_finite_differences(levels):
    base, B, H = 8, 2, 8
    net = UNetOracle(base, levels, "fp64")
    p = rand_params(base, levels, 1)
    rng = np.random.default_rng(2)
    x = rng.random((B, H, H))
    t = rng.random((B, H, H))
    loss, g = net.loss_and_grad(p, x, t)
    lay, n = layers(base, levels)
    idx = []
    for d in lay.values():                       # a few entries of every layer, weights and biases
        lo, hi = d["w"], d["b"] + (d["cout"] if d["kind"] != "head" else 1)
        cand = np.arange(lo, hi)
        if d["name"] == "enc0a":                 # only input channel 0 is live
            cand = cand[(cand >= d["b"]) | ((cand - lo) % d["cin"] == 0)]
        idx += list(rng.choice(cand, size=min(4, cand.size), replace=False))
    eps = 1e-6
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += eps
        pm[i] -= eps
        fd = (np.mean((net.forward(pp, x) - t) ** 2) - np.mean((net.forward(pm, x) - t) ** 2)) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-5 * max(1e-3, abs(fd)), (i, fd, g[i])


def test_conv_and_upconv_match_explicit_loops():
    rng = np.random.default_rng(3)
    B, H, W, Ci, Co = 2, 5, 4, 3, 2
    x = rng.standard_normal((B, H, W, Ci))
    K = rng.standard_normal((Co, 9, Ci))
    b = rng.standard_normal(Co)
    ref = np.zeros((B, H, W, Co))
    for bb in range(B):
        for y in range(H):
            for xx in range(W):
                for co in range(Co):
                    s = b[co]
                    for ty in range(3):
                        for tx in range(3):
                            yy, xs = y + ty - 1, xx + tx - 1
                            if 0 <= yy < H and 0 <= xs < W:
                                for ci in range(Ci):
                                    s += x[bb, yy, xs, ci] * K[co, 3 * ty + tx, ci]
                    ref[bb, y, xx, co] = s
    orc = UNetOracle(8, 2)
    np.testing.assert_allclose(orc.conv(x, K, b), ref, atol=1e-12)
    # the FP32-accumulation mode computes the same sums up to FP32 rounding
    np.testing.assert_allclose(UNetOracle(8, 2, acc="fp32").conv(x, K, b), ref, rtol=0,
                               atol=1e-5 * np.abs(ref).max())
    U = rng.standard_normal((4, Co, Ci))
    up = orc.up(x, U, b)
    for bb in range(B):
        for y in range(2 * H):
            for xx in range(2 * W):
                d = 2 * (y % 2) + (xx % 2)
                np.testing.assert_allclose(up[bb, y, xx], U[d] @ x[bb, y // 2, xx // 2] + b, atol=1e-12)


def test_bf16_rounding():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 2 ** -9, -2.5, 3.0e-3])
    r = to_bf16(vals)
    assert r[0] == 1.0
    assert r[1] == 1.0                    # halfway: ties to even (mantissa ...0)
    assert r[2] == 1.0 + 4 * 2 ** -8      # halfway: ties to even (rounds up)
    assert r[3] == 1.0
    assert r[4] == -2.5
    assert abs(r[5] - 3.0e-3) <= 3.0e-3 * 2 ** -8


def test_pool_tie_goes_to_first():
    x = np.zeros((1, 2, 2, 1))
    x[0, 0, 1, 0] = x[0, 1, 0, 0] = 2.0
    m, a = UNetOracle.pool(x)
    assert m[0, 0, 0, 0] == 2.0 and a[0, 0, 0, 0] == 1


def test_adam_first_step():
    p = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -0.01, 0.0])
    p1, m, v = UNetOracle.adam(p, g, np.zeros(3), np.zeros(3), 1, lr=0.1)
    np.testing.assert_allclose(p1, p - 0.1 * g / (np.abs(g) + 1e-8), rtol=1e-12)
