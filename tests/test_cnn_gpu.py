"""GPU U-Net (MFMA BF16 kernels) against the BF16-emulating NumPy oracle:
forward output, every layer's weight and bias gradient, one Adam step, and a
short overfitting run.  One layer fed with the GPU's own inputs: 2e-3 relative
L2 (FP32 vs FP64 accumulation can flip single BF16 roundings).  The whole
network: twice the spread that the oracle itself shows between exact and FP32
sums on the same inputs, per output (tests/golden/cnn_fp32_spread.json, written
by tests/golden/cnn_tolerance.py from the oracle alone), never below 2e-3."""
import json
import math
import os
import sys

import numpy as np
import pytest
import torch

from oracle.cnn import UNetOracle, layers
from paper_1306_1392_amd.cnn import UNet, init_params

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
from cnn_tolerance import CASES, case_data, case_params, key  # noqa: E402

pytestmark = pytest.mark.gpu
TOL = 2e-3        # one layer: FP32 vs FP64 accumulation flips isolated BF16 roundings
with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "cnn_fp32_spread.json")) as _f:
    SPREAD = json.load(_f)["cases"]


def bar(case, name):
    """Whole-network bar of one output: twice the oracle's own FP32-accumulation spread, at least TOL."""
    return max(TOL, 2.0 * SPREAD[key(case)][name])


def rel(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def params_with_bias(base, levels, seed):
    return case_params(base, levels, seed)


@pytest.mark.parametrize("base,levels,B,H", CASES)
def test_forward_and_gradients_match_oracle(dev, base, levels, B, H):
    case = (base, levels, B, H)
    p = case_params(base, levels, 1)
    x, t = case_data(B, H, 5)
    net = UNet(B + 1, H, H, base, levels)           # batch larger than used: n < batch path
    net.set_params(p)
    xt, tt = torch.from_numpy(x).to(dev), torch.from_numpy(t).to(dev)
    out = net.forward(xt).cpu().numpy()
    orc = UNetOracle(base, levels, "bf16")
    ref = orc.forward(p, x)
    assert rel(out - x, ref - x) <= bar(case, "out"), rel(out - x, ref - x)
    loss = net.backward(xt, tt)
    g = net.get_grads().cpu().numpy()
    lref, gref = orc.loss_and_grad(p, x, t)
    assert abs(float(loss) - lref) <= 1e-3 * lref
    lay, _ = layers(base, levels)
    for d in lay.values():
        nb = d["cout"] if d["kind"] != "head" else 1
        w = slice(d["w"], d["b"])
        b = slice(d["b"], d["b"] + nb)
        if d["name"] == "enc0a":     # only input channel 0 is live
            gw = g[w].reshape(d["cout"], 9, 8)
            assert np.all(gw[:, :, 1:] == 0)
        assert rel(g[w], gref[w]) <= bar(case, d["name"] + ".w"), (d["name"], "w", rel(g[w], gref[w]))
        assert rel(g[b], gref[b]) <= bar(case, d["name"] + ".b"), (d["name"], "b", rel(g[b], gref[b]))


def test_adam_step_matches_oracle(dev):
    base, levels, B, H = 8, 3, 2, 32
    p = params_with_bias(base, levels, 2)
    rng = np.random.default_rng(6)
    x = rng.random((B, H, H)).astype(np.float32)
    t = rng.random((B, H, H)).astype(np.float32)
    net = UNet(B, H, H, base, levels)
    net.set_params(p)
    net.train_step(torch.from_numpy(x).to(dev), torch.from_numpy(t).to(dev), lr=1e-3)
    got = net.get_params().cpu().numpy()
    orc = UNetOracle(base, levels, "bf16")
    _, g = orc.loss_and_grad(p, x, t)
    ref, _, _ = orc.adam(p.astype(np.float64), g, np.zeros_like(g), np.zeros_like(g), 1, lr=1e-3)
    # the first Adam step moves each weight by ~lr sign(g): compare the step itself
    live = np.abs(g) > 1e-6 * np.abs(g).max()
    assert rel((got - p)[live], (ref - p)[live]) <= 2e-2


def test_training_overfits_a_fixed_batch(dev):
    base, levels, B, H = 16, 3, 4, 64
    net = UNet(B, H, H, base, levels)
    net.set_params(init_params(base, levels, 3))
    rng = np.random.default_rng(7)
    t = np.zeros((B, H, H), dtype=np.float32)
    t[:, 16:48, 16:48] = 1.0
    x = (t + 0.3 * rng.standard_normal((B, H, H))).astype(np.float32)
    xt, tt = torch.from_numpy(x).to(dev), torch.from_numpy(t).to(dev)
    losses = [float(net.train_step(xt, tt, lr=2e-3)) for _ in range(150)]
    assert losses[-1] < 0.2 * losses[0], (losses[0], losses[-1])


def test_data_scale_inside_the_network(dev):
    """With data scale c the network computes x + f(c x)/c and trains on (c x, c target): the same numbers
    as scaling by hand around a scale-1 network (forward bit for bit; the training step's loss and weights
    too, since the scale enters only at the input, the target and the output).  c is a power of two, so
    every product and quotient by it is exact in FP32 whichever way either side rounds or fuses it."""
    base, levels, B, H, c = 8, 3, 2, 32, 8.0
    p = case_params(base, levels, 4)
    x, t = case_data(B, H, 6)
    xt, tt = torch.from_numpy(x).to(dev), torch.from_numpy(t).to(dev)
    a, b = UNet(B, H, H, base, levels), UNet(B, H, H, base, levels)
    a.set_params(p)
    b.set_params(p)
    a.set_scale(c)
    assert a.scale == c and b.scale == 1.0
    fa = a.forward(xt)
    fb = b.forward((xt * c).contiguous()) / c
    assert torch.equal(fa, fb)
    la = float(a.train_step(xt, tt, lr=1e-3))
    lb = float(b.train_step((xt * c).contiguous(), (tt * c).contiguous(), lr=1e-3))
    assert la == lb
    assert torch.equal(a.get_params(), b.get_params())
    with pytest.raises(Exception):
        a.set_scale(0.0)


@pytest.mark.parametrize("base,levels,H,W", [(32, 4, 48, 80), (16, 3, 32, 72), (8, 4, 40, 56)])
def test_inference_upsampling_fused_into_decoder_conv(dev, base, levels, H, W):
    """Inference runs a decoder level's up-sampling inside its first conv wherever that conv has at most
    32 inputs from each side and 32 outputs (the concatenation is never stored there): its output equals
    the unfused up-sampling + conv of the training forward bit for bit at every level, on ragged tiles."""
    B = 2
    p = case_params(base, levels, 7)
    rng = np.random.default_rng(11)
    x = rng.random((B, H, W)).astype(np.float32)
    t = (x + 0.1 * rng.standard_normal((B, H, W))).astype(np.float32)
    net = UNet(B, H, W, base, levels)
    net.set_params(p)
    xt, tt = torch.from_numpy(x).to(dev), torch.from_numpy(t).to(dev)
    out = net.forward(xt)
    torch.cuda.synchronize()
    fused = [net.tensor("da", l).clone() for l in range(levels - 1)]
    net.backward(xt, tt)   # training forward: up-sampling kernel, concatenation, conv
    torch.cuda.synchronize()
    for l in range(levels - 1):
        assert torch.equal(fused[l], net.tensor("da", l)), l
    assert torch.isfinite(out).all()


def test_every_layer_teacher_forced(dev):
    """Each layer of the GPU U-Net against the oracle's layer fed with the GPU's own BF16
    inputs (no compounding of rounding differences across layers): forward activations,
    activation gradients and weight / bias gradients of the 4-level, 32-base network."""
    from oracle.cnn import to_bf16
    base, levels, B, H = 32, 4, 2, 64
    L = levels
    p = params_with_bias(base, levels, 3).astype(np.float64)
    rng = np.random.default_rng(8)
    x = rng.random((B, H, H)).astype(np.float32)
    t = (x + 0.1 * rng.standard_normal((B, H, H))).astype(np.float32)
    net = UNet(B, H, H, base, levels)
    net.set_params(p.astype(np.float32))
    xt, tt = torch.from_numpy(x).to(dev), torch.from_numpy(t).to(dev)
    out = net.forward(xt).cpu().numpy().astype(np.float64)
    net.backward(xt, tt)
    g = net.get_grads().cpu().numpy().astype(np.float64)
    orc = UNetOracle(base, levels, "bf16")
    lay, _ = layers(base, levels)

    def T(kind, l=0, grad=False):
        return net.tensor(kind, l, grad).double().cpu().numpy()

    relu = lambda a: np.maximum(a, 0.0)
    checks = []

    def cmp(name, got, ref, tol=TOL):
        r = rel(got, ref)
        checks.append((name, r))
        assert r <= tol, (name, r)

    def cmp_grads(name, dW, db):
        d = lay[name]
        nb = d["cout"] if d["kind"] != "head" else 1
        cmp(name + ".dW", g[d["w"]:d["b"]], dW.ravel())
        cmp(name + ".db", g[d["b"]:d["b"] + nb], db)

    # forward
    for l in range(L):
        c = base << l
        xin = T("x8") if l == 0 else T("pool", l - 1)
        Wa, ba = orc.weights(p, f"enc{l}a")
        cmp(f"enc{l}a", T("ea", l), to_bf16(relu(orc.conv(xin, Wa, ba))))
        Wb, bb = orc.weights(p, f"enc{l}b")
        eb = T("cat", l)[..., :c] if l < L - 1 else T("bott")
        cmp(f"enc{l}b", eb, to_bf16(relu(orc.conv(T("ea", l), Wb, bb))))
        if l < L - 1:
            assert np.array_equal(T("pool", l), orc.pool(eb)[0])
    for l in range(L - 2, -1, -1):
        c = base << l
        below = T("bott") if l == L - 2 else T("db", l + 1)
        U, bu = orc.weights(p, f"up{l}")
        cmp(f"up{l}", T("cat", l)[..., c:], to_bf16(relu(orc.up(below, U, bu))))
        Wa, ba = orc.weights(p, f"dec{l}a")
        cmp(f"dec{l}a", T("da", l), to_bf16(relu(orc.conv(T("cat", l), Wa, ba))))
        Wb, bb = orc.weights(p, f"dec{l}b")
        cmp(f"dec{l}b", T("db", l), to_bf16(relu(orc.conv(T("da", l), Wb, bb))))
    wh, bh = orc.weights(p, "head")
    cmp("head", out - x, bh[0] + T("db", 0) @ wh, tol=1e-5)

    # backward
    n = out.size
    dout = (2.0 * (out - t) / n)
    d0 = T("db", 0)
    cmp("head.dD", T("db", 0, True), to_bf16(np.where(d0 > 0, dout[..., None] * wh, 0.0)))
    cmp_grads("head", (d0 * dout[..., None]).reshape(-1, base).sum(0), np.array([dout.sum()]))

    def conv_layer(name, xin, dz, dx_gpu=None):
        W, _ = orc.weights(p, name)
        dW, db, dx = orc.conv_bwd(xin, W, dz)
        cmp_grads(name, dW, db)
        if dx_gpu is not None:
            cmp(name + ".dX", dx_gpu, to_bf16(np.where(xin > 0, dx, 0.0)))

    for l in range(L - 1):
        c = base << l
        conv_layer(f"dec{l}b", T("da", l), T("db", l, True), T("da", l, True))
        dcat = T("cat", l, True)
        W, _ = orc.weights(p, f"dec{l}a")
        dW, db, dx = orc.conv_bwd(T("cat", l), W, T("da", l, True))
        cmp_grads(f"dec{l}a", dW, db)
        ref = to_bf16(np.where(T("cat", l) > 0, dx, 0.0))
        cmp(f"dec{l}a.dX(up half)", dcat[..., c:], ref[..., c:])
        below = T("bott") if l == L - 2 else T("db", l + 1)
        dbelow = T("bott", 0, True) if l == L - 2 else T("db", l + 1, True)
        U, _ = orc.weights(p, f"up{l}")
        dU, dbu, dxu = orc.up_bwd(below, U, dcat[..., c:])
        cmp_grads(f"up{l}", dU, dbu)
        cmp(f"up{l}.dX", dbelow, to_bf16(np.where(below > 0, dxu, 0.0)))
        if l == 0:
            # skip half of level 0 plus the pooled gradient routed back by pool 0
            add = orc.unpool_add(ref[..., :c], T("pool", 0, True), orc.pool(T("cat", 0)[..., :c])[1],
                                 T("pool", 0))
            cmp("cat0.dX(skip + pool)", dcat[..., :c], np.where(add != 0, to_bf16(ref[..., :c] + add), ref[..., :c]))
    for l in range(L - 1, -1, -1):
        c = base << l
        dz = T("bott", 0, True) if l == L - 1 else T("cat", l, True)[..., :c]
        conv_layer(f"enc{l}b", T("ea", l), dz, T("ea", l, True))
        xin = T("x8") if l == 0 else T("pool", l - 1)
        conv_layer(f"enc{l}a", xin, T("ea", l, True), None if l == 0 else T("pool", l - 1, True))
    assert len(checks) > 40
