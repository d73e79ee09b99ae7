"""Whole-network tolerance of the GPU U-Net tests, derived from the oracle alone.

Two correct implementations of the BF16-storage / FP32-accumulate network (section
"learned corrector" of the design; not in the paper) differ by more than rounding of
one layer: a different FP32 summation order flips isolated BF16 roundings of stored
activations and gradients, and those flips compound through the layers and back.
This script measures that spread on the oracle itself: the BF16-emulating oracle with
exact (FP64) sums against the same oracle with FP32 matrix products in two summation
orders, on the inputs of each whole-network test case, per output (the residual output
and every layer's weight and bias gradients), keeping the larger of the two.  The GPU
test allows twice the measured spread for each of them (never less than the
single-layer bar).

Run from the repository root:  python tests/golden/cnn_tolerance.py
It writes tests/golden/cnn_fp32_spread.json.  Only oracle/ and numpy are used.
"""
from __future__ import annotations

import json
import math
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle.cnn import UNetOracle, layers  # noqa: E402

# (base channels, levels, batch, image size) of the whole-network GPU test cases
CASES = [(8, 2, 2, 16), (8, 3, 2, 32), (32, 4, 2, 64), (16, 3, 3, 48)]
OUT = os.path.join(HERE, "cnn_fp32_spread.json")


def case_params(base: int, levels: int, seed: int) -> np.ndarray:
    """Float32 parameters: He-normal conv / transposed-conv weights (the first conv reads only input
    channel 0), biases U[0, 0.05], head weights N(0, 0.1^2)."""
    lay, n = layers(base, levels)
    rng = np.random.default_rng(np.random.SeedSequence([4, 9, seed]))
    p = np.zeros(n)
    for d in lay.values():
        if d["kind"] == "conv":
            real = 1 if d["name"] == "enc0a" else d["cin"]
            W = rng.standard_normal((d["cout"], 9, d["cin"])) * math.sqrt(2.0 / (9 * real))
            if d["name"] == "enc0a":
                W[:, :, 1:] = 0.0
            p[d["w"]:d["b"]] = W.ravel()
            p[d["b"]:d["b"] + d["cout"]] = rng.uniform(0.0, 0.05, d["cout"])
        elif d["kind"] == "up":
            p[d["w"]:d["b"]] = (rng.standard_normal((4, d["cout"], d["cin"])) * math.sqrt(2.0 / d["cin"])).ravel()
            p[d["b"]:d["b"] + d["cout"]] = rng.uniform(0.0, 0.05, d["cout"])
        else:
            p[d["w"]:d["b"]] = rng.standard_normal(d["cin"]) * 0.1
            p[d["b"]] = rng.uniform(0.0, 0.05)
    return p.astype(np.float32)


def case_data(B: int, H: int, seed: int):
    """Input x ~ U[0, 1) and target x + N(0, 0.1^2), float32 [B][H][H]."""
    rng = np.random.default_rng(np.random.SeedSequence([4, 10, seed]))
    x = rng.random((B, H, H)).astype(np.float32)
    t = (x + 0.1 * rng.standard_normal((B, H, H))).astype(np.float32)
    return x, t


def rel(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def spread(base: int, levels: int, B: int, H: int) -> dict:
    """{output name: rel-L2 between the FP64-sum and FP32-sum BF16 oracles} for one case."""
    p = case_params(base, levels, 1)
    x, t = case_data(B, H, 5)
    ref = UNetOracle(base, levels, "bf16")
    o64 = ref.forward(p, x)
    _, g64 = ref.loss_and_grad(p, x, t)
    lay, _ = layers(base, levels)
    res = {}
    for acc in ("fp32", "fp32rev"):
        alt = UNetOracle(base, levels, "bf16", acc=acc)
        o32 = alt.forward(p, x)
        _, g32 = alt.loss_and_grad(p, x, t)
        cur = {"out": rel(o32 - x, o64 - x)}
        for d in lay.values():
            nb = d["cout"] if d["kind"] != "head" else 1
            cur[d["name"] + ".w"] = rel(g32[d["w"]:d["b"]], g64[d["w"]:d["b"]])
            cur[d["name"] + ".b"] = rel(g32[d["b"]:d["b"] + nb], g64[d["b"]:d["b"] + nb])
        for k, v in cur.items():
            res[k] = max(res.get(k, 0.0), v)
    return res


def key(case) -> str:
    return "base%d_levels%d_batch%d_size%d" % case


def main():
    table = {}
    for case in CASES:
        table[key(case)] = {k: float("%.4g" % v) for k, v in spread(*case).items()}
        worst = max(table[key(case)].items(), key=lambda kv: kv[1])
        print(key(case), "largest spread:", worst, flush=True)
    with open(OUT, "w") as f:
        json.dump({"what": "largest rel-L2 between the BF16-emulating oracle with FP64 sums and with FP32 "
                           "matrix products (two summation orders), per output of each whole-network case",
                   "script": "tests/golden/cnn_tolerance.py", "cases": table}, f, indent=1, sort_keys=True)
        f.write("\n")
    print("wrote", OUT)


if __name__ == "__main__":
    main()
