"""Throughput of the FBP path on one MI355X.

Workload (one step = the whole path over one batch, replayed as one HIP graph):
64 slices of 2048 x 2048, 2048 detector bins, 1800 projections over 180
degrees, raw uint16 radiographs with two flats and a dark, rotation axis 3.5
bins right of the detector centre, 20 random ellipses per slice.  The path is
normalise + -log (fused into the filter load) -> ramp filter -> backprojection.

Printed: one JSON line with GUPS (giga voxel-angle updates per second),
slices/s, the backprojector's roofline position and the FP64 CPU oracle timed
on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "backprojection GUPS (voxel·angle/s) + slices/s at 2048²; learned vs TV RMSE"
# VALU peak of MI355X: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz (wave64 instruction = 64 lane-ops)
VALU_LANE_OPS_PEAK = 256 * 64 * 2.4e9
BP_OPS_PER_UPDATE = 6   # t, trunc, fract, LDS address, add, fma
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_hash(path):
    return hashlib.sha256(open(path, "rb").read()).hexdigest()[:16]


def traffic_for(kernel_src: str, per_launch_key: str):
    """HBM bytes per launch from the committed counter summary, if it was taken on this kernel source."""
    f = os.path.join(ROOT, "profiles", "bp_fbp2048_traffic.json")
    if not os.path.exists(f):
        return None
    d = json.load(open(f))
    if d.get("source_sha256_16") != source_hash(kernel_src):
        return None
    return d.get(per_launch_key)


def cpu_baseline(R, N, K, cfg):
    """FP64 oracle on a bounded sample: normalise + filter of one whole slice, and
    backprojection of 1/32 of its pixels; extrapolated to the full workload."""
    import numpy as np
    import oracle
    oracle.build()
    r = 0
    raw = cfg["raw"][:, r:r + 1, :].cpu().numpy().astype(np.float64)
    flats = cfg["flats"][:, r:r + 1, :].cpu().numpy()
    dark = cfg["dark"][r:r + 1].cpu().numpy()
    g = oracle.Geom(N, N, N, cfg["angles"], cfg["axis"])
    t0 = time.perf_counter()
    sino = oracle.normalize(raw, flats, cfg["flat_pos"], dark)
    filt = oracle.fbp_filter(sino, g)[0]
    t1 = time.perf_counter()
    rows = np.arange(0, N, 32)
    ix = np.tile(np.arange(N), rows.shape[0])
    iy = np.repeat(rows, N)
    oracle.backproject_points(filt, g, ix, iy, extended=True)
    t2 = time.perf_counter()
    t_slice = (t1 - t0) + (t2 - t1) * 32
    t_full = t_slice * R
    return {"value": R * N * N * K / t_full / 1e9, "unit": "GUPS", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"1 of {R} slices: normalise + direct Ram-Lak filter of all {K} rows, backprojection of "
                      f"every 32nd image row ({N // 32} x {N} pixels x {K} angles); measured "
                      f"{t2 - t0:.1f} s, extrapolated x32 (backprojection) and x{R} (slices)",
            "seconds_measured": round(t2 - t0, 2)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--slices", type=int, default=64)
    ap.add_argument("--n", type=int, default=2048)
    ap.add_argument("--angles", type=int, default=1800)
    ap.add_argument("--tile", type=int, default=-1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile-only", action="store_true", help="warmup + steps only, no extra measurements")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a plain 2 GiB device copy (reference kernel for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build measures one GPU only (the slices of a batch are independent; "
              "see DESIGN.md for how the path shards across GPUs)", file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    import paper_1306_1392_amd as ph

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    R, N, K = args.slices, args.n, args.angles
    log(f"bench: generating {R} x {N}^2 slices, {K} angles, raw uint16 ...")
    cfg = synth.cfg_batched_raw(R=R, N=N, K=K, device=dev)
    torch.cuda.synchronize()
    geo = ph.Geometry(N, N, N, cfg["angles"], cfg["axis"])
    plan = ph.Plan(geo, n_slices=R)
    plan.set_tiles(args.tile, False)
    tile = plan.get_tiles()[0]
    raw, flats, dark = cfg["raw"], cfg["flats"], cfg["dark"]
    out = torch.empty(plan.img_shape(), device=dev, dtype=torch.float32)
    work = torch.empty(ph.work_bytes(plan, raw=raw, method=ph.FBP), device=dev, dtype=torch.uint8)
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())

    def step():
        ph.reconstruct_slices(plan, raw=raw, flats=flats, flat_pos=cfg["flat_pos"], dark=dark, method=ph.FBP,
                              out=out, work=work, use_graph=True, stream=stream)

    log(f"bench: warmup {args.warmup}")
    for _ in range(args.warmup):
        step()
    stream.synchronize()
    torch.cuda.synchronize()
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    t_start.record(stream)
    w0 = time.perf_counter()
    for i in range(args.steps):
        step()
    t_end.record(stream)
    stream.synchronize()
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms = t_start.elapsed_time(t_end) / args.steps
    log(f"bench: {args.steps} steps, {ms:.2f} ms/step (wall {wall / args.steps * 1e3:.2f} ms/step)")
    U = float(R) * N * N * K
    gups = U / (ms * 1e-3) / 1e9
    res = {"metric": METRIC, "value": round(gups, 2), "unit": "GUPS", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(ms, 3), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"batched FBP from raw uint16: {R} slices of {N}x{N}, {N} bins, {K} angles over "
                                  f"180 deg, 2 flats + dark, axis +3.5 bins, 20-ellipse phantoms, one HIP graph "
                                  f"per step (normalise+filter, backprojection)",
                      "slices": R, "n": N, "bins": N, "angles": K, "bp_tile": tile},
           "slices_per_s": round(R / (ms * 1e-3), 2)}
    if args.calib_copy:
        src = torch.empty(2 ** 29, device=dev, dtype=torch.float32).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        res["calib_copy_bytes"] = 2 * src.numel() * 4
        del src, dst
    if args.profile_only:
        print(json.dumps(res), flush=True)
        return

    # dominant kernel: the backprojector, timed alone in the same launch configuration
    filt = work[: plan.filt_elems * 4].view(torch.float32)
    nbp = max(3, args.steps)
    for _ in range(2):
        ph.backproject(plan, filt, 1, out=out, stream=stream)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record(stream)
    for _ in range(nbp):
        ph.backproject(plan, filt, 1, out=out, stream=stream)
    ev[1].record(stream)
    stream.synchronize()
    bp_ms = ev[0].elapsed_time(ev[1]) / nbp
    # the fused normalise + filter kernel
    ev2 = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    sino_f = torch.empty(plan.sino_shape(), device=dev, dtype=torch.float32)
    ph.normalize(plan, raw, flats, cfg["flat_pos"], dark, out=sino_f, stream=stream)
    ev2[0].record(stream)
    for _ in range(nbp):
        ph.fbp_filter(plan, sino_f, out=filt, stream=stream)
    ev2[1].record(stream)
    stream.synchronize()
    filt_ms = ev2[0].elapsed_time(ev2[1]) / nbp
    achieved = U * BP_OPS_PER_UPDATE / (bp_ms * 1e-3) / 1e12
    peak = VALU_LANE_OPS_PEAK / 1e12
    res["roofline"] = {"bound": "alu", "achieved": round(achieved, 3), "peak": round(peak, 3), "unit": "Tops/s",
                       "frac": round(achieved / peak, 4),
                       "traffic": traffic_for(os.path.join(ROOT, "paper_1306_1392_amd", "csrc", "k_bp.hip"),
                                              "hbm_bytes_per_launch"),
                       "kernel": "bp_kernel (backprojection)", "kernel_ms": round(bp_ms, 3),
                       "ops_per_update": BP_OPS_PER_UPDATE, "updates_per_launch": U,
                       "bp_gups": round(U / (bp_ms * 1e-3) / 1e9, 2)}
    res["filter_ms"] = round(filt_ms, 3)
    res["filter_hbm_gbs"] = round((plan.sino_elems * 4 + plan.filt_elems * 4) / (filt_ms * 1e-3) / 1e9, 1)
    if not args.no_cpu_baseline:
        log("bench: CPU oracle baseline on a bounded sample ...")
        res["cpu_baseline"] = cpu_baseline(R, N, K, cfg)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
