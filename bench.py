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
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "backprojection GUPS (voxel·angle/s) + slices/s at 2048²; learned vs TV RMSE"
# MI355X FP32 vector peak 157.3 TFLOP/s = 256 CU x 2.4 GHz x 128 FMA lanes/clk x 2 flops:
# one VALU lane-op per FMA slot gives 78.6 T lane-ops/s.
VALU_LANE_OPS_PEAK = 157.3e12 / 2
BP_OPS_PER_UPDATE = 6   # t = t0 + off, trunc, fract, LDS address, acc += q, acc = fma(f, dq, acc)


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
    """FP64 oracle on a bounded sample: the whole FBP of one of the R slices
    (normalise, direct Ram-Lak filter, backprojection of all N^2 pixels), x R."""
    import numpy as np
    import oracle
    oracle.build()
    r = 0
    raw = cfg["raw"][:, r:r + 1, :].cpu().numpy().astype(np.float64)
    flats = cfg["flats"][:, r:r + 1, :].cpu().numpy()
    dark = cfg["dark"][r:r + 1].cpu().numpy()
    g = oracle.Geom(N, N, N, cfg["angles"], cfg["axis"])
    t0 = time.perf_counter()
    oracle.fbp_raw(raw, flats, cfg["flat_pos"], dark, g)
    t1 = time.perf_counter()
    return {"value": round(R * N * N * K / ((t1 - t0) * R) / 1e9, 4), "unit": "GUPS", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"FBP of 1 of the {R} slices from raw (normalise, direct Ram-Lak filter of {K} rows, "
                      f"backprojection of all {N}x{N} pixels), {t1 - t0:.1f} s, scaled by {R} slices"}


def quick_data(R, N, K, dev):
    """Cheap stand-in input for profiler runs (traffic and timing do not depend on the values)."""
    import numpy as np
    import torch
    g = torch.Generator(device=dev)
    g.manual_seed(5)
    raw = torch.randint(2000, 30000, (K, R, N), device=dev, generator=g, dtype=torch.int32).to(torch.uint16)
    flats = torch.full((2, R, N), 35000.0, device=dev)
    dark = torch.full((R, N), 100.0, device=dev)
    return dict(raw=raw, flats=flats, dark=dark, flat_pos=np.array([0.0, K - 1.0]),
                angles=np.arange(K) * (np.pi / K), axis=(N - 1) / 2 + 3.5)


def measure_peaks(dev):
    """VALU FMA rate, the backprojector's op mix rate and LDS ds_read_b64 bandwidth."""
    import torch
    import paper_1306_1392_amd as ph
    from paper_1306_1392_amd import _lib
    L = ph.lib()
    blocks, iters = 256 * 16, 4096
    sink = torch.zeros(blocks * 256, device=dev)
    st = torch.cuda.current_stream()
    out = {}
    for kind, name, per in ((0, "valu_fma_lane_ops_per_s", 8), (1, "bp_mix_lane_ops_per_s", 64),
                            (2, "lds_read_bytes_per_s", 64)):
        _lib.check(L.pyhst_microbench(kind, blocks, iters, ctypes_ptr(sink), ctypes_stream(st)), "microbench")
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        _lib.check(L.pyhst_microbench(kind, blocks, iters, ctypes_ptr(sink), ctypes_stream(st)), "microbench")
        e1.record()
        torch.cuda.synchronize()
        s = e0.elapsed_time(e1) * 1e-3
        out[name] = blocks * 256.0 * iters * per / s
    return out


def ctypes_ptr(t):
    import ctypes
    return ctypes.c_void_p(t.data_ptr())


def ctypes_stream(s):
    import ctypes
    return ctypes.c_void_p(s.cuda_stream)


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
    ap.add_argument("--quick-data", action="store_true", help="random raw counts instead of phantoms (profiling)")
    ap.add_argument("--profile-only", action="store_true", help="warmup + steps only, no extra measurements")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a plain 2 GiB device copy (reference kernel for HBM byte counters)")
    ap.add_argument("--tile-sweep", action="store_true", help="time the backprojector for every tile shape")
    ap.add_argument("--peaks", action="store_true", help="run the roofline microbenchmarks")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build measures one GPU only (the slices of a batch are independent; "
              "DESIGN.md describes how the path shards across GPUs)", file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    import paper_1306_1392_amd as ph

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    R, N, K = args.slices, args.n, args.angles
    log(f"bench: generating {R} x {N}^2 slices, {K} angles, raw uint16 ...")
    cfg = quick_data(R, N, K, dev) if args.quick_data else synth.cfg_batched_raw(R=R, N=N, K=K, device=dev)
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
    if args.quick_data:
        res["data"] = "synthetic (random counts, profiling run)"
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

    def time_bp():
        for _ in range(2):
            ph.backproject(plan, filt, 1, out=out, stream=stream)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record(stream)
        for _ in range(nbp):
            ph.backproject(plan, filt, 1, out=out, stream=stream)
        ev[1].record(stream)
        stream.synchronize()
        return ev[0].elapsed_time(ev[1]) / nbp

    bp_ms = time_bp()
    if args.tile_sweep:
        sweep = {}
        for t in range(5):
            plan.set_tiles(t, False)
            sweep[t] = round(time_bp(), 3)
            log(f"bench: tile {t}: {sweep[t]} ms")
        plan.set_tiles(args.tile, False)
        res["bp_tile_sweep_ms"] = sweep
    # the normalise + filter kernel on its own
    ev2 = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    sino_f = torch.empty(plan.sino_shape(), device=dev, dtype=torch.float32)
    ph.normalize(plan, raw, flats, cfg["flat_pos"], dark, out=sino_f, stream=stream)
    ev2[0].record(stream)
    for _ in range(nbp):
        ph.fbp_filter(plan, sino_f, out=filt, stream=stream)
    ev2[1].record(stream)
    stream.synchronize()
    filt_ms = ev2[0].elapsed_time(ev2[1]) / nbp
    del sino_f
    achieved = U * BP_OPS_PER_UPDATE / (bp_ms * 1e-3) / 1e12
    peak = VALU_LANE_OPS_PEAK / 1e12
    res["roofline"] = {"bound": "alu", "achieved": round(achieved, 3), "peak": round(peak, 3), "unit": "Tops/s",
                       "frac": round(achieved / peak, 4),
                       "traffic": traffic_for(os.path.join(ROOT, "paper_1306_1392_amd", "csrc", "k_bp.hip"),
                                              "hbm_bytes_per_launch"),
                       "kernel": "bp_kernel (backprojection)", "kernel_ms": round(bp_ms, 3),
                       "ops_per_update": BP_OPS_PER_UPDATE, "updates_per_launch": U,
                       "bp_gups": round(U / (bp_ms * 1e-3) / 1e9, 2),
                       "lds_tbytes_per_s": round(8.0 * U / (bp_ms * 1e-3) / 1e12, 2)}
    res["filter_ms"] = round(filt_ms, 3)
    res["filter_hbm_gbs"] = round((plan.sino_elems * 4 + plan.filt_elems * 4) / (filt_ms * 1e-3) / 1e9, 1)
    if args.peaks:
        res["measured_peaks"] = {k: float(f"{v:.4g}") for k, v in measure_peaks(dev).items()}
    if not args.no_cpu_baseline:
        log("bench: CPU oracle baseline on a bounded sample ...")
        res["cpu_baseline"] = cpu_baseline(R, N, K, cfg)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
