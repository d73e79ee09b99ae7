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
import ctypes
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
# The headline batch runs the two-slice backprojector: per pixel and projection one 16-byte LDS read of
# both slices' (q[j], q[j+1] - q[j]) pairs (8 B per update) and t = t0 + off, trunc, fract, LDS address
# shared by the two slices plus acc += q, acc = fma(f, dq, acc) per slice (4 lane-ops per update).
BP_OPS_PER_UPDATE = 4
BP_LDS_BYTES_PER_UPDATE = 8
# LDS read port for 16-byte reads: 256 B/clk/CU x 256 CU x 2.4 GHz (ds_read_b128 measures 136 TB/s on the
# chip, ds_read_b64 78 TB/s, i.e. 128 B/clk)
LDS_PEAK_GBS = 256 * 256 * 2.4


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
    """VALU FMA rate, the backprojector's op mix rate and LDS read bandwidth (ds_read_b64,
    ds_read_b128, ds_read_b128 with lanes 1.25 entries apart as in the projector, and
    ds_read_b128 with half of the lanes masked off; bytes count active lanes only)."""
    import torch
    import paper_1306_1392_amd as ph
    from paper_1306_1392_amd import _lib
    L = ph.lib()
    blocks, iters = 256 * 16, 4096
    sink = torch.zeros(blocks * 256, device=dev)
    st = torch.cuda.current_stream()
    out = {}
    for kind, name, per in ((0, "valu_fma_lane_ops_per_s", 8), (1, "bp_mix_lane_ops_per_s", 64),
                            (2, "lds_read_bytes_per_s", 64), (3, "lds_read128_bytes_per_s", 128),
                            (4, "lds_read128_spread_bytes_per_s", 128),
                            (5, "lds_read128_even_lanes_bytes_per_s", 64),
                            (6, "lds_read128_low_half_bytes_per_s", 64)):
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


def run_uneven(args):
    """Uneven batch: 500 slices of 512^2 / 1024^2 / 2048^2, 90..3600 projections, half of them
    360 degree half-acquisition scans, per-projection axis shifts; one plan, autotuned
    backprojector, the whole FBP of the batch replayed as one HIP graph, then the U-Net corrector
    on the sparse-angle 512^2 slices (at most 180 projections) inside the same timed step."""
    import numpy as np
    import torch
    import synth
    import paper_1306_1392_amd as ph
    dev = torch.device("cuda:0")
    n = args.uneven_slices
    log(f"bench(uneven): generating {n} slices ...")
    d = synth.configs.cfg_uneven(n_slices=n, device=dev)
    geos = [ph.Geometry(s["N"], s["N"], s["nb"], s["angles"], s["axis"], s["shifts"], s["scan"])
            for s in d["specs"]]
    plan = ph.Plan(geos, slice_geom=np.arange(n))
    sino = torch.cat([x.reshape(-1) for x in d["sinos"]]).contiguous()
    del d["sinos"]
    U = float(sum(s["N"] ** 2 * s["K"] for s in d["specs"]))
    img = torch.empty(plan.img_elems, device=dev)
    filt = torch.empty(plan.filt_elems, device=dev)
    ph.fbp_filter(plan, sino, out=filt)
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    t_default = None
    plan.set_tiles(-1, False)
    e = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    e[0].record(stream)
    ph.backproject(plan, filt, 1, out=img, stream=stream)
    e[1].record(stream)
    stream.synchronize()
    t_default = e[0].elapsed_time(e[1])
    best_ms = plan.autotune(filt, img, reps=2, stream=stream)
    tile, pers = plan.get_tiles()
    work = torch.empty(ph.work_bytes(plan, sino=sino, method=ph.FBP), device=dev, dtype=torch.uint8)
    # the sparse-angle 512^2 slices (K <= 180) also go through the U-Net corrector, read in place from the
    # packed FBP output (random-init weights of the corrector's architecture: throughput only)
    from paper_1306_1392_amd.cnn import UNet, init_params
    sub = [i for i, s in enumerate(d["specs"]) if s["N"] == 512 and s["K"] <= 180]
    net = cnn_out = None
    if sub:
        net = UNet(1, 512, 512)
        net.set_params(init_params(32, 4, seed=0))
        cnn_out = torch.empty(len(sub), 512, 512, device=dev)
        sub_ptrs = [ctypes.c_void_p(img.data_ptr() + 4 * plan.slice_info(i).img_offset) for i in sub]
    sptr = ctypes.c_void_p(stream.cuda_stream)

    def corrector():
        for k, ptr in enumerate(sub_ptrs):
            rc = net.L.pyhst_unet_forward(net.handle, ptr, 1, ctypes.c_void_p(cnn_out[k].data_ptr()), sptr)
            if rc != 0:
                raise RuntimeError(f"pyhst_unet_forward failed: {rc}")

    def step():
        ph.reconstruct_slices(plan, sino=sino, method=ph.FBP, out=img, work=work, use_graph=True, stream=stream)
        if sub:
            corrector()

    for _ in range(args.warmup):
        step()
    stream.synchronize()
    e[0].record(stream)
    for _ in range(args.steps):
        step()
    e[1].record(stream)
    stream.synchronize()
    ms = e[0].elapsed_time(e[1]) / args.steps
    cnn_ms = _timed(stream, corrector, 3) if sub else 0.0
    classes = {}
    for s in d["specs"]:
        key = f"{s['N']}{'_half' if s['scan'] == 2 else ''}"
        c = classes.setdefault(key, {"slices": 0, "updates": 0.0})
        c["slices"] += 1
        c["updates"] += s["N"] ** 2 * s["K"]
    res = {"metric": "uneven-batch FBP aggregate GUPS", "value": round(U / (ms * 1e-3) / 1e9, 2), "unit": "GUPS",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3),
           "higher_is_better": True, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"{n} slices, N in {{512,1024,2048}}, K in 90..3600, half of them 360-degree "
                                  f"half acquisition, axis shifts N(0,0.5^2); one plan, one HIP graph per step; "
                                  f"U-Net on the 512^2 slices with K <= 180",
                      "updates": U, "classes": classes},
           "slices_per_s": round(n / (ms * 1e-3), 2),
           "autotune": {"tile": tile, "persistent": pers, "bp_ms_tuned": round(best_ms, 3),
                        "bp_ms_default": round(t_default, 3)},
           "corrector": {"slices": len(sub), "ms_per_step": round(cnn_ms, 3),
                         "rule": "512^2 slices with at most 180 projections: FBP + U-Net"}}
    print(json.dumps(res), flush=True)


def run_single(args):
    """Single-slice FBP: 256^2 image, 256 bins, 180 projections over 180 degrees, 10-ellipse
    phantoms with 1 % Gaussian noise.  Latency of one slice (one graph replay per call) and
    throughput of a 1024-slice batch (64 distinct phantoms, each repeated 16 times)."""
    import numpy as np
    import torch
    import synth
    import oracle
    import paper_1306_1392_amd as ph
    dev = torch.device("cuda:0")
    N, K, R, distinct = 256, 180, 1024, 64
    ds = [synth.cfg_single_slice(index=i, device=dev) for i in range(distinct)]
    sino1 = ds[0]["sino"][None].contiguous()
    sinoB = torch.stack([ds[i % distinct]["sino"] for i in range(R)]).contiguous()
    g = ph.Geometry(N, N, N, ds[0]["angles"], ds[0]["axis"])
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    e = [torch.cuda.Event(enable_timing=True) for _ in range(2)]

    def timed(plan, sino, reps, graph=True):
        out = torch.empty(plan.img_shape(), device=dev)
        work = torch.empty(ph.work_bytes(plan, sino=sino, method=ph.FBP), device=dev, dtype=torch.uint8)
        for _ in range(3):
            ph.reconstruct_slices(plan, sino=sino, method=ph.FBP, out=out, work=work, use_graph=graph, stream=stream)
        stream.synchronize()
        t0 = time.perf_counter()
        e[0].record(stream)
        for _ in range(reps):
            ph.reconstruct_slices(plan, sino=sino, method=ph.FBP, out=out, work=work, use_graph=graph, stream=stream)
        e[1].record(stream)
        stream.synchronize()
        wall = (time.perf_counter() - t0) * 1e3 / reps
        return e[0].elapsed_time(e[1]) / reps, wall, out

    def timed_c(plan, sino, reps):
        # the same call made straight through the C ABI with a prepared argument block (no Python wrapper)
        from paper_1306_1392_amd import _lib
        L = _lib.lib()
        out = torch.empty(plan.img_shape(), device=dev)
        work = torch.empty(ph.work_bytes(plan, sino=sino, method=ph.FBP), device=dev, dtype=torch.uint8)
        a = _lib.ReconArgs()
        a.sino = ctypes.c_void_p(sino.data_ptr())
        a.method, a.use_graph, a.eps, a.n_inner = ph.FBP, 1, 1e-6, 20
        a.out = ctypes.c_void_p(out.data_ptr())
        a.work = ctypes.c_void_p(work.data_ptr())
        a.work_bytes = work.numel()
        sp, pa = ctypes.c_void_p(stream.cuda_stream), ctypes.byref(a)
        for _ in range(3):
            assert L.reconstruct_slices(plan.handle, pa, sp) == 0
        stream.synchronize()
        e[0].record(stream)
        for _ in range(reps):
            L.reconstruct_slices(plan.handle, pa, sp)
        e[1].record(stream)
        stream.synchronize()
        return e[0].elapsed_time(e[1]) / reps

    p1 = ph.Plan(g)
    lat_ms, lat_wall, out1 = timed(p1, sino1, 200)
    lat_nograph_ms = timed(p1, sino1, 200, graph=False)[0]
    lat_c_ms = timed_c(p1, sino1, 200)
    pB = ph.Plan(g, n_slices=R)
    pB.autotune(ph.fbp_filter(pB, sinoB), torch.empty(pB.img_shape(), device=dev), reps=2, stream=stream)
    bat_ms, _, outB = timed(pB, sinoB, max(args.steps, 5))
    ref = oracle.fbp(ds[0]["sino"].double().cpu().numpy(), oracle.Geom(N, N, N, ds[0]["angles"], ds[0]["axis"]))
    par = float(np.linalg.norm(out1[0].cpu().numpy() - ref) / np.linalg.norm(ref))
    rmse = float(torch.sqrt(((outB[0].double() - ds[0]["truth"]) ** 2).mean()))
    U = float(N * N * K)
    res = {"metric": "single-slice FBP latency and batch throughput", "value": round(R / (bat_ms * 1e-3), 1),
           "unit": "slices/s", "higher_is_better": True, "n_gpus": 1, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "256x256, 256 bins, 180 angles over 180 deg, 10-ellipse phantoms, 1 % noise; "
                                  "batch of 1024 slices, one HIP graph per call"},
           "latency_ms_one_slice": round(lat_ms, 4), "latency_wall_ms_one_slice": round(lat_wall, 4),
           "latency_ms_one_slice_direct_launches": round(lat_nograph_ms, 4),
           "latency_ms_one_slice_c_call": round(lat_c_ms, 4),
           "batch_ms": round(bat_ms, 3), "gups_batch": round(R * U / (bat_ms * 1e-3) / 1e9, 1),
           "bp_tile": pB.get_tiles()[0], "parity_rel_l2_vs_oracle": par, "rmse_vs_phantom": rmse}
    if not args.no_cpu_baseline:
        og = oracle.Geom(N, N, N, ds[0]["angles"], ds[0]["axis"])
        sc = np.stack([ds[i]["sino"].double().cpu().numpy() for i in range(16)])
        t0 = time.time()
        oracle.fbp(sc, og)
        dt = time.time() - t0
        res["cpu_baseline"] = {"value": round(16 / dt, 2), "unit": "slices/s", "cores": oracle.num_threads(),
                               "kind": "oracle", "sample": f"FBP of 16 slices (direct Ram-Lak convolution, "
                                                           f"backprojection), {dt:.2f} s"}
    print(json.dumps(res), flush=True)


def _timed(stream, fn, reps):
    import torch
    e = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    fn()
    stream.synchronize()
    e[0].record(stream)
    for _ in range(reps):
        fn()
    e[1].record(stream)
    stream.synchronize()
    return e[0].elapsed_time(e[1]) / reps


def run_preproc(args):
    """Preprocessing of section 2.3 inside the batched FBP workload (64 x 2048^2, 1800 angles, raw uint16):
    time per step of the plain fused path, with the hot-spot filter, with the ring filter, and with the
    ring filter plus thresholded-object subtraction (one HIP graph per step each)."""
    import torch
    import synth
    import paper_1306_1392_amd as ph
    dev = torch.device("cuda:0")
    R, N, K = args.slices, args.n, args.angles
    cfg = quick_data(R, N, K, dev) if args.quick_data else synth.cfg_batched_raw(R=R, N=N, K=K, device=dev)
    plan = ph.Plan(ph.Geometry(N, N, N, cfg["angles"], cfg["axis"]), n_slices=R)
    out = torch.empty(plan.img_shape(), device=dev, dtype=torch.float32)
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    variants = {"plain": {}, "hot_spot": {"hot_threshold": 0.05}, "ring": {"ring_width": 8},
                "ring_object": {"ring_width": 8, "ring_object_threshold": 0.02},
                "hot_spot_ring_object": {"hot_threshold": 0.05, "ring_width": 8, "ring_object_threshold": 0.02}}
    res_ms = {}
    for name, kw in variants.items():
        work = torch.empty(ph.work_bytes(plan, raw=cfg["raw"], method=ph.FBP, **kw), device=dev, dtype=torch.uint8)

        def step():
            ph.reconstruct_slices(plan, raw=cfg["raw"], flats=cfg["flats"], flat_pos=cfg["flat_pos"], dark=cfg["dark"],
                                  method=ph.FBP, out=out, work=work, use_graph=True, stream=stream, **kw)

        res_ms[name] = round(_timed(stream, step, max(3, args.steps)), 3)
        del work
        log(f"preproc: {name} {res_ms[name]} ms")
    U = float(R) * N * N * K
    res = {"metric": "FBP step time with the preprocessing of section 2.3", "value": res_ms["hot_spot_ring_object"],
           "unit": "ms", "higher_is_better": False, "n_gpus": 1, "dtype": "f32",
           "data": "synthetic" + (" (random counts)" if args.quick_data else ""),
           "config": {"workload": f"{R} slices of {N}x{N}, {K} angles, raw uint16; hot-spot threshold 0.05, ring "
                                  f"half-width 8, object threshold 0.02"},
           "ms_per_step": res_ms, "gups": {k: round(U / (v * 1e-3) / 1e9, 1) for k, v in res_ms.items()}}
    print(json.dumps(res), flush=True)


def run_fp(args):
    """Matched forward projector alone, next to the backprojector in the same launch configuration:
    1024^2 x 128 angles (the TV workload) and 64 x 2048^2 x 1800 angles (the FBP batch).  Unit:
    voxel-angle pairs per second (the same count as the backprojector's updates)."""
    import torch
    import synth
    import paper_1306_1392_amd as ph
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    cases = {}
    kinds = {"blocks": ph.FP_BLOCKS, "staged": ph.FP_STAGED, "lines": ph.FP_LINES}
    shapes = {"tv1024": (1, 1024, 128), "mid1024": (8, 1024, 720), "fbp2048": (args.slices, 2048, 1800)}
    for name, (R, N, K) in shapes.items():
        plan = ph.Plan(ph.Geometry(N, N, N, synth.uniform_angles(K), (N - 1) / 2 + 3.5), n_slices=R)
        g = torch.Generator(device=dev)
        g.manual_seed(7)
        img = torch.rand(plan.img_shape(), device=dev, generator=g)
        sino = torch.empty(plan.sino_shape(), device=dev)
        reps = 20 if R == 1 else 3
        U = float(R) * N * N * K
        # every kernel forced in turn (the line-split one only where it finishes quickly), then automatic
        per_kind = {}
        for kn, kv in kinds.items():
            if kn == "lines" and U > 2e10:
                continue
            plan.set_fp_kernel(kv)
            per_kind[kn] = round(_timed(stream, lambda: ph.forward_project(plan, img, out=sino, stream=stream), reps), 3)
        plan.set_fp_kernel(ph.FP_AUTO)
        fp_ms = _timed(stream, lambda: ph.forward_project(plan, img, out=sino, stream=stream), reps)
        bp_ms = _timed(stream, lambda: ph.backproject(plan, sino, 0, out=img, stream=stream), reps)
        cases[name] = {"slices": R, "n": N, "angles": K, "fp_ms": round(fp_ms, 3), "bp_ms": round(bp_ms, 3),
                       "fp_gups": round(U / (fp_ms * 1e-3) / 1e9, 1), "bp_gups": round(U / (bp_ms * 1e-3) / 1e9, 1),
                       "fp_ms_by_kernel": per_kind}
        if R == 1:
            # the backprojector as the solvers use it: accumulating (beta = 1), alternating with the projector,
            # and for every tile shape
            cases[name]["bp_ms_beta1"] = round(_timed(stream, lambda: ph.backproject(
                plan, sino, 0, out=img, alpha=-1e-6, beta=1.0, stream=stream), reps), 3)

            def pair():
                ph.forward_project(plan, img, out=sino, stream=stream)
                ph.backproject(plan, sino, 0, out=img, alpha=1e-6, beta=0.0, stream=stream)
            cases[name]["fp_then_bp_ms"] = round(_timed(stream, pair, reps), 3)
            by_tile = {}
            for t in range(6):
                for pers in (False, True):
                    plan.set_tiles(t, pers)
                    by_tile[f"{t}{'p' if pers else ''}"] = round(_timed(stream, lambda: ph.backproject(
                        plan, sino, 0, out=img, stream=stream), reps), 3)
            plan.set_tiles(-1, False)
            cases[name]["bp_ms_by_tile"] = by_tile
        log(f"fp: {name} {cases[name]}")
        del img, sino, plan
    res = {"metric": "forward projector GUPS (voxel-angle pairs/s)", "value": cases["fbp2048"]["fp_gups"],
           "unit": "GUPS", "higher_is_better": True, "n_gpus": 1, "dtype": "f32", "data": "synthetic (uniform random image)",
           "config": {"workload": "A = s^2 B^T alone: 1024^2 x 128 angles, 8 x 1024^2 x 720 angles and 64 x 2048^2 x 1800 angles"},
           "cases": cases}
    print(json.dumps(res), flush=True)


def run_bpcache(args):
    """Backprojector of one 1024^2 slice x 128 projections (the solvers' launch) timed right after
    different predecessor kernels: what its time depends on (the L2 contents it inherits)."""
    import numpy as np
    import torch
    import synth
    import paper_1306_1392_amd as ph
    dev = torch.device("cuda:0")
    N, K = 1024, 128
    plan = ph.Plan(ph.Geometry(N, N, N, synth.uniform_angles(K), (N - 1) / 2 + 3.5))
    small = ph.Plan(ph.Geometry(256, 256, 256, synth.uniform_angles(K), 127.5 + 3.5))
    small.set_tiles(plan.get_tiles()[0], False)
    g = torch.Generator(device=dev)
    g.manual_seed(3)
    img, img2, img3 = [torch.rand(plan.img_shape(), device=dev, generator=g) for _ in range(3)]
    sino, sino2 = [torch.rand(plan.sino_shape(), device=dev, generator=g) for _ in range(2)]
    simg = torch.rand(small.img_shape(), device=dev, generator=g)
    ssino = torch.rand(small.sino_shape(), device=dev, generator=g)
    big = torch.rand(16 << 20, device=dev, generator=g)
    big2 = torch.empty_like(big)
    st = torch.cuda.current_stream()

    def bp():
        ph.backproject(plan, sino, 0, out=img, alpha=1e-6)

    def fp_then_small_bp():
        ph.forward_project(plan, img3, out=sino2)
        ph.backproject(small, ssino, 0, out=simg, alpha=1e-6)

    variants = {
        "after_backprojection": lambda: ph.backproject(plan, sino2, 0, out=img3, alpha=1e-6),
        "after_projector": lambda: ph.forward_project(plan, img3, out=sino2),
        "after_projector_reading_the_output_image": lambda: ph.forward_project(plan, img, out=sino2),
        "after_64MB_copy": lambda: big2.copy_(big),
        "after_projector_on_256sq_image": lambda: ph.forward_project(small, simg, out=ssino),
        "after_projector_then_small_backprojection": fp_then_small_bp,
        "after_sum_of_the_output_image": lambda: img.sum(),
        "after_copy_of_the_output_image": lambda: img2.copy_(img),
    }
    res = {}
    for name, pre in variants.items():
        for _ in range(3):
            pre()
            bp()
        torch.cuda.synchronize()
        ts = []
        for _ in range(30):
            pre()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(st)
            bp()
            e1.record(st)
            ts.append((e0, e1))
        torch.cuda.synchronize()
        res[name] = round(1e3 * float(np.median([a.elapsed_time(b) for a, b in ts])), 1)
        log(f"bpcache: {name} {res[name]} us")
    out = {"metric": "backprojector time after a predecessor kernel (median of 30)", "value": res["after_projector"],
           "unit": "us", "higher_is_better": False, "n_gpus": 1, "dtype": "f32", "data": "synthetic (uniform random)",
           "config": {"workload": "backprojection of one 1024x1024 slice, 1024 bins, 128 projections (32x32 tiles)"},
           "us_by_predecessor": res}
    print(json.dumps(out), flush=True)


def run_beta(args):
    """Choice of beta (section 3.1) on the TV workload (1024^2, 128 angles, Poisson 1e4): FISTA (300
    iterations, 10 inner prox steps) at 8 beta values, cross-validation over 3 excluded projections
    (24 more reconstructions) and the decoherence estimator; whole sweep timed."""
    import numpy as np
    import torch
    import synth
    import paper_1306_1392_amd as ph
    from paper_1306_1392_amd.beta import select_beta
    dev = torch.device("cuda:0")
    d = synth.cfg_tv_sparse(N=1024, K=128, device=dev)
    g = ph.Geometry(1024, 1024, 1024, d["angles"], d["axis"])
    y = d["y"][None].contiguous()
    betas = np.geomspace(0.01, 3.0, 8)
    select_beta(g, y, betas[:1], n_iter=5)        # warm-up (plans, graphs of the kernels)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = select_beta(g, y, betas, n_iter=300, n_inner=10)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    truth = d["truth"].to(dev).float() if torch.is_tensor(d.get("truth")) else None
    res = {"metric": "beta sweep time (cross-validation + decoherence)", "value": round(dt, 3), "unit": "s",
           "higher_is_better": False, "n_gpus": 1, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "1024x1024, 1024 bins, 128 angles, Poisson 1e4; FISTA 300 iterations, 10 inner; "
                                  "8 betas x (1 + 3 excluded projections) reconstructions"},
           "reconstructions": int(len(betas) * 4 + 1), "betas": [float(b) for b in betas],
           "cv": [float(v) for v in r["cv"][:, 0]], "e_cohe": [float(v) for v in r["e_cohe"][:, 0]],
           "beta_cv": float(betas[int(np.argmin(r["cv"][:, 0]))]),
           "beta_ecohe": float(betas[int(np.argmin(np.abs(r["e_cohe"][:, 0])))])}
    if truth is not None:
        rm = torch.sqrt(((r["x"][:, 0] - truth) ** 2).mean(dim=(1, 2))).cpu().numpy()
        res["rmse_vs_truth"] = [float(v) for v in rm]
        res["beta_truth"] = float(betas[int(np.argmin(rm))])
    print(json.dumps(res), flush=True)


def run_patch(args):
    """Overlapping-patch dictionary prior (section 3.2) at the paper's experiment size: 2048^2 slice,
    150 projections, 8x8 patches every 4 pixels, 128 atoms (64 DCT + 64 random), FISTA 150 iterations
    (its Lipschitz estimate included).  The oracle beside it: one iteration of the NumPy oracle on a
    128^2 / 24-angle problem, scaled by the number of coefficients."""
    import numpy as np
    import torch
    import synth
    import paper_1306_1392_amd as ph
    from synth import dct_dictionary
    dev = torch.device("cuda:0")
    N, K, m, st, n_it = 2048, 150, 8, 4, 150
    ang = synth.uniform_angles(K)
    ell = synth.random_ellipses(synth.rng_for(12, 0, 0), 20)
    y = synth.ellipse_sinogram(ell, ang, N, (N - 1) / 2, N, device=dev)
    y = (y + 0.02 * float(y.max()) * torch.randn(y.shape, device=dev, dtype=y.dtype,
                                                  generator=torch.Generator(device=dev).manual_seed(3))).float()
    yt = y[None].contiguous()
    plan = ph.Plan(ph.Geometry(N, N, N, ang, (N - 1) / 2))
    D = torch.from_numpy(dct_dictionary(m, extra=64, seed=3).astype(np.float32)).to(dev)
    ph.patch_fista(plan, yt, D, m, st, 5.0, 8.0, 2)              # warm-up + Lipschitz estimate
    Lf = plan.last_lipschitz
    torch.cuda.synchronize()
    e = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    e[0].record()
    x, W = ph.patch_fista(plan, yt, D, m, st, 5.0, 8.0, n_it, lipschitz=Lf)
    e[1].record()
    torch.cuda.synchronize()
    ms = e[0].elapsed_time(e[1])
    n_coef = W.numel()
    res = {"metric": "patch-prior FISTA time per iteration", "value": round(ms / n_it, 3), "unit": "ms",
           "higher_is_better": False, "n_gpus": 1, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"{N}x{N}, {K} angles, 20-ellipse phantom, 2 % noise; {m}x{m} patches every {st} px, "
                                  f"128 atoms, rho 5, beta 8, {n_it} FISTA iterations"},
           "coefficients": n_coef, "patches": int(W.shape[1]), "total_s": round(ms / 1e3, 3), "lipschitz": Lf,
           "nonzero_fraction": float((W != 0).float().mean())}
    if not args.no_cpu_baseline:
        import oracle
        from oracle.patches import PatchGrid, PatchProblem, fista
        n2, k2 = 128, 24
        og = oracle.Geom(n2, n2, n2, synth.uniform_angles(k2), (n2 - 1) / 2)
        ys = synth.ellipse_sinogram(ell, og.angles, n2, og.axis, n2).numpy()
        prob = PatchProblem(PatchGrid(n2, n2, m, st), dct_dictionary(m, extra=64, seed=3), ys, rho=5.0, beta=8.0,
                            project=lambda v: oracle.forward_project(v, og), backproject=lambda r: oracle.backproject(r, og))
        t0 = time.time()
        fista(prob, 3, 1e4)
        dt = (time.time() - t0) / 3
        scale = n_coef / (prob.g.n_p * 128)
        res["cpu_baseline"] = {"value": round(dt * scale * 1e3, 1), "unit": "ms", "cores": oracle.num_threads(),
                               "kind": "oracle",
                               "sample": f"3 iterations of the NumPy oracle at {n2}^2 / {k2} angles ({dt:.3f} s each), "
                                         f"scaled by the coefficient count ({scale:.0f}x)"}
    print(json.dumps(res), flush=True)


def run_tv(args):
    """TV-regularised sparse-angle reconstruction: 1024^2, 128 projections, Poisson data at 1e4
    photons, 300 Chambolle-Pock iterations (lambda 0.01) replayed as one HIP graph."""
    import torch
    import synth
    import paper_1306_1392_amd as ph
    dev = torch.device("cuda:0")
    d = synth.cfg_tv_sparse(N=1024, K=128, device=dev)
    g = ph.Geometry(1024, 1024, 1024, d["angles"], d["axis"])
    plan = ph.Plan(g)
    y = d["y"][None].contiguous()
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    work = torch.empty(ph.work_bytes(plan, sino=y, method=ph.TV_CP, n_iter=300), device=dev, dtype=torch.uint8)
    out = torch.empty(plan.img_shape(), device=dev)
    # operator norm once per geometry (GPU power iteration inside the library, synchronous)
    ph.reconstruct_slices(plan, sino=y, method=ph.TV_CP, lam=0.01, n_iter=1, op_norm=0.0, out=out, work=work,
                          stream=stream)
    stream.synchronize()
    Lk = plan.last_op_norm

    def run():
        ph.reconstruct_slices(plan, sino=y, method=ph.TV_CP, lam=0.01, n_iter=300, op_norm=Lk, out=out, work=work,
                              use_graph=True, stream=stream)

    run()
    stream.synchronize()
    e = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    reps = max(1, args.steps // 5)
    e[0].record(stream)
    for _ in range(reps):
        run()
    e[1].record(stream)
    stream.synchronize()
    ms = e[0].elapsed_time(e[1]) / reps
    U = 2.0 * 1024 * 1024 * 128 * 300

    # the paper's own solvers on the same data: 300 ISTA / FISTA iterations, 10 inner prox steps each
    fi = {}
    for name, meth in (("ista", ph.ISTA), ("fista", ph.FISTA)):
        wk = torch.empty(ph.work_bytes(plan, sino=y, method=meth, n_iter=300), device=dev, dtype=torch.uint8)
        ph.reconstruct_slices(plan, sino=y, method=meth, lam=0.01, n_iter=1, op_norm=0.0, n_inner=10, out=out,
                              work=wk, stream=stream)
        La = plan.last_op_norm

        def run_fi():
            ph.reconstruct_slices(plan, sino=y, method=meth, lam=0.01, n_iter=300, op_norm=La, n_inner=10,
                                  out=out, work=wk, use_graph=True, stream=stream)

        run_fi()
        stream.synchronize()
        e[0].record(stream)
        for _ in range(reps):
            run_fi()
        e[1].record(stream)
        stream.synchronize()
        fi[name] = {"s_300_iterations": round(e[0].elapsed_time(e[1]) / reps / 1e3, 4), "op_norm_A": La,
                    "n_inner": 10}

    res = {"metric": "TV-CP reconstruction time (300 iterations)", "value": round(ms / 1e3, 4), "unit": "s",
           "higher_is_better": False, "n_gpus": 1, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "1024x1024, 1024 bins, 128 angles, Poisson 1e4 photons, 300 Chambolle-Pock "
                                  "iterations, lambda 0.01, one HIP graph", "op_norm": Lk},
           "gups_in_projectors": round(U / (ms * 1e-3) / 1e9, 2), "slices_per_s": round(1e3 / ms, 3),
           "paper_solvers": fi}
    if not args.no_cpu_baseline:
        import oracle
        og = oracle.Geom(1024, 1024, 1024, d["angles"], d["axis"])
        yc = d["y"].double().cpu().numpy()
        t0 = time.time()
        oracle.cp_tv(yc, og, 0.01, 3, Lk)
        dt = time.time() - t0
        res["cpu_baseline"] = {"value": round(dt * 100, 1), "unit": "s", "cores": oracle.num_threads(),
                               "kind": "oracle",
                               "sample": f"3 of the 300 Chambolle-Pock iterations (FP64 scatter projector, "
                                         f"pixel-driven backprojector), {dt:.1f} s, scaled by 100"}
    print(json.dumps(res), flush=True)


PROFILE_CMDS = {
    "trace": "rocprofv3 --kernel-trace --stats --output-format csv -d <dir>/prof_trace -o bench -- "
             "python -u bench.py --steps 5 --warmup 2 --no-cpu-baseline --quick-data --profile-only",
    "pmc": "rocprofv3 --pmc <COUNTER> --output-format csv -d <dir>/pmc_<name> -o pmc -- "
           "python -u bench.py --steps 1 --warmup 1 --no-cpu-baseline --quick-data --profile-only --calib-copy "
           "(one pass per counter: FETCH_SIZE, then WRITE_SIZE; then one pass of SQ_INSTS_VALU SQ_INSTS_LDS "
           "SQ_LDS_BANK_CONFLICT SQ_ACTIVE_INST_LDS SQ_WAVES without --calib-copy, into <dir>/pmc_sq)",
}


def summarize_profiles(d):
    """Turn rocprofv3 CSV output under d into the text summaries and the traffic record in profiles/."""
    import csv
    import collections
    out_dir = os.path.join(ROOT, "profiles")
    os.makedirs(out_dir, exist_ok=True)

    def short(name):
        for key in ("bp2_kernel", "bp_kernel", "filter", "normalize_kernel", "copyBuffer", "fp_kernel"):
            if key in name:
                return name.replace("pyhst::(anonymous namespace)::", "").split("(")[0].replace("void ", "")
        return None

    lines = []
    ks = os.path.join(d, "prof_trace", "bench_kernel_stats.csv")
    if os.path.exists(ks):
        lines.append("# kernel time summary: " + PROFILE_CMDS["trace"].replace("<dir>", d))
        lines.append(f"{'kernel':40s} {'calls':>6s} {'avg_ms':>10s} {'min_ms':>10s} {'max_ms':>10s} {'pct':>6s}")
        for r in csv.DictReader(open(ks)):
            n = short(r["Name"])
            if n:
                lines.append(f"{n:40s} {int(r['Calls']):6d} {float(r['AverageNs']) / 1e6:10.3f} "
                             f"{float(r['MinNs']) / 1e6:10.3f} {float(r['MaxNs']) / 1e6:10.3f} "
                             f"{float(r['Percentage']):6.2f}")
    counters = collections.defaultdict(list)
    for sub in sorted(os.listdir(d)):
        f = os.path.join(d, sub, "pmc_counter_collection.csv")
        if sub.startswith("pmc_") and os.path.exists(f):
            for r in csv.DictReader(open(f)):
                n = short(r["Kernel_Name"])
                if n:
                    counters[(n, r["Counter_Name"])].append(float(r["Counter_Value"]))
    if counters:
        lines.append("")
        lines.append("# counters per dispatch (mean over dispatches): " + PROFILE_CMDS["pmc"].replace("<dir>", d))
        for (n, c), v in sorted(counters.items()):
            lines.append(f"{n:40s} {c:24s} {sum(v) / len(v):14.6g}  (n={len(v)})")
    txt = os.path.join(out_dir, "bp_fbp2048_rocprof.txt")
    open(txt, "w").write("\n".join(lines) + "\n")
    log(f"wrote {txt}")
    # traffic: FETCH_SIZE / WRITE_SIZE (KiB) scaled by the same counters on a 2 GiB device copy
    cp = [k for k in counters if "copyBuffer" in k[0]]
    bp = [k for k in counters if "bp2_kernel" in k[0]] or [k for k in counters if "bp_kernel" in k[0]]
    if cp and bp:
        copy_bytes = 2 * 2 ** 29 * 4
        cf = sum(counters[(cp[0][0], "FETCH_SIZE")]) / len(counters[(cp[0][0], "FETCH_SIZE")]) * 1024
        cw = sum(counters[(cp[0][0], "WRITE_SIZE")]) / len(counters[(cp[0][0], "WRITE_SIZE")]) * 1024
        f_scale, w_scale = (copy_bytes / 2) / cf, (copy_bytes / 2) / cw
        bname = bp[0][0]
        bf = sum(counters[(bname, "FETCH_SIZE")]) / len(counters[(bname, "FETCH_SIZE")]) * 1024
        bw = sum(counters[(bname, "WRITE_SIZE")]) / len(counters[(bname, "WRITE_SIZE")]) * 1024
        rec = {"kernel": bname, "source_sha256_16": source_hash(os.path.join(ROOT, "paper_1306_1392_amd", "csrc",
                                                                             "k_bp.hip")),
               "fetch_scale": f_scale, "write_scale": w_scale,
               "fetch_bytes_per_launch": bf * f_scale, "write_bytes_per_launch": bw * w_scale,
               "hbm_bytes_per_launch": bf * f_scale + bw * w_scale,
               "calibration": "a device copy of 2 GiB reads 2 GiB and writes 2 GiB; scale = true bytes / counter bytes",
               "command": PROFILE_CMDS["pmc"].replace("<dir>", d)}
        jf = os.path.join(out_dir, "bp_fbp2048_traffic.json")
        json.dump(rec, open(jf, "w"), indent=1)
        log(f"wrote {jf}: {rec['hbm_bytes_per_launch'] / 1e9:.2f} GB per launch")


def run_cnn(args):
    """U-Net corrector throughput at the learned workload's shape: 512^2 slices, batch 32,
    4 levels, 32 base channels (BF16 MFMA, FP32 accumulate).  Times one training step
    (forward + MSE + backward + Adam) and inference."""
    import torch
    from paper_1306_1392_amd.cnn import UNet, init_params
    dev = torch.device("cuda:0")
    B, H = 32, 512
    net = UNet(B, H, H, 32, 4)
    net.set_params(init_params(32, 4, 0))
    g = torch.Generator(device=dev)
    g.manual_seed(1)
    x = torch.rand((B, H, H), device=dev, generator=g)
    t = torch.rand((B, H, H), device=dev, generator=g)
    out = torch.empty_like(x)
    st = torch.cuda.current_stream()
    for _ in range(2):
        net.train_step(x, t, 1e-4)
        net.forward(x, out=out)
    torch.cuda.synchronize()
    e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    reps = max(2, args.steps // 2)
    e[0].record(st)
    for _ in range(reps):
        net.train_step(x, t, 1e-4)
    e[1].record(st)
    for _ in range(reps):
        net.forward(x, out=out)
    e[2].record(st)
    torch.cuda.synchronize()
    train_ms = e[0].elapsed_time(e[1]) / reps
    infer_ms = e[1].elapsed_time(e[2]) / reps
    fwd_flop = 73.4e9 * B   # 3x3 convs + transposed convs of the 4-level, 32-base U-Net at 512^2
    res = {"metric": "U-Net corrector throughput", "value": round(B / (infer_ms * 1e-3), 1), "unit": "slices/s",
           "higher_is_better": True, "n_gpus": 1, "dtype": "bf16 (fp32 accumulate)", "data": "synthetic",
           "config": {"workload": "U-Net 4 levels, 32 base channels, batch 32 of 512x512"},
           "train_step_ms": round(train_ms, 3), "infer_ms": round(infer_ms, 3),
           "infer_tflops": round(fwd_flop / (infer_ms * 1e-3) / 1e12, 1),
           "train_tflops": round(3 * fwd_flop / (train_ms * 1e-3) / 1e12, 1),
           "mfma_bf16_peak_tflops": 2500.0}
    if not args.no_cpu_baseline:
        from oracle import num_threads
        from oracle.cnn import UNetOracle
        xc = x[:1].double().cpu().numpy()
        p64 = net.get_params().double().cpu().numpy()
        t0 = time.time()
        UNetOracle(32, 4, "fp64").forward(p64, xc)
        dt = time.time() - t0
        res["cpu_baseline"] = {"value": round(1.0 / dt, 4), "unit": "slices/s", "cores": num_threads(),
                               "kind": "oracle",
                               "sample": f"FP64 NumPy forward pass of 1 slice of 512x512, {dt:.1f} s"}
    print(json.dumps(res), flush=True)


def learned_data(indices, stream, plan_hi, plan_b, N, K, B, dev):
    """(FBP input, truth) for the given phantom indices, in batches of B (data from synth)."""
    import torch
    import synth
    import paper_1306_1392_amd as ph

    def project(tex):
        return ph.forward_project(plan_hi, tex)

    xs, ts, ys = [], [], []
    for i0 in range(0, len(indices), B):
        idx = list(indices[i0:i0 + B])
        y, tr, _, _ = synth.configs.cfg_learned(idx, stream, project, N=N, K=K, device=dev)
        n = y.shape[0]
        if n < B:   # pad the last batch for the fixed-size plan
            y = torch.cat([y, y[:1].expand(B - n, -1, -1)])
        fb = ph.reconstruct_slices(plan_b, sino=y.contiguous(), method=ph.FBP)[:n]
        xs.append(fb.clone())
        ts.append(tr)
        ys.append(y[:n])
    return torch.cat(xs), torch.cat(ts), torch.cat(ys)


def learned_experiment(N, K, B, n_train, epochs, n_test, n_val, dev, save_params=None):
    """Learned sparse-angle corrector: U-Net (4 levels, 32 base) trained on ellipse + Perlin
    phantoms (N^2, K projections, Poisson 1e4) by the library's own MFMA kernels, then applied as
    the product ships it (Corrector: FBP, U-Net, data-consistency check against a threshold
    calibrated on validation phantoms, TV for the slices that fail it), against TV (the better of
    Chambolle-Pock with the balanced gradient block and FISTA, 300 iterations, lambda calibrated on
    the validation phantoms) on test phantoms."""
    import numpy as np
    import torch
    import paper_1306_1392_amd as ph
    from paper_1306_1392_amd.cnn import UNet, init_params
    from paper_1306_1392_amd import corrector as cr
    SCALE = 10.0
    ang = np.arange(K) * (np.pi / K)
    axis = (N - 1) / 2.0
    geo = ph.Geometry(N, N, N, ang, axis)
    plan_b = ph.Plan(geo, n_slices=B)
    plan_hi = ph.Plan(ph.Geometry(2 * N, 2 * N, N, ang, axis, pixel_size=0.5))
    t0 = time.perf_counter()
    log(f"learned: generating {n_train} training phantoms ({N}^2, {K} angles) ...")
    xtr, ttr, _ = learned_data(np.arange(n_train), 0, plan_hi, plan_b, N, K, B, dev)
    xva, tva, yva = learned_data(np.arange(n_val), 2, plan_hi, plan_b, N, K, B, dev)
    xte, tte, yte = learned_data(np.arange(n_test), 1, plan_hi, plan_b, N, K, B, dev)
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t0
    log(f"learned: data in {t_gen:.1f} s")
    net = UNet(B, N, N, 32, 4)
    net.set_params(init_params(32, 4, 0))
    net.set_scale(SCALE)
    steps = epochs * (xtr.shape[0] // B)
    t1 = time.perf_counter()
    losses = cr.train(net, xtr, ttr, steps, lr=1e-3, log=log)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    del xtr, ttr

    # TV reference (section 3.1: lambda by ground-truth calibration on validation phantoms)
    t2 = time.perf_counter()
    plan_te = ph.Plan(geo, n_slices=yte.shape[0])
    tvres = {}
    for name, meth in (("fista", ph.FISTA), ("cp", ph.TV_CP)):
        lam, cal, norm, mu = cr.calibrate_tv_lambda(geo, yva, tva, method=meth)
        x_tv = ph.reconstruct_slices(plan_te, sino=yte.contiguous(), method=meth, lam=lam, n_iter=300, op_norm=norm,
                                     n_inner=10, tv_mu=mu)
        tvres[name] = {"method": meth, "lambda": lam, "op_norm": norm, "tv_mu": mu, "val_rmse": cal[lam],
                       "test_rmse": cr.rmse(x_tv, tte), "calibration": {str(k): v for k, v in sorted(cal.items())}}
        log(f"learned: TV {name}: lambda {lam}, validation RMSE {cal[lam]:.4g}")
    t_cal = time.perf_counter() - t2
    ref = min(tvres, key=lambda k: tvres[k]["val_rmse"])
    J = tvres[ref]

    # the corrector as shipped: FBP + U-Net, data-consistency check, TV for the slices that fail it
    corr = cr.Corrector.from_net(geo, net, tv_lambda=J["lambda"], tv_iters=300, tv_method=J["method"],
                                 op_norm=J["op_norm"], tv_mu=J["tv_mu"])
    tau = corr.calibrate(yva)
    x_c, fell = corr.reconstruct_all(yte)
    r_fbp, r_cnn, r_tv = cr.rmse(xte, tte), cr.rmse(x_c, tte), J["test_rmse"]
    # throughput: the corrector over the test set in batches of B vs the TV reference on the whole test set
    stream = torch.cuda.current_stream()
    ycs = [yte[i:i + B].contiguous() for i in range(0, yte.shape[0], B)]
    e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    torch.cuda.synchronize()
    e[0].record(stream)
    for yb in ycs:
        corr.reconstruct(yb)
    e[1].record(stream)
    ph.reconstruct_slices(plan_te, sino=yte.contiguous(), method=J["method"], lam=J["lambda"], n_iter=300,
                          op_norm=J["op_norm"], n_inner=10, tv_mu=J["tv_mu"])
    e[2].record(stream)
    torch.cuda.synchronize()
    sps_cnn = yte.shape[0] / (e[0].elapsed_time(e[1]) * 1e-3)
    sps_tv = yte.shape[0] / (e[1].elapsed_time(e[2]) * 1e-3)
    for v in tvres.values():
        del v["method"]
    if save_params:
        cr.save_weights(save_params, net.get_params(), SCALE, 32, 4)
    return {"rmse_ratio": round(r_cnn / r_tv, 4),
            "workload": f"ellipse+Perlin phantoms {N}^2, {K} angles, Poisson 1e4; train {n_train} x {epochs} "
                        f"epochs, batch {B}; validation {n_val}; test {n_test}; corrector: FBP + U-Net (4 levels, "
                        f"32 base, BF16) with the data-consistency check and TV fallback; TV reference: better "
                        f"of Chambolle-Pock and FISTA on validation, 300 iterations, calibrated lambda",
            "rmse": {"fbp": r_fbp, "corrector": r_cnn, "tv": r_tv}, "tv_reference": ref, "tv_solvers": tvres,
            "slices_per_s": {"corrector": round(sps_cnn, 1), "tv": round(sps_tv, 2),
                             "ratio": round(sps_cnn / sps_tv, 1)},
            "fallback_slices": int(fell.sum()), "dc_threshold": tau,
            "pass": {"rmse_within_5pct_of_tv": r_cnn <= 1.05 * r_tv, "speed_20x": sps_cnn >= 20 * sps_tv,
                     "gain_over_fbp": r_cnn < r_fbp},
            "seconds": {"data": round(t_gen, 1), "train": round(t_train, 1), "tv_calibration": round(t_cal, 1)},
            "train_steps": steps, "loss_trace": losses[::max(1, len(losses) // 20)]}


def run_learned(args):
    import torch
    L = learned_experiment(args.learned_n, 90, 32, args.learned_train, args.learned_epochs, args.learned_test,
                           args.learned_val, torch.device("cuda:0"), save_params=args.save_params)
    res = {"metric": f"learned vs TV RMSE (sparse-angle {args.learned_n}^2, 90 angles)", "value": L["rmse_ratio"],
           "unit": "RMSE_corrector / RMSE_TV", "higher_is_better": False, "n_gpus": 1, "dtype": "bf16 CNN, f32 TV",
           "data": "synthetic", "config": {"workload": L.pop("workload")}}
    res.update(L)
    print(json.dumps(res), flush=True)


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
    ap.add_argument("--workload", default="fbp2048", choices=["fbp2048", "single", "uneven", "tv", "cnn", "learned", "preproc", "beta", "patch", "fp",
                             "bpcache"],
                    help="fbp2048: the headline batch; uneven / tv: the other measured workloads")
    ap.add_argument("--uneven-slices", type=int, default=500)
    ap.add_argument("--learned-train", type=int, default=10000)
    ap.add_argument("--learned-test", type=int, default=256)
    ap.add_argument("--learned-epochs", type=int, default=6)
    ap.add_argument("--learned-n", type=int, default=512)
    ap.add_argument("--learned-val", type=int, default=32)
    ap.add_argument("--no-learned", action="store_true", help="leave the learned-corrector record out of the line")
    ap.add_argument("--line-learned-train", type=int, default=10000)
    ap.add_argument("--line-learned-epochs", type=int, default=6)
    ap.add_argument("--save-params", default=None)
    ap.add_argument("--summarize", metavar="DIR", help="write profiles/ summaries from rocprofv3 output in DIR")
    args = ap.parse_args()
    if args.summarize:
        return summarize_profiles(args.summarize)
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: measures one GPU only; the slices of a batch are independent, so N GPUs would "
              "each reconstruct 1/N of them with no exchange (no multi-GPU run is made here)", file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    import paper_1306_1392_amd as ph

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.workload == "single":
        return run_single(args)
    if args.workload == "preproc":
        return run_preproc(args)
    if args.workload == "beta":
        return run_beta(args)
    if args.workload == "fp":
        return run_fp(args)
    if args.workload == "bpcache":
        return run_bpcache(args)
    if args.workload == "patch":
        return run_patch(args)
    if args.workload == "uneven":
        return run_uneven(args)
    if args.workload == "tv":
        return run_tv(args)
    if args.workload == "cnn":
        return run_cnn(args)
    if args.workload == "learned":
        return run_learned(args)
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
    # roofline: the two-slice backprojector reads 8 LDS bytes per update (one 16-byte read per pixel,
    # projection and slice pair) against the 16-byte read port (256 B/clk/CU); the VALU mix
    # (4 lane-ops/update) is the other bound
    lds_achieved = BP_LDS_BYTES_PER_UPDATE * U / (bp_ms * 1e-3) / 1e9
    valu_achieved = U * BP_OPS_PER_UPDATE / (bp_ms * 1e-3) / 1e12
    res["roofline"] = {"bound": "lds", "achieved": round(lds_achieved, 1), "peak": round(LDS_PEAK_GBS, 1),
                       "unit": "GB/s", "frac": round(lds_achieved / LDS_PEAK_GBS, 4),
                       "traffic": traffic_for(os.path.join(ROOT, "paper_1306_1392_amd", "csrc", "k_bp.hip"),
                                              "hbm_bytes_per_launch"),
                       "algorithmic_hbm_bytes": (plan.filt_elems + plan.img_elems) * 4,
                       "kernel": "bp2_kernel (backprojection, two slices per workgroup)", "kernel_ms": round(bp_ms, 3),
                       "lds_bytes_per_update": BP_LDS_BYTES_PER_UPDATE, "updates_per_launch": U,
                       "bp_gups": round(U / (bp_ms * 1e-3) / 1e9, 2),
                       "valu": {"achieved_tops": round(valu_achieved, 2), "ops_per_update": BP_OPS_PER_UPDATE,
                                "peak_tops": round(VALU_LANE_OPS_PEAK / 1e12, 2),
                                "frac": round(valu_achieved / (VALU_LANE_OPS_PEAK / 1e12), 4)}}
    res["filter_ms"] = round(filt_ms, 3)
    res["filter_hbm_gbs"] = round((plan.sino_elems * 4 + plan.filt_elems * 4) / (filt_ms * 1e-3) / 1e9, 1)
    if args.peaks:
        res["measured_peaks"] = {k: float(f"{v:.4g}") for k, v in measure_peaks(dev).items()}
    if not args.no_cpu_baseline:
        log("bench: CPU oracle baseline on a bounded sample ...")
        res["cpu_baseline"] = cpu_baseline(R, N, K, cfg)
    if not args.no_learned:
        # second half of the metric, outside the timed region: the learned corrector against TV on the
        # sparse-angle workload, with a bounded training set
        del raw, flats, dark, out, work, filt, cfg
        torch.cuda.empty_cache()
        log(f"bench: learned corrector vs TV ({args.line_learned_train} training phantoms) ...")
        t0 = time.perf_counter()
        res["learned"] = learned_experiment(512, 90, 32, args.line_learned_train, args.line_learned_epochs,
                                            256, 32, dev)
        res["learned"]["seconds"]["total"] = round(time.perf_counter() - t0, 1)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
