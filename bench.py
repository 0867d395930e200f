"""Benchmark of the neural visibility query path on one MI355X.

Workload (the single-object frame): 1920 x 1080 = 2,073,600 shadow rays from a
4 x 4 ground quad to a 0.5 x 0.5 area light, one object (a 1M-triangle displaced
sphere; only its AABB is used by the query), grids of 8 levels 16..512 with 2
binary16 latents per vertex (2.1 GB), MLP 48 -> 4 x 64 ReLU -> 1, Xavier weights,
latents U(-1e-4, 1e-4).  Inputs are synthetic and seeded, resident in HBM
before timing.  A step is one nif_query over all 2,073,600 (ray, object)
queries: AABB clip, normalisation, multi-resolution encoding, MLP, sigmoid,
write-back.

Prints ONE JSON line (see the keys below).  --gpus N > 1 is refused: this path
runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HEADLINE_DTYPE = "bf16"
PEAK_TFLOPS = {"bf16": 2500.0, "f16": 2500.0, "fp8": 5000.0, "f32": 157.3}
HBM_PEAK_GBS = 8000.0
GRID_SEED = 2024


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def time_launches(fn, steps: int, warmup: int):
    """Average seconds per call, HIP events on the stream the kernels use."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(steps):
        fn()
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3 / steps


def measured_traffic():
    """HBM bytes per launch of the fused kernel from the committed counter run,
    or None when the kernel source has changed since those counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "query_frame_bf16_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    src = b"".join(open(os.path.join(ROOT, "paper_2306_07191_amd", "csrc", f), "rb").read()
                   for f in ("nif_forward.hip", "nif_device.h"))
    if hashlib.sha256(src).hexdigest() != rec["source_sha256"]:
        return None
    return rec["traffic_bytes_per_launch"]


def cpu_baseline(w, gpu_y, budget_s: float = 12.0):
    """The binary64 oracle on the host cores over a bounded sample of the same
    queries; also the error of the GPU outputs on that sample."""
    from oracle import oracle as O
    model = O.Model(w["shape"], w["aabb"], w["mlps"], grid_seed=GRID_SEED, grid_amp=1e-4)
    cores = len(os.sched_getaffinity(0))
    n_all = w["ids"].shape[0]
    pilot = min(20000, n_all)
    t0 = time.perf_counter()
    model.forward(w["rays"][:pilot], w["ids"][:pilot], w["tmax"][:pilot], nthreads=cores)
    rate = pilot / (time.perf_counter() - t0)
    n = int(min(n_all, max(pilot, rate * budget_s)))
    sel = np.linspace(0, n_all - 1, n).astype(np.int64)
    t0 = time.perf_counter()
    ref = model.forward(w["rays"][sel], w["ids"][sel], w["tmax"][sel], nthreads=cores)
    dt = time.perf_counter() - t0
    errs = {}
    for dt_name, y in gpu_y.items():
        e = np.abs(y[sel].astype(np.float64) - ref["y"])
        errs[dt_name] = {"max_abs": float(e.max()), "max_rel": float((e / ref["y"]).max())}
    return ({"value": n / dt, "unit": "queries/s", "cores": cores, "kind": "oracle",
             "sample": f"{n} of {n_all} frame queries (evenly strided), binary64 encode+MLP, {cores} threads"},
            errs)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run three 1 GiB device copies (scales FETCH_SIZE / WRITE_SIZE counters)")
    ap.add_argument("--quick", action="store_true",
                    help="time the headline step only (no per-dtype sweep, no CPU baseline): for profilers")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this path runs on one GPU; --gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2306_07191_amd import nif, synth as S

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.copy_calibration:
        a = torch.ones(256 * 1024 * 1024, dtype=torch.float32, device="cuda")
        c = torch.empty_like(a)
        for _ in range(3):
            c.copy_(a)
        torch.cuda.synchronize()
        log("copied 1 GiB three times")
        return
    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    w = S.frame_workload(with_mesh=False)
    sh = w["shape"]
    n = w["ids"].shape[0]
    log(f"workload ready in {time.perf_counter() - t0:.1f}s: {n} queries")
    ctx = nif.Context(sh)
    ctx.set_mlp(0, torch.from_numpy(w["mlps"][0]).cuda())
    grid = ctx.alloc_grid()
    ctx.set_object(0, w["aabb"][0], grid, 0)
    ctx.init_grid(0, GRID_SEED, 1e-4)
    rays = torch.from_numpy(w["rays"]).cuda()
    ids = torch.from_numpy(w["ids"]).cuda()
    tmax = torch.from_numpy(w["tmax"]).cuda()
    y = torch.empty(n, dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()

    flops = 2 * (sh.din * sh.width + (sh.hidden - 1) * sh.width * sh.width + sh.width)  # 30,848 per query
    ws = torch.empty(max(1, ctx.workspace_bytes(n)), dtype=torch.uint8, device="cuda")
    per_dtype = {}
    gpu_y = {}
    for order in (() if args.quick else (0, 2)):
        ctx.set_option(nif.NIF_OPT_ORDER, order)
        for dtype in ("f32", "f16", "bf16"):
            ctx.prepare(dtype)
            sec = time_launches(lambda: ctx.query(rays, ids, tmax, dtype=dtype, out=y, ws=ws), max(5, args.steps // 5), 2)
            key = dtype if order else dtype + "_unordered"
            per_dtype[key] = {"queries_per_s": n / sec, "us_per_call": sec * 1e6}
            if order:
                gpu_y[dtype] = y.cpu().numpy().copy()
            log(f"{key}: {sec * 1e6:.1f} us/call, {n / sec / 1e9:.3f} G queries/s")

    # the contract timing for the headline dtype: a step is the ordering pass plus
    # the fused query kernel; events around the kernel give its own duration
    ctx.prepare(HEADLINE_DTYPE)
    perm = torch.empty(n, dtype=torch.int32, device="cuda")
    ows = torch.empty(max(1, nif.lib().nif_order_workspace_bytes(ctx.h, n)), dtype=torch.uint8, device="cuda")

    def step():
        ctx.order(rays, ids, tmax, perm=perm, ws=ows)
        ctx.query_ordered(rays, ids, tmax, perm, dtype=HEADLINE_DTYPE, out=y)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * args.steps + 1)]
    w0 = time.perf_counter()
    ev[0].record(s)
    for k in range(args.steps):
        ctx.order(rays, ids, tmax, perm=perm, ws=ows)
        ev[2 * k + 1].record(s)
        ctx.query_ordered(rays, ids, tmax, perm, dtype=HEADLINE_DTYPE, out=y)
        ev[2 * k + 2].record(s)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    sec = ev[0].elapsed_time(ev[-1]) / 1e3 / args.steps
    kern = sum(ev[2 * k + 1].elapsed_time(ev[2 * k + 2]) for k in range(args.steps)) / 1e3 / args.steps
    value = n / sec
    achieved_tflops = flops * n / kern / 1e12
    roofline = {"bound": "mfma", "achieved": achieved_tflops, "peak": PEAK_TFLOPS[HEADLINE_DTYPE],
                "unit": "TFLOP/s", "frac": achieved_tflops / PEAK_TFLOPS[HEADLINE_DTYPE], "traffic": measured_traffic(),
                "kernel": "nif_query_kernel<bf16, L=8, f16 grid> (fused clip+encode+MLP)",
                "algorithmic_flop_per_launch": flops * n, "kernel_us": kern * 1e6,
                "step_us": sec * 1e6, "order_us": (sec - kern) * 1e6}
    log(f"step {sec * 1e6:.1f} us (order {(sec - kern) * 1e6:.1f} us, fused kernel {kern * 1e6:.1f} us)")

    cpu = None
    errs = None
    if not (args.no_cpu or args.quick):
        cpu, errs = cpu_baseline(w, gpu_y)
        log(f"cpu oracle: {cpu['value']:.0f} queries/s on {cpu['cores']} cores")

    out = {
        "metric": "shadow-ray visibility queries/sec at stated error vs FP64 oracle",
        "value": value,
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": HEADLINE_DTYPE,
        "data": "synthetic (seeded frame scene: 2,073,600 ground-to-area-light shadow rays; init-distribution latents and Xavier weights)",
        "config": {"workload": "frame: 1920x1080 shadow rays, 1 object, 8 levels 16..512, 2 binary16 latents, MLP 48-64x4-1",
                   "queries": n, "levels": sh.levels, "res_min": sh.res_min, "res_max": sh.res_max,
                   "hidden": sh.hidden, "width": sh.width, "grid_dtype": sh.grid_dtype},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "per_dtype": per_dtype,
        "error_vs_oracle_on_cpu_sample": errs,
        "wall_s_timed_region": wall,
    }
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
