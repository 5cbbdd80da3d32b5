"""Benchmark: site-updates/s and HBM-roofline fraction of the fused (3+1)D
leap-frog step on a 512^3 lattice, FP32 (complex64) vs FP64 (complex128), at
the stated drift of the conserved functional E_r.

One timed step = one full time step of the scheme (both half-steps with the
mass and V(z) terms) over the whole lattice; every 10th step also evaluates the
conserved functional E_r of its result in FP64 (inside the same fused pass).
Inputs are synthetic and already resident in HBM when timing starts.  Prints
one JSON line.

Usage: python bench.py [--gpus 1] [--steps 1000] [--warmup 10] [--n 512]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
NORM_EVERY = 10


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=512, help="lattice edge (cells)")
    ap.add_argument("--fp64-steps", type=int, default=None, help="timed FP64 steps (default: --steps)")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--tile-y", type=int, default=0)
    ap.add_argument("--zchunk", type=int, default=0)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="first copy BYTES with a plain device copy (3 times): the reference dispatch "
                         "for scaling hardware byte counters")
    return ap.parse_args()


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("fused.hip", "stencil3.h", "device.h", "internal.h"):
        with open(os.path.join(ROOT, "paper_1309_3452_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def profiled_traffic(dtype_tag, n):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "fused3d_%s_%d_counters.md" % (dtype_tag, n))
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"kernel_source_sha:\s*([0-9a-f]+)", text)
    t = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not m or not t or m.group(1) != kernel_source_hash():
        return None
    return float(t.group(1))


def run_gpu(n, dtype, steps, warmup, tile_y, zchunk):
    import torch

    import paper_1309_3452_amd as P
    import workloads

    cfg = workloads.config_step3d(n, dtype=dtype, device="cuda")
    lat = P.Lattice3D(n, n, n, dtype=dtype, dt=cfg["dt"])
    lat.set_kernel("fused", tile_y, zchunk)
    lat.set_potential_z(cfg["m"], cfg["v_int"], cfg["v_half"])
    lat.load(cfg["state"])
    del cfg["state"]
    torch.cuda.synchronize()
    e_start = lat.norm()
    lat.step(warmup)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    norms = torch.zeros((steps // NORM_EVERY + 1, 2), dtype=torch.float64, device="cuda")
    w0 = torch.cuda.Event(enable_timing=True)
    w1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    w0.record(stream)
    for s in range(steps):
        ev[s][0].record(stream)
        if (s + 1) % NORM_EVERY == 0:
            lat.step_norm(1, norms[(s + 1) // NORM_EVERY])   # step + E_r of the new state in one pass
        else:
            lat.step(1)
        ev[s][1].record(stream)
    w1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kernel_ms = sum(a.elapsed_time(b) for a, b in ev) / steps
    region_ms = w0.elapsed_time(w1)
    e_end = lat.norm()
    nr = norms[1:].cpu().numpy()
    drift_series = float(abs(nr[:, 0] - e_start[0]).max() / abs(e_start[0])) if len(nr) else 0.0
    out = dict(wall_s=wall, region_ms=region_ms, kernel_ms=kernel_ms, e_start=e_start, e_end=e_end,
               drift=abs(e_end[0] - e_start[0]) / abs(e_start[0]), drift_max=drift_series,
               plain_norm_change=abs(e_end[2] - e_start[2]) / e_start[2], steps_total=steps + warmup)
    del lat
    torch.cuda.empty_cache()
    return out


def cpu_baseline():
    import numpy as np

    import oracle
    import workloads
    n, nsteps = 128, 300
    ol = oracle.Lattice3(n, n, n, workloads.DT3)
    vi, vh = workloads.step_potential(n, 1.5, n / 2.0, 4.0)
    th = ol.theta_vz(0.5, vi, vh)
    st = workloads.packet3d(n, n, n, (n / 2.0, n / 2.0, n / 4.0), 12.0, (0.0, 0.0, 0.56), 0.5, workloads.DT3)
    f = [np.ascontiguousarray(t.numpy()) for t in st]
    t0 = time.perf_counter()
    ol.step(f, th, nsteps)
    dt = time.perf_counter() - t0
    return {"value": n ** 3 * nsteps / dt, "unit": "site-updates/s", "cores": oracle.threads(), "kind": "oracle",
            "sample": "FP64 C oracle, same physics on a %d^3 lattice, %d steps (%.1f s); "
                      "site-updates/s is per cell-step, independent of lattice size" % (n, nsteps, dt)}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(z-slab sharding is described in DESIGN.md); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    n, K, W = args.n, args.steps, args.warmup
    cells = n ** 3
    if args.calibrate_copy:
        src = torch.ones(args.calibrate_copy // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        torch.cuda.empty_cache()
    r32 = run_gpu(n, torch.complex64, K, W, args.tile_y, args.zchunk)
    r64 = None
    if not args.no_fp64:
        r64 = run_gpu(n, torch.complex128, args.fp64_steps or K, W, 0, 0)
    value = cells * K / r32["wall_s"]
    alg_bytes = 128.0 * cells           # 16 amplitudes x 8 B per cell-step, FP32
    achieved = alg_bytes / (r32["kernel_ms"] * 1e-3) / 1e9
    traffic = profiled_traffic("fp32", n)
    line = {
        "metric": "site-updates/s & HBM-roofline %, FP32 vs FP64 3+1D 512^3 at stated norm error",
        "value": value,
        "unit": "site-updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": r32["wall_s"] * 1e3 / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "(3+1)D %d^3 periodic lattice, complex64 storage and FP32 arithmetic, m=0.5, "
                               "V(z)=1.5(1+tanh((z-%d)/4))/2, Gaussian packet sigma=12 k0=(0,0,0.56), "
                               "dt=0.9x stability bound, fused z-march kernel, FP64 E_r evaluated in-step every %d steps"
                               % (n, n // 2, NORM_EVERY),
                   "nx": n, "ny": n, "nz": n, "cells": cells},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic,
                     "kernel": "k3_fused<float> (one launch per step; every 10th launch also sums E_r)",
                     "alg_bytes_per_launch": alg_bytes,
                     "avg_launch_ms": r32["kernel_ms"]},
        "norm_error": {"E_r_rel_drift_fp32": r32["drift"], "E_r_rel_drift_fp32_max_every10": r32["drift_max"],
                       "steps_total": r32["steps_total"], "plain_norm_rel_change": r32["plain_norm_change"]},
        "amplitude_updates_per_s": 8 * value,
    }
    if r64 is not None:
        v64 = cells * (args.fp64_steps or K) / r64["wall_s"]
        a64 = 256.0 * cells / (r64["kernel_ms"] * 1e-3) / 1e9
        line["fp64"] = {"value": v64, "unit": "site-updates/s", "ms_per_step": r64["wall_s"] * 1e3 / (args.fp64_steps or K),
                        "roofline_frac": a64 / HBM_PEAK_GBS, "achieved_GBs": a64, "avg_launch_ms": r64["kernel_ms"],
                        "E_r_rel_drift": r64["drift"]}
        line["fp32_speedup_over_fp64"] = value / v64
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
