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
# 256 CUs x 4 SIMDs x 16 lanes x 2 FLOP per FMA x 2.4 GHz (packed FP32, which would double it, is not used)
FP32_NONPACKED_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
# per amplitude update: S (3 complex differences, 3 real scalings, 2 complex sums) 16 FLOP + the update
# (two complex products and a difference) 16 FLOP; a cell holds 8 amplitudes, each updated once per step
ALU_FLOP_PER_CELL_STEP = 8 * 32
NORM_EVERY = 10
ACCURACY_STEPS = 1000          # the norm-drift and phase-error horizon, independent of --steps


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=512, help="lattice edge (cells)")
    ap.add_argument("--fp64-steps", type=int, default=None, help="timed FP64 steps (default: --steps)")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--precision", default="both", choices=["both", "f64"],
                    help="f64: time the complex128 step alone (for profiler runs of that kernel)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true",
                    help="skip the untimed 1000-step accuracy passes (for profiler runs of the timed kernels)")
    ap.add_argument("--tile-y", type=int, default=0)
    ap.add_argument("--zchunk", type=int, default=0)
    ap.add_argument("--kernel", default="auto", choices=["auto", "fused", "fused2"],
                    help="auto = fused2 (two steps per launch) where it applies")
    ap.add_argument("--workload", default="step3d",
                    choices=["step3d", "batched2d", "adjoint3d", "plane2d", "links3d", "links2d", "klein2d",
                             "slab3d", "site3d", "reverse3d", "norm3d"],
                    help="step3d (default): the 512^3 FP32-vs-FP64 headline; the others print their own line")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="first copy BYTES with a plain device copy (3 times): the reference dispatch "
                         "for scaling hardware byte counters")
    return ap.parse_args()


def kernel_source_hash(steps_per_launch=1):
    """Hash of the kernel sources' code (comments and blank space removed), so
    that a profile stays attached to the code it measured."""
    h = hashlib.sha256()
    for f in ("fused2.hip" if steps_per_launch == 2 else "fused.hip", "stencil3.h", "device.h", "internal.h"):
        with open(os.path.join(ROOT, "paper_1309_3452_amd", "csrc", f)) as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        h.update("\n".join(line.strip() for line in text.split("\n") if line.strip()).encode())
    return h.hexdigest()[:16]


def profiled_traffic(dtype_tag, n, steps_per_launch=1):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source; else None."""
    name = "fused3d_%s_%d_counters.md" if steps_per_launch == 1 else "fused3dx2_%s_%d_counters.md"
    path = os.path.join(ROOT, "profiles", name % (dtype_tag, n))
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"kernel_source_sha:\s*([0-9a-f]+)", text)
    t = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not m or not t or m.group(1) != kernel_source_hash(steps_per_launch):
        return None
    return float(t.group(1))


def profiled_valu_busy(n, steps_per_launch):
    """Vector-ALU busy fraction of the FP32 march kernel from the committed SQ
    counter summary, if it was taken on the current kernel source; else None."""
    if steps_per_launch != 2:
        return None
    path = os.path.join(ROOT, "profiles", "fused3dx2_fp32_%d_sq.md" % n)
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"kernel_source_sha:\s*([0-9a-f]+)", text)
    v = re.search(r"valu_busy:\s*([0-9.eE+-]+)", text)
    if not m or not v or m.group(1) != kernel_source_hash(2):
        return None
    return float(v.group(1))


def run_gpu(n, dtype, steps, warmup, tile_y, zchunk, kernel, keep=False):
    import torch

    import paper_1309_3452_amd as P
    import workloads

    cfg = workloads.config_step3d(n, dtype=dtype, device="cuda")
    lat = P.Lattice3D(n, n, n, dtype=dtype, dt=cfg["dt"])
    lat.set_kernel(kernel, tile_y, zchunk)
    lat.set_potential_z(cfg["m"], cfg["v_int"], cfg["v_half"])
    lat.load(cfg["state"])
    del cfg["state"]
    torch.cuda.synchronize()
    e_start = lat.norm()
    lat.step(warmup)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    # one launch advances G steps (two-step kernel: 2); every NORM_EVERY steps the
    # launch that ends there also sums E_r of its result
    G = 2 if kernel in ("fused2", "auto") else 1
    groups = []
    s = 0
    while s < steps:
        g = min(G, steps - s)
        groups.append((g, (s + g) % NORM_EVERY == 0))
        s += g
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in groups]
    norms = torch.zeros((steps // NORM_EVERY + 1, 2), dtype=torch.float64, device="cuda")
    w0 = torch.cuda.Event(enable_timing=True)
    w1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    w0.record(stream)
    done = 0
    for q, (g, with_norm) in enumerate(groups):
        ev[q][0].record(stream)
        if with_norm:
            lat.step_norm(g, norms[(done + g) // NORM_EVERY])   # steps + E_r of the new state in the same pass
        else:
            lat.step(g)
        ev[q][1].record(stream)
        done += g
    w1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    full = [q for q, (g, _) in enumerate(groups) if g == G]
    launch_ms = sum(ev[q][0].elapsed_time(ev[q][1]) for q in full) / max(1, len(full))
    region_ms = w0.elapsed_time(w1)
    e_end = lat.norm()
    nr = norms[1:].cpu().numpy()
    drift_series = float(abs(nr[:, 0] - e_start[0]).max() / abs(e_start[0])) if len(nr) else 0.0
    out = dict(wall_s=wall, region_ms=region_ms, launch_ms=launch_ms, steps_per_launch=G, launches=len(groups),
               e_start=e_start, e_end=e_end,
               drift=abs(e_end[0] - e_start[0]) / abs(e_start[0]), drift_max=drift_series,
               plain_norm_change=abs(e_end[2] - e_start[2]) / e_start[2], steps_total=steps + warmup)
    if keep:
        out["lat"] = lat          # reused by the accuracy pass
    else:
        del lat
        torch.cuda.empty_cache()
    return out


def accuracy_pass(lat, n, dtype, steps=ACCURACY_STEPS):
    """The headline packet from its initial state for `steps` steps in the
    timed launch sequence (two-step launches, E_r in-step every NORM_EVERY
    steps): the relative drift of E_r at the end and its largest excursion."""
    import torch

    import workloads
    cfg = workloads.config_step3d(n, dtype=dtype, device="cuda")
    lat.load(cfg["state"])
    del cfg
    e0 = lat.norm()
    G = 2
    norms = torch.zeros((steps // NORM_EVERY + 1, 2), dtype=torch.float64, device="cuda")
    done = 0
    while done < steps:
        g = min(G, steps - done)
        if (done + g) % NORM_EVERY == 0:
            lat.step_norm(g, norms[(done + g) // NORM_EVERY])
        else:
            lat.step(g)
        done += g
    e1 = lat.norm()
    nr = norms[1:].cpu().numpy()
    return {"E_r_rel_drift": abs(e1[0] - e0[0]) / abs(e0[0]),
            "E_r_rel_drift_max_every10": float(abs(nr[:, 0] - e0[0]).max() / abs(e0[0])),
            "plain_norm_rel_change": abs(e1[2] - e0[2]) / e0[2]}


def plane_wave_z(nx, ny, nz, kz, m, dt, dtype, t_shift=0.0):
    """Eigen plane wave psi^(1) of Sect. 2.1 travelling along z (k = (0, 0, kz)):
    every amplitude is its spinor component times exp(i (kz z_s - w t)) at its own
    site and time sheet, with w from Eq. (pwdsip); built in FP64 on the device."""
    import torch
    Pz = 2.0 * math.sin(kz / 2.0)
    X = math.sqrt((m * m + Pz * Pz) / (m * m + (2.0 / dt) ** 2))
    w = 2.0 / dt * math.asin(X)
    E, mk = 2.0 / dt * X, m * math.sqrt(1.0 - X * X)
    spinor = [1.0, 0.0, Pz / (E + mk), 0.0]                 # A, B, C, D of psi^(1) with Px = Py = 0
    zoff = [0.0, 0.0, 0.5, 0.5, 0.5, 0.5, 0.0, 0.0]           # z offsets of A0 A1 B0 B1 C0 C1 D0 D1
    z = torch.arange(nz, dtype=torch.float64, device="cuda")
    out = []
    for a in range(8):
        t = (-0.5 * dt if a < 4 else 0.0) + t_shift
        col = spinor[a // 2] * torch.exp(1j * (kz * (z + zoff[a]) - w * t))
        out.append(col.view(nz, 1, 1).expand(nz, ny, nx).to(dtype).contiguous())
    return out, w


def plane_wave_phase_error(dtype, nz=512, nxy=128, kz_index=46, m=0.5, steps=ACCURACY_STEPS):
    """Phase of <psi_exact, psi> after `steps` steps of a plane wave at
    kz = 2 pi kz_index / nz against the closed-form e^{-i w t} (Eq. pwdsip), and
    its amplitude error.  x and y are uniform, so every cell computes the same
    values and the error does not depend on nx, ny."""
    import torch

    import paper_1309_3452_amd as P
    import workloads
    kz = 2 * math.pi * kz_index / nz
    st, w = plane_wave_z(nxy, nxy, nz, kz, m, workloads.DT3, dtype)
    lat = P.Lattice3D(nxy, nxy, nz, dtype=dtype, dt=workloads.DT3)
    lat.set_potential_z(m)
    lat.load(st)
    del st
    lat.step(steps)
    ex, _ = plane_wave_z(nxy, nxy, nz, kz, m, workloads.DT3, torch.complex128, t_shift=steps * workloads.DT3)
    inner = sum(complex(torch.sum(torch.conj(b) * a.to(torch.complex128))) for a, b in zip(lat.state(), ex))
    nrm = sum(float(torch.sum(torch.abs(b) ** 2)) for b in ex)
    del lat, ex
    torch.cuda.empty_cache()
    return {"phase_error_rad": abs(math.atan2(inner.imag, inner.real)), "amplitude_error": abs(abs(inner) / nrm - 1.0),
            "k_z": kz, "omega": w, "m": m, "steps": steps, "lattice": "%dx%dx%d" % (nxy, nxy, nz)}


def compare_states(s32, s64):
    """Relative L2 distance of the FP32 state from the FP64 one and the phase of
    their overlap <psi64, psi32>, summed in FP64 array by array."""
    import torch
    num = den = 0.0
    ov = 0j
    for a, b in zip(s32, s64):
        a64 = a.to(torch.complex128)
        num += float(torch.sum(torch.abs(a64 - b) ** 2))
        den += float(torch.sum(torch.abs(b) ** 2))
        ov += complex(torch.sum(torch.conj(b) * a64))
        del a64
    import cmath
    return math.sqrt(num / den), cmath.phase(ov)


def copy_ceiling_gbs(nbytes=4 << 30, reps=5, detail=None):
    """Device-to-device copy rate (read + write bytes per second) of nbytes, the
    practical HBM ceiling the stencil kernels are compared with: the faster of the
    runtime's copy (torch copy_) and the library's plain streaming copy."""
    import torch

    import paper_1309_3452_amd as P
    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    ms_rt = _timed(lambda: dst.copy_(src), reps)
    P.stream_copy(dst, src)
    ms_lib = _timed(lambda: P.stream_copy(dst, src), reps)
    del src, dst
    torch.cuda.empty_cache()
    rates = {"runtime_copy_GBs": 2.0 * nbytes / (ms_rt * 1e-3) / 1e9,
             "stream_copy_GBs": 2.0 * nbytes / (ms_lib * 1e-3) / 1e9}
    if detail is not None:
        detail.update(rates)
    return max(rates.values())


def cpu_model():
    """The host CPU's model name with its family, model and stepping numbers
    (a virtualised host may report only a generic name)."""
    info = {}
    try:
        for line in open("/proc/cpuinfo"):
            if ":" in line:
                k, v = line.split(":", 1)
                k = k.strip()
                if k in ("model name", "cpu family", "model", "stepping", "vendor_id") and k not in info:
                    info[k] = v.strip()
            elif info:
                break
    except OSError:
        pass
    name = info.get("model name", "unknown")
    extra = ", ".join("%s %s" % (k, info[k]) for k in ("vendor_id", "cpu family", "model", "stepping") if k in info)
    return "%s (%s)" % (name, extra) if extra else name


def cpu_baseline(n=512, steps_all=3, steps_one=1):
    """The FP64 oracle on the host cores, on the headline workload itself (n^3,
    same packet, mass and V(z)): steps_all steps on all cores, then steps_one
    step(s) on one thread; the input is built on the GPU and copied to host
    memory before timing."""
    import numpy as np
    import torch

    import oracle
    import workloads
    ol = oracle.Lattice3(n, n, n, workloads.DT3)
    vi, vh = workloads.step_potential(n, 1.5, n / 2.0, 4.0)
    th = ol.theta_vz(0.5, vi, vh)
    st = workloads.packet3d(n, n, n, (n / 2.0, n / 2.0, n / 4.0), 12.0, (0.0, 0.0, 0.56), 0.5, workloads.DT3,
                            device="cuda")
    f = [np.ascontiguousarray(t.cpu().numpy()) for t in st]
    del st
    torch.cuda.empty_cache()
    cores = oracle.threads()
    t0 = time.perf_counter()
    ol.step(f, th, steps_all)
    t_all = time.perf_counter() - t0
    oracle.set_threads(1)
    try:
        t0 = time.perf_counter()
        ol.step(f, th, steps_one)
        t_one = time.perf_counter() - t0
    finally:
        oracle.set_threads(cores)
    cells = float(n) ** 3
    return {"value": cells * steps_all / t_all, "unit": "site-updates/s", "cores": cores, "kind": "oracle",
            "cpu_model": cpu_model(), "value_1thread": cells * steps_one / t_one, "cores_1thread": 1,
            "sample": "FP64 C oracle on the headline workload (%d^3, m=0.5, V(z) step, same packet): %d steps on "
                      "%d threads (%.1f s), then %d step(s) on 1 thread (%.1f s)"
                      % (n, steps_all, cores, t_all, steps_one, t_one)}


def _timed(fn, reps=1):
    import torch
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def bench_batched(steps):
    """64 uneven 2D lattices (sizes from {64, 96, ..., 1024}^2, per-site theta), complex64."""
    import tempfile

    import torch

    import paper_1309_3452_amd as P
    import workloads
    lats = workloads.config_batched(device="cuda")
    cells = sum(L["nx"] * L["ny"] for L in lats)
    B = P.BatchedLattices(lats, dtype=torch.complex64, dt=workloads.DT2)
    snap = [[t.clone() for t in B.state(b)] for b in range(B.count)]
    cache = os.path.join(tempfile.gettempdir(), "dirac_tune_cache.json")
    choice = B.autotune(cache)
    res = {}
    for mode, graph in ((1, False), (1, True), (0, False), (0, True)):
        for b in range(B.count):                     # same initial state for every variant
            for t, s0 in zip(B.state(b), snap[b]):
                t.copy_(s0)
        B.run(2, mode=mode, graph=False)
        if graph:
            B.run(steps, mode=mode, graph=True)      # capture + first replay
        ms = _timed(lambda: B.run(steps, mode=mode, graph=graph))
        res["mode%d%s" % (mode, "_graph" if graph else "")] = ms
    # 64 single-lattice runs one after another (fused 2D kernel, same inputs)
    solo_ms = 0.0
    for L in lats:
        lat = P.Lattice2D(L["nx"], L["ny"], dtype=torch.complex64, dt=workloads.DT2)
        lat.load(L["state"])
        lat.set_fields(L["m"], L["v_site"])
        lat.step(2)
        solo_ms += _timed(lambda: lat.step(steps))
    best = min(res, key=res.get)
    value = cells * steps / (res[best] * 1e-3)
    alg = 96.0 * cells            # 4 complex64 amplitudes read + 4 written, 4 complex64 per-site records read, per cell-pass
    # tuning candidates 8..14 of the batch library make two-step passes (mode 1 only;
    # the persistent mode makes one-step passes); a two-step pass moves each byte once
    spp = 2 if (best.startswith("mode1") and choice[0] >= 8) else 1
    return {"metric": "site-updates/s, 64 batched (2+1)D lattices, complex64, 500 steps", "value": value,
            "unit": "site-updates/s", "n_gpus": 1, "steps": steps, "warmup": 2,
            "ms_per_step": res[best] / steps, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f32", "data": "synthetic",
            "config": {"workload": "64 uneven 2D lattices, sizes iid from {64,...,1024}^2, sum of 4 Gaussians V, "
                                   "m in [0,1], per-site coefficient records, complex64", "cells": cells, "best": best,
                       "tile_choice": choice},
            "variants_ms": res, "sequential_single_lattice_ms": solo_ms, "speedup_vs_sequential": solo_ms / res[best],
            # per pass (one launch) every amplitude is read and written once and every
            # record read once: 96 B per cell and pass, whatever the steps per pass
            "roofline": {"bound": "hbm", "achieved": alg * steps / spp / (res[best] * 1e-3) / 1e9,
                         "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": alg * steps / spp / (res[best] * 1e-3) / 1e9 / HBM_PEAK_GBS,
                         "traffic": None, "alg_bytes_per_launch": alg, "steps_per_pass": spp,
                         "effective_GBs_per_step_model": alg * steps / (res[best] * 1e-3) / 1e9}}


def bench_adjoint(steps, dtype_name):
    """Gradient of the transmitted probability w.r.t. 32 V(z) nodes on 128^3, by the reversible adjoint."""
    import numpy as np
    import torch

    import paper_1309_3452_amd as P
    import workloads
    cfg = workloads.config_adjoint(128)
    dtype = torch.complex128 if dtype_name == "f64" else torch.complex64
    n = cfg["n"]
    st = workloads.packet3d(n, n, n, cfg["center"], cfg["sigma"], cfg["k0"], cfg["m"], cfg["dt"], dtype=dtype,
                            device="cuda")
    # the forward runs the library's default (fastest) step kernel, in the timed
    # forward and inside the gradient alike; every kernel gives the same bits,
    # so the reversal rebuilds the same states
    lat = P.Lattice3D(n, n, n, dtype=dtype, dt=cfg["dt"])
    H_int = torch.from_numpy(cfg["H_int"])
    H_half = torch.from_numpy(cfg["H_half"])
    p = torch.tensor(cfg["p"], dtype=torch.float64, requires_grad=True)
    vi = (H_int @ p.detach()).numpy()
    vh = (H_half @ p.detach()).numpy()
    lat.load(st)
    lat.set_potential_z(cfg["m"], vi, vh)
    lat.step(2)
    lat.load(st)
    fwd = _timed(lambda: lat.step(steps))
    loss = P.DiracLoss.apply(p, lat, st, cfg["m"], H_int, H_half, steps, cfg["z0"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    loss = P.DiracLoss.apply(p, lat, st, cfg["m"], H_int, H_half, steps, cfg["z0"])
    loss.backward()
    torch.cuda.synchronize()
    total = (time.perf_counter() - t0) * 1e3
    rebuilt = [t.clone() for t in lat.state()]
    err = math.sqrt(sum(float(torch.sum(torch.abs(a.to(torch.complex128) - b.to(torch.complex128)) ** 2))
                        for a, b in zip(rebuilt, st)) / sum(float(torch.sum(torch.abs(b.to(torch.complex128)) ** 2))
                                                            for b in st))
    cells = n ** 3
    return {"metric": "adjoint gradient time / forward time, (3+1)D 128^3, 400 steps, 32 V(z) nodes",
            "value": total / fwd, "unit": "x forward", "n_gpus": 1, "steps": steps, "warmup": 2,
            "ms_per_step": total / steps, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
            "dtype": dtype_name, "data": "synthetic",
            "config": {"workload": "(3+1)D 128^3 adjoint, V(z) from 32 periodic hat nodes, loss = P(z >= 64)",
                       "cells": cells},
            "forward_ms": fwd, "forward_plus_gradient_ms": total, "backward_ms": total - fwd,
            "backward_ms_per_step": (total - fwd) / steps, "loss": float(loss.detach()),
            "grad_norm": float(p.grad.norm()), "rebuilt_initial_state_rel_l2": err}


def bench_links3d(n, steps, dtype_name):
    """(3+1)D n^3 step with a vector potential as gauge links (split kernels with links)."""
    import torch

    import paper_1309_3452_amd as P
    import workloads
    dtype = torch.complex64 if dtype_name == "f32" else torch.complex128
    cfg = workloads.config_step3d(n, dtype=dtype, device="cuda")
    lat = P.Lattice3D(n, n, n, dtype=dtype, dt=cfg["dt"])
    lat.set_potential_z(cfg["m"], cfg["v_int"], cfg["v_half"])
    lat.load(cfg["state"])
    del cfg["state"]
    lat.set_links(workloads.peierls_links3d(n, n, n, 0.05, 31, dtype=dtype, device="cuda"))
    torch.cuda.empty_cache()
    e0 = lat.norm()
    # the split link kernels (two launches per step) for comparison, then the z-march
    # link kernel (one launch per step, the default); the state keeps evolving
    lat.set_kernel("split")
    lat.step(2)
    split_ms = _timed(lambda: lat.step(steps // 2)) / (steps // 2)
    lat.set_kernel("auto")
    lat.step(2)
    ms = _timed(lambda: lat.step(steps))
    e1 = lat.norm()
    cells = n ** 3
    b = 8 if dtype_name == "f32" else 16
    # per step and cell: 16 amplitudes read or written once and 24 link factors read once
    alg_launch = (16 + 24) * b * cells
    launch_ms = ms / steps
    achieved = alg_launch / (launch_ms * 1e-3) / 1e9
    return {"metric": "site-updates/s, (3+1)D %d^3 with gauge links (vector potential)" % n,
            "value": cells * steps / (ms * 1e-3), "unit": "site-updates/s", "n_gpus": 1, "steps": steps,
            "warmup": 2, "ms_per_step": ms / steps, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": dtype_name, "data": "synthetic",
            "config": {"workload": "(3+1)D %d^3 Klein-step lattice of the headline workload plus Peierls links of "
                                   "a smooth periodic vector potential (amplitude 0.05 rad/cell), z-march "
                                   "link kernel" % n, "cells": cells},
            "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                         "kernel": "k3_fused_links (one launch per step)", "avg_launch_ms": launch_ms,
                         "alg_bytes_per_launch": alg_launch},
            "split_kernels_ms_per_step": split_ms,
            "E_r_rel_drift": abs(e1[0] - e0[0]) / abs(e0[0]), "plain_norm_rel_change": abs(e1[2] - e0[2]) / e0[2]}


def bench_norm3d(n, reps, dtype_name):
    """The conserved-functional reduction alone on the n^3 headline lattice (asynchronous
    device-output calls back to back: the LDS-staged z-march plus the final sum of its
    fixed 1024 partials)."""
    import torch

    import paper_1309_3452_amd as P
    import workloads
    dtype = torch.complex64 if dtype_name == "f32" else torch.complex128
    cfg = workloads.config_step3d(n, dtype=dtype, device="cuda")
    lat = P.Lattice3D(n, n, n, dtype=dtype, dt=cfg["dt"])
    lat.set_potential_z(cfg["m"], cfg["v_int"], cfg["v_half"])
    lat.load(cfg["state"])
    del cfg["state"]
    torch.cuda.empty_cache()
    e = lat.norm()
    lat.norm_device()
    ms = _timed(lambda: lat.norm_device(), reps)
    # the observables reduction of the same state (synchronous calls: host copy-out included)
    obs = lat.observables(n / 2.0)
    obs_ms = _timed(lambda: lat.observables(n / 2.0), reps)
    cells = n ** 3
    b = 8 if dtype_name == "f32" else 16
    alg = 8 * b * cells                    # each of the eight arrays read once
    achieved = alg / (ms * 1e-3) / 1e9
    return {"metric": "cells/s of the conserved-functional reduction, (3+1)D %d^3" % n,
            "value": cells / (ms * 1e-3), "unit": "cells/s", "n_gpus": 1, "steps": reps, "warmup": 1,
            "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": dtype_name, "data": "synthetic",
            "config": {"workload": "(3+1)D %d^3 periodic lattice of the headline workload, E_r in both "
                                   "forms and the plain norm, FP64 sums" % n, "cells": cells},
            "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                         "kernel": "k3_norm_lds + k_final_sum per call", "avg_call_ms": ms,
                         "alg_bytes_per_call": alg},
            "E_r": e[0], "E_r_cd_form": e[1], "plain_norm": e[2],
            "observables": {"ms_per_call": obs_ms, "GBs_read_once": alg / (obs_ms * 1e-3) / 1e9,
                            "kernel": "k3_obs (synchronous call)", "P_z_ge_half": obs[0], "plain_norm": obs[4]}}


def bench_site3d(n, steps, dtype_name):
    """(3+1)D n^3 step with per-site coefficient records (a potential V(x, y, z)):
    the one-step and the two-step z-march kernels on the same lattice."""
    import torch

    import paper_1309_3452_amd as P
    import workloads
    dtype = torch.complex64 if dtype_name == "f32" else torch.complex128
    cfg = workloads.config_step3d(n, dtype=dtype, device="cuda")
    lat = P.Lattice3D(n, n, n, dtype=dtype, dt=cfg["dt"])
    lat.load(cfg["state"])
    del cfg["state"]
    # V at each array's own sites: the headline's step in z plus 0.05 N(0, 1)
    # site noise (seeded), so that no two sites share a record
    gen = torch.Generator(device="cuda")
    gen.manual_seed(13093452)
    V = []
    for a in range(8):
        z = torch.arange(n, dtype=torch.float64, device="cuda") + workloads.OFF3[a][2]
        vz = 1.5 * (1.0 + torch.tanh((z - n / 2.0) / 4.0)) / 2.0
        noise = torch.randn((n, n, n), generator=gen, dtype=torch.float64, device="cuda")
        V.append((vz.view(n, 1, 1) + 0.05 * noise).to(lat.real_dtype).contiguous())
        del noise
    lat.set_fields(cfg["m"], V)
    del V
    lat._vsite = None
    torch.cuda.empty_cache()
    e0 = lat.norm()
    out = {}
    for kern in ("fused", "fused2"):
        lat.set_kernel(kern)
        lat.step(2)
        out[kern] = _timed(lambda: lat.step(steps)) / steps
    e1 = lat.norm()
    cells = n ** 3
    b = 8 if dtype_name == "f32" else 16
    # per cell-step: 16 amplitudes read or written once, 8 per-site records read
    # once (complex64 gamma or float64 theta, 8 B each)
    alg_step = (16 * b + 8 * 8) * cells
    ms = out["fused2"]
    # the two-step launch reads and writes each amplitude and reads each record
    # once at least: alg_step bytes per launch (two steps)
    achieved = alg_step / (2 * ms * 1e-3) / 1e9
    return {"metric": "site-updates/s, (3+1)D %d^3 with per-site potential records" % n,
            "value": cells / (ms * 1e-3), "unit": "site-updates/s", "n_gpus": 1, "steps": steps,
            "warmup": 2, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": dtype_name, "data": "synthetic",
            "config": {"workload": "(3+1)D %d^3 lattice of the headline workload with V(x, y, z) = the z-step "
                                   "plus 0.05 N(0,1) per site as per-site coefficient records, m = 0.5, "
                                   "two-step z-march kernel" % n, "cells": cells},
            "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                         "kernel": "k3_fused2 per-site (two steps per launch)", "avg_launch_ms": 2 * ms,
                         "alg_bytes_per_launch": alg_step,
                         "effective_GBs_per_step_model": alg_step / (ms * 1e-3) / 1e9},
            "one_step_kernel_ms_per_step": out["fused"],
            "E_r_rel_drift": abs(e1[0] - e0[0]) / abs(e0[0])}


def bench_reverse3d(n, steps, dtype_name):
    """The reversed step on the n^3 headline workload: the forward default, the
    reversed steps on the march kernels (the default) and on the split kernels."""
    import torch

    import paper_1309_3452_amd as P
    import workloads
    dtype = torch.complex64 if dtype_name == "f32" else torch.complex128
    cfg = workloads.config_step3d(n, dtype=dtype, device="cuda")
    lat = P.Lattice3D(n, n, n, dtype=dtype, dt=cfg["dt"])
    lat.set_potential_z(cfg["m"], cfg["v_int"], cfg["v_half"])
    lat.load(cfg["state"])
    del cfg["state"]
    torch.cuda.empty_cache()
    e0 = lat.norm()
    lat.step(2)
    fwd = _timed(lambda: lat.step(steps)) / steps
    lat.reverse(2)
    rev = _timed(lambda: lat.reverse(steps)) / steps
    lat.set_kernel("fused")
    fwd1 = _timed(lambda: lat.step(steps)) / steps
    lat.set_kernel("split")
    rev_split = _timed(lambda: lat.reverse(steps // 4)) / (steps // 4)
    lat.set_kernel("auto")
    lat.step(steps // 4)
    e1 = lat.norm()
    cells = n ** 3
    b = 8 if dtype_name == "f32" else 16
    # per march launch: every amplitude read once and written once (two steps per launch)
    alg = 16 * b * cells
    return {"metric": "site-updates/s of the reversed step, (3+1)D %d^3" % n,
            "value": cells / (rev * 1e-3), "unit": "site-updates/s", "n_gpus": 1, "steps": steps, "warmup": 2,
            "ms_per_step": rev, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": dtype_name, "data": "synthetic",
            "config": {"workload": "(3+1)D %d^3 headline Klein-step lattice, %d reversed steps per call: one split "
                                   "reversed C,D half-step, the forward march with r, theta negated, one split "
                                   "reversed A,B half-step" % (n, steps), "cells": cells},
            "roofline": {"bound": "hbm", "achieved": alg / (2 * rev * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": alg / (2 * rev * 1e-3) / 1e9 / HBM_PEAK_GBS, "traffic": None,
                         "kernel": "k3_fused2 with the reversed tables", "alg_bytes_per_launch": alg},
            "forward_ms_per_step": fwd, "forward_one_step_kernel_ms_per_step": fwd1,
            "reverse_split_ms_per_step": rev_split, "reverse_over_forward": rev / fwd,
            "reverse_over_one_step_forward": rev / fwd1,
            "E_r_rel_change_after_round_trips": abs(e1[0] - e0[0]) / abs(e0[0])}


def bench_klein2d(phi_deg):
    """(2+1)D Klein-step scattering (m = 0, step height twice the packet energy,
    absorbing frame), complex64: steps timed; the transmitted probability and
    refraction angle of the run are reported beside the rate."""
    import torch

    import paper_1309_3452_amd as P
    import workloads
    cfg = workloads.config_klein2d(phi_deg, dtype=torch.complex64, device="cuda", absorbing=True)
    nx, ny = cfg["nx"], cfg["ny"]
    lat = P.Lattice2D(nx, ny, dtype=torch.complex64, dt=cfg["dt"])
    lat.set_fields(0.0, [torch.from_numpy(v) for v in cfg["v_site"]], [torch.from_numpy(w) for w in cfg["w_site"]])
    # warm-up on a copy of the initial state, then the measured run from it
    lat.load(cfg["state"])
    lat.step(4)
    lat.load(cfg["state"])
    seg = [int(round(250.0 / cfg["dt"])), int(round(100.0 / cfg["dt"]))]
    ms, meas = 0.0, []
    xs = [(torch.arange(nx, dtype=torch.float64, device="cuda") + workloads.OFF2[a][0]) for a in range(4)]
    ys = [(torch.arange(ny, dtype=torch.float64, device="cuda") + workloads.OFF2[a][1]) for a in range(4)]
    for n in seg:
        ms += _timed(lambda: lat.step(n))
        obs = lat.observables(cfg["xc"])
        pm = sx = sy = 0.0
        for a, t in enumerate(lat.state()):
            d = (t.to(torch.complex128).abs() ** 2) * (xs[a] > cfg["xc"] + 40.0)[None, :]
            pm += float(d.sum())
            sx += float((d * xs[a][None, :]).sum())
            sy += float((d * ys[a][:, None]).sum())
        meas.append((obs[0], sx / pm, sy / pm))
    steps = sum(seg)
    cells = nx * ny
    angle = math.degrees(math.atan2(meas[1][2] - meas[0][2], meas[1][1] - meas[0][1]))
    # launch variants of the same steps (every kernel gives the same bits): one step per
    # launch, two steps per launch, and two-step launches replayed from a captured graph
    # (an even launch count, so the replay starts from the buffers it was captured on)
    variants = {"auto": ms / steps}
    for kind in ("fused", "fused2"):
        lat.set_kernel(kind)
        lat.load(cfg["state"])
        lat.step(2)
        variants[kind] = _timed(lambda: lat.step(steps)) / steps
    gsteps = 4 * (steps // 4)
    lat.set_kernel("fused2")
    lat.load(cfg["state"])
    st = torch.cuda.Stream()
    st.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(st):
        lat.step(2)
        torch.cuda.synchronize()
        with torch.cuda.graph(graph, stream=st):
            lat.step(gsteps)
    torch.cuda.current_stream().wait_stream(st)
    graph.replay()
    variants["fused2_graph"] = _timed(lambda: graph.replay(), reps=3) / gsteps
    best = min(variants, key=variants.get)
    ms_step = variants[best]
    spp = 1 if best == "fused" else 2        # steps per launch (auto is the two-step march at this size)
    alg = 96.0 * cells          # per launch: 4 complex64 amplitudes read + written, 4 complex64 coefficient records read
    return {"metric": "site-updates/s, (2+1)D Klein-step scattering %dx%d complex64" % (nx, ny),
            "value": cells / (ms_step * 1e-3), "unit": "site-updates/s", "n_gpus": 1, "steps": steps,
            "warmup": 4, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "(2+1)D %dx%d, m=0, smoothed step V0=0.4 (width 3) at x=400, packet E=0.2 "
                                   "sigma=30 at %g deg from the step normal, absorbing frame of width 32, "
                                   "per-site complex coefficient records" % (nx, ny, phi_deg), "cells": cells},
            "variants_ms_per_step": variants, "best": best,
            "roofline": {"bound": "hbm", "achieved": alg / (spp * ms_step * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": alg / (spp * ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS, "traffic": None,
                         "alg_bytes_per_launch": alg, "steps_per_launch": spp,
                         "effective_GBs_per_step_model": alg / (ms_step * 1e-3) / 1e9},
            "physics": {"transmitted_probability_t250": meas[0][0], "transmitted_probability_t350": meas[1][0],
                        "refraction_angle_deg": angle}}


def bench_links2d(n, steps):
    """(2+1)D n^2 complex64 lattice in a uniform magnetic field (Landau-gauge links),
    the link y-march against the split link kernels."""
    import torch

    import paper_1309_3452_amd as P
    import workloads
    st = workloads.packet2d(n, n, (n / 2.0, n / 2.0), n / 16.0, (0.3, 0.0), 0.3, workloads.DT2,
                            dtype=torch.complex64, device="cuda")
    lat = P.Lattice2D(n, n, dtype=torch.complex64, dt=workloads.DT2)
    lat.set_potential_z(0.3)
    lat.load(st)
    lat.set_links(workloads.landau_links2d(n, n, 1, dtype=torch.complex64, device="cuda"))
    e0 = lat.norm()
    lat.set_kernel("split")
    lat.step(2)
    split_ms = _timed(lambda: lat.step(steps)) / steps
    lat.set_kernel("auto")
    lat.step(2)
    ms = _timed(lambda: lat.step(steps)) / steps
    e1 = lat.norm()
    cells = n * n
    alg = (8 + 8) * 8.0 * cells      # 4 amplitudes read + 4 written, 8 link factors read, per cell-step
    return {"metric": "site-updates/s, (2+1)D %d^2 complex64 in a uniform magnetic field (gauge links)" % n,
            "value": cells / (ms * 1e-3), "unit": "site-updates/s", "n_gpus": 1, "steps": steps, "warmup": 2,
            "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
            "data": "synthetic",
            "config": {"workload": "(2+1)D %d^2, m=0.3, Landau-gauge links of one flux pair across the torus, "
                                   "Gaussian packet, link y-march" % n, "cells": cells},
            "roofline": {"bound": "hbm", "achieved": alg / (ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, "traffic": None,
                         "kernel": "k2_fused_links (one launch per step)", "alg_bytes_per_step": alg},
            "split_kernels_ms_per_step": split_ms, "E_r_rel_drift": abs(e1[0] - e0[0]) / abs(e0[0])}


def bench_slab3d(steps):
    """One device's share of the 512^3 headline lattice split into 8 z-slabs: a
    512 x 512 x 64 slab (complex64) with two halo planes per side, stepped by the
    two-step kernel (the two halo planes serve two steps), halos refilled after
    every launch (here from the slab's own opposite boundary: a one-slab
    decomposition, the same bytes a device would receive from its neighbours)."""
    import torch

    import paper_1309_3452_amd as P
    import workloads
    n, nzs = 512, 64
    v_int, v_half = workloads.step_potential(nzs, 1.5, nzs / 2.0, 4.0)
    st = workloads.packet3d(n, n, nzs, (n / 2.0, n / 2.0, nzs / 2.0), 12.0, (0.0, 0.0, 0.56), 0.5, workloads.DT3,
                            dtype=torch.complex64, device="cuda")
    sl = P.SlabDecomposition(n, n, nzs, 1, dtype=torch.complex64, dt=workloads.DT3)
    sl.set_potential_z(0.5, v_int, v_half)
    sl.load(st)
    del st
    torch.cuda.empty_cache()
    e0 = sl.norm()
    lat = sl.parts[0]
    k = lat.halo_steps
    sl.step(2 * k)
    stream = torch.cuda.current_stream()
    launches = steps // k
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(launches)]
    torch.cuda.synchronize()
    for q in range(launches):
        ev[q][0].record(stream)
        lat.step(k)
        ev[q][1].record(stream)
        sl.exchange()
        ev[q][2].record(stream)
    torch.cuda.synchronize()
    k_ms = sum(e[0].elapsed_time(e[1]) for e in ev) / launches
    x_ms = sum(e[1].elapsed_time(e[2]) for e in ev) / launches
    e1 = sl.norm()
    cells = n * n * nzs
    plane = n * n * 8
    alg = 128.0 * cells          # per launch: each amplitude read and written once
    ms = (k_ms + x_ms) / k
    return {"metric": "site-updates/s of one device's z-slab (512x512x64 of a 512^3 lattice over 8 devices), complex64",
            "value": cells / (ms * 1e-3), "unit": "site-updates/s", "n_gpus": 1, "steps": launches * k,
            "warmup": 2 * k, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "(3+1)D z-slab 512x512x64 + 2 halo planes per side, headline physics, "
                                   "%d step(s) per launch and per halo refill, refill on the device" % k,
                       "cells": cells, "steps_per_refill": k},
            "slab_kernel_ms_per_launch": k_ms, "halo_fill_ms_per_refill": x_ms,
            "slab_kernel_ms_per_step": k_ms / k, "halo_fill_ms_per_step": x_ms / k,
            "roofline": {"bound": "hbm", "achieved": alg / (k_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": alg / (k_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, "traffic": None,
                         "kernel": "k3_fused2<float> in z-slab mode" if k == 2 else "k3_fused<float> in z-slab mode",
                         "steps_per_launch": k, "alg_bytes_per_launch": alg,
                         "effective_GBs_per_step_model": alg * k / (k_ms * 1e-3) / 1e9},
            "halo": {"bytes_per_face_filled": 8 * 2 * plane, "refills_per_step": 1.0 / k, "xgmi_link_GBs": 153.0,
                     "modeled_link_ms_per_face": 8 * 2 * plane / 153e9 * 1e3},
            "E_r_rel_drift": abs(e1[0] - e0[0]) / abs(e0[0])}


def bench_plane2d(steps):
    """(2+1)D 128^2, complex128, 200 steps: launch-bound; plain launches vs one
    captured graph, for the one-step march and the two-step march."""
    import torch

    import paper_1309_3452_amd as P
    import workloads
    cfg = workloads.config1()
    lat = P.Lattice2D(128, 128, dtype=torch.complex128, dt=cfg["dt"])
    lat.set_potential_z(0.0)
    lat.load(cfg["state"])

    def measure(kind):
        lat.set_kernel(kind)
        lat.step(2)
        plain = _timed(lambda: lat.step(steps))
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        g = torch.cuda.CUDAGraph()
        with torch.cuda.stream(s):
            lat.step(2)
            torch.cuda.synchronize()
            with torch.cuda.graph(g, stream=s):
                lat.step(steps)
        torch.cuda.current_stream().wait_stream(s)
        return plain, _timed(lambda: g.replay(), reps=5)

    variants = {k: measure(k) for k in ("fused", "fused2")}
    best = min(variants, key=lambda k: variants[k][1])
    plain, graph = variants[best]
    cells = 128 * 128
    return {"metric": "site-updates/s, (2+1)D 128^2 complex128, 200 steps", "value": cells * steps / (graph * 1e-3),
            "unit": "site-updates/s", "n_gpus": 1, "steps": steps, "warmup": 2, "ms_per_step": graph / steps,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "(2+1)D 128^2 Gaussian packet, m=0, V=0, y-march kernel", "cells": cells,
                       "kernel": best},
            "plain_launches_ms": plain, "graph_replay_ms": graph,
            "plain_value": cells * steps / (plain * 1e-3),
            "variants_ms": {k: {"plain": v[0], "graph": v[1]} for k, v in variants.items()}}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU: a lattice is stepped on one device (a z-slab context is the "
              "per-device unit of a multi-device run); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    if args.calibrate_copy:
        src = torch.ones(args.calibrate_copy // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        torch.cuda.empty_cache()
    if args.workload == "batched2d":
        print(json.dumps(bench_batched(500)), flush=True)
        return
    if args.workload == "adjoint3d":
        for d in ("f64", "f32"):
            print(json.dumps(bench_adjoint(400, d)), flush=True)
        return
    if args.workload == "plane2d":
        print(json.dumps(bench_plane2d(200)), flush=True)
        return
    if args.workload == "links2d":
        print(json.dumps(bench_links2d(2048, 200)), flush=True)
        return
    if args.workload == "slab3d":
        print(json.dumps(bench_slab3d(200)), flush=True)
        return
    if args.workload == "klein2d":
        for phi in (0.0, 37.0):
            print(json.dumps(bench_klein2d(phi)), flush=True)
        return
    if args.workload == "site3d":
        for d in ("f32", "f64"):
            print(json.dumps(bench_site3d(args.n, 100 if d == "f32" else 50, d)), flush=True)
            torch.cuda.empty_cache()
        return
    if args.workload == "reverse3d":
        for d in ("f32", "f64"):
            print(json.dumps(bench_reverse3d(args.n, 100 if d == "f32" else 50, d)), flush=True)
            torch.cuda.empty_cache()
        return
    if args.workload == "norm3d":
        for d in ("f32", "f64"):
            print(json.dumps(bench_norm3d(args.n, 50, d)), flush=True)
        return
    if args.workload == "links3d":
        for d in ("f32", "f64"):
            print(json.dumps(bench_links3d(args.n, 100 if d == "f32" else 50, d)), flush=True)
            torch.cuda.empty_cache()
        return
    n, K, W = args.n, args.steps, args.warmup
    cells = n ** 3
    K64 = args.fp64_steps or K
    if args.precision == "f64":
        r64 = run_gpu(n, torch.complex128, K64, W, 0, 0, args.kernel)
        l64 = r64["launch_ms"] * 1e-3
        v64 = cells * K64 / r64["wall_s"]
        t64 = profiled_traffic("fp64", n, r64["steps_per_launch"])
        print(json.dumps({"metric": "site-updates/s, (3+1)D %d^3 complex128 step" % n, "value": v64,
                          "unit": "site-updates/s", "n_gpus": 1, "steps": K64, "warmup": W,
                          "ms_per_step": r64["wall_s"] * 1e3 / K64, "higher_is_better": True, "scaling": "weak",
                          "vs_baseline": None, "dtype": "f64", "data": "synthetic",
                          "config": {"workload": "(3+1)D %d^3 headline physics, complex128" % n, "cells": cells},
                          "roofline": {"bound": "hbm", "achieved": 256.0 * cells / l64 / 1e9, "peak": HBM_PEAK_GBS,
                                       "unit": "GB/s", "frac": 256.0 * cells / l64 / 1e9 / HBM_PEAK_GBS,
                                       "traffic": t64, "avg_launch_ms": r64["launch_ms"],
                                       "alg_bytes_per_launch": 256.0 * cells,
                                       "kernel_source_sha": kernel_source_hash(r64["steps_per_launch"])}}),
              flush=True)
        return
    r32 = run_gpu(n, torch.complex64, K, W, args.tile_y, args.zchunk, args.kernel, keep=True)
    G = r32["steps_per_launch"]
    # accuracy over a fixed horizon, from the initial packet (untimed)
    acc = not args.no_accuracy
    acc32 = accuracy_pass(r32["lat"], n, torch.complex64) if acc else {}
    r64 = acc64 = packet = None
    if args.no_fp64:
        del r32["lat"]
        torch.cuda.empty_cache()
    else:
        r64 = run_gpu(n, torch.complex128, K64, W, 0, 0, args.kernel, keep=True)
        if acc:
            acc64 = accuracy_pass(r64["lat"], n, torch.complex128)
            # both lattices now hold the packet after ACCURACY_STEPS steps
            l2, ph = compare_states(r32["lat"].state(), r64["lat"].state())
            packet = {"rel_l2_fp32_vs_fp64": l2, "overlap_phase_rad": ph, "steps": ACCURACY_STEPS}
        del r32["lat"], r64["lat"]
        torch.cuda.empty_cache()
    pw32 = plane_wave_phase_error(torch.complex64) if acc else None
    pw64 = plane_wave_phase_error(torch.complex128) if acc else None
    value = cells * K / r32["wall_s"]
    launch_s = r32["launch_ms"] * 1e-3
    # algorithmic bytes of one launch: every amplitude of the state read once and
    # written once (16 x 8 B per cell for complex64), whatever the number of steps
    # the launch advances -- the least any launch can move
    alg_bytes = 128.0 * cells
    achieved = alg_bytes / launch_s / 1e9
    traffic = profiled_traffic("fp32", n, G)
    copy_detail = {}
    copy_gbs = copy_ceiling_gbs(detail=copy_detail)
    kname = "k3_fused2<float> (two steps per launch" if G == 2 else "k3_fused<float> (one step per launch"
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
                               "dt=0.9x stability bound, fused z-march kernel (%d steps per launch), "
                               "FP64 E_r evaluated in-step every %d steps" % (n, n // 2, G, NORM_EVERY),
                   "nx": n, "ny": n, "nz": n, "cells": cells},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic,
                     "kernel": kname + "; every fifth launch also sums E_r)" if G == 2 else kname + "; every tenth launch also sums E_r)",
                     "steps_per_launch": G,
                     "alg_bytes_per_launch": alg_bytes,
                     "alg_unit": "cell-launch: 16 amplitudes x 8 B, each read once and written once per launch",
                     "avg_launch_ms": r32["launch_ms"],
                     # bus view from the committed counters: bytes that crossed HBM per launch over
                     # the launch time, and their excess over the algorithmic bytes
                     "hbm_GBs": (traffic / launch_s / 1e9) if traffic else None,
                     "hbm_frac": (traffic / launch_s / 1e9 / HBM_PEAK_GBS) if traffic else None,
                     "traffic_over_alg": (traffic / alg_bytes) if traffic else None,
                     "kernel_source_sha": kernel_source_hash(G),
                     "copy_ceiling_GBs": copy_gbs,
                     "copy_probes_GBs": copy_detail,
                     "hbm_frac_of_copy_ceiling": (traffic / launch_s / 1e9 / copy_gbs) if traffic else None,
                     # the rate a kernel moving 128 B per cell-step (one step per pass) would need
                     # to match this one: an effective bandwidth, not a fraction of any peak
                     "effective_GBs_per_step_model": 128.0 * cells * G / launch_s / 1e9,
                     # useful FP32 arithmetic (32 FLOP per amplitude update, 8 updates per cell-step)
                     # against the non-packed FP32 vector peak
                     # instruction view from the committed SQ counters: the share of time the
                     # vector ALUs issue (ring recomputation and bookkeeping included)
                     "valu_busy": profiled_valu_busy(n, G),
                     "alu": {"flop_per_cell_step": ALU_FLOP_PER_CELL_STEP,
                             "achieved_TFLOPs": ALU_FLOP_PER_CELL_STEP * value / 1e12,
                             "peak_TFLOPs": FP32_NONPACKED_TFLOPS,
                             "frac": ALU_FLOP_PER_CELL_STEP * value / 1e12 / FP32_NONPACKED_TFLOPS}},
        "norm_error": {"steps": ACCURACY_STEPS if acc else None,
                       "E_r_rel_drift_fp32": acc32.get("E_r_rel_drift"),
                       "E_r_rel_drift_fp32_max_every10": acc32.get("E_r_rel_drift_max_every10"),
                       "plain_norm_rel_change_fp32": acc32.get("plain_norm_rel_change"),
                       "plane_wave_fp32": pw32, "plane_wave_fp64": pw64,
                       "timed_run_E_r_rel_drift_fp32": r32["drift"], "timed_run_steps": r32["steps_total"]},
        "amplitude_updates_per_s": 8 * value,
    }
    if r64 is not None:
        v64 = cells * K64 / r64["wall_s"]
        G64 = r64["steps_per_launch"]
        l64 = r64["launch_ms"] * 1e-3
        a64 = 256.0 * cells / l64 / 1e9
        t64 = profiled_traffic("fp64", n, G64)
        line["fp64"] = {"value": v64, "unit": "site-updates/s", "ms_per_step": r64["wall_s"] * 1e3 / K64,
                        "roofline_frac": a64 / HBM_PEAK_GBS, "achieved_GBs": a64,
                        "alg_bytes_per_launch": 256.0 * cells, "avg_launch_ms": r64["launch_ms"],
                        "traffic": t64, "hbm_frac": (t64 / l64 / 1e9 / HBM_PEAK_GBS) if t64 else None,
                        "effective_GBs_per_step_model": 256.0 * cells * G64 / l64 / 1e9,
                        "steps_per_launch": G64, "kernel_source_sha": kernel_source_hash(G64)}
        line["fp32_speedup_over_fp64"] = value / v64
        line["norm_error"]["E_r_rel_drift_fp64"] = acc64["E_r_rel_drift"] if acc64 else None
        line["norm_error"]["packet_vs_fp64"] = packet
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(n)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
