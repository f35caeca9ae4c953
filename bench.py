#!/usr/bin/env python3
"""Throughput of the free-stream-preserving residual + TVD RK3 on one MI355X.

Metric: cell-stage updates/s = interior nodes x 3 RK stages x steps / time,
with the state, metrics and workspace resident in HBM before the timed
region (metrics are computed once, outside it).  One "step" is one full
third-order TVD Runge-Kutta step (three residual evaluations and updates),
replayed from the library's captured step graph.

Prints ONE JSON line.  Extra fields: the per-kernel roofline of the dominant
sweep kernel (timed with HIP events on the stream it runs on), the
stage-level HBM figure of the method's compulsory traffic, and the FP64 CPU
oracle timed on the host on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks
PEAK_HBM_GBS = 8000.0
PEAK_FP64_TFLOPS = 78.6
PEAK_FP32_TFLOPS = 157.3

# Compulsory HBM bytes per cell-stage of the method (read the stage input,
# Q^n in stages 2-3, the metrics, write the stage output; FP64 storage):
# 3D: (160 + 2*200)/3 = 186.7 B, 2D: (104 + 2*136)/3 = 125.3 B.
STAGE_BYTES = {3: 560.0 / 3.0, 2: 376.0 / 3.0}

# Floating-point operations per face evaluation of each face kernel, counted
# from the kernels' instruction mix with rocprofv3 PMC counters (add, mul,
# transcendental = 1, fma = 2; FP64 plus FP32): profiles/flops_per_face.json,
# written from the counter summaries in profiles/.
FLOPS_FILE = os.path.join(ROOT, "profiles", "flops_per_face.json")
# HBM bytes per launch of the sweep kernels from FETCH_SIZE / WRITE_SIZE
# counter runs scaled by a plain copy kernel: profiles/hbm_traffic.json.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic.json")


def csrc_hash():
    """hash of the kernel sources; counter tables carry the hash they were
    taken with, and a table taken on other sources is reported as stale"""
    import glob
    import hashlib
    h = hashlib.sha256()
    for p in sorted(glob.glob(os.path.join(ROOT, "paper_2101_05886_amd", "csrc", "*"))):
        h.update(os.path.basename(p).encode())
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def counter_table(path):
    try:
        with open(path) as f:
            table = json.load(f)
    except (OSError, ValueError):
        return {}, False
    return table, table.get("csrc_sha256") == csrc_hash()

WORKLOADS = {
    "c2": dict(name="3D isentropic vortex (strength 5, radius 1), 128^3 periodic wavy grid "
                    "(amplitude 0.1), linear-upwind-5 with 6th-order metrics, FP64",
               ndim=3, n=128, Y=6, recon="linup5", prec="fp64", L=12.0, amp=0.1, jitter=0.0,
               seed=2, mach=0.5, vortex=True, cfl=0.5),
    "c3": dict(name="3D 256^3 periodic wavy grid (amplitude 0.1, 5% jitter), Mach 0.8 + vortex, "
                    "WENO5-JS with 6th-order metrics, FP64",
               ndim=3, n=256, Y=6, recon="weno5", prec="fp64", L=12.0, amp=0.1, jitter=0.05,
               seed=3, mach=0.8, vortex=True, cfl=0.5),
    "c3m": dict(name="3D 256^3 periodic wavy grid (amplitude 0.1, 5% jitter), Mach 0.8 + vortex, "
                     "WENO5-JS with 6th-order metrics, FP32-mixed reconstruction",
                ndim=3, n=256, Y=6, recon="weno5", prec="mixed", L=12.0, amp=0.1, jitter=0.05,
                seed=3, mach=0.8, vortex=True, cfl=0.5),
    "c1": dict(name="2D free stream, 64^2 periodic wavy grid (5% jitter), Mach 0.5 at 20 deg, "
                    "WENO5-JS with 2nd-order metrics, FP64",
               ndim=2, n=64, Y=2, recon="weno5", prec="fp64", L=20.0, amp=0.1, jitter=0.05,
               seed=1, mach=0.5, vortex=False, cfl=0.5),
}


def make_inputs(w):
    from paper_2101_05886_amd import inputs as I
    ndim, n, Y, g = w["ndim"], w["n"], w["Y"], max(3, w["Y"] // 2)
    xyz = I.wavy_grid(ndim, n, w["L"], g, Y, amp=w["amp"], jitter=w["jitter"], seed=w["seed"])
    if ndim == 3:
        vel = I.mach_velocity(w["mach"], I.direction_3d())
    else:
        vel = I.mach_velocity(w["mach"], [math.cos(math.radians(20)), math.sin(math.radians(20))])
    if w["vortex"]:
        v3 = tuple(vel) + (0.0,) * (3 - len(vel))
        q = I.Vortex(vel_inf=v3).state(I.state_nodes(xyz, g, Y), period=w["L"])
    else:
        q = I.uniform_state(ndim, n, g, 1.4, vel, 1.0)
    return xyz, q, g


def cpu_baseline(w, xyz, q, g, budget_s=20.0):
    """FP64 oracle on the host: whole RK3 steps of the same grid and state,
    as many as fit in about budget_s seconds (at least one)."""
    import oracle as O
    og = O.Grid(w["ndim"], w["n"], g)
    met = O.metrics(og, w["Y"], xyz)
    sc = O.Scheme(w["recon"], w["Y"], True)
    dt = O.max_dt(og, sc, met, q, w["cfl"])
    qq = q.copy()
    t0 = time.perf_counter()
    steps = 0
    while True:
        qq = O.rk3_step(og, sc, met, qq, dt)
        steps += 1
        if time.perf_counter() - t0 > budget_s * 0.5 or steps >= 1000:
            break
    el = time.perf_counter() - t0
    nodes = w["n"] ** w["ndim"]
    return {"value": nodes * 3 * steps / el, "unit": "cell-stage updates/s", "cores": O.num_threads(),
            "kind": "oracle",
            "sample": f"{steps} full RK3 step(s) of the same {w['n']}^{w['ndim']} grid and state, "
                      f"FP64 oracle (gcc -O2, OpenMP over grid lines), {el:.1f} s"}


COPY_BYTES = 1 << 30


def copy_calibration(torch):
    """A plain copy kernel of known size: every launch reads and writes
    COPY_BYTES of HBM once (the arrays are far larger than the L2 and MALL)."""
    src = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": COPY_BYTES, "launches": 5}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c2", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--kernel-reps", type=int, default=10)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of 1 GiB five times (the reference "
                         "kernel that scales the FETCH_SIZE / WRITE_SIZE counters to bytes)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(the design notes describe how the method would shard)", file=sys.stderr)
        sys.exit(2)

    import torch

    if args.copy_calibration:
        copy_calibration(torch)
        return
    from paper_2101_05886_amd import fp

    w = WORKLOADS[args.workload]
    xyz, q, g = make_inputs(w)
    ndim, n, Y = w["ndim"], w["n"], w["Y"]
    G = fp.Grid(ndim, n, g)
    S = fp.Scheme(w["recon"], Y, True, precision=w["prec"])
    dev = torch.device("cuda")
    met = fp.metrics(G, Y, torch.from_numpy(xyz).to(dev))
    qg = torch.from_numpy(q).to(dev)
    work = torch.zeros(G.work_shape(), dtype=torch.float64, device=dev)
    dt = float(fp.max_dt(G, S, met, qg, w["cfl"]).item())

    # warmup (captures the step graph), then the timed region
    fp.solve(G, S, met, qg, work, dt, max(args.warmup, 1))
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    fp.solve(G, S, met, qg, work, dt, args.steps)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_total = e0.elapsed_time(e1)
    ms_step = ms_total / args.steps
    nodes = n ** ndim
    value = nodes * 3 * args.steps / (ms_total * 1e-3)

    # state sanity after the timed steps
    flag = fp.check_state(G, S, qg)
    torch.cuda.synchronize()
    healthy = int(flag.item()) == 0

    # per-kernel timing of the three sweep kernels an RK stage runs, one
    # kernel per call with the stage's launch configuration (fp_residual_dir
    # launches exactly the stage's kernel of that direction), HIP events on
    # torch's current stream, which is the stream the kernels are launched on
    acc = torch.zeros_like(qg)
    names = ["k_sweep_x", "k_sweep_wg<eta>", "k_sweep_wg<zeta>"]
    kt = {}
    for d in range(ndim):
        fp.residual_dir(G, S, met, qg, d, acc, accumulate=d > 0)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(args.kernel_reps):
            fp.residual_dir(G, S, met, qg, d, acc, accumulate=d > 0)
        b.record()
        torch.cuda.synchronize()
        kt[d] = a.elapsed_time(b) / args.kernel_reps
    dom = max(kt, key=kt.get)
    ftab, fcur = counter_table(FLOPS_FILE)
    ttab, tcur = counter_table(TRAFFIC_FILE)
    fpf = ftab.get(f"{w['recon']}/{ndim}d/{w['prec']}")
    traffic = ttab.get(f"{args.workload}/{names[dom]}") if tcur else None
    peak = PEAK_FP64_TFLOPS if w["prec"] == "fp64" else PEAK_FP32_TFLOPS
    # algorithmic units of one launch: one face per node (periodic lines)
    if fpf:
        achieved = fpf * nodes / (kt[dom] * 1e-3) / 1e12
        roof = {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                "frac": achieved / peak, "traffic": traffic}
    else:
        roof = {"bound": "alu", "achieved": None, "peak": peak, "unit": "TFLOP/s", "frac": None,
                "traffic": traffic}
    roof.update({"kernel": names[dom], "kernel_ms": kt[dom], "flops_per_face": fpf,
                 "counters_current": fcur,
                 "traffic_gbs": traffic / (kt[dom] * 1e-3) / 1e9 if traffic else None,
                 "kernel_ms_by_dir": [round(kt[d], 4) for d in range(ndim)]})
    stage_gbs = STAGE_BYTES[ndim] * value / 1e9
    out = {
        "metric": "cell-stage updates/s", "value": value, "unit": "cell-stage updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if w["prec"] == "fp64" else "f64 state, f32 reconstruction",
        "data": "synthetic",
        "config": {"workload": w["name"], "nodes": nodes, "metric_order": Y,
                   "recon": w["recon"], "precision": w["prec"], "dt": dt},
        "roofline": roof,
        "hbm_stage": {"bytes_per_cell_stage": STAGE_BYTES[ndim], "achieved": stage_gbs,
                      "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": stage_gbs / PEAK_HBM_GBS},
        "wall_s": wall, "state_ok": healthy,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, xyz, q, g)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
