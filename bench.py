#!/usr/bin/env python3
"""Throughput of the free-stream-preserving residual + TVD RK3 on one MI355X.

Metric: cell-stage updates/s = interior nodes x 3 RK stages x steps / time,
with the state, metrics and workspace resident in HBM before the timed
region (metrics are computed once, outside it).  One "step" is one full
third-order TVD Runge-Kutta step (three residual evaluations and updates),
replayed from the library's captured step graph.

Default workload (c4): 48 uneven O-grid blocks advanced together by the
batched path, FP32-mixed reconstruction as `value`, FP64 timed beside it
(`fp64`, `mixed_over_fp64`), and the serving stream (500 requests, p50/p99
latency) reported under `serving` (--no-serving skips it).  Single-block
workloads: --workload c1/c2/c3/c3m/c3w7/c3cu6 and c3v (Navier-Stokes); linked
blocks: c3x8; the double Mach reflection with its boundary faces: dmr; the
serving stream alone: --workload c5.

Prints ONE JSON line.  Extra fields: the roofline of the dominant sweep
kernel (timed with HIP events on the stream it runs on): the method's
algorithmic flops per face over the launch time against the 78.6 TFLOP/s
vector-ALU ceiling, with the VALU issue rate and the algorithmic HBM rate of
the same launch beside it; the stage-level HBM figure of the method's
compulsory traffic; the median of repeated timed regions; the serving stream
at 0.5x, 0.8x and 1.1x load; and the FP64 CPU oracle timed on the host on a
bounded sample of the same workload, with all threads and with one.
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
# The ALU ceiling the library can reach, from the chip's unit counts: 256 CUs
# x 4 SIMDs x 16 lanes x 2 flop (fma) x 2.4 GHz = 78.6 TFLOP/s for FP64 and
# for non-packed FP32 alike (the published 157.3 TFLOP/s FP32 needs packed
# FP32 instructions, which the library's compile flags disable).
CU, SIMD_PER_CU, LANES, CLOCK_HZ = 256, 4, 16, 2.4e9
PEAK_ALU_TFLOPS = CU * SIMD_PER_CU * LANES * 2 * CLOCK_HZ / 1e12
# VALU issue: one wave64 instruction occupies a SIMD for 4 cycles
VALU_ISSUE_PER_S = CU * SIMD_PER_CU * CLOCK_HZ / 4.0

# Compulsory HBM bytes per cell-stage of the method (read the stage input,
# Q^n in stages 2-3, the metrics, write the stage output; FP64 storage):
# 3D: (160 + 2*200)/3 = 186.7 B, 2D: (104 + 2*136)/3 = 125.3 B.
STAGE_BYTES = {3: 560.0 / 3.0, 2: 376.0 / 3.0}

# Floating-point operations per face evaluation of each face kernel, counted
# from the kernels' instruction mix with rocprofv3 PMC counters (add, mul,
# transcendental = 1, fma = 2; FP64 plus FP32), keyed by reconstruction,
# dimension, precision and metric order: profiles/flops_per_face.json,
# written from the counter summaries in profiles/.
FLOPS_FILE = os.path.join(ROOT, "profiles", "flops_per_face.json")
# HBM bytes per launch of the sweep kernels from FETCH_SIZE / WRITE_SIZE
# counter runs scaled by a plain copy kernel: profiles/hbm_traffic.json.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic.json")
# VALU wave instructions per launch (SQ_INSTS_VALU) of the sweep kernels:
# profiles/valu_insts.json.
VALU_FILE = os.path.join(ROOT, "profiles", "valu_insts.json")
# Active shader cycles of each sweep launch (GRBM_GUI_ACTIVE counter runs):
# profiles/active_cycles.json.
CYCLES_FILE = os.path.join(ROOT, "profiles", "active_cycles.json")


def alg_flops_per_face(recon, ndim, Y):
    """Floating-point operations of one face flux of the method (add, mul,
    div, sqrt = 1, fma = 2), counted step by step from the algorithm, not
    from a kernel: the face reference state (interpolation of 1/J, s and
    Q/J of order Y, Q*, F(Q*).s), per stencil node the reference-subtracted
    dQ~ and dF~, the Roe average and eigen-structure with the local speeds,
    two characteristic projections per node (structured Euler form), the
    split a +- lambda b, the reconstructions, the back-projection, add-back
    and the flux difference.  3D WENO5-JS with sixth-order metrics: 1,897."""
    D = ndim
    nv = D + 2
    S = 8 if recon == "weno7" else 6  # stencil nodes
    ref = 2 * Y * (1 + D) + 3 * Y * nv + nv + 8 * D + 6
    node = (2 * nv + 12 * D + 10) * S
    tang = 29 if D == 3 else 3
    eig = (11 * D + 20) + (3 * D + 2) + (2 * D - 1) + tang + (2 * D + 9) * S + 3
    proj = 2 * (2 * D - 1) + (D - 1) * (2 * D - 1) + 4 + 3 + 2 + 1 + 2 * (D - 1) + 2
    back = 35 if D == 3 else 24
    if recon == "linup5":
        recon_f = nv * 22 + proj + nv + 2 * nv
        return ref + node + eig + recon_f + back + nv + nv
    per = {"weno5": 60, "weno7": 150, "wenocu6": 155}[recon]
    return ref + node + eig + 2 * S * proj + 4 * nv * S + 2 * nv * per + back + nv + nv


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

def faces_along(n, d):
    """faces of every line along axis d of a block of interior extents n"""
    f = n[d] + 1
    for e, m in enumerate(n):
        if e != d:
            f *= m
    return f


def roofline(recon, ndim, Y, prec, kernel, kernel_ms, faces, nodes, key):
    """Roofline of one sweep launch.  Bound: the vector ALU.  `achieved` is
    the method's algorithmic flops (alg_flops_per_face x the faces the
    launch evaluates) over the launch's duration, against the 78.6 TFLOP/s
    ALU ceiling.  Beside it: the VALU issue rate (SQ_INSTS_VALU of the same
    launch from profiles/valu_insts.json, 4 cycles per wave instruction, over
    the issue capacity of 1,024 SIMDs at 2.4 GHz), the algorithmic HBM rate
    (the method's compulsory bytes per cell-stage split over the stage's
    ndim sweeps), and the measured HBM bytes of the launch (FETCH_SIZE +
    WRITE_SIZE, calibrated, profiles/hbm_traffic.json).  Counter tables
    taken on other kernel sources are reported as null."""
    fpf = alg_flops_per_face(recon, ndim, Y)
    t = kernel_ms * 1e-3
    achieved = fpf * faces / t / 1e12
    ttab, tcur = counter_table(TRAFFIC_FILE)
    vtab, vcur = counter_table(VALU_FILE)
    ftab, fcur = counter_table(FLOPS_FILE)
    traffic = ttab.get(key) if tcur else None
    insts = vtab.get(key) if vcur else None
    counted = ftab.get(f"{recon}/{ndim}d/{prec}/m{Y}") if fcur else None
    alg_bytes = STAGE_BYTES[ndim] / ndim * nodes
    return {"bound": "alu", "achieved": achieved, "peak": PEAK_ALU_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / PEAK_ALU_TFLOPS, "traffic": traffic,
            "peak_basis": "256 CUs x 4 SIMDs x 16 lanes x 2 flop (fma) x 2.4 GHz: FP64 and non-packed FP32",
            "kernel": kernel, "kernel_ms": kernel_ms, "faces_per_launch": faces,
            "alg_flops_per_face": fpf, "counters_current": bool(tcur and vcur),
            "valu_issue": ({"insts_per_launch": insts, "insts_per_face": insts * 64.0 / faces,
                            "frac": insts / (VALU_ISSUE_PER_S * t)} if insts else None),
            "hbm_alg": {"bytes_per_launch": alg_bytes, "achieved_gbs": alg_bytes / t / 1e9,
                        "peak_gbs": PEAK_HBM_GBS, "frac": alg_bytes / t / 1e9 / PEAK_HBM_GBS},
            "traffic_gbs": traffic / t / 1e9 if traffic else None,
            "traffic_bytes_per_node": traffic / nodes if traffic else None,
            "counted_flops_per_face": counted,
            "clock": clock_view(key, achieved, insts, t)}


def clock_view(key, achieved, insts, t):
    """The same launch against the shader clock it ran at: VALU-bound
    launches run below the 2.4 GHz peak clock (power management), so the
    ALU ceiling they can reach is peak x clock / 2.4 GHz.  The launch's
    active cycles come from a separate GRBM_GUI_ACTIVE counter run
    (profiles/active_cycles.json; none for launches too short to measure);
    the clock of the live launch is those cycles over its live duration,
    and the VALU issue per active cycle is SQ_INSTS_VALU x 4 over (1,024
    SIMDs x the cycles), independent of either run's duration."""
    ctab, ccur = counter_table(CYCLES_FILE)
    rec = ctab.get(key) if ccur else None
    if not rec:
        return None
    cyc = rec["active_cycles"]
    ghz = cyc / t / 1e9
    scale = ghz * 1e9 / CLOCK_HZ
    return {"active_cycles": cyc, "live_ghz": ghz, "counter_run_ghz": rec["ghz"],
            "alu_peak_at_clock": PEAK_ALU_TFLOPS * scale, "frac_at_clock": achieved / (PEAK_ALU_TFLOPS * scale),
            "valu_issue_per_cycle": insts * 4.0 / (CU * SIMD_PER_CU * cyc) if insts else None}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def median_rate(times_ms, work):
    """median, min and max of work / time over repeated timed regions"""
    rates = sorted(work / (t * 1e-3) for t in times_ms)
    return {"n": len(rates), "median": rates[len(rates) // 2], "min": rates[0], "max": rates[-1]}


WORKLOADS = {
    "c2": dict(name="3D isentropic vortex (strength 5, radius 1), 128^3 periodic wavy grid "
                    "(amplitude 0.1), linear-upwind-5 with 6th-order metrics, FP64",
               ndim=3, n=128, Y=6, recon="linup5", prec="fp64", L=12.0, amp=0.1, jitter=0.0,
               seed=2, mach=0.5, vortex=True, cfl=0.5, convergence=(32, 64)),
    "c3": dict(name="3D 256^3 periodic wavy grid (amplitude 0.1, 5% jitter), Mach 0.8 + vortex, "
                    "WENO5-JS with 6th-order metrics, FP64",
               ndim=3, n=256, Y=6, recon="weno5", prec="fp64", L=12.0, amp=0.1, jitter=0.05,
               seed=3, mach=0.8, vortex=True, cfl=0.5),
    "c3m": dict(name="3D 256^3 periodic wavy grid (amplitude 0.1, 5% jitter), Mach 0.8 + vortex, "
                     "WENO5-JS with 6th-order metrics, FP32-mixed reconstruction",
                ndim=3, n=256, Y=6, recon="weno5", prec="mixed", L=12.0, amp=0.1, jitter=0.05,
                seed=3, mach=0.8, vortex=True, cfl=0.5),
    "c3w7": dict(name="3D 256^3 periodic wavy grid (amplitude 0.1, 5% jitter), Mach 0.8 + vortex, "
                      "WENO7-JS with 8th-order metrics, FP32-mixed reconstruction",
                 ndim=3, n=256, Y=8, recon="weno7", prec="mixed", L=12.0, amp=0.1, jitter=0.05,
                 seed=3, mach=0.8, vortex=True, cfl=0.5),
    "c3cu6": dict(name="3D 256^3 periodic wavy grid (amplitude 0.1, 5% jitter), Mach 0.8 + vortex, "
                       "WENOCU6 (C = 20, q = 2, eps = 1e-6) with 6th-order metrics, FP32-mixed reconstruction",
                  ndim=3, n=256, Y=6, recon="wenocu6", prec="mixed", L=12.0, amp=0.1, jitter=0.05,
                  seed=3, mach=0.8, vortex=True, cfl=0.5, cpu_n=128),
    "c3v": dict(name="3D 256^3 periodic wavy grid (amplitude 0.1, 5% jitter), Mach 0.8 + vortex, "
                     "Navier-Stokes: WENO5-JS inviscid fluxes with 6th-order metrics plus sixth-order central "
                     "viscous fluxes (mu 1e-3, Prandtl 0.72), FP64",
                ndim=3, n=256, Y=6, recon="weno5", prec="fp64", L=12.0, amp=0.1, jitter=0.05,
                seed=3, mach=0.8, vortex=True, cfl=0.5, mu=1e-3, prandtl=0.72, cpu_n=128),
    "c3x8": dict(name="the 256^3 periodic wavy grid (amplitude 0.1, 5% jitter, Mach 0.8 + vortex) cut into "
                      "2x2x2 blocks of 128^3 joined by interface links on every axis (the outer faces linked "
                      "around the period), batched, WENO5-JS with 6th-order metrics, FP32-mixed",
                 ndim=3, n=256, Y=6, recon="weno5", prec="mixed", L=12.0, amp=0.1, jitter=0.05,
                 seed=3, mach=0.8, vortex=True, cfl=0.5, cuts=(2, 2, 2)),
    "c1": dict(name="2D free stream, 64^2 periodic wavy grid (5% jitter), Mach 0.5 at 20 deg, "
                    "WENO5-JS with 2nd-order metrics, FP64",
               ndim=2, n=64, Y=2, recon="weno5", prec="fp64", L=20.0, amp=0.1, jitter=0.05,
               seed=1, mach=0.5, vortex=False, cfl=0.5),
    "c5": dict(name="serving: Poisson stream of 500 solve requests (seed 5) at 0.8x the measured "
                    "closed-loop capacity; grids 2D 64^2 to 3D 160^3 (log-uniform nodes), wavy periodic "
                    "with a vortex or O-grid with frozen ghosts; Mach U(0.3, 2.0), angle U(0, 10) deg; "
                    "200 RK3 steps each; WENO5-JS with 6th-order metrics, FP32-mixed; continuous batching",
               ndim=3, Y=6, recon="weno5", prec="mixed", requests=500, seed=5, load=0.8,
               capacity_requests=100, slots=64, round_steps=10, other_loads=(0.5, 1.1), other_requests=300),
    "dmr": dict(name="2D double Mach reflection (Mach 10, 60 deg), 961x241 nodes on [0,4]x[0,1] with a 5% "
                     "random grid (seed 11), WENO5-JS with 6th-order metrics and global Lax-Friedrichs "
                     "splitting, FP64, boundary faces (held inflow, outflow, slip wall, exact moving shock) "
                     "applied every stage, CFL 0.6 from the initial state",
                ndim=2, nx=961, ny=241, rand=0.05, Y=6, recon="weno5", prec="fp64", cfl=0.6, seed=11,
                shock=True),
    "c4": dict(name="48 O-grid sector blocks (seed 4; n_theta 32..192, n_r 32..128, n_z 16..64; wall "
                    "spacing 0.01 stretched x1.1; skew up to 30 deg), uniform Mach 3 along x with frozen "
                    "free-stream ghosts, WENO5-JS with 6th-order metrics, batched: one persistent launch "
                    "per sweep direction and RK stage, FP32-mixed (FP64 timed beside it)",
               ndim=3, Y=6, recon="weno5", prec="mixed", mach=3.0, cfl=0.5, blocks=48, seed=4),
}


def make_inputs(w):
    from paper_2101_05886_amd import inputs as I
    ndim, n, Y = w["ndim"], w["n"], w["Y"]
    g = 4 if (w["recon"] == "weno7" or Y == 8) else 3
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
    note = ""
    if "cpu_n" in w:
        # a slow scheme: the same recipe on a smaller grid keeps the sample short
        w = dict(w, n=w["cpu_n"])
        xyz, q, g = make_inputs(w)
        note = f" (the workload's recipe at {w['n']}^{w['ndim']}: one step at full size takes over a minute)"
    og = O.Grid(w["ndim"], w["n"], g)
    met = O.metrics(og, w["Y"], xyz)
    sc = O.Scheme(w["recon"], w["Y"], True, mu=w.get("mu", 0.0), prandtl=w.get("prandtl", 0.72))
    dt = O.max_dt(og, sc, met, q, w["cfl"])
    nodes = w["n"] ** w["ndim"]

    def timed(limit):
        qq = q.copy()
        t0 = time.perf_counter()
        steps = 0
        while True:
            qq = O.rk3_step(og, sc, met, qq, dt)
            steps += 1
            if time.perf_counter() - t0 > limit or steps >= 1000:
                break
        return steps, time.perf_counter() - t0

    threads = O.num_threads()
    progress(f"cpu baseline: {threads} threads")
    steps, el = timed(budget_s * 0.5)
    out = {"value": nodes * 3 * steps / el, "unit": "cell-stage updates/s", "cores": threads,
           "kind": "oracle", "cpu_model": cpu_model(), "nproc": os.cpu_count(),
           "sample": f"{steps} full RK3 step(s) of the same {w['n']}^{w['ndim']} grid and state, "
                     f"FP64 oracle (gcc -O2, OpenMP over grid lines, {threads} threads), {el:.1f} s{note}"}
    # one thread: the same recipe on a grid small enough that one step
    # takes about budget_s / 4 at the per-node cost just measured, taken as
    # if the threads had scaled perfectly (so the sample is never longer)
    per_node = el / (steps * nodes) * threads
    n1 = int((budget_s * 0.25 / per_node) ** (1.0 / w["ndim"]))
    n1 = max(16, min(w["n"], n1))
    w1 = dict(w, n=n1)
    xyz1, q1, g1 = make_inputs(w1)
    og1 = O.Grid(w["ndim"], n1, g1)
    met1 = O.metrics(og1, w["Y"], xyz1)
    dt1 = O.max_dt(og1, sc, met1, q1, w["cfl"])
    progress(f"cpu baseline: one thread, {n1}^{w['ndim']}")
    O.set_num_threads(1)
    try:
        t0 = time.perf_counter()
        O.rk3_step(og1, sc, met1, q1, dt1)
        el1 = time.perf_counter() - t0
    finally:
        O.set_num_threads(threads)
    out["single_thread"] = {"value": n1 ** w["ndim"] * 3 / el1, "cores": 1,
                            "sample": f"one full RK3 step of the same recipe at {n1}^{w['ndim']}, one thread, "
                                      f"{el1:.1f} s"}
    if "convergence" in w:
        out["convergence_runs"] = cpu_convergence_runs(w, sc, threads)
    return out


def cpu_convergence_runs(w, sc, threads):
    """The oracle over whole convergence runs of the workload's recipe (t = 0
    to 1, dt = dt_32 (32/n)^(5/3) with dt_32 the CFL step of the coarsest
    grid): the coarsest grid with all threads and with one, the next with
    all threads."""
    import oracle as O
    runs, dt32 = [], None
    n0, n1 = w["convergence"]
    for n, nt in ((n0, threads), (n0, 1), (n1, threads)):
        wn = dict(w, n=n)
        xyz, q, g = make_inputs(wn)
        og = O.Grid(w["ndim"], n, g)
        met = O.metrics(og, w["Y"], xyz)
        if dt32 is None:
            dt32 = O.max_dt(og, sc, met, q, w["cfl"])
        steps = math.ceil(1.0 / (dt32 * (n0 / n) ** (5.0 / 3.0)))
        progress(f"cpu baseline: convergence run {n}^{w['ndim']}, {steps} steps, {nt} thread(s)")
        O.set_num_threads(nt)
        try:
            t0 = time.perf_counter()
            O.solve(og, sc, met, q, 1.0 / steps, steps)
            el = time.perf_counter() - t0
        finally:
            O.set_num_threads(threads)
        runs.append({"n": n, "steps": steps, "cores": nt, "seconds": el,
                     "value": n ** w["ndim"] * 3 * steps / el, "unit": "cell-stage updates/s"})
    return runs


def nodes_of(w):
    return w["n"] ** w["ndim"]


def profiled_kinds(fp, G, S, met, qg, work, dt, steps, bcs=None, t=0.0, vwork=None):
    """mean duration (ms) per launch kind over `steps` instrumented RK3 steps
    (fp_profile_step: every launch of the step followed by a HIP event)"""
    acc = {}
    for i in range(max(1, steps)):
        for kind, ms in fp.profile_step(G, S, met, qg, work, dt, bcs=bcs, t=t + i * dt, vwork=vwork):
            acc.setdefault(kind, []).append(ms)
    return {k: sum(v) / len(v) for k, v in acc.items()}


def c4_inputs(w):
    """coordinates and states of the 48 O-grid blocks (host arrays)"""
    from paper_2101_05886_amd import inputs as I
    g, Y = 3, w["Y"]
    out = []
    for spec in I.multiblock_specs(w["blocks"], seed=w["seed"]):
        xyz = I.ogrid_sector_block(spec.n, g, Y, spec.sector, spec.skew_deg, spec.rotation)
        q = I.uniform_state(3, spec.n, g, 1.4, I.mach_velocity(w["mach"], [1.0, 0.0, 0.0]), 1.0)
        out.append((list(spec.n), xyz, q))
    return out, g


def cpu_baseline_blocks(w, blocks, g, budget_s=20.0):
    """FP64 oracle on the host: one RK3 step of as many of the blocks (in
    order) as fit in about budget_s seconds (at least one)."""
    import oracle as O
    sc = O.Scheme(w["recon"], w["Y"], True)

    def timed(limit):
        nodes = used = 0
        el = 0.0
        for n, xyz, q in blocks:
            og = O.Grid(3, n, g, bc=[1, 1, 1])
            met = O.metrics(og, w["Y"], xyz)
            dt = O.max_dt(og, sc, met, q, w["cfl"])
            t0 = time.perf_counter()
            O.rk3_step(og, sc, met, q, dt)
            el += time.perf_counter() - t0
            nodes += int(np.prod(n))
            used += 1
            if el > limit:
                break
        return nodes, used, el

    threads = O.num_threads()
    progress(f"cpu baseline: {threads} threads")
    nodes, used, el = timed(budget_s * 0.5)
    out = {"value": nodes * 3 / el, "unit": "cell-stage updates/s", "cores": threads, "kind": "oracle",
           "cpu_model": cpu_model(), "nproc": os.cpu_count(),
           "sample": f"one RK3 step of each of the first {used} of the {len(blocks)} blocks "
                     f"({nodes} nodes), FP64 oracle (gcc -O2, OpenMP over grid lines, {threads} threads), "
                     f"{el:.1f} s"}
    progress("cpu baseline: one thread")
    O.set_num_threads(1)
    try:
        nodes1, used1, el1 = timed(budget_s * 0.25)
    finally:
        O.set_num_threads(threads)
    out["single_thread"] = {"value": nodes1 * 3 / el1, "cores": 1,
                            "sample": f"one RK3 step of each of the first {used1} blocks ({nodes1} nodes), "
                                      f"one thread, {el1:.1f} s"}
    return out


def bench_dmr(args, w):
    """The double Mach reflection through fp_solve_bcs: every stage applies
    the boundary faces and reduces the global LF speeds before its sweeps."""
    import torch
    from paper_2101_05886_amd import fp
    from paper_2101_05886_amd import inputs as I
    g, Y, nx, ny = 3, w["Y"], w["nx"], w["ny"]
    xyz = I.dmr_grid(nx, ny, w["rand"], g, Y, w["seed"])
    nodes = I.state_nodes(xyz, g, Y)
    q = I.dmr_state(nodes, g)
    f = I.dmr_faces(nodes, g)
    dev = torch.device("cuda")
    G = fp.Grid(2, (nx, ny), g, bc=[fp.FP_BC_FROZEN, fp.FP_BC_FROZEN])
    S = fp.Scheme(w["recon"], Y, True, splitting="glf")
    met = fp.metrics(G, Y, torch.from_numpy(xyz).to(dev))
    bcs = fp.Bcs(f["kind"], mask={k: torch.from_numpy(v).to(dev) for k, v in f["mask"].items()},
                 nodes=torch.from_numpy(nodes).to(dev), pre=f["pre"], post=f["post"], normal=f["normal"],
                 offset=f["offset"], speed=f["speed"])
    qg = torch.from_numpy(q).to(dev)
    work = torch.zeros(G.work_shape(), dtype=torch.float64, device=dev)
    dt = float(fp.max_dt(G, S, met, qg, w["cfl"]).item())
    clock = {"t": 0.0}

    def run_bcs(k):
        fp.solve_bcs(G, S, bcs, met, qg, work, clock["t"], dt, k)
        clock["t"] += k * dt

    warmup = warm_up(run_bcs, args.warmup)
    t = clock["t"]
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    fp.solve_bcs(G, S, bcs, met, qg, work, t, dt, args.steps)
    e1.record()
    torch.cuda.synchronize()
    ms_total = e0.elapsed_time(e1)
    nodes_n = nx * ny
    value = nodes_n * 3 * args.steps / (ms_total * 1e-3)
    reps = [ms_total]
    for i in range(args.repeats - 1):
        e0.record()
        fp.solve_bcs(G, S, bcs, met, qg, work, t + (i + 1) * args.steps * dt, dt, args.steps)
        e1.record()
        torch.cuda.synchronize()
        reps.append(e0.elapsed_time(e1))
    t += (args.repeats - 1) * args.steps * dt
    healthy = int(fp.check_state(G, S, qg).item()) == 0
    # per-launch durations of instrumented steps of the same run (boundary
    # faces, global speeds and sweeps of every stage), after the timed region
    names = ["k_sweep_x", "k_sweep_wg<eta>"]
    t_end = t + args.steps * dt
    per_kind = profiled_kinds(fp, G, S, met, qg, work, dt, args.kernel_reps, bcs=bcs, t=t_end)
    kt = {d: per_kind[d] for d in range(2)}
    dom = max(kt, key=kt.get)
    # algorithmic units of one launch: the n_d + 1 faces of every line
    roof = roofline(w["recon"], 2, Y, "fp64", names[dom], kt[dom], faces_along([nx, ny], dom), nodes_n,
                    f"dmr/{names[dom]}")
    roof.update({"kernel_ms_by_dir": [round(kt[d], 4) for d in range(2)],
                 "glf_ms_per_stage": per_kind.get(5), "bc_faces_ms_per_stage": per_kind.get(6),
                 "sweeps_share_of_step": 3 * (kt[0] + kt[1]) / (ms_total / args.steps)})
    out = {
        "metric": "cell-stage updates/s", "value": value, "unit": "cell-stage updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": warmup, "ms_per_step": ms_total / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w["name"], "nodes": nodes_n, "metric_order": Y, "recon": w["recon"],
                   "precision": "fp64", "splitting": "glf", "dt": dt},
        "roofline": roof,
        "repeats": median_rate(reps, nodes_n * 3 * args.steps),
        "state_ok": healthy,
    }
    if not args.no_cpu_baseline:
        import oracle as O
        og = O.Grid(2, (nx, ny), g, bc=[1, 1])
        ob = O.Bcs(f["kind"], mask=f["mask"], nodes=nodes, pre=f["pre"], post=f["post"], normal=f["normal"],
                   offset=f["offset"], speed=f["speed"])
        omet = O.metrics(og, Y, xyz)
        osc = O.Scheme(w["recon"], Y, True, splitting="glf")
        threads = O.num_threads()
        t0 = time.perf_counter()
        O.solve_bcs(og, osc, ob, omet, q, 0.0, dt, 2)
        el = time.perf_counter() - t0
        O.set_num_threads(1)
        try:
            t0 = time.perf_counter()
            O.solve_bcs(og, osc, ob, omet, q, 0.0, dt, 1)
            el1 = time.perf_counter() - t0
        finally:
            O.set_num_threads(threads)
        out["cpu_baseline"] = {"value": nodes_n * 3 * 2 / el, "unit": "cell-stage updates/s",
                               "cores": threads, "kind": "oracle", "cpu_model": cpu_model(),
                               "nproc": os.cpu_count(),
                               "sample": f"2 RK3 steps of the same grid and state with its boundary faces, "
                                         f"FP64 oracle ({threads} threads), {el:.1f} s",
                               "single_thread": {"value": nodes_n * 3 / el1, "cores": 1,
                                                 "sample": f"one RK3 step, one thread, {el1:.1f} s"}}
    print(json.dumps(out), flush=True)


def bench_links(args, w):
    """One periodic grid cut into linked blocks, advanced by the batched path:
    before every stage the interface exchange fills each block's linked ghost
    slabs from its neighbour's stage register."""
    import torch
    from paper_2101_05886_amd import fp

    xyz, q, g = make_inputs(w)
    n, Y, cuts = w["n"], w["Y"], w["cuts"]
    gc = g + Y // 2
    sizes = [n // c for c in cuts]
    dev = torch.device("cuda")
    sc = fp.Scheme(w["recon"], Y, True, precision=w["prec"])
    ent, index = [], {}
    for c in np.ndindex(*cuts):
        lo = [c[d] * sizes[d] for d in range(3)]
        sl_x = (slice(None),) + tuple(slice(lo[d], lo[d] + sizes[d] + 2 * gc) for d in reversed(range(3)))
        sl_q = (slice(None),) + tuple(slice(lo[d], lo[d] + sizes[d] + 2 * g) for d in reversed(range(3)))
        G = fp.Grid(3, sizes, g, bc=[fp.FP_BC_FROZEN] * 3)
        met = fp.metrics(G, Y, torch.from_numpy(np.ascontiguousarray(xyz[sl_x])).to(dev))
        qg = torch.from_numpy(np.ascontiguousarray(q[sl_q])).to(dev)
        work = torch.zeros(G.work_shape(), dtype=torch.float64, device=dev)
        index[c] = len(ent)
        ent.append([G, met, qg, work, 0.0])
    dt = min(float(fp.max_dt(e[0], sc, e[1], e[2], w["cfl"]).item()) for e in ent)
    for e in ent:
        e[4] = dt
    links = []
    for c, i in index.items():
        for d in range(3):
            for side in (0, 1):
                nb = list(c)
                nb[d] = (c[d] + (1 if side else -1)) % cuts[d]
                links.append((i, d, side, index[tuple(nb)]))
    b = fp.Batch(sc, len(ent))
    b.set([tuple(e) for e in ent])
    b.set_links(links)
    seg = b.autotune()
    tiles = b.tiles()
    warmup = warm_up(b.solve, args.warmup)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    b.solve(args.steps)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    nodes = n ** 3
    value = nodes * 3 * args.steps / (ms * 1e-3)
    reps = [ms]
    for _ in range(args.repeats - 1):
        e0.record()
        b.solve(args.steps)
        e1.record()
        torch.cuda.synchronize()
        reps.append(e0.elapsed_time(e1))
    healthy = all(int(fp.check_state(e[0], sc, e[2]).item()) == 0 for e in ent)
    kinds = {}
    for _, kind, t in b.profile_step():
        kinds.setdefault(kind, []).append(t)
    pk = {k: sum(v) / len(v) for k, v in kinds.items()}
    b.close()
    names = {0: "kb_sweep_x", 1: "kb_sweep_wg<eta>", 2: "kb_sweep_wg<zeta>", 3: "kb_frozen_ghosts",
             4: "kb_halo"}
    dom = max((k for k in pk if k < 3), key=pk.get)
    faces = len(ent) * faces_along(sizes, dom)
    roof = roofline(w["recon"], 3, Y, w["prec"], names[dom], pk[dom], faces, nodes, f"c3x8/{names[dom]}")
    roof["kernel_ms_by_kind"] = {names[k]: round(v, 4) for k, v in sorted(pk.items())}
    # the exchange moves g ghost layers of every linked face: NV values read
    # from the neighbour and written into the block, FP64
    halo_bytes = len(links) * g * sizes[0] * sizes[1] * 5 * 8 * 2
    out = {
        "metric": "cell-stage updates/s", "value": value, "unit": "cell-stage updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": warmup, "ms_per_step": ms / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if w["prec"] == "fp64" else "f64 state, f32 reconstruction", "data": "synthetic",
        "config": {"workload": w["name"], "blocks": len(ent), "links": len(links), "nodes": nodes,
                   "metric_order": Y, "recon": w["recon"], "precision": w["prec"], "segment": seg, "tiles": tiles,
                   "dt": dt},
        "roofline": roof,
        "repeats": median_rate(reps, nodes * 3 * args.steps),
        "interfaces": {"kernel": "kb_halo", "ms_per_stage": pk.get(4), "bytes_per_stage": halo_bytes,
                       "achieved_gbs": halo_bytes / (pk[4] * 1e-3) / 1e9 if pk.get(4) else None,
                       "peak_gbs": PEAK_HBM_GBS},
        "state_ok": healthy,
    }
    if not args.no_cpu_baseline:
        progress("cpu baseline (FP64 oracle, the undivided grid)")
        cb = cpu_baseline(w, xyz, q, g)
        cb["sample"] += " (the undivided grid: the linked blocks reproduce its arithmetic node for node)"
        out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)


def bench_batch(args, w):
    import torch
    from paper_2101_05886_amd import fp

    blocks, g = c4_inputs(w)
    dev = torch.device("cuda")
    nodes = sum(int(np.prod(n)) for n, _, _ in blocks)
    res = {}
    per_kernel = {}
    for prec in ("fp64", "mixed"):
        sc = fp.Scheme(w["recon"], w["Y"], True, precision=prec)
        ent = []
        for n, xyz, q in blocks:
            G = fp.Grid(3, n, g, bc=[1, 1, 1])
            met = fp.metrics(G, w["Y"], torch.from_numpy(xyz).to(dev))
            qg = torch.from_numpy(q).to(dev)
            work = torch.zeros(G.work_shape(), dtype=torch.float64, device=dev)
            dt = float(fp.max_dt(G, sc, met, qg, w["cfl"]).item())
            ent.append((G, met, qg, work, dt))
        b = fp.Batch(sc, len(ent))
        b.set(ent)
        seg = b.autotune()
        tiles = b.tiles()
        warmup = warm_up(b.solve, args.warmup)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.solve(args.steps)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        reps = [ms]
        for _ in range(args.repeats - 1):
            e0.record()
            b.solve(args.steps)
            e1.record()
            torch.cuda.synchronize()
            reps.append(e0.elapsed_time(e1))
        flag_ok = True
        for G, met, qg, work, dt in ent:
            flag_ok = flag_ok and int(fp.check_state(G, sc, qg).item()) == 0
        # per-launch durations of one instrumented step (HIP events on the
        # stream the batched kernels run on)
        prof = b.profile_step()
        kinds = {}
        for ndim, kind, t in prof:
            kinds.setdefault(kind, []).append(t)
        per_kernel[prec] = {k: sum(v) / len(v) for k, v in kinds.items()}
        res[prec] = dict(value=nodes * 3 * args.steps / (ms * 1e-3), ms_step=ms / args.steps, seg=seg,
                         ok=flag_ok, repeats=median_rate(reps, nodes * 3 * args.steps), tiles=tiles,
                         warmup=warmup)
        progress(f"batch {prec}: {res[prec]['value']:.3e} cell-stage/s (segment {seg})")
        b.close()
        del ent
        torch.cuda.empty_cache()
    names = {0: "kb_sweep_x", 1: "kb_sweep_wg<eta>", 2: "kb_sweep_wg<zeta>", 3: "kb_frozen_ghosts",
             4: "kb_halo"}
    pk = per_kernel["mixed"]
    dom = max((k for k in pk if k < 3), key=pk.get)
    faces = sum(faces_along(n, dom) for n, _, _ in blocks)
    roof = roofline(w["recon"], 3, w["Y"], "mixed", names[dom], pk[dom], faces, nodes, f"c4/{names[dom]}")
    roof["kernel_ms_by_kind"] = {names[k]: round(v, 4) for k, v in sorted(pk.items())}
    pk64 = per_kernel["fp64"]
    dom64 = max((k for k in pk64 if k < 3), key=pk64.get)
    roof64 = roofline(w["recon"], 3, w["Y"], "fp64", names[dom64], pk64[dom64],
                      sum(faces_along(n, dom64) for n, _, _ in blocks), nodes, f"c4fp64/{names[dom64]}")
    roof64["kernel_ms_by_kind"] = {names[k]: round(v, 4) for k, v in sorted(pk64.items())}
    value = res["mixed"]["value"]
    stage_gbs = STAGE_BYTES[3] * value / 1e9
    out = {
        "metric": "cell-stage updates/s", "value": value, "unit": "cell-stage updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": res["mixed"]["warmup"], "ms_per_step": res["mixed"]["ms_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64 state, f32 reconstruction", "data": "synthetic",
        "config": {"workload": w["name"], "blocks": len(blocks), "nodes": nodes, "metric_order": w["Y"],
                   "recon": w["recon"], "precision": "mixed", "segment": res["mixed"]["seg"],
                   "tiles": res["mixed"]["tiles"]},
        "fp64": {"value": res["fp64"]["value"], "ms_per_step": res["fp64"]["ms_step"], "warmup": res["fp64"]["warmup"],
                 "segment": res["fp64"]["seg"], "tiles": res["fp64"]["tiles"], "repeats": res["fp64"]["repeats"],
                 "roofline": roof64},
        "mixed_over_fp64": value / res["fp64"]["value"],
        "repeats": res["mixed"]["repeats"],
        "roofline": roof,
        "hbm_stage": with_copy({"bytes_per_cell_stage": STAGE_BYTES[3], "achieved": stage_gbs,
                                "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": stage_gbs / PEAK_HBM_GBS}),
        "state_ok": res["mixed"]["ok"] and res["fp64"]["ok"],
    }
    if not args.no_serving:
        out["serving"] = serve_measure(WORKLOADS["c5"])
    if not args.no_cpu_baseline:
        progress("cpu baseline (FP64 oracle)")
        out["cpu_baseline"] = cpu_baseline_blocks(w, blocks, g)
    print(json.dumps(out), flush=True)


def progress(msg):
    print(f"bench: {msg}", file=sys.stderr, flush=True)


WARMUP_S = 0.3


def warm_up(run, requested):
    """Untimed steps before the timed region: `requested` of them, or (when
    none is requested) at least three and about WARMUP_S seconds of them, so
    that a workload of short steps starts its timed region with the GPU out
    of its idle clocks.  run(k) enqueues k steps.  Returns the steps run."""
    import torch
    if requested is not None:
        run(max(requested, 1))
        torch.cuda.synchronize()
        return requested
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    run(3)
    e1.record()
    e1.synchronize()
    per_step = max(e0.elapsed_time(e1) / 3, 1e-3) * 1e-3
    extra = max(0, math.ceil(WARMUP_S / per_step) - 3)
    if extra:
        run(extra)
    torch.cuda.synchronize()
    return 3 + extra


def serve_measure(w):
    """The serving stream: closed-loop capacity on the first requests, then
    the open-loop Poisson stream at w['load'] x that capacity."""
    import torch
    from paper_2101_05886_amd import fp
    from paper_2101_05886_amd import serve as S

    sc = fp.Scheme(w["recon"], w["Y"], True, precision=w["prec"])
    free, total = torch.cuda.mem_get_info()
    budget = int(0.85 * total) - (8 << 30)

    def run(reqs):
        be = S.GpuBackend(sc, w["slots"])
        try:
            st, _ = S.Scheduler(be, budget, w["slots"], w["round_steps"]).run(reqs)
        finally:
            be.close()
        return st

    # closed loop (all requests at t = 0) on the first requests of the
    # stream: the capacity the open-loop arrival rate is scaled from
    closed = run(S.make_requests(w["capacity_requests"], seed=w["seed"], rate=None))
    cap = closed.summary()["requests_per_s"]
    rate = w["load"] * cap
    progress(f"serving: closed-loop capacity {cap:.2f} requests/s; open loop at {rate:.2f}/s")
    st = run(S.make_requests(w["requests"], seed=w["seed"], rate=rate))
    s = st.summary()
    progress(f"serving: {s['requests']} requests, p50 {s['p50_latency_s']:.2f} s, p99 {s['p99_latency_s']:.2f} s")
    # the same stream (its first requests) at lighter and heavier load
    loads = []
    for load in sorted(set(w.get("other_loads", ())) | {w["load"]}):
        if load == w["load"]:
            o, count = s, w["requests"]
        else:
            count = w["other_requests"]
            o = run(S.make_requests(count, seed=w["seed"], rate=load * cap)).summary()
            progress(f"serving at {load}x: p50 {o['p50_latency_s']:.2f} s, p99 {o['p99_latency_s']:.2f} s")
        loads.append({"load": load, "requests": count, "arrival_rate_per_s": load * cap,
                      "p50_latency_s": o["p50_latency_s"], "p99_latency_s": o["p99_latency_s"],
                      "mean_queue_wait_s": o["mean_queue_wait_s"], "requests_per_s": o["requests_per_s"],
                      "cell_stage_per_s": o["cell_stage_per_s"], "peak_active": o["peak_active"]})
    return {"workload": w["name"], "requests": w["requests"], "slots": w["slots"],
            "round_steps": w["round_steps"], "hbm_budget_bytes": budget,
            "cell_stage_per_s": s["cell_stage_per_s"],
            "p50_latency_s": s["p50_latency_s"], "p99_latency_s": s["p99_latency_s"],
            "requests_per_s": s["requests_per_s"], "mean_queue_wait_s": s["mean_queue_wait_s"],
            "arrival_rate_per_s": rate, "closed_loop_capacity_per_s": cap,
            "closed_loop_cell_stage_per_s": closed.summary()["cell_stage_per_s"],
            "makespan_s": s["makespan_s"], "rounds": s["rounds"], "peak_active": s["peak_active"],
            "peak_bytes": s["peak_bytes"], "by_load": loads}


def bench_serve(args, w):
    sv = serve_measure(w)
    out = {
        "metric": "cell-stage updates/s", "value": sv["cell_stage_per_s"], "unit": "cell-stage updates/s",
        "n_gpus": 1, "steps": 200, "warmup": 0, "ms_per_step": None,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64 state, f32 reconstruction", "data": "synthetic",
        "config": {"workload": w["name"], "requests": w["requests"], "slots": w["slots"],
                   "round_steps": w["round_steps"], "hbm_budget_bytes": sv["hbm_budget_bytes"]},
        "serving": sv,
    }
    print(json.dumps(out), flush=True)


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


def copy_bandwidth():
    """Achievable HBM bandwidth on this GPU: a plain device copy of 1 GiB
    (read + write), five launches timed with HIP events; the median."""
    import torch
    src = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    times = []
    for _ in range(5):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
    del src, dst
    torch.cuda.empty_cache()
    ms = sorted(times)[len(times) // 2]
    return 2 * COPY_BYTES / (ms * 1e-3) / 1e9


def with_copy(hbm):
    """hbm_stage plus the measured copy bandwidth it can be read against"""
    gbs = copy_bandwidth()
    hbm["copy_gbs"] = gbs
    hbm["frac_of_copy"] = hbm["achieved"] / gbs
    return hbm


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=None,
                    help="untimed steps before the timed region (default: at least 3 and about "
                         f"{WARMUP_S} s of steps)")
    ap.add_argument("--workload", default="c4", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serving", action="store_true",
                    help="batched workload only: skip the serving stream reported beside it")
    ap.add_argument("--kernel-reps", type=int, default=10)
    ap.add_argument("--repeats", type=int, default=5,
                    help="timed regions of --steps steps: the first gives `value`, all of them the "
                         "median in `repeats`")
    ap.add_argument("--n", type=int, default=None,
                    help="single-block workloads only: nodes per axis instead of the workload's own "
                         "(a size sweep; the workload's configuration is the default)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of 1 GiB five times (the reference "
                         "kernel that scales the FETCH_SIZE / WRITE_SIZE counters to bytes)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(the design notes describe how the method would shard)", file=sys.stderr)
        sys.exit(2)

    import torch

    if args.copy_calibration:
        copy_calibration(torch)
        return
    from paper_2101_05886_amd import fp

    w = WORKLOADS[args.workload]
    if args.n is not None:
        if "n" not in w or "cuts" in w:
            print("--n applies to the single-block workloads only", file=sys.stderr)
            sys.exit(2)
        w = dict(w, n=args.n, name=w["name"] + f" (resized to {args.n} nodes per axis)")
    if "blocks" in w:
        bench_batch(args, w)
        return
    if "requests" in w:
        bench_serve(args, w)
        return
    if "shock" in w:
        bench_dmr(args, w)
        return
    if "cuts" in w:
        bench_links(args, w)
        return
    xyz, q, g = make_inputs(w)
    ndim, n, Y = w["ndim"], w["n"], w["Y"]
    G = fp.Grid(ndim, n, g)
    mu = w.get("mu", 0.0)
    S = fp.Scheme(w["recon"], Y, True, precision=w["prec"], mu=mu, prandtl=w.get("prandtl", 0.72))
    # the inviscid scheme: the sweep kernels a viscous stage runs are its kernels
    SI = fp.Scheme(w["recon"], Y, True, precision=w["prec"])
    dev = torch.device("cuda")
    met = fp.metrics(G, Y, torch.from_numpy(xyz).to(dev))
    qg = torch.from_numpy(q).to(dev)
    work = torch.zeros(G.work_shape(), dtype=torch.float64, device=dev)
    dt = float(fp.max_dt(G, SI, met, qg, w["cfl"]).item())
    if mu > 0:
        vwork = fp.viscous_work(G)
        run = lambda k: fp.solve_ns(G, S, met, qg, work, vwork, dt, k)  # noqa: E731
    else:
        run = lambda k: fp.solve(G, S, met, qg, work, dt, k)  # noqa: E731

    # warmup (captures the step graph), then the timed region
    warmup = warm_up(run, args.warmup)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    run(args.steps)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_total = e0.elapsed_time(e1)
    ms_step = ms_total / args.steps
    nodes = n ** ndim
    value = nodes * 3 * args.steps / (ms_total * 1e-3)
    reps = [ms_total]
    for _ in range(args.repeats - 1):
        e0.record()
        run(args.steps)
        e1.record()
        torch.cuda.synchronize()
        reps.append(e0.elapsed_time(e1))

    # state sanity after the timed steps
    flag = fp.check_state(G, S, qg)
    torch.cuda.synchronize()
    healthy = int(flag.item()) == 0

    # per-launch durations of instrumented RK3 steps run right after the
    # timed region: the same launches the step graph replays, each followed
    # by a HIP event on the stream the kernels run on
    names = ["k_sweep_x", "k_sweep_wg<eta>", "k_sweep_wg<zeta>"]
    per_kind = profiled_kinds(fp, G, S, met, qg, work, dt, args.kernel_reps,
                              vwork=vwork if mu > 0 else None)
    kt = {d: per_kind[d] for d in range(ndim)}
    dom = max(kt, key=kt.get)
    viscous = None
    if mu > 0:
        # the viscous part of a stage (node fluxes, then their divergence)
        # against its algorithmic bytes per node: read q (nv) and the metrics
        # (ndim^2 + 1), write and read back the ndim (ndim + 1) contravariant
        # fluxes, write the residual (nv); FP64
        nv = ndim + 2
        vb = (nv + ndim * ndim + 1 + 2 * ndim * (ndim + 1) + nv) * 8
        vms = per_kind[7] + per_kind[8]
        viscous = {"kernels": "k_visc_flux3 + k_visc_div3" if ndim == 3 else "k_visc_flux + k_visc_div",
                   "ms_per_stage": vms, "fluxes_ms": per_kind[7], "divergence_ms": per_kind[8], "bytes_per_node": vb,
                   "achieved_gbs": vb * nodes_of(w) / (vms * 1e-3) / 1e9, "peak_gbs": PEAK_HBM_GBS}
    # algorithmic units of one launch: the n + 1 faces of every line
    roof = roofline(w["recon"], ndim, Y, w["prec"], names[dom], kt[dom], faces_along([n] * ndim, dom), nodes,
                    f"{args.workload}/{names[dom]}")
    roof["kernel_ms_by_dir"] = [round(kt[d], 4) for d in range(ndim)]
    stage_gbs = STAGE_BYTES[ndim] * value / 1e9
    out = {
        "metric": "cell-stage updates/s", "value": value, "unit": "cell-stage updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if w["prec"] == "fp64" else "f64 state, f32 reconstruction",
        "data": "synthetic",
        "config": {"workload": w["name"], "nodes": nodes, "metric_order": Y,
                   "recon": w["recon"], "precision": w["prec"], "dt": dt},
        "roofline": roof,
        "repeats": median_rate(reps, nodes * 3 * args.steps),
        "hbm_stage": with_copy({"bytes_per_cell_stage": STAGE_BYTES[ndim], "achieved": stage_gbs,
                                "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": stage_gbs / PEAK_HBM_GBS}),
        "wall_s": wall, "state_ok": healthy,
    }
    if mu > 0:
        out["config"].update({"mu": mu, "prandtl": w.get("prandtl", 0.72)})
        out["viscous"] = viscous
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, xyz, q, g)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
