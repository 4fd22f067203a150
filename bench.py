#!/usr/bin/env python3
"""Throughput benchmark of the DSMC hot path on one MI355X.

A step is one pass of the whole hot path (move with body force and diffuse
walls, stable counting sort by collision cell, NTC collisions, FP64 moment
sampling) over every particle of the workload.  The default workload is the
single-instance FP32-velocity / FP64-accumulator channel at Kn = 0.1 with 300
cells x 1000 particles per cell (3e5 particles), inputs resident in HBM.  The
timed steps are sampling steps (the warm-up steps are the transient).

Prints one JSON line: particle-steps/s, the roofline of the dominant kernel
(its algorithmic bytes over its average duration from HIP events on the
library's stream), the plain FP64 deterministic path on the same workload, and
the CPU oracle timed on this host for a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = ("particle-steps/s at fixed moment accuracy (FP32 batched vs FP64 plain); "
          "p50/p99 solve latency")


def kernel_bytes(phase: str, N: int, Cc: int, rb: int, coll_frac: float, sampling: bool) -> float:
    """Algorithmic HBM bytes of one launch of a phase kernel: the particle
    record and per-cell traffic the method itself must move (library tables
    such as per-tile histograms are not counted)."""
    if phase == "move_hist":   # read y, v; write y, vx and the cell index
        return N * (4 * rb + 2 * rb + 4)
    if phase == "scatter":     # read cell + record, write the record
        return N * (4 + 4 * rb + 4 * rb)
    if phase == "collide":     # read v, write the collided particles' v; cell tables
        b = N * 3 * rb + coll_frac * N * 3 * rb + Cc * (8 + 8 + 4 + 4 + 4)
        if sampling:
            b += Cc * 12 * 8 * 2
        return b
    if phase == "scan":
        return Cc * 4 * 2
    return 0.0


PROFILE_TAGS = {"cfg1": "kernels_cfg1_kn0.1_300x1000_fp32"}


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in ("kernels.hip", "rng.hpp", "common.hpp"):
        with open(os.path.join(ROOT, "paper_2311_14140_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload: str, kernel: str):
    """Copy-calibrated HBM bytes per launch of a kernel from the committed
    rocprofv3 counter summary, or None when there is none or the kernels have
    changed since the counters were taken."""
    import json as _json
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    tag = PROFILE_TAGS.get(workload)
    if not tag or not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = _json.load(fh).get(tag)
    if not rec or rec.get("kernel_source_hash") != kernel_source_hash():
        return None
    return rec["bytes_per_launch"].get(kernel)


def cpu_oracle_rate(params, seconds: float):
    import oracle
    o = oracle.Oracle(params)
    steps = 0
    t0 = time.perf_counter()
    while True:
        o.step(2)
        steps += 2
        el = time.perf_counter() - t0
        if el >= seconds:
            break
    return o.N * steps / el, steps, el


def _timed(torch, step, sync, n):
    sync()
    torch.cuda.synchronize()
    t = time.perf_counter()
    step(n)
    sync()
    torch.cuda.synchronize()
    return time.perf_counter() - t


def time_single(dsmc, torch, p, steps):
    """particle-steps/s of one instance (sampling steps, graph-replayed)."""
    p = p.with_(n_transient=4)
    with dsmc.Solver(p) as s:
        s.step(8)
        el = _timed(torch, s.step, s.sync, steps)
        prof = s.profile(4)
        return {"value": s.N * steps / el, "unit": "particle-steps/s", "particles": s.N,
                "steps": steps, "ms_per_step": 1e3 * el / steps,
                "workload": f"Kn={p.kn}, F={p.body_force}, {p.n_cells} cells x "
                            f"{p.particles_per_cell}/cell, n_sub={p.n_sub}, FP32",
                "kernel_ms_per_step": {k: prof[k] / 4 for k in dsmc.Solver.PHASES}}


def time_batched(dsmc, torch, steps):
    """particle-steps/s of the 256-instance mix stepped as one group."""
    import synth
    ps = synth.config3_instances(256)
    g = dsmc.Group()
    sols = []
    for p in ps:
        s = dsmc.Solver(p.with_(n_transient=4))
        g.add(s)
        sols.append(s)
    N = sum(s.N for s in sols)
    g.step(8)
    el = _timed(torch, g.step, g.sync, steps)
    prof = sols[0].profile(4)
    out = {"value": N * steps / el, "unit": "particle-steps/s", "particles": N,
           "instances": len(sols), "steps": steps, "ms_per_step": 1e3 * el / steps,
           "workload": "256 instances: Kn log-uniform [0.05, 10], F uniform [0.001, 0.02], "
                       "cells uniform [50, 2000], particles/cell uniform [20, 200], FP32",
           "kernel_ms_per_step": {k: prof[k] / 4 for k in dsmc.Solver.PHASES}}
    g.close()
    for s in sols:
        s.close()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--workload", default="cfg1", choices=["cfg0", "cfg1", "cfg2"])
    ap.add_argument("--profile-steps", type=int, default=100)
    ap.add_argument("--fp64-steps", type=int, default=40)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the large-instance and batched-mix measurements")
    ap.add_argument("--extra-steps", type=int, default=20)
    ap.add_argument("--copy-mib", type=int, default=256,
                    help="size of the plain device copy run after the timed region, whose "
                         "HBM counters calibrate the kernels' (0 = skip)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: this build runs a single instance or group on one "
              "MI355X and has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2311_14140_amd import dsmc
    from synth import WORKLOADS, FP64_DETERMINISTIC

    torch.cuda.set_device(0)
    base, _ = WORKLOADS[args.workload]
    p = base.with_(n_transient=args.warmup)
    rb = 4 if p.precision == dsmc.DSMC_FP32_FAST else 8
    s = dsmc.Solver(p)
    N, Cc = s.N, s.Cc
    print(f"# workload {args.workload}: N={N} cells={p.n_cells} n_sub={p.n_sub} "
          f"precision={p.precision} warmup={args.warmup} steps={args.steps}",
          file=sys.stderr, flush=True)
    s.step(args.warmup)
    s.sync()
    s.sample(reset=True)

    # ---- timed region: K steps, graph-replayed, inputs resident in HBM
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(args.steps)
    s.sync()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    el = t1 - t0
    rate = N * args.steps / el
    est = s.sample(reset=True)
    coll_frac = 2.0 * est["n_collisions"] / (N * args.steps)
    print(f"# timed {args.steps} steps in {el:.4f} s: {rate:.4e} particle-steps/s; "
          f"mass flow {est['mass_flow']:.6f}", file=sys.stderr, flush=True)

    # ---- per-kernel durations: HIP events around every kernel on the
    # library's stream, over separately launched steps of the same run
    prof = s.profile(args.profile_steps)
    kern = {k: prof[k] / args.profile_steps for k in dsmc.Solver.PHASES}
    dom = max(kern, key=kern.get)
    dom_bytes = kernel_bytes(dom, N, Cc, rb, coll_frac, True)
    achieved = dom_bytes / (kern[dom] * 1e-3) / 1e9
    step_bytes = sum(kernel_bytes(k, N, Cc, rb, coll_frac, True) for k in kern)
    print("# per-kernel ms/step: " + ", ".join(f"{k}={v:.4f}" for k, v in kern.items()),
          file=sys.stderr, flush=True)
    s.close()

    # ---- the plain FP64 deterministic path on the same workload
    fp64 = None
    if args.fp64_steps > 0:
        q = base.with_(n_transient=0, precision=FP64_DETERMINISTIC)
        with dsmc.Solver(q) as d:
            d.step(2)
            d.sync()
            torch.cuda.synchronize()
            a = time.perf_counter()
            d.step(args.fp64_steps)
            d.sync()
            b = time.perf_counter()
        fp64 = {"value": N * args.fp64_steps / (b - a), "unit": "particle-steps/s",
                "steps": args.fp64_steps, "dtype": "f64",
                "note": "sequential-per-cell NTC, bit-identical to the oracle"}

    # ---- other workloads of the same hot path, timed the same way
    extra = {}
    if not args.no_extra:
        extra["cfg2_large_instance"] = time_single(dsmc, torch, WORKLOADS["cfg2"][0].with_(
            n_sub=2), args.extra_steps)
        extra["cfg3_batched_256"] = time_batched(dsmc, torch, args.extra_steps)

    # a plain copy of known size (outside the timed region): what the
    # FETCH_SIZE / WRITE_SIZE counters read for it calibrates the kernels'
    if args.copy_mib > 0:
        n = args.copy_mib * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    cpu = None
    if not args.no_cpu_baseline:
        cq = base.with_(precision=FP64_DETERMINISTIC)
        r, st, sec = cpu_oracle_rate(cq, args.cpu_seconds)
        cpu = {"value": r, "unit": "particle-steps/s", "cores": 1, "kind": "oracle",
               "sample": f"{st} steps of the same {N}-particle instance from its initial "
                         f"state, FP64, one thread, {sec:.1f} s"}

    line = {
        "metric": METRIC,
        "value": rate,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * el / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if rb == 4 else "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: Kn={p.kn}, F={p.body_force}, "
                               f"{p.n_cells} cells x {p.particles_per_cell} particles/cell, "
                               f"n_sub={p.n_sub}, FP32 velocities + FP64 accumulators"
                   if rb == 4 else f"{args.workload}", "particles": N,
                   "collision_cells": Cc, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(args.workload, dom), "kernel_ms": kern[dom],
                     "algorithmic_bytes_per_launch": dom_bytes},
        "step_roofline": {"algorithmic_bytes_per_step": step_bytes,
                          "achieved_GBps": step_bytes / (el / args.steps) / 1e9,
                          "frac": step_bytes / (el / args.steps) / 1e9 / HBM_PEAK_GBS},
        "kernel_ms_per_step": kern,
        "fp64_plain": fp64,
        "cpu_baseline": cpu,
        "mass_flow": est["mass_flow"],
        "other_workloads": extra,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
