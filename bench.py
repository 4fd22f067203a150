#!/usr/bin/env python3
"""Throughput benchmark of the DSMC hot path on one MI355X.

A step is one pass of the whole hot path (move with body force and diffuse
walls, stable counting sort by collision cell, NTC collisions, FP64 moment
sampling) over every particle of the workload.  The default workload is the
batched mix: 256 independent force-driven channel instances (Kn log-uniform
in [0.05, 10], force uniform in [0.001, 0.02], 50..2000 cells, 20..200
particles per cell; 2.6e7 particles in all) in FP32 velocities with FP64
moment accumulators, stepped as one group with graph-replayed steps and
inputs resident in HBM.  The timed steps are sampling steps (the warm-up
steps are the transient).

Prints one JSON line: particle-steps/s, the roofline of the dominant kernel
(its algorithmic bytes over its average duration from HIP events on the
library's stream), the plain FP64 path (each instance alone, sequential
per-cell NTC) on the same instances, the served request stream (p50/p99 time
from arrival to moments on the host, FP32 batched against plain FP64), the
single-instance workloads, and the CPU oracle timed on this host for a
bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = ("particle-steps/s at fixed moment accuracy (FP32 batched vs FP64 plain); "
          "p50/p99 solve latency")
MIX_DESC = ("256 instances: Kn log-uniform [0.05, 10], F uniform [0.001, 0.02], "
            "cells uniform [50, 2000], particles/cell uniform [20, 200]")


def kernel_bytes(phase: str, N: int, Cc: int, rb: int, coll_frac: float, sampling: bool,
                 bucketed: bool) -> float:
    """Algorithmic HBM bytes of one launch of a phase kernel: the particle
    record and per-cell traffic its part of the method must move (library
    tables such as per-tile histograms are not counted).  rb is the bytes of
    a real; a record is y, vx, vy, vz."""
    if phase == "count":         # position-only flight: read y, vy
        return N * 2 * rb
    if phase == "move_scatter":  # read the record, write it moved to its sorted slot
        return N * 8 * rb
    if phase == "collide":
        if bucketed:             # finishes the sort: read and write the whole record
            b = N * 8 * rb
        else:                    # read v, write v back
            b = N * 6 * rb
        b += Cc * (8 + 8 + 4 + 4 + 4)  # crmax, rem, count, offset, collisions
        if sampling:             # thirteen FP64 sums per cell, read and written
            b += Cc * 13 * 8 * 2
        return b
    if phase == "scan":
        return Cc * 4 * 2
    return 0.0


PROFILE_TAGS = {"cfg1": "kernels_cfg1_kn0.1_300x1000_fp32",
                "cfg2": "kernels_cfg2_kn0.01_1000x20000_fp32",
                "cfg3": "kernels_cfg3_batched256_fp32"}


def kernel_source_hash() -> str:
    """Hash of the kernels and of the runtime that chooses their launch
    shapes: the committed counters hold only for the sources they were
    taken with."""
    from paper_2311_14140_amd.rocprof_summary import source_hash
    return source_hash()


def measured_traffic(workload: str, kernel: str):
    """Copy-calibrated HBM bytes per launch of a kernel from the committed
    rocprofv3 counter summary, or None when there is none or the kernels have
    changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    tag = PROFILE_TAGS.get(workload)
    if not tag or not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh).get(tag)
    if not rec or rec.get("kernel_source_hash") != kernel_source_hash():
        return None
    return rec["bytes_per_launch"].get(kernel)


class Subject:
    """The timed workload: one instance, or the batched mix as one group."""

    def __init__(self, dsmc, params_list):
        self.sols = [dsmc.Solver(p) for p in params_list]
        self.group = None
        if len(self.sols) > 1:
            self.group = dsmc.Group()
            for s in self.sols:
                self.group.add(s)
        self.N = sum(s.N for s in self.sols)
        self.Cc = sum(s.Cc for s in self.sols)

    def step(self, n):
        (self.group or self.sols[0]).step(n)

    def sync(self):
        (self.group or self.sols[0]).sync()

    def profile(self, n):
        # profiling a member of a group profiles the group's steps
        return self.sols[0].profile(n)

    def lanes(self):
        """(multi-kernel lanes, particles and collision cells in them): each
        multi-kernel phase of a step is launched once per such lane; members
        small enough run resident in a lane of their own."""
        if not self.group:
            return 1, self.N, self.Cc
        li = self.group.lane_info()
        return (li["lanes"] - li["resident_lanes"], self.N - li["resident_particles"],
                self.Cc - li["resident_cells"])

    def sample(self):
        return [s.sample(reset=True) for s in self.sols]

    def close(self):
        if self.group:
            self.group.close()
        for s in self.sols:
            s.close()


def _timed(torch, step, sync, n):
    sync()
    torch.cuda.synchronize()
    t = time.perf_counter()
    step(n)
    sync()
    torch.cuda.synchronize()
    return time.perf_counter() - t


def time_single(dsmc, torch, p, steps, label):
    """particle-steps/s of one instance (sampling steps, graph-replayed)."""
    p = p.with_(n_transient=4)
    with dsmc.Solver(p) as s:
        s.step(10)  # past the capture of the instance's step graph
        el = _timed(torch, s.step, s.sync, steps)
        prof = s.profile(4)
        return {"value": s.N * steps / el, "unit": "particle-steps/s", "particles": s.N,
                "steps": steps, "ms_per_step": 1e3 * el / steps,
                "workload": f"{label}: Kn={p.kn}, F={p.body_force}, {p.n_cells} cells x "
                            f"{p.particles_per_cell}/cell, n_sub={p.n_sub}, FP32",
                "kernel_ms_per_step": {k: prof[k] / 4 for k in dsmc.Solver.PHASES}}


def fp64_plain(dsmc, torch, params_list, steps):
    """The plain FP64 path: each instance alone, deterministic mode
    (sequential per-cell NTC, bit-identical to the oracle)."""
    from synth import FP64_DETERMINISTIC
    ps_total, el_total = 0, 0.0
    for p in params_list:
        with dsmc.Solver(p.with_(n_transient=0, precision=FP64_DETERMINISTIC)) as d:
            d.step(10)  # past the capture of the instance's step graph
            el_total += _timed(torch, d.step, d.sync, steps)
            ps_total += d.N * steps
    return {"value": ps_total / el_total, "unit": "particle-steps/s", "steps": steps,
            "instances": len(params_list), "dtype": "f64",
            "note": "each instance alone, sequential-per-cell NTC, bit-identical to the oracle"}


def fp64_fast_rates(dsmc, torch, plist, sample, steps):
    """The parallel-NTC scheme of the fast mode with FP64 state: the sampled
    instances each alone, and the whole workload as one group."""
    FP64_FAST = dsmc.DSMC_FP64_FAST
    ps_total, el_total = 0, 0.0
    for p in sample:
        with dsmc.Solver(p.with_(n_transient=0, precision=FP64_FAST)) as d:
            d.step(10)
            el_total += _timed(torch, d.step, d.sync, steps)
            ps_total += d.N * steps
    alone = {"value": ps_total / el_total, "unit": "particle-steps/s", "steps": steps,
             "instances": len(sample)}
    sols = [dsmc.Solver(p.with_(n_transient=0, precision=FP64_FAST)) for p in plist]
    g = dsmc.Group()
    try:
        for s in sols:
            g.add(s)
        g.step(16)
        el = _timed(torch, g.step, g.sync, steps)
        N = sum(s.N for s in sols)
    finally:
        g.close()
        for s in sols:
            s.close()
    batched = {"value": N * steps / el, "unit": "particle-steps/s", "steps": steps,
               "instances": len(plist), "ms_per_step": 1e3 * el / steps}
    return {"alone": alone, "batched": batched, "dtype": "f64",
            "note": "the fast mode's parallel NTC with FP64 positions and velocities"}


def serve(n_requests, rate_hz, precision, batched, budget):
    """Serve the first n requests of the Poisson trace; returns the summary."""
    import synth
    from paper_2311_14140_amd.serve import GpuExecutor, PlainGpuExecutor, Request, Server
    trace = synth.serving_trace(n_requests, rate_hz=rate_hz, precision=precision)
    reqs = [Request(i, t, p, steps) for i, (t, p, steps) in enumerate(trace)]
    if batched:
        ex = GpuExecutor()
        srv = Server(ex, budget_bytes=budget, max_slots=256, quantum=100)
    else:
        ex = PlainGpuExecutor()
        srv = Server(ex, budget_bytes=budget, max_slots=1, quantum=1000)
    _, summ = srv.run(reqs)
    if batched:
        ex.close()
    summ["rate_hz"] = rate_hz
    summ["mode"] = "FP32 batched (one group, up to 256 running)" if batched else \
        "FP64 plain (one solve at a time)"
    return summ


def cpu_oracle_rate(params_list, seconds: float):
    """The oracle stepping the given instances in turn, 2 steps at a time,
    for about ``seconds`` of stepping (set-up not timed)."""
    import oracle
    from synth import FP64_DETERMINISTIC
    orc = [oracle.Oracle(p.with_(precision=FP64_DETERMINISTIC)) for p in params_list]
    ps, el = 0, 0.0
    while el < seconds:
        for o in orc:
            t = time.perf_counter()
            o.step(2)
            el += time.perf_counter() - t
            ps += 2 * o.N
            if el >= seconds:
                break
    return ps / el, ps, el


def host_cores() -> int:
    """Cores this process may use, capped at 16 (the host share of one GPU)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def host_identity() -> dict:
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "usable_cores": host_cores(), "cpu_model": model}


def cpu_oracle_rate_all_cores(params_list, seconds: float, threads: int):
    """Aggregate oracle throughput on ``threads`` host cores: every thread
    steps its own independent instances (the oracle's C calls release the
    interpreter lock) for about ``seconds`` of wall time."""
    import threading
    import oracle
    from synth import FP64_DETERMINISTIC
    work = [[] for _ in range(threads)]
    for i, p in enumerate(params_list):
        work[i % threads].append(p)
    work = [w for w in work if w]
    orcs = [[oracle.Oracle(p.with_(precision=FP64_DETERMINISTIC)) for p in w] for w in work]
    done = [0] * len(orcs)
    t0 = time.perf_counter()
    stop = t0 + seconds

    def run(k):
        while time.perf_counter() < stop:
            for o in orcs[k]:
                o.step(2)
                done[k] += 2 * o.N
                if time.perf_counter() >= stop:
                    break

    ts = [threading.Thread(target=run, args=(k,)) for k in range(len(orcs))]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    el = time.perf_counter() - t0
    return sum(done) / el, sum(done), el, len(ts)


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--workload", default="cfg3", choices=["cfg0", "cfg1", "cfg2", "cfg3"])
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the automatic launch shape of the batched mix")
    ap.add_argument("--profile-steps", type=int, default=20)
    ap.add_argument("--fp64-steps", type=int, default=40)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the single-instance workloads and the served stream")
    ap.add_argument("--extra-steps", type=int, default=200)
    ap.add_argument("--serve-requests", type=int, default=2000,
                    help="requests of the Poisson trace served FP32-batched (2000 = the full trace)")
    ap.add_argument("--serve-plain-requests", type=int, default=40,
                    help="requests of the same trace served by the plain FP64 path")
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
    import synth
    from synth import WORKLOADS

    def log(msg):
        print("# " + msg, file=sys.stderr, flush=True)

    torch.cuda.set_device(0)
    tune_budget = 0 if (args.workload != "cfg3" or args.no_autotune) else 64
    if args.workload == "cfg3":
        plist = [p.with_(n_transient=args.warmup + tune_budget) for p in synth.config3_instances(256)]
        wdesc = f"cfg3: {MIX_DESC}, FP32 velocities + FP64 accumulators, one group"
    else:
        base, _ = WORKLOADS[args.workload]
        plist = [base.with_(n_transient=args.warmup)]
        wdesc = (f"{args.workload}: Kn={base.kn}, F={base.body_force}, {base.n_cells} cells x "
                 f"{base.particles_per_cell} particles/cell, n_sub={base.n_sub}")
    rb = 4 if plist[0].precision == dsmc.DSMC_FP32_FAST else 8
    sub = Subject(dsmc, plist)
    N, Cc = sub.N, sub.Cc
    log(f"workload {args.workload}: {len(plist)} instance(s), N={N}, collision cells={Cc}, "
        f"warmup={args.warmup} steps={args.steps}")
    tuning = None
    if tune_budget:
        t = time.perf_counter()
        tm, ppb, wpc = sub.group.autotune()
        # the tuner's steps are transient steps of the members: the warm-up
        # makes up the rest, so the timed steps are sampling steps
        small = min(range(len(sub.sols)), key=lambda i: sub.sols[i].N)
        done = sub.sols[small].get_state()[5]
        tuning = {"tile_mult": tm, "particles_per_block": ppb, "waves_per_cu": wpc,
                  "tuner_steps": done, "tuner_seconds": time.perf_counter() - t,
                  "searched": "tile_mult {1,2,4} x particles_per_block {auto,1024,4096} "
                              "at automatic occupancy, then waves_per_cu {8,12,16}"}
        log(f"autotuned: tile_mult={tm} particles_per_block={ppb} waves_per_cu={wpc} "
            f"({done} steps)")
        sub.step(max(0, args.warmup + tune_budget - done))
    else:
        sub.step(args.warmup)
    sub.sync()
    sub.sample()
    # one more graph chunk past the warm-up, right before the timed steps:
    # it replays the step graphs (captured when a group's lanes are built)
    # once, and keeps the device busy up to the timed region (after the
    # host-side window reads above, an idle device ran the first timed
    # steps some 5% slower)
    sub.step(8)
    sub.sync()

    # ---- timed region: K steps, graph-replayed, inputs resident in HBM
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sub.step(args.steps)
    sub.sync()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    rate = N * args.steps / el
    # the window holds the extra chunk and the timed steps
    est = sub.sample()
    n_coll = sum(e["n_collisions"] for e in est)
    coll_frac = 2.0 * n_coll / sum(s.N * e["n_sampled_steps"] for s, e in zip(sub.sols, est))
    log(f"timed {args.steps} steps in {el:.4f} s: {rate:.4e} particle-steps/s")

    # ---- per-kernel durations: HIP events around every kernel on the
    # library's stream, over separately launched steps of the same run
    prof = sub.profile(args.profile_steps)
    kern = {k: prof[k] / args.profile_steps for k in dsmc.Solver.PHASES}
    dom = max(kern, key=kern.get)
    bucketed = rb == 4 and all(p.particles_per_cell / p.n_sub < 256 for p in plist)
    # per launch: a step launches each kernel once per lane, on that lane's
    # share of the particles (the profiler's dispatches are these launches)
    lanes, n_multi, cc_multi = sub.lanes()
    resident_note = None
    dom_total_ms = kern[dom]
    if n_multi != N:
        # small members run resident in a lane of their own, whose whole step
        # is one kernel timed in the collide slot: the dominant kernel's
        # figures cover the multi-kernel lanes only
        resident_note = (f"{N - n_multi} particles of small members stepped resident in a lane "
                         f"of their own ({prof['resident'] / args.profile_steps:.4f} ms/step); "
                         f"per-launch figures cover the other {n_multi}")
        if dom == "collide":
            dom_total_ms -= prof["resident"] / args.profile_steps
    dom_bytes = kernel_bytes(dom, n_multi, cc_multi, rb, coll_frac, True, bucketed) / max(lanes, 1)
    dom_ms = dom_total_ms / max(lanes, 1)
    achieved = dom_bytes / (dom_ms * 1e-3) / 1e9
    step_bytes = sum(kernel_bytes(k, N, Cc, rb, coll_frac, True, bucketed) for k in kern)
    log("per-kernel ms/step: " + ", ".join(f"{k}={v:.4f}" for k, v in kern.items()))
    sub.close()

    # ---- the FP64 paths on the same instances (a sample of the mix): the
    # plain deterministic path (sequential per-cell NTC), and the parallel NTC
    # of the fast mode in FP64, alone and as one group
    fp64 = fp64_fast = None
    if args.fp64_steps > 0:
        sample = plist[::16]
        fp64 = fp64_plain(dsmc, torch, sample, args.fp64_steps)
        fp64["sample"] = f"{len(sample)} instances (every 16th), {args.fp64_steps} steps each" \
            if len(plist) > 1 else "the same instance"
        log(f"fp64 plain: {fp64['value']:.4e} particle-steps/s")
        fp64_fast = fp64_fast_rates(dsmc, torch, plist, sample, args.fp64_steps)
        log(f"fp64 fast: alone {fp64_fast['alone']['value']:.4e}, "
            f"batched {fp64_fast['batched']['value']:.4e} particle-steps/s")

    # ---- other workloads of the same hot path, and the served stream
    extra, serving = {}, None
    if not args.no_extra:
        extra["cfg1_single_instance"] = time_single(dsmc, torch, WORKLOADS["cfg1"][0],
                                                    args.extra_steps, "cfg1")
        log(f"cfg1: {extra['cfg1_single_instance']['value']:.4e}")
        extra["cfg2_large_instance"] = time_single(dsmc, torch, WORKLOADS["cfg2"][0],
                                                   max(2, args.extra_steps // 10), "cfg2")
        log(f"cfg2: {extra['cfg2_large_instance']['value']:.4e}")
        from paper_2311_14140_amd.hybrid import time_patch_group
        for resident in (True, False):
            t = time_patch_group(0.1, True, replicas=64, steps=2000, profile_steps=4,
                                 resident=resident)
            key = "hybrid_patches_kn0.1_" + ("resident" if resident else "multi_kernel")
            extra[key] = {"value": t["particle_steps_per_s"], "unit": "particle-steps/s",
                          "particles": t["particles"], "ms_per_step": t["ms_per_step"],
                          "workload": "64 open patches of the MMS hybrid at Kn 0.1 (45 cells x 50/cell, "
                                      "Chapman-Enskog inflow), FP32, one group"}
            log(f"{key}: {t['particle_steps_per_s']:.4e}")
        if args.serve_requests > 0:
            free, _ = torch.cuda.mem_get_info()
            budget = int(0.8 * free)
            fp32 = serve(args.serve_requests, 200.0, synth.FP32_FAST, True, budget)
            log(f"served FP32 batched ({args.serve_requests} requests at 200/s): "
                f"p50 {fp32['p50_s']:.3f} s, p99 {fp32['p99_s']:.3f} s")
            plain = None
            if args.serve_plain_requests > 0:
                plain = serve(args.serve_plain_requests, 200.0, synth.FP64_DETERMINISTIC, False,
                              budget)
                log(f"served FP64 plain ({args.serve_plain_requests} requests): "
                    f"p50 {plain['p50_s']:.3f} s, p99 {plain['p99_s']:.3f} s")
            # capacity: requests/s the batched path sustains, from the
            # saturated run's throughput and the mean work of a request
            per_req = fp32["particle_steps"] / max(1, fp32["served"])
            cap = fp32["throughput"] / per_req
            low = serve(args.serve_requests, 0.7 * cap, synth.FP32_FAST, True, budget)
            log(f"served FP32 at 0.7 capacity ({0.7 * cap:.1f}/s): p50 {low['p50_s']:.3f} s, "
                f"p99 {low['p99_s']:.3f} s")
            serving = {"trace": f"Poisson trace (PCG64 seeds 4 and 40), parameters from the "
                                f"batched-mix distribution, transient per Kn + 5000 sampling "
                                f"steps each; FP32 batched: the first {args.serve_requests} "
                                f"requests; FP64 plain: the first {args.serve_plain_requests}",
                       "budget_bytes": budget, "capacity_req_per_s": cap,
                       "fp32_batched": fp32, "fp64_plain": plain,
                       "fp32_batched_0.7_capacity": low}

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
        sample = plist[::16]
        host = host_identity()
        r1, ps1, sec1 = cpu_oracle_rate(sample, args.cpu_seconds)
        log(f"cpu oracle, one core: {r1:.4e} particle-steps/s")
        # every core: the whole mix, instances dealt to the threads
        rn, psn, secn, used = cpu_oracle_rate_all_cores(plist, args.cpu_seconds, host["usable_cores"])
        log(f"cpu oracle, {used} cores: {rn:.4e} particle-steps/s")
        cpu = {"value": rn, "unit": "particle-steps/s", "cores": used, "kind": "oracle",
               "sample": f"{psn} particle-steps in {secn:.1f} s: the {len(plist)} instance(s) of "
                         f"the workload dealt to {used} threads, each stepping its own from "
                         f"their initial state, FP64",
               "one_core": {"value": r1, "cores": 1,
                            "sample": f"{ps1} particle-steps: {len(sample)} instance(s) (every "
                                      f"16th) stepped in turn, one thread, {sec1:.1f} s"},
               "host": host}

    survey_bytes = 79.0 * N if rb == 4 else 149.0 * N
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
        "config": {"workload": wdesc, "instances": len(plist), "particles": N,
                   "collision_cells": Cc, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(args.workload, dom), "kernel_ms": dom_ms,
                     "algorithmic_bytes_per_launch": dom_bytes, "launches_per_step": lanes,
                     "note": resident_note},
        "step_roofline": {"algorithmic_bytes_per_step": step_bytes,
                          "achieved_GBps": step_bytes / (el / args.steps) / 1e9,
                          "frac": step_bytes / (el / args.steps) / 1e9 / HBM_PEAK_GBS,
                          "three_pass_bytes_per_step": survey_bytes,
                          "three_pass_frac": survey_bytes / (el / args.steps) / 1e9 / HBM_PEAK_GBS},
        "kernel_ms_per_step": kern,
        "tuning": tuning,
        "fp64_plain": fp64,
        "speedup_vs_fp64_plain": rate / fp64["value"] if fp64 else None,
        "fp64_fast": fp64_fast,
        "speedup_vs_fp64_fast_batched": rate / fp64_fast["batched"]["value"] if fp64_fast else None,
        "serving": serving,
        "cpu_baseline": cpu,
        "other_workloads": extra,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
