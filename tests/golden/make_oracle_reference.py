#!/usr/bin/env python3
"""Write the CPU-oracle reference statistics the FP32 parity tests compare
against.  Calls only the oracle (and the seeded workload definitions).

For a workload it runs R independent replicas (seed of replica r:
synth.seed_of(k, 0, r)), each with the workload's transient followed by its
sampling steps, and stores every replica's time-averaged profiles (density,
x velocity, temperature, shear stress, x heat flux per sampling cell) and
mass flow rate.  Replicas are independent, so the across-replica spread
gives the standard error of the mean profiles.

    python tests/golden/make_oracle_reference.py --workload cfg1 --replicas 64

For the batched mix (``--workload cfg3``) every one of its instances is run
with ``--replicas`` replicas (seed of instance i, replica r:
synth.seed_of(3, i, r)) on a short common schedule (MIX_TRANSIENT steps, then
MIX_SAMPLING sampling steps).  Both sides of a comparison run the same
schedule, so the expected profiles agree whether or not the flow is steady.
To keep the file small each profile is stored as MIX_BINS averages over
equal runs of cells (bin j of an instance with C cells holds the plain mean
over cells floor(j C / B) .. floor((j + 1) C / B) - 1).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

QUANTITIES = ("n", "ux", "T", "pxy", "qx")
MIX_TRANSIENT, MIX_SAMPLING, MIX_BINS = 100, 1000, 16

SCHEDULES = {
    # workload: (params, workload index for seeds, transient, sampling steps)
    "cfg0": (synth.CONFIG0, 0, 1000, 1000),
    "cfg1": (synth.CONFIG1, 1, 1000, 20000),
    # an open patch of the hybrid with a fixed Chapman-Enskog inflow
    "patch0": (synth.PATCH0, 11, synth.PATCH0.n_transient,
               synth.PATCH0_STEPS - synth.PATCH0.n_transient),
}
INFLOWS = {"patch0": synth.PATCH0_INFLOW}
EXTRA = {"patch0": ("pxy_mid",)}


def run_replica(params, transient, sampling, inflow=None, extra=()):
    o = oracle.Oracle(params.with_(n_transient=transient))
    if inflow:
        o.set_inflow(**inflow)
    o.step(transient + sampling)
    e = o.estimators()
    assert e["n_sampled_steps"] == sampling
    return {q: e[q].copy() for q in QUANTITIES + tuple(extra)}, e["mass_flow"]


def bin_means(profile, bins=MIX_BINS):
    c = len(profile)
    edges = [(j * c) // bins for j in range(bins + 1)]
    return np.array([np.mean(profile[edges[j]:edges[j + 1]]) for j in range(bins)])


def run_mix_replica(params):
    prof, q = run_replica(params, MIX_TRANSIENT, MIX_SAMPLING)
    return {name: bin_means(prof[name]) for name in QUANTITIES}, q


def main_mix(args):
    inst = synth.config3_instances()
    jobs = [(i, r - args.first, inst[i].with_(seed=synth.seed_of(3, i, r), precision=0))
            for i in range(len(inst)) for r in range(args.first, args.first + args.replicas)]
    # longest first keeps the pool busy to the end
    jobs.sort(key=lambda j: -j[2].n_particles)
    t0 = time.time()
    out = {q: np.zeros((len(inst), args.replicas, MIX_BINS)) for q in QUANTITIES}
    Q = np.zeros((len(inst), args.replicas))
    with ThreadPoolExecutor(args.workers) as ex:
        for n, ((i, r, _), (prof, q)) in enumerate(
                zip(jobs, ex.map(lambda j: run_mix_replica(j[2]), jobs))):
            for name in QUANTITIES:
                out[name][i, r] = prof[name]
            Q[i, r] = q
            if n % 16 == 15 or n == len(jobs) - 1:
                print(f"{n + 1}/{len(jobs)} runs ({time.time() - t0:.0f} s)", flush=True)
    src = open(oracle.SRC, "rb").read()
    meta = dict(workload="cfg3", instances=len(inst), transient=MIX_TRANSIENT,
                sampling_steps=MIX_SAMPLING, bins=MIX_BINS, replicas=args.replicas,
                first_replica=args.first, seed_rule="synth.seed_of(3, i, r)",
                mix="synth.config3_instances()", oracle_sha256=hashlib.sha256(src).hexdigest())
    path = os.path.join(args.out or HERE, f"oracle_cfg3_mix_s{MIX_SAMPLING}_r{args.first}_"
                                          f"{args.first + args.replicas}.npz")
    np.savez_compressed(path, mass_flow=Q, **out, meta=json.dumps(meta))
    print("wrote", path, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", choices=sorted(SCHEDULES) + ["cfg3"], required=True)
    ap.add_argument("--replicas", type=int, default=64)
    ap.add_argument("--workers", type=int, default=max(1, (os.cpu_count() or 2) - 2))
    ap.add_argument("--first", type=int, default=0, help="index of the first replica")
    ap.add_argument("--out", default=None, help="directory of the written file (default: here)")
    args = ap.parse_args()
    if args.workload == "cfg3":
        return main_mix(args)
    base, k, transient, sampling = SCHEDULES[args.workload]
    inflow = INFLOWS.get(args.workload)
    extra = EXTRA.get(args.workload, ())
    reps = [base.with_(seed=synth.seed_of(k, 0, r))
            for r in range(args.first, args.first + args.replicas)]
    t0 = time.time()
    out = {q: [] for q in QUANTITIES + extra}
    Q = []
    with ThreadPoolExecutor(args.workers) as ex:
        for i, (prof, q) in enumerate(ex.map(lambda p: run_replica(p, transient, sampling, inflow,
                                                                   extra), reps)):
            for name in QUANTITIES + extra:
                out[name].append(prof[name])
            Q.append(q)
            print(f"replica {args.first + i}: mass flow {q:.6f} ({time.time() - t0:.0f} s)",
                  flush=True)
    src = open(oracle.SRC, "rb").read()
    meta = dict(workload=args.workload, params=base.as_dict(), transient=transient,
                sampling_steps=sampling, replicas=args.replicas, first_replica=args.first,
                seed_rule="synth.seed_of(%d, 0, r)" % k, inflow=inflow,
                oracle_sha256=hashlib.sha256(src).hexdigest())
    path = os.path.join(HERE, f"oracle_{args.workload}_r{args.first}_{args.first + args.replicas}.npz")
    np.savez_compressed(path, mass_flow=np.array(Q),
                        **{q: np.array(out[q]) for q in QUANTITIES + extra}, meta=json.dumps(meta))
    print("wrote", path, flush=True)


if __name__ == "__main__":
    main()
