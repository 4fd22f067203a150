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
SCHEDULES = {
    # workload: (params, workload index for seeds, transient, sampling steps)
    "cfg0": (synth.CONFIG0, 0, 1000, 1000),
    "cfg1": (synth.CONFIG1, 1, 1000, 20000),
}


def run_replica(params, transient, sampling):
    o = oracle.Oracle(params.with_(n_transient=transient))
    o.step(transient + sampling)
    e = o.estimators()
    assert e["n_sampled_steps"] == sampling
    return {q: e[q].copy() for q in QUANTITIES}, e["mass_flow"]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", choices=sorted(SCHEDULES), required=True)
    ap.add_argument("--replicas", type=int, default=64)
    ap.add_argument("--workers", type=int, default=max(1, (os.cpu_count() or 2) - 2))
    ap.add_argument("--first", type=int, default=0, help="index of the first replica")
    args = ap.parse_args()
    base, k, transient, sampling = SCHEDULES[args.workload]
    reps = [base.with_(seed=synth.seed_of(k, 0, r))
            for r in range(args.first, args.first + args.replicas)]
    t0 = time.time()
    out = {q: [] for q in QUANTITIES}
    Q = []
    with ThreadPoolExecutor(args.workers) as ex:
        for i, (prof, q) in enumerate(ex.map(lambda p: run_replica(p, transient, sampling), reps)):
            for name in QUANTITIES:
                out[name].append(prof[name])
            Q.append(q)
            print(f"replica {args.first + i}: mass flow {q:.6f} ({time.time() - t0:.0f} s)",
                  flush=True)
    src = open(oracle.SRC, "rb").read()
    meta = dict(workload=args.workload, params=base.as_dict(), transient=transient,
                sampling_steps=sampling, replicas=args.replicas, first_replica=args.first,
                seed_rule="synth.seed_of(%d, 0, r)" % k,
                oracle_sha256=hashlib.sha256(src).hexdigest())
    path = os.path.join(HERE, f"oracle_{args.workload}_r{args.first}_{args.first + args.replicas}.npz")
    np.savez_compressed(path, mass_flow=np.array(Q),
                        **{q: np.array(out[q]) for q in QUANTITIES}, meta=json.dumps(meta))
    print("wrote", path, flush=True)


if __name__ == "__main__":
    main()
