"""One-way verification of the micro-macro coupling (Sec. 3.1): DSMC over the
whole gap generates the training windows, the surrogates are trained and
selected, the corrected macro model is solved once with its Monte Carlo
uncertainty, and the result is compared with a low-noise benchmark DSMC of
the same flow (500 particles per cell, 10^6 sampled steps after the
transient, Sec. 3).

Both DSMC runs use the GPU solver.  Each can run as an ensemble of
independent replicas advanced together in one batched group: R replicas of
S/R steps carry the statistics of one run of S steps (the benchmark), or give
R training samples per window (the training), in 1/R of the steps.

    python -m paper_2311_14140_amd.mms --kn 1 --replicas 32 --training-steps 4
"""
from __future__ import annotations

import argparse
import json
import math
import time
from dataclasses import dataclass

import numpy as np

from . import surrogate as sg
from .macro import MmsSolution, solve_selected


@dataclass
class Benchmark:
    """Time- and ensemble-averaged profiles of a benchmark DSMC run."""
    y: np.ndarray
    ux: np.ndarray
    ux_se: np.ndarray          # standard error per cell (batch means)
    pxy: np.ndarray            # time-centred shear stress
    pxy_se: np.ndarray
    mass_flow: float
    mass_flow_se: float
    sampled_steps: int         # per replica
    replicas: int
    seconds: float


def run_benchmark(params_list, sampling_steps: int, n_batches: int = 20) -> Benchmark:
    """Run every instance through its transient, then ``sampling_steps``
    sampled steps in ``n_batches`` windows; average windows and replicas
    (all instances must describe the same flow)."""
    from . import dsmc
    if sampling_steps % n_batches:
        raise ValueError("sampling_steps must be a multiple of n_batches")
    p0 = params_list[0]
    for p in params_list:
        if (p.kn, p.body_force, p.n_cells) != (p0.kn, p0.body_force, p0.n_cells):
            raise ValueError("benchmark replicas must share Kn, force and cells")
    t0 = time.perf_counter()
    solvers, group = [], None
    try:
        solvers = [dsmc.Solver(p) for p in params_list]
        if len(solvers) > 1:
            group = dsmc.Group()
            for s in solvers:
                group.add(s)
        longest = max(int(p.n_transient) for p in params_list)
        _advance(solvers, group, longest)
        for s in solvers:
            s.sample(reset=True)
        per = sampling_steps // n_batches
        ux, pxy, q = [], [], []
        for _ in range(n_batches):
            _advance(solvers, group, per)
            ws = group.sample(reset=True) if group is not None else [s.sample(reset=True) for s in solvers]
            for w in ws:
                if w["n_sampled_steps"] != per:
                    raise RuntimeError("benchmark window shorter than asked")
                ux.append(w["ux"])
                pxy.append(w["pxy_mid"])
                q.append(w["mass_flow"])
    finally:
        if group is not None:
            group.close()
        for s in solvers:
            s.close()
    ux, pxy, q = np.array(ux), np.array(pxy), np.array(q)
    nb = len(ux)
    C = p0.n_cells
    return Benchmark((np.arange(C) + 0.5) / C, ux.mean(0), ux.std(0, ddof=1) / math.sqrt(nb),
                     pxy.mean(0), pxy.std(0, ddof=1) / math.sqrt(nb), float(q.mean()),
                     float(q.std(ddof=1) / math.sqrt(nb)), sampling_steps, len(params_list),
                     time.perf_counter() - t0)


def _advance(solvers, group, n):
    if group is not None:
        group.step(n)
    else:
        for s in solvers:
            s.step(n)


@dataclass
class OneWay:
    kn: float
    trainer: sg.SurrogateTrainer
    run: sg.TrainingRun
    solution: MmsSolution
    benchmark: Benchmark | None

    def compare(self) -> dict:
        """MMS velocity against the benchmark at the benchmark's cells."""
        if self.benchmark is None:
            return {}
        return compare_with_benchmark(self.solution, self.trainer.history[-1], self.benchmark)


def compare_with_benchmark(solution: MmsSolution, step: sg.TrainingStep, b: Benchmark) -> dict:
    """Errors of a macro solution's velocity at the benchmark's cells,
    relative to the benchmark's largest velocity, and the fraction of cells
    within two combined standard deviations (the posterior spread of the
    macro velocity and the benchmark's standard error)."""
    from .macro import velocity_basis
    model = solution.model
    u = model.velocity(b.y)
    scale = float(np.max(np.abs(b.ux)))
    err = u - b.ux
    B = velocity_basis(b.y, model.kn, model.force, model.b)
    cov = np.zeros((1 + len(model.b), 1 + len(model.b)))
    if solution.slip:
        cov[0, 0] = step.boundary[1].S[0, 0]
    cov[1:, 1:] = step.constitutive[solution.order].S
    sd = np.sqrt(np.einsum("ij,jk,ik->i", B, cov, B))
    z = err / np.sqrt(sd ** 2 + b.ux_se ** 2)
    return dict(max_rel_err=float(np.max(np.abs(err)) / scale),
                rms_rel_err=float(np.sqrt(np.mean(err ** 2)) / scale),
                wall_rel_err=float(max(abs(err[0]), abs(err[-1])) / scale),
                frac_within_2sd=float(np.mean(np.abs(z) <= 2.0)),
                mass_flow_mms=float(model.mass_flow()), mass_flow_bench=b.mass_flow,
                mass_flow_bench_se=b.mass_flow_se,
                mass_flow_rel_err=float(model.mass_flow() / b.mass_flow - 1.0))


def one_way(kn: float, training_steps: int = 1000, samples_per_step: int = 100,
            replicas: int = 1, bench_steps: int = 10 ** 6, bench_replicas: int = 1,
            n_trials: int = 1000, n_points: int = 201, precision: int | None = None) -> OneWay:
    """The Sec. 3.1 pipeline at ``kn`` with the seeded training runs of the
    workload definitions; ``bench_steps`` = 0 skips the benchmark."""
    import synth
    prec = synth.FP32_FAST if precision is None else precision
    ps = [synth.training_case(kn, replica=r, precision=prec) for r in range(replicas)]
    run = sg.train_on_gpu(ps, training_steps, samples_per_step, flows=[0] * replicas)
    trainer = run.trainers[0]
    step = trainer.history[-1]
    sol = solve_selected(trainer, step, np.linspace(0.0, 1.0, n_points), n_trials=n_trials,
                         rng=np.random.default_rng(int(1000 * kn)))
    bench = None
    if bench_steps:
        bp = [synth.benchmark_case(kn, replica=r, precision=prec) for r in range(bench_replicas)]
        bench = run_benchmark(bp, bench_steps // bench_replicas)
    return OneWay(kn, trainer, run, sol, bench)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--kn", type=float, nargs="+", default=[1.0])
    ap.add_argument("--training-steps", type=int, default=1000)
    ap.add_argument("--samples-per-step", type=int, default=100)
    ap.add_argument("--replicas", type=int, default=1)
    ap.add_argument("--bench-steps", type=int, default=10 ** 6)
    ap.add_argument("--bench-replicas", type=int, default=1)
    ap.add_argument("--trials", type=int, default=1000)
    a = ap.parse_args()
    for kn in a.kn:
        r = one_way(kn, a.training_steps, a.samples_per_step, a.replicas, a.bench_steps,
                    a.bench_replicas, a.trials)
        s = r.trainer.history[-1]
        out = dict(kn=kn, samples=s.n_samples, p_slip=float(s.p_boundary[1]),
                   sigma_p=s.sigma_p, p_constitutive=[float(v) for v in s.p_constitutive],
                   order=s.order, weights=[float(v) for v in s.stress_weights],
                   seconds_training_dsmc=r.run.seconds_dsmc, seconds_train=r.run.seconds_train,
                   seconds_macro=r.solution.seconds,
                   seconds_bench=r.benchmark.seconds if r.benchmark else None, **r.compare())
        out["p_constitutive_history"] = [[round(float(v), 4) for v in h.p_constitutive]
                                         for h in r.trainer.history]
        out["p_slip_history"] = [round(float(h.p_boundary[1]), 6) for h in r.trainer.history]
        print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
