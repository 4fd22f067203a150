"""The micro-macro-surrogate (MMS) hybrid of Sec. 3.2 on the GPU.

The macro model covers the whole gap.  DSMC runs only in patches at the
plates: each patch spans the cells within two mean free paths of its plate
(the training cells) and a buffer of 5 cells beyond them, and ends at an
open boundary where particles enter from the Chapman-Enskog distribution at
the macro state there (Sec. 2).  The loop of Sec. 2 and Sec. 3.2, iterated
until the solution is steady:

  1. the macro model is solved with the current surrogates (at the start
     Newton's law and no slip);
  2. its velocity and gradient at the patches' open boundary become their
     inflow;
  3. the patches run one training step of windows (100 steps each);
  4. the surrogates are trained on the samples so far (the buffer cells are
     not used), and the most probable boundary and constitutive models are
     selected.

The channel is symmetric, so the patch at the top plate, seen from its plate,
is the same problem as the patch at the bottom: both are run as independent
replicas of one patch and their samples train the same (antisymmetric)
models.  R replicas advanced together in one batched group give R samples per
window.

Readings: the patch is 2 lambda of training cells (rounded up to whole
cells, at least 3) plus the 5 buffer cells; the samples of the first
``burn_in`` iterations, taken while the inflow is still far from steady,
are dropped; the patch starts at rest and samples after about five of its
viscous relaxation times.

    python -m paper_2311_14140_amd.hybrid --kn 0.1 --replicas 64 --iterations 16
"""
from __future__ import annotations

import argparse
import json
import math
import time
from dataclasses import dataclass, field

import numpy as np

from . import surrogate as sg
from .macro import MacroModel, MmsSolution, solve_selected

BUFFER_CELLS = 5


@dataclass(frozen=True)
class Patch:
    """Cells of one patch: n_train training cells of width dy from the plate,
    then the buffer; length = its extent (the open boundary's position)."""
    n_train: int
    n_buffer: int
    dy: float

    @property
    def n_cells(self) -> int:
        return self.n_train + self.n_buffer

    @property
    def length(self) -> float:
        return self.n_cells * self.dy


def patch_for(kn: float, dy: float = 0.005, mean_free_paths: float = 2.0,
              buffer_cells: int = BUFFER_CELLS) -> Patch:
    n_train = max(3, int(math.ceil(mean_free_paths * kn / dy - 1e-9)))
    p = Patch(n_train, buffer_cells, dy)
    if p.length > 0.5:
        raise ValueError(f"a patch of {p.length:.3f} H would reach past the centre line")
    return p


def patch_transient(kn: float, length: float) -> int:
    """Steps for five viscous relaxation times of a patch, L^2 / nu with
    nu = mu / rho of hard spheres (0.796 Kn in H sqrt(kT/m)) and the default
    step 0.2 lambda / sqrt(2); at least 500."""
    nu = 0.796 * kn
    dt = 0.2 * min(kn, 1.0) / math.sqrt(2.0)
    return max(500, int(math.ceil(5.0 * length * length / nu / dt)))


@dataclass
class HybridRun:
    kn: float
    force: float
    patch: Patch
    trainer: sg.SurrogateTrainer
    solution: MmsSolution
    history: list = field(default_factory=list)   # per iteration
    seconds_dsmc: float = 0.0
    seconds_train: float = 0.0
    replicas: int = 0
    samples: int = 0


def _select(trainer: sg.SurrogateTrainer, step: sg.TrainingStep) -> MacroModel:
    k = step.order
    return MacroModel(trainer.kn, trainer.force, step.sigma_p if step.slip else 0.0,
                      tuple(float(v) for v in step.constitutive[k].m), trainer.exponents[:k])


def hybrid(kn: float, force: float | None = None, iterations: int = 16,
           samples_per_iteration: int = 100, replicas: int = 64, steps_per_sample: int = 100,
           dy: float = 0.005, particles_per_cell: int = 50, burn_in: int = 2,
           n_trials: int = 1000, n_points: int = 201, precision: int | None = None,
           seed_base: int = 10, verbose: bool = False) -> HybridRun:
    """Run the MMS hybrid at ``kn`` with ``replicas`` patch replicas on the GPU."""
    import synth
    from . import dsmc
    prec = synth.FP32_FAST if precision is None else precision
    F = synth.training_force(kn) if force is None else force
    patch = patch_for(kn, dy)
    ps = [synth.Params(kn=kn, body_force=F, n_cells=patch.n_cells,
                       particles_per_cell=particles_per_cell,
                       n_transient=patch_transient(kn, patch.length),
                       seed=synth.seed_of(seed_base, int(round(1000 * kn)), r), precision=prec,
                       domain_length=patch.length) for r in range(replicas)]

    def new_trainer():
        return sg.SurrogateTrainer(kn, F, patch.n_cells, cells=np.arange(patch.n_train), dy=dy,
                                   plates=1)

    trainer = new_trainer()
    model = MacroModel(kn, F)       # Newton's law, no slip
    run = HybridRun(kn, F, patch, trainer, None, replicas=replicas)
    solvers, group = [], None
    try:
        solvers = [dsmc.Solver(p) for p in ps]
        group = dsmc.Group()
        for s in solvers:
            group.add(s)
        started = False
        for it in range(iterations):
            u_in = float(model.velocity(patch.length))
            g_in = float(model.velocity_gradient(patch.length))
            for s in solvers:
                s.set_inflow(u=u_in, dudy=g_in)
            t0 = time.perf_counter()
            if not started:
                group.step(ps[0].n_transient)
                group.sample(reset=True)
                started = True
            pending = []
            run.seconds_dsmc += sg.collect_windows(
                solvers, samples_per_iteration, steps_per_sample, group,
                lambda k, ux, pxy: pending.append((ux, pxy)))
            t1 = time.perf_counter()
            if it == burn_in:
                trainer = new_trainer()
            trainer.add(np.stack([w[0] for w in pending]), np.stack([w[1] for w in pending]))
            step = trainer.train()
            model = _select(trainer, step)
            run.seconds_train += time.perf_counter() - t1
            rec = dict(iteration=it, samples=step.n_samples, u_in=u_in, dudy_in=g_in,
                       sigma_p=step.sigma_p, p_slip=float(step.p_boundary[1]),
                       order=step.order, p_constitutive=[float(v) for v in step.p_constitutive],
                       mass_flow=float(model.mass_flow()),
                       u_centre=float(model.velocity(0.5)), burn_in=it < burn_in)
            run.history.append(rec)
            if verbose:
                print(json.dumps(rec), flush=True)
    finally:
        if group is not None:
            group.close()
        for s in solvers:
            s.close()
    run.trainer = trainer
    run.samples = trainer.n_samples
    run.solution = solve_selected(trainer, trainer.history[-1], np.linspace(0.0, 1.0, n_points),
                                  n_trials=n_trials, rng=np.random.default_rng(int(1000 * kn)))
    return run


def time_patch_group(kn: float, open_boundary: bool = True, replicas: int = 64,
                     steps: int = 2000, profile_steps: int = 50, dy: float = 0.005,
                     particles_per_cell: int = 50, u_in: float = 0.03,
                     dudy_in: float = 0.07, resident: bool = True) -> dict:
    """Cost of one step of the hybrid's DSMC: ``replicas`` patches at ``kn``
    (FP32) batched in one group, with their open boundary and a fixed inflow,
    or closed at the same size for comparison; resident (one workgroup per
    patch, whole steps per launch) where the patches are small enough, or
    with the multi-kernel step.  Wall time per step over ``steps`` steps, and
    device time per kernel slot from ``profile_steps`` eagerly launched steps
    timed with HIP events (a resident step is one kernel, in the collide
    slot)."""
    import synth
    from . import dsmc
    patch = patch_for(kn, dy)
    F = synth.training_force(kn)
    ps = [synth.Params(kn=kn, body_force=F, n_cells=patch.n_cells,
                       particles_per_cell=particles_per_cell, n_transient=10,
                       seed=synth.seed_of(12, r), precision=synth.FP32_FAST,
                       domain_length=patch.length if open_boundary else 0.0)
          for r in range(replicas)]
    solvers, group = [], None
    try:
        solvers = [dsmc.Solver(p) for p in ps]
        group = dsmc.Group()
        group.set_resident(resident)
        for s in solvers:
            if open_boundary:
                s.set_inflow(u=u_in, dudy=dudy_in)
            group.add(s)
        group.step(200)
        group.sync()
        prof = solvers[0].profile(profile_steps)
        t0 = time.perf_counter()
        group.step(steps)
        group.sync()
        wall = (time.perf_counter() - t0) / steps
        live = sum(s.live() for s in solvers)
    finally:
        if group is not None:
            group.close()
        for s in solvers:
            s.close()
    return dict(kn=kn, open=open_boundary, resident=resident, replicas=replicas,
                patch_cells=patch.n_cells,
                particles=live, ms_per_step=wall * 1e3, particle_steps_per_s=live / wall,
                kernel_ms_per_step={k: prof[k] / profile_steps for k in dsmc.Solver.PHASES})


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--kn", type=float, nargs="+", default=[0.1])
    ap.add_argument("--iterations", type=int, default=16)
    ap.add_argument("--samples-per-iteration", type=int, default=100)
    ap.add_argument("--replicas", type=int, default=64)
    ap.add_argument("--burn-in", type=int, default=2)
    ap.add_argument("--bench-steps", type=int, default=10 ** 6)
    ap.add_argument("--bench-replicas", type=int, default=8)
    ap.add_argument("--verbose", action="store_true")
    ap.add_argument("--time-patches", action="store_true",
                    help="only time the patch group per step at each Kn: open and closed, "
                         "resident and multi-kernel")
    a = ap.parse_args()
    if a.time_patches:
        for kn in a.kn:
            for open_boundary in (True, False):
                for resident in (True, False):
                    print(json.dumps(time_patch_group(kn, open_boundary, replicas=a.replicas,
                                                      resident=resident)), flush=True)
        return
    import synth
    from .mms import compare_with_benchmark, run_benchmark
    for kn in a.kn:
        r = hybrid(kn, iterations=a.iterations, samples_per_iteration=a.samples_per_iteration,
                   replicas=a.replicas, burn_in=a.burn_in, verbose=a.verbose)
        s = r.trainer.history[-1]
        out = dict(kn=kn, patch_cells=r.patch.n_cells, training_cells=r.patch.n_train,
                   patch_length=r.patch.length, replicas=r.replicas, samples=r.samples,
                   p_slip=float(s.p_boundary[1]), sigma_p=s.sigma_p, order=s.order,
                   p_constitutive=[float(v) for v in s.p_constitutive],
                   weights=[float(v) for v in s.stress_weights],
                   seconds_dsmc=r.seconds_dsmc, seconds_train=r.seconds_train,
                   mass_flow_history=[round(h["mass_flow"], 6) for h in r.history],
                   p_slip_history=[round(h["p_slip"], 6) for h in r.history])
        if a.bench_steps:
            bp = [synth.benchmark_case(kn, replica=q) for q in range(a.bench_replicas)]
            b = run_benchmark(bp, a.bench_steps // a.bench_replicas)
            out.update(compare_with_benchmark(r.solution, s, b))
            out["seconds_bench"] = b.seconds
        print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
