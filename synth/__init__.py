"""Seeded synthetic workloads for the force-driven parallel-plate DSMC solver.

This module only describes inputs: the parameter sets of the workloads, the
seeds, and the seeded draws of the batched and served request mixes.  It holds
none of the solver's arithmetic (no moves, collisions, random streams of the
method or estimators), so both the CPU oracle and the GPU path can take their
inputs from here without sharing any code of the method.

Parameters are in the units of the paper's statement of the problem (Sec. 2.1
and the dimensionless groups of Eq. 6): Kn is the hard-sphere mean free path
over the plate gap, ``body_force`` is F = F' H / v0^2, the wall temperature is
relative to the reference temperature, and ``dt`` is in H / sqrt(k T_ref / m);
``dt <= 0`` asks the solver for its default step.

Workload shapes follow the paper's DSMC runs (Sec. 3: cell size 0.005, 50
particles per cell for training data, a 500-per-cell benchmark, Mach about
0.05) scaled to the sizes listed below.  There is no public dataset: every
input is generated from a seed.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, asdict, replace

import numpy as np

FP64_DETERMINISTIC = 0
FP32_FAST = 1


def seed_of(k: int, i: int = 0, r: int = 0) -> int:
    """Seed of instance ``i``, replica ``r`` of workload ``k``."""
    return (k << 48) + (r << 32) + i


@dataclass(frozen=True)
class Params:
    kn: float
    body_force: float
    wall_temperature: float = 1.0
    n_cells: int = 100
    particles_per_cell: int = 50
    dt: float = 0.0
    n_transient: int = 1000
    seed: int = 0
    precision: int = FP64_DETERMINISTIC
    n_sub: int = 1
    domain_length: float = 0.0   # 0: the closed gap; L > 0: wall at 0, open boundary at L

    @property
    def n_particles(self) -> int:
        return self.n_cells * self.particles_per_cell

    def with_(self, **kw) -> "Params":
        return replace(self, **kw)

    def as_dict(self) -> dict:
        return asdict(self)


def transient_steps(kn: float) -> int:
    """Transient length: five e-folds of the slowest viscous mode, at least 1000."""
    return max(1000, int(math.ceil(4.5 / (kn * kn))))


# Plain FP64, Kn = 1, 100 cells x 50 per cell, 1000 transient + 1000 sampling steps.
CONFIG0 = Params(kn=1.0, body_force=0.01, n_cells=100, particles_per_cell=50,
                 n_transient=1000, seed=seed_of(0), precision=FP64_DETERMINISTIC)
CONFIG0_STEPS = 2000

# Single instance, FP32 velocities with FP64 accumulators: Kn = 0.1,
# 300 cells x 1000 per cell, 1000 transient + 20000 sampling steps.
CONFIG1 = Params(kn=0.1, body_force=0.005, n_cells=300, particles_per_cell=1000,
                 n_transient=1000, seed=seed_of(1), precision=FP32_FAST)
CONFIG1_STEPS = 21000

# Large near-continuum instance: Kn = 0.01, 1000 cells x 20000 per cell (2e7
# particles), 1000 transient + 10000 sampling steps.  Two collision sub-cells per
# sampling cell (10^4 particles, 0.05 lambda wide) keep a collision cell small
# enough to stage on chip.
CONFIG2 = Params(kn=0.01, body_force=0.001, n_cells=1000, particles_per_cell=20000,
                 n_transient=1000, seed=seed_of(2), precision=FP32_FAST, n_sub=2)
CONFIG2_STEPS = 11000


def config3_instances(n: int = 256, seed: int = 3, precision: int = FP32_FAST,
                      kn_range=(0.05, 10.0), force_range=(0.001, 0.02),
                      cells_range=(50, 2000), ppc_range=(20, 200)) -> list[Params]:
    """The batched mix: Kn log-uniform, force uniform, cells and particles per
    cell integer-uniform, drawn with numpy's PCG64 from ``seed``."""
    rng = np.random.Generator(np.random.PCG64(seed))
    lo, hi = math.log10(kn_range[0]), math.log10(kn_range[1])
    out = []
    for i in range(n):
        kn = float(10.0 ** rng.uniform(lo, hi))
        f = float(rng.uniform(*force_range))
        c = int(rng.integers(cells_range[0], cells_range[1] + 1))
        ppc = int(rng.integers(ppc_range[0], ppc_range[1] + 1))
        out.append(Params(kn=kn, body_force=f, n_cells=c, particles_per_cell=ppc,
                          n_transient=transient_steps(kn), seed=seed_of(3, i),
                          precision=precision))
    return out


CONFIG3_SAMPLING_STEPS = 5000


def serving_trace(n_requests: int = 2000, rate_hz: float = 200.0, seed: int = 4,
                  param_seed: int = 40, precision: int = FP32_FAST,
                  sampling_steps: int = CONFIG3_SAMPLING_STEPS):
    """Poisson arrivals (exponential gaps, mean 1/rate) of solves drawn from the
    batched mix.  Returns a list of (arrival_time_s, Params, total_steps)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    gaps = rng.exponential(1.0 / rate_hz, size=n_requests)
    t = np.cumsum(gaps)
    ps = config3_instances(n_requests, seed=param_seed, precision=precision)
    out = []
    for i, (ti, p) in enumerate(zip(t, ps)):
        p = p.with_(seed=seed_of(4, i))
        out.append((float(ti), p, p.n_transient + sampling_steps))
    return out


# The surrogate-training runs (Sec. 3): cells of 0.005 (200 across the gap),
# 50 particles per cell, one training sample per 100 steps, 100 samples per
# training step, 1000 training steps.
TRAINING_CELLS = 200
TRAINING_PPC = 50
STEPS_PER_SAMPLE = 100
SAMPLES_PER_TRAINING_STEP = 100
TRAINING_STEPS = 1000


def training_force(kn: float, mach: float = 0.05) -> float:
    """Body force F giving a centre-line Mach number near ``mach`` (Sec. 3):
    the no-slip Stokes centre speed sqrt(pi) F / (8 Kn) plus a slip speed of
    about F, with the speed of sound sqrt(5/6) v0 of a monatomic gas."""
    return mach * math.sqrt(5.0 / 6.0) / (math.sqrt(math.pi) / (8.0 * kn) + 1.0)


def training_case(kn: float, replica: int = 0, precision: int = FP32_FAST) -> Params:
    """One surrogate-training run at ``kn`` (seeds of workload 5)."""
    return Params(kn=kn, body_force=training_force(kn), n_cells=TRAINING_CELLS,
                  particles_per_cell=TRAINING_PPC, n_transient=transient_steps(kn),
                  seed=seed_of(5, int(round(1000 * kn)), replica), precision=precision)


# The benchmark DSMC of Sec. 3: the training flow with 500 particles per cell,
# sampled 10^6 steps after the transient.
BENCHMARK_PPC = 500
BENCHMARK_STEPS = 10 ** 6


def benchmark_case(kn: float, replica: int = 0, precision: int = FP32_FAST) -> Params:
    """One benchmark run at ``kn`` (seeds of workload 6)."""
    return training_case(kn, precision=precision).with_(
        particles_per_cell=BENCHMARK_PPC, seed=seed_of(6, int(round(1000 * kn)), replica))


# A patch of the hybrid at Kn = 0.1 (two mean free paths of cells of 0.005
# plus a 5-cell buffer: 45 cells, wall at 0, open boundary at 0.225) with the
# Chapman-Enskog inflow of a slip-flow macro state there (sigma_P 0.8, no
# stress correction): the open-boundary workload of the parity tests.
PATCH0 = Params(kn=0.1, body_force=training_force(0.1), n_cells=45, particles_per_cell=50,
                n_transient=500, seed=seed_of(11), precision=FP64_DETERMINISTIC,
                domain_length=0.225)
PATCH0_INFLOW = dict(u=0.0333, dudy=0.069)
PATCH0_STEPS = 6500


WORKLOADS = {
    "cfg0": (CONFIG0, CONFIG0_STEPS),
    "cfg1": (CONFIG1, CONFIG1_STEPS),
    "cfg2": (CONFIG2, CONFIG2_STEPS),
}
