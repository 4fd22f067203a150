"""Macroscopic model of the micro-macro coupling for force-driven flow between
parallel plates (Sec. 2.1, Eqs. 5-10), corrected by the trained surrogates,
and the one-way verification pipeline of Sec. 3.1.

In the units of Eq. 6 the corrected Newton law (Eq. 7) is
P = -c du/dy + c S(y) with c = 2 Kn / sqrt(pi), and the macro equation
(Eq. 8) is u'' = -(sqrt(pi) / Kn) F + S'(y).  With the stress correction of
Eq. 14, S(y) = sum_l a_l (exp(-b_l y) - exp(-b_l (1 - y))), the equation
integrates in closed form, so the macro model is solved exactly rather than
on a grid: with either boundary condition (no-slip, Eq. 9; slip
u(0) = -sigma_P P(0), u(1) = sigma_P P(1), Eq. 10)

    P(y) = 2 F (y - 1/2)
    u(y) = (F / c) y (1 - y) + sigma_P F + I(y) - I(0),
    I(y) = -sum_l (a_l / b_l) (exp(-b_l y) + exp(-b_l (1 - y))),

(sigma_P = 0 for no-slip).  The stress is the momentum balance's whatever
the correction and the slip coefficient, which the paper notes for this
flow; the velocity is linear in (sigma_P, a_1..a_k).

The uncertainty of the macro velocity is propagated from the weight
posteriors by Monte Carlo (Sec. 2.2, Sec. 3: weights drawn from the
posteriors of the selected models, the macro model solved per draw, the
standard deviation taken across draws); ``exact_std`` gives the same
quantity from the posterior covariances, the velocity being linear in the
weights.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass

import numpy as np

from .surrogate import SurrogateTrainer, TrainingStep


@dataclass
class MacroModel:
    """Eq. 8 with the boundary condition and stress correction of the
    selected surrogates: ``sigma_p`` = 0 is no-slip; ``a`` the weights of the
    exponential correction with exponents ``b``."""
    kn: float
    force: float
    sigma_p: float = 0.0
    a: tuple = ()
    b: tuple = ()

    @property
    def c(self) -> float:
        return 2.0 * self.kn / math.sqrt(math.pi)

    def correction(self, y) -> np.ndarray:
        """S(y) of Eq. 14."""
        y = np.asarray(y, dtype=np.float64)
        s = np.zeros_like(y)
        for al, bl in zip(self.a, self.b):
            s = s + al * (np.exp(-bl * y) - np.exp(-bl * (1.0 - y)))
        return s

    def velocity(self, y) -> np.ndarray:
        y = np.asarray(y, dtype=np.float64)
        u = (self.force / self.c) * y * (1.0 - y) + self.sigma_p * self.force
        for al, bl in zip(self.a, self.b):
            u = u + (al / bl) * ((1.0 + math.exp(-bl)) - np.exp(-bl * y) - np.exp(-bl * (1.0 - y)))
        return u

    def shear_stress(self, y) -> np.ndarray:
        return 2.0 * self.force * (np.asarray(y, dtype=np.float64) - 0.5)

    def velocity_gradient(self, y) -> np.ndarray:
        """du/dy = (F / c)(1 - 2y) + S(y)."""
        y = np.asarray(y, dtype=np.float64)
        return (self.force / self.c) * (1.0 - 2.0 * y) + self.correction(y)

    def mass_flow(self) -> float:
        """Integral of u over the gap (density uniform, in the units of the
        solver's mass-flow estimator)."""
        q = self.force / (6.0 * self.c) + self.sigma_p * self.force
        for al, bl in zip(self.a, self.b):
            q += (al / bl) * ((1.0 + math.exp(-bl)) - 2.0 * (1.0 - math.exp(-bl)) / bl)
        return q


def velocity_basis(y, kn: float, force: float, b) -> np.ndarray:
    """Columns of du_macro/d(sigma_P, a_1..a_k) at the points y: the velocity
    is u_0(y) + this matrix times (sigma_P, a)."""
    y = np.asarray(y, dtype=np.float64)
    cols = [np.full_like(y, force)]
    for bl in b:
        cols.append(((1.0 + math.exp(-bl)) - np.exp(-bl * y) - np.exp(-bl * (1.0 - y))) / bl)
    return np.stack(cols, axis=1)


@dataclass
class MmsSolution:
    """Macro velocity of the selected surrogates with its uncertainty."""
    y: np.ndarray
    u: np.ndarray               # velocity at the posterior means
    u_mc_mean: np.ndarray       # mean over the Monte Carlo trials
    u_std: np.ndarray           # standard deviation over the trials
    u_std_exact: np.ndarray     # the same from the posterior covariances
    pxy: np.ndarray
    model: MacroModel
    slip: bool
    order: int
    n_trials: int
    seconds: float

    @property
    def ci95(self):
        """Two standard deviations about the mean (Sec. 3)."""
        return self.u - 2.0 * self.u_std, self.u + 2.0 * self.u_std


def solve_selected(trainer: SurrogateTrainer, step: TrainingStep, y, n_trials: int = 1000,
                   rng: np.random.Generator | None = None, draws=None) -> MmsSolution:
    """Macro solution with the most probable boundary and constitutive
    models of ``step`` (selected independently, Sec. 2.2), and its Monte
    Carlo uncertainty from ``n_trials`` weight draws.  ``draws`` =
    (sigma_P draws (n,), stress-weight draws (n, k)) replaces the draws
    from the posteriors."""
    t0 = time.perf_counter()
    rng = np.random.default_rng(0) if rng is None else rng
    y = np.asarray(y, dtype=np.float64)
    slip, k = step.slip, step.order
    bnd = step.boundary[1] if slip else step.boundary[0]
    con = step.constitutive[k]
    b = trainer.exponents[:k]
    model = MacroModel(trainer.kn, trainer.force, float(bnd.m[0]) if slip else 0.0,
                       tuple(float(v) for v in con.m), tuple(b))
    u = model.velocity(y)
    # Monte Carlo over the weights of the two selected models, drawn
    # independently from their posteriors; one macro solve per draw is one
    # row of the linear map below
    if draws is None:
        ws = bnd.draw(n_trials, rng) if slip else np.zeros((n_trials, 1))
        wa = con.draw(n_trials, rng)
    else:
        ws = np.asarray(draws[0], dtype=np.float64).reshape(-1, 1)
        wa = np.asarray(draws[1], dtype=np.float64).reshape(len(ws), k)
        n_trials = len(ws)
    B = velocity_basis(y, trainer.kn, trainer.force, b)
    u0 = (trainer.force / model.c) * y * (1.0 - y)
    W = np.concatenate([ws, wa], axis=1)
    trials = u0[None, :] + W @ B.T
    cov = np.zeros((1 + k, 1 + k))
    if slip:
        cov[0, 0] = bnd.S[0, 0]
    cov[1:, 1:] = con.S
    std_exact = np.sqrt(np.maximum(np.einsum("ij,jk,ik->i", B, cov, B), 0.0))
    return MmsSolution(y, u, trials.mean(axis=0), trials.std(axis=0, ddof=1), std_exact,
                       model.shear_stress(y), model, slip, k, n_trials, time.perf_counter() - t0)
