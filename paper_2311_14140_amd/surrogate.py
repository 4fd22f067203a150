"""Surrogate boundary and constitutive models of the micro-macro coupling,
trained on windows of the GPU DSMC solver (Sec. 2.2, Eqs. 11-17, Appendix A).

A training sample is one window of the solver: the x velocity and shear
stress profiles averaged over 100 steps (Sec. 3), which ``dsmc_sample`` with a
window reset hands back to the host.  From the samples the module builds

  * the boundary models: no-slip (Eq. 11, no weight) and first-order slip
    (Eq. 12, one weight sigma_P, the wall velocity against the wall stress
    of the macro model);
  * the constitutive models C_0 .. C_3 (Eqs. 13-14): the error of Newton's
    law E = P + 2 Kn / sqrt(pi) du/dy against 0, 1, 2 or 3 antisymmetric
    exponential basis functions with the Table 1 exponents;

trains each by Bayesian ridge regression, the weight prior a zero-mean
isotropic Gaussian of precision alpha, the noise Gaussian of precision beta,
both chosen to maximise the evidence by MacKay's re-estimation (Tipping's
Appendix A), and turns the evidences into model probabilities with equal
priors (Eq. 17), separately for the two families.  The selected model is the
most probable one and its weights are the posterior mean; ``Posterior.draw``
samples weights for the Monte Carlo uncertainty of the macro solution.

Everything here is host FP64 on purpose: a window is a few kB, the models have
at most three weights, and the regression needs only the sufficient statistics
of the samples (Phi' Phi, Phi' t, t' t, the sum and count of t), which are
accumulated as windows arrive, so a training step costs the same however many
samples came before it.  The regression works in the eigenbasis of Phi' Phi,
where every re-estimation is a few elementwise products.

Points the paper leaves open are taken as follows: du/dy by second-order
central differences inside and second-order one-sided differences in the two
end cells; the wall velocity u(y_bot), u(y_top) of Eqs. 11-12 is the profile
extrapolated linearly to the plate from its two nearest cells (the nearest
cell's own value, half a cell away, is an option); the
macro wall stress of the force-driven channel is -F at the bottom plate and +F
at the top (the momentum balance in the units of Eq. 6 fixes P = 2F(y - 1/2)
whatever the constitutive law); Table 1 is looked up at the tabulated Kn nearest
in log(Kn); the regression starts from alpha = 1 and beta = 1/Var(t), puts
Gamma(1e-6, 1e-6) hyperpriors on both precisions, and stops when the weights
move by less than 1e-3 in the sum of absolute changes or after 300 updates;
the evidence is the log marginal likelihood at the final precisions, and a
model without weights keeps the noise precision as its only parameter.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field

import numpy as np

# Table 1: exponents b_1, b_2, b_3 of the stress-correction basis per Kn.
_TABLE_KN = np.array([0.01, 0.05, 0.1, 0.2, 0.5, 1.0, 5.0])
_TABLE_B = np.array([[130.0, 30.0, 20.0, 20.0, 10.0, 8.0, 7.0],
                     [150.0, 40.0, 40.0, 12.0, 7.0, 6.0, 6.0],
                     [200.0, 70.0, 10.0, 8.0, 6.0, 20.0, 5.0]])

MAX_ORDER = 3
_LOG_2PI = math.log(2.0 * math.pi)


def table_exponents(kn: float) -> tuple:
    """The Table 1 exponents at the tabulated Kn nearest to ``kn`` in log(Kn)."""
    q = int(np.argmin(np.abs(np.log(_TABLE_KN / kn))))
    return tuple(float(b) for b in _TABLE_B[:, q])


def stress_basis(y: np.ndarray, kn: float, exponents) -> np.ndarray:
    """Columns 2 Kn / sqrt(pi) (exp(-b y) - exp(-b (1 - y))) for each exponent b
    (Eq. 14 with the factor of Eq. 13), plates at y = 0 and y = 1."""
    y = np.asarray(y, dtype=np.float64)[:, None]
    b = np.asarray(exponents, dtype=np.float64)[None, :]
    return (2.0 * kn / math.sqrt(math.pi)) * (np.exp(-b * y) - np.exp(-b * (1.0 - y)))


@dataclass
class Posterior:
    """Posterior of one model's weights and its evidence."""
    m: np.ndarray            # posterior mean of the weights
    S: np.ndarray            # posterior covariance
    alpha: float             # weight precision (nan for a model without weights)
    beta: float              # noise precision
    log_evidence: float      # log p(D | model)
    n_iter: int              # re-estimation updates made
    n_data: int              # targets the model was trained on

    def draw(self, n: int, rng: np.random.Generator) -> np.ndarray:
        """``n`` weight vectors from N(m, S), shape (n, M)."""
        M = len(self.m)
        if M == 0:
            return np.zeros((n, 0))
        w, V = np.linalg.eigh(self.S)
        L = V * np.sqrt(np.maximum(w, 0.0))
        return self.m[None, :] + rng.standard_normal((n, M)) @ L.T


def fit_stats(G, h, tt: float, tsum: float, n: int, tol: float = 1e-3, max_iter: int = 300,
              hyper: float = 1e-6) -> Posterior:
    """Evidence-maximising Bayesian ridge regression from sufficient statistics:
    G = Phi' Phi, h = Phi' t, tt = t' t, tsum = sum of t, n = len(t)."""
    G = np.asarray(G, dtype=np.float64)
    h = np.asarray(h, dtype=np.float64)
    M = h.shape[0]
    if n <= 0:
        raise ValueError("no training data")
    if M == 0:
        beta = (n + 2.0 * hyper) / (tt + 2.0 * hyper)
        log_ev = 0.5 * n * math.log(beta) - 0.5 * beta * tt - 0.5 * n * _LOG_2PI
        return Posterior(np.zeros(0), np.zeros((0, 0)), float("nan"), beta, log_ev, 0, n)
    lam, V = np.linalg.eigh(G)
    lam = np.maximum(lam, 0.0)
    hv = V.T @ h
    var_t = max(tt / n - (tsum / n) ** 2, 0.0)
    beta = 1.0 / (var_t + np.finfo(np.float64).eps)
    alpha = 1.0

    def mean(alpha, beta):
        mv = beta * hv / (alpha + beta * lam)
        rss = max(tt - 2.0 * float(mv @ hv) + float(mv @ (lam * mv)), 0.0)
        return mv, rss

    m_old = None
    it = 0
    for it in range(1, max_iter + 1):
        mv, rss = mean(alpha, beta)
        gamma = float(np.sum(beta * lam / (alpha + beta * lam)))
        alpha = (gamma + 2.0 * hyper) / (float(mv @ mv) + 2.0 * hyper)
        beta = (n - gamma + 2.0 * hyper) / (rss + 2.0 * hyper)
        m = V @ mv
        if m_old is not None and float(np.sum(np.abs(m_old - m))) < tol:
            break
        m_old = m
    mv, rss = mean(alpha, beta)
    d = alpha + beta * lam
    log_ev = (0.5 * M * math.log(alpha) + 0.5 * n * math.log(beta) - 0.5 * beta * rss
              - 0.5 * alpha * float(mv @ mv) - 0.5 * float(np.sum(np.log(d))) - 0.5 * n * _LOG_2PI)
    return Posterior(V @ mv, (V / d) @ V.T, alpha, beta, log_ev, it, n)


def probabilities(log_evidences) -> np.ndarray:
    """Model probabilities from log evidences with equal priors (Eq. 17)."""
    le = np.asarray(log_evidences, dtype=np.float64)
    w = np.exp(le - le.max())
    return w / w.sum()


@dataclass
class TrainingStep:
    """Outcome of one training step: every model's posterior and the two
    families' probabilities."""
    n_samples: int
    boundary: list                 # [no-slip, slip] posteriors
    constitutive: list             # [C_0 .. C_K] posteriors
    p_boundary: np.ndarray
    p_constitutive: np.ndarray

    @property
    def slip(self) -> bool:
        return bool(self.p_boundary[1] > self.p_boundary[0])

    @property
    def order(self) -> int:
        return int(np.argmax(self.p_constitutive))

    @property
    def sigma_p(self) -> float:
        return float(self.boundary[1].m[0])

    @property
    def stress_weights(self) -> np.ndarray:
        return self.constitutive[self.order].m


class SurrogateTrainer:
    """Accumulates DSMC windows of one flow and trains the surrogates.

    ``kn`` and ``force`` are the Kn and F of Eq. 6 for the flow; ``n_cells``
    the cells of the profiles, of equal width across the gap.  ``cells`` (an
    index array or boolean mask) restricts the constitutive targets to a set
    of cells, the gradient still being taken over the whole profile.
    ``wall`` picks the wall velocity of the boundary models:
    ``"extrapolated"`` (to the plate) or ``"cell"`` (the nearest cell).

    For a patch of the hybrid (Sec. 3.2) the profiles cover only the cells
    next to the bottom plate: ``dy`` is their width (default 1/n_cells, the
    whole gap), ``cells`` the training cells (the patch without its buffer)
    and ``plates=1`` takes the wall velocity of the bottom plate alone."""

    def __init__(self, kn: float, force: float, n_cells: int, exponents=None,
                 max_order: int = MAX_ORDER, cells=None, wall: str = "extrapolated",
                 dy: float | None = None, plates: int = 2):
        if wall not in ("extrapolated", "cell"):
            raise ValueError("wall must be 'extrapolated' or 'cell'")
        if plates not in (1, 2):
            raise ValueError("plates must be 1 or 2")
        self.wall = wall
        self.plates = plates
        if n_cells < 3:
            raise ValueError("the gradient needs at least three cells")
        if not 0 <= max_order <= MAX_ORDER:
            raise ValueError("max_order must be 0..3")
        self.kn, self.force, self.n_cells = float(kn), float(force), int(n_cells)
        self.exponents = tuple(exponents) if exponents is not None else table_exponents(kn)
        self.max_order = max_order
        self.dy = 1.0 / n_cells if dy is None else float(dy)
        self.y = (np.arange(n_cells) + 0.5) * self.dy
        self.visc = 2.0 * self.kn / math.sqrt(math.pi)
        sel = np.arange(n_cells) if cells is None else np.arange(n_cells)[cells]
        self.cells = sel
        self.basis = stress_basis(self.y[sel], self.kn, self.exponents[:max_order])
        self._BtB = self.basis.T @ self.basis
        self.n_samples = 0
        # constitutive sufficient statistics
        self._hE = np.zeros(max_order)
        self._EE = 0.0
        self._Esum = 0.0
        # boundary sufficient statistics (one design column)
        self._xx = 0.0
        self._xu = 0.0
        self._uu = 0.0
        self._usum = 0.0
        self.history: list[TrainingStep] = []

    def newton_error(self, ux: np.ndarray, pxy: np.ndarray) -> np.ndarray:
        """E = P + 2 Kn / sqrt(pi) du/dy per sample and cell (Eq. 13)."""
        return pxy + self.visc * np.gradient(ux, self.dy, axis=-1, edge_order=2)

    def add(self, ux, pxy, wall_stress=None):
        """Add samples: ``ux`` and ``pxy`` of shape (n_cells,) or (S, n_cells).
        ``wall_stress`` is the macro shear stress (bottom, top) the slip model
        correlates with; default (-F, +F)."""
        ux = np.atleast_2d(np.asarray(ux, dtype=np.float64))
        pxy = np.atleast_2d(np.asarray(pxy, dtype=np.float64))
        if ux.shape != pxy.shape or ux.shape[1] != self.n_cells:
            raise ValueError("profiles must have shape (samples, n_cells)")
        if not (np.all(np.isfinite(ux)) and np.all(np.isfinite(pxy))):
            raise ValueError("non-finite sample (a window without sampled steps?)")
        S = ux.shape[0]
        E = self.newton_error(ux, pxy)[:, self.cells]
        self._hE += (E @ self.basis).sum(axis=0)
        self._EE += float(np.sum(E * E))
        self._Esum += float(np.sum(E))
        p_bot, p_top = (-self.force, self.force) if wall_stress is None else wall_stress
        x_bot, x_top = -float(p_bot), float(p_top)
        if self.wall == "cell":
            u_bot, u_top = ux[:, 0], ux[:, -1]
        else:
            u_bot = 1.5 * ux[:, 0] - 0.5 * ux[:, 1]
            u_top = 1.5 * ux[:, -1] - 0.5 * ux[:, -2]
        self._xx += S * x_bot * x_bot
        self._xu += x_bot * float(u_bot.sum())
        self._uu += float(u_bot @ u_bot)
        self._usum += float(u_bot.sum())
        if self.plates == 2:
            self._xx += S * x_top * x_top
            self._xu += x_top * float(u_top.sum())
            self._uu += float(u_top @ u_top)
            self._usum += float(u_top.sum())
        self.n_samples += S

    def train(self, **fit_kw) -> TrainingStep:
        """Train every model on all samples so far; appends to ``history``."""
        S = self.n_samples
        nE = S * len(self.cells)
        cons = [fit_stats(S * self._BtB[:k, :k], self._hE[:k], self._EE, self._Esum, nE, **fit_kw)
                for k in range(self.max_order + 1)]
        nw = self.plates * S
        no_slip = fit_stats(np.zeros((0, 0)), np.zeros(0), self._uu, self._usum, nw, **fit_kw)
        slip = fit_stats(np.array([[self._xx]]), np.array([self._xu]), self._uu, self._usum, nw,
                         **fit_kw)
        step = TrainingStep(S, [no_slip, slip], cons,
                            probabilities([no_slip.log_evidence, slip.log_evidence]),
                            probabilities([c.log_evidence for c in cons]))
        self.history.append(step)
        return step


def collect_windows(solvers, n_windows: int, steps_per_sample: int = 100, group=None,
                    on_window=None):
    """Run ``n_windows`` sampling windows of ``steps_per_sample`` steps on the
    GPU and hand each solver's window to ``on_window(k, ux, pxy)``, the
    stress being the time-centred estimate (the mean of the kinetic stresses
    before and after the collisions, which keeps the momentum balance; the
    value after the collisions alone lies a first-order amount in dt below
    the momentum flux).

    ``solvers`` are ``dsmc.Solver`` objects past their transient; with
    ``group`` (a ``dsmc.Group`` holding exactly them, in order) one group
    step advances them together and one group call takes all their windows.
    Returns the seconds spent stepping and sampling."""
    t0 = time.perf_counter()
    if group is not None and list(group.members) != list(solvers):
        raise ValueError("the group must hold exactly the solvers, in order")
    for _ in range(n_windows):
        if group is not None:
            group.step(steps_per_sample)
            ws = group.sample(reset=True)
        else:
            ws = []
            for s in solvers:
                s.step(steps_per_sample)
            for s in solvers:
                ws.append(s.sample(reset=True))
        for k, w in enumerate(ws):
            if w["n_sampled_steps"] != steps_per_sample:
                raise RuntimeError(f"window of {w['n_sampled_steps']} sampled steps, "
                                   f"expected {steps_per_sample} (transient not over?)")
            if on_window is not None:
                on_window(k, w["ux"], w["pxy_mid"])
    return time.perf_counter() - t0


@dataclass
class TrainingRun:
    """The Sec. 3 training schedule on a batch of flows."""
    trainers: list
    seconds_dsmc: float = 0.0
    seconds_train: float = 0.0
    windows: int = 0                                # windows per instance
    log: list = field(default_factory=list)         # (flow, ux, pxy) if kept


def train_on_gpu(params_list, training_steps: int, samples_per_step: int = 100,
                 steps_per_sample: int = 100, grouped: bool = True, flows=None,
                 keep_windows: bool = False, on_step=None) -> TrainingRun:
    """Run the training schedule on the GPU for every parameter set in
    ``params_list``: step through the transient, then per training step
    collect ``samples_per_step`` windows of ``steps_per_sample`` steps from
    every instance and train.

    ``flows[i]`` names the trainer instance ``i`` feeds (default: one trainer
    per instance).  Instances of one flow (same Kn, force and cells, other
    seeds) are independent realisations, so pooling R of them gives R
    samples per window: the paper's sample count in 1/R of its steps.
    With ``grouped`` all instances advance in one batched group.
    ``on_step(i, run)`` is called after training step i."""
    from . import dsmc
    flows = list(range(len(params_list))) if flows is None else list(flows)
    if len(flows) != len(params_list):
        raise ValueError("flows must name one trainer per parameter set")
    n_flows = max(flows) + 1
    first = {}
    for i, f in enumerate(flows):
        p = params_list[i]
        q = params_list[first.setdefault(f, i)]
        if (p.kn, p.body_force, p.n_cells) != (q.kn, q.body_force, q.n_cells):
            raise ValueError("instances pooled into one flow must share Kn, force and cells")
    trainers = [SurrogateTrainer(params_list[first[f]].kn, params_list[first[f]].body_force,
                                 params_list[first[f]].n_cells) for f in range(n_flows)]
    run = TrainingRun(trainers)
    solvers, group = [], None
    try:
        solvers = [dsmc.Solver(p) for p in params_list]
        if grouped and len(solvers) > 1:
            group = dsmc.Group()
            for s in solvers:
                group.add(s)
        # every instance samples after its own transient; start the windows
        # once the longest transient is over
        longest = max(int(p.n_transient) for p in params_list)
        if group is not None:
            group.step(longest)
        else:
            for s in solvers:
                s.step(longest)
        for s in solvers:
            s.sample(reset=True)
        pending = [[] for _ in range(n_flows)]

        def feed(k, ux, pxy):
            pending[flows[k]].append((ux, pxy))

        for _ in range(training_steps):
            run.seconds_dsmc += collect_windows(solvers, samples_per_step, steps_per_sample,
                                                group, feed)
            t0 = time.perf_counter()
            for f, t in enumerate(trainers):
                ux = np.stack([w[0] for w in pending[f]])
                pxy = np.stack([w[1] for w in pending[f]])
                t.add(ux, pxy)
                if keep_windows:
                    run.log.append((f, ux, pxy))
                pending[f] = []
                t.train()
            run.seconds_train += time.perf_counter() - t0
            run.windows += samples_per_step
            if on_step is not None:
                on_step(len(trainers[0].history) - 1, run)
        return run
    finally:
        if group is not None:
            group.close()
        for s in solvers:
            s.close()
