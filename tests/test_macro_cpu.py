"""Parity of the closed-form macro model (Eqs. 7-10 with the correction of
Eq. 14) and its uncertainty propagation with the finite-difference oracle."""
import math

import numpy as np
import pytest
from scipy.integrate import simpson

from oracle import macro as om
from oracle.surrogate import exponents
from paper_2311_14140_amd import macro as mc
from paper_2311_14140_amd import surrogate as sg


def richardson(kn, F, sig, a, b, n):
    """Oracle velocity at the nodes i/n, extrapolated from n and 2n (the
    scheme's error is second order in h, so the estimate is third order)."""
    y, u, P = om.solve(kn, F, sig, list(a), list(b), n)
    _, u2, P2 = om.solve(kn, F, sig, list(a), list(b), 2 * n)
    return y, (4 * u2[::2] - u) / 3, (4 * P2[::2] - P) / 3


CASES = [(0.01, 0.002, 0.9, (-0.01, 0.02, 0.004)), (0.1, 0.0142, 0.84, (-0.047, 0.1, 0.068)),
         (0.5, 0.0316, 1.0, (0.03, -0.05, 0.02)), (1.0, 0.0374, 1.05, (-0.27, 0.29, 0.12)),
         (5.0, 0.0437, 1.9, (0.4, -0.3, 0.1)), (1.0, 0.0374, 0.0, (-0.27, 0.29)),
         (0.1, 0.0142, 0.84, ())]


@pytest.mark.parametrize("kn,F,sig,a", CASES)
def test_velocity_and_stress_match_the_oracle(kn, F, sig, a):
    b = exponents(kn)[:len(a)]
    y, u_ref, P_ref = richardson(kn, F, sig, a, b, 1000)
    m = mc.MacroModel(kn, F, sig, a, b)
    u = m.velocity(y)
    # the extrapolated oracle is good to a few 1e-7 of the peak velocity; its
    # one-sided wall differences are the coarsest part at b h = 0.2 (Kn 0.01)
    assert np.abs(u - u_ref).max() < 2e-6 * np.abs(u_ref).max()
    assert np.abs(m.shear_stress(y) - P_ref).max() < 1e-4 * F
    grad_ref = m.correction(y) - P_ref / m.c      # Eq. 7 solved for du/dy
    assert np.abs(m.velocity_gradient(y) - grad_ref).max() < 5e-5 * np.abs(grad_ref).max()
    assert math.isclose(m.mass_flow(), simpson(u_ref, x=y), rel_tol=2e-6)


def test_monte_carlo_matches_oracle_solves():
    """The same weight draws through the closed form and through one
    oracle solve per draw give the same spread."""
    rng = np.random.default_rng(3)
    kn, F = 1.0, 0.0374
    ux = 0.05 + rng.normal(scale=0.01, size=(100, 100))
    pxy = 2 * F * ((np.arange(100) + 0.5) / 100 - 0.5) + rng.normal(scale=0.004, size=(100, 100))
    t = sg.SurrogateTrainer(kn, F, 100, max_order=2)
    t.add(ux, pxy)
    step = t.train()
    step.p_constitutive = np.array([0.0, 0.0, 1.0])        # select C_2, slip
    step.p_boundary = np.array([0.0, 1.0])
    n_tr = 60
    sd_sig = np.array([1.0, 0.9, 1.15])[rng.integers(0, 3, n_tr)] + rng.normal(0, 0.05, n_tr)
    sd_a = rng.normal(size=(n_tr, 2)) * [0.05, 0.04] + [-0.2, 0.25]
    y_ref, _, _ = om.solve(kn, F, 0.0, [], [], 200)
    sol = mc.solve_selected(t, step, y_ref, draws=(sd_sig, sd_a))
    b = t.exponents[:2]
    runs = []
    for i in range(n_tr):
        runs.append(richardson(kn, F, sd_sig[i], sd_a[i], b, 200)[1])
    runs = np.array(runs)
    assert sol.n_trials == n_tr
    assert np.allclose(sol.u_mc_mean, runs.mean(0), rtol=0, atol=1e-5 * np.abs(runs).max())
    assert np.allclose(sol.u_std, runs.std(0, ddof=1), rtol=1e-3, atol=1e-9)


def test_monte_carlo_spread_matches_the_posterior():
    """1000 trials (Sec. 3) estimate the exact linear-propagation spread to
    within their sampling error; more trials tighten it."""
    rng = np.random.default_rng(4)
    kn, F = 0.1, 0.0142
    y = (np.arange(200) + 0.5) / 200
    ux = 0.84 * F + F / (2 * kn / math.sqrt(math.pi)) * y * (1 - y) + rng.normal(scale=0.002, size=(300, 200))
    pxy = 2 * F * (y - 0.5) + rng.normal(scale=0.004, size=(300, 200))
    t = sg.SurrogateTrainer(kn, F, 200)
    t.add(ux, pxy)
    step = t.train()
    yy = np.linspace(0, 1, 101)
    sol = mc.solve_selected(t, step, yy, n_trials=1000, rng=np.random.default_rng(5))
    assert sol.slip
    # relative standard error of a standard deviation from n draws: 1/sqrt(2(n-1))
    assert np.all(np.abs(sol.u_std / sol.u_std_exact - 1) < 5 / math.sqrt(2 * 999))
    big = mc.solve_selected(t, step, yy, n_trials=200000, rng=np.random.default_rng(6))
    assert np.all(np.abs(big.u_std / big.u_std_exact - 1) < 5 / math.sqrt(2 * 199999))
    lo, hi = sol.ci95
    assert np.all(hi - lo > 0) and np.allclose(hi - sol.u, 2 * sol.u_std)


def test_no_slip_selection_gives_zero_wall_velocity():
    t = sg.SurrogateTrainer(0.1, 0.0142, 50)
    rng = np.random.default_rng(7)
    t.add(rng.normal(scale=0.01, size=(50, 50)), rng.normal(scale=0.01, size=(50, 50)))
    step = t.train()
    step.p_boundary = np.array([1.0, 0.0])
    step.p_constitutive = np.array([1.0, 0.0, 0.0, 0.0])
    sol = mc.solve_selected(t, step, np.array([0.0, 0.5, 1.0]), n_trials=100)
    assert not sol.slip and sol.order == 0
    assert sol.u[0] == 0.0 and sol.u[2] == 0.0
    assert np.all(sol.u_std < 1e-15) and np.all(sol.u_std_exact == 0.0)
