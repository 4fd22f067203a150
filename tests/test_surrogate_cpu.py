"""Parity of the surrogate trainer (sufficient statistics, eigenbasis
regression) with the plain oracle (full design matrices, step-by-step
re-estimation) on identical seeded windows, and its host-side behaviour."""
import math

import numpy as np
import pytest

from oracle import surrogate as ref
from paper_2311_14140_amd import surrogate as sg


def synthetic_windows(kn, force, n_cells, n_samples, seed, sigma=1.1, a=(-0.03, 0.02, 0.0),
                      noise_u=0.01, noise_p=0.004):
    """Profiles shaped like DSMC windows of the force-driven channel: a slip
    parabola for u, the momentum-balance line plus a Knudsen-layer correction
    for P, and independent Gaussian noise per cell and window."""
    rng = np.random.default_rng(seed)
    y = (np.arange(n_cells) + 0.5) / n_cells
    c = 2 * kn / math.sqrt(math.pi)
    u0 = sigma * force + force / c * y * (1 - y)
    b = ref.exponents(kn)
    corr = sum(a[l] * c * (np.exp(-b[l] * y) - np.exp(-b[l] * (1 - y))) for l in range(3))
    p0 = 2 * force * (y - 0.5) + corr
    ux = u0[None, :] + rng.normal(scale=noise_u, size=(n_samples, n_cells))
    pxy = p0[None, :] + rng.normal(scale=noise_p, size=(n_samples, n_cells))
    return ux, pxy


def oracle_step(ux, pxy, kn, force, wall="extrapolated"):
    us, Ps = list(ux), list(pxy)
    cons = [ref.bayesian_ridge(*ref.constitutive_system(us, Ps, kn, k)) for k in range(4)]
    bnd = [ref.bayesian_ridge(*ref.slip_system(us, force, s, wall)) for s in (False, True)]
    return cons, bnd


def assert_posterior_equal(p, r, what):
    assert p.n_iter == r["n_iter"], what
    assert np.allclose(p.m, r["m"], rtol=1e-9, atol=1e-13), what
    assert np.allclose(p.S, r["S"], rtol=1e-8, atol=1e-16), what
    if len(p.m):
        assert math.isclose(p.alpha, r["alpha"], rel_tol=1e-9), what
    assert math.isclose(p.beta, r["beta"], rel_tol=1e-9), what
    assert abs(p.log_evidence - r["log_evidence"]) < 1e-7 * max(1.0, abs(r["log_evidence"])), what


@pytest.mark.parametrize("kn,force,n_cells,n_samples,seed,wall", [
    (0.1, 0.0142, 200, 100, 1, "extrapolated"), (1.0, 0.0374, 200, 100, 2, "extrapolated"),
    (0.5, 0.03, 64, 300, 3, "cell"), (0.05, 0.0084, 200, 40, 4, "extrapolated"),
    (1.0, 0.0374, 200, 100, 2, "cell")])
def test_training_step_matches_oracle(kn, force, n_cells, n_samples, seed, wall):
    ux, pxy = synthetic_windows(kn, force, n_cells, n_samples, seed)
    t = sg.SurrogateTrainer(kn, force, n_cells, wall=wall)
    assert t.exponents == ref.exponents(kn)
    t.add(ux, pxy)
    step = t.train()
    cons, bnd = oracle_step(ux, pxy, kn, force, wall)
    for k in range(4):
        assert_posterior_equal(step.constitutive[k], cons[k], f"C_{k}")
    assert_posterior_equal(step.boundary[0], bnd[0], "no-slip")
    assert_posterior_equal(step.boundary[1], bnd[1], "slip")
    assert np.allclose(step.p_constitutive, ref.model_probabilities([c["log_evidence"] for c in cons]),
                       atol=1e-9)
    assert np.allclose(step.p_boundary, ref.model_probabilities([b["log_evidence"] for b in bnd]),
                       atol=1e-9)


def test_newton_error_matches_oracle():
    ux, pxy = synthetic_windows(0.2, 0.02, 37, 3, 8)
    t = sg.SurrogateTrainer(0.2, 0.02, 37)
    E = t.newton_error(ux, pxy)
    for j in range(3):
        want = ref.newton_error(list(ux[j]), list(pxy[j]), 1.0 / 37, 0.2)
        assert np.allclose(E[j], want, rtol=1e-12, atol=1e-15)


def test_windows_accumulate():
    """Training on windows added one batch at a time equals training on all
    of them at once (the sufficient statistics are sums)."""
    ux, pxy = synthetic_windows(0.1, 0.014, 200, 300, 5)
    a = sg.SurrogateTrainer(0.1, 0.014, 200)
    for lo in range(0, 300, 100):
        a.add(ux[lo:lo + 100], pxy[lo:lo + 100])
        a.train()
    b = sg.SurrogateTrainer(0.1, 0.014, 200)
    for j in range(300):
        b.add(ux[j], pxy[j])
    sb = b.train()
    sa = a.history[-1]
    assert len(a.history) == 3 and sa.n_samples == 300
    for k in range(4):
        assert np.allclose(sa.constitutive[k].m, sb.constitutive[k].m, rtol=1e-10, atol=1e-14)
        assert math.isclose(sa.constitutive[k].log_evidence, sb.constitutive[k].log_evidence,
                            rel_tol=1e-11)
    assert np.allclose(sa.p_boundary, sb.p_boundary)


def test_cell_subset_matches_oracle_rows():
    """Constitutive targets restricted to a set of cells equal the oracle's
    system with the other rows dropped (the gradient still over the whole
    profile)."""
    kn, F, C, S = 0.2, 0.02, 80, 50
    ux, pxy = synthetic_windows(kn, F, C, S, 6)
    cells = np.r_[0:20, 60:80]
    t = sg.SurrogateTrainer(kn, F, C, cells=cells)
    t.add(ux, pxy)
    step = t.train()
    keep = np.concatenate([j * C + cells for j in range(S)])
    for k in range(4):
        Phi, tv = ref.constitutive_system(list(ux), list(pxy), kn, k)
        r = ref.bayesian_ridge(Phi[keep], tv[keep])
        assert_posterior_equal(step.constitutive[k], r, f"C_{k}")


def test_selection_on_planted_models():
    """Slip data select the slip model at once; a planted two-term stress
    correction rejects C_0 and C_1 and recovers the planted weights."""
    kn, F = 0.1, 0.0142
    # (u noise small: the finite-difference gradient multiplies it by 1/dy)
    ux, pxy = synthetic_windows(kn, F, 200, 200, 7, sigma=1.1, a=(-0.05, 0.04, 0.0),
                                noise_u=0.0002)
    t = sg.SurrogateTrainer(kn, F, 200)
    t.add(ux, pxy)
    s = t.train()
    assert s.slip and s.p_boundary[1] > 1 - 1e-12
    # extrapolated to the plate, the planted parabola's wall value is sigma F
    assert abs(s.sigma_p - 1.1) < 4 * math.sqrt(s.boundary[1].S[0, 0])
    # read in the first cell, half a cell from the plate, it is larger
    c = sg.SurrogateTrainer(kn, F, 200, wall="cell")
    c.add(ux, pxy)
    y0 = 0.5 / 200
    sigma_cell = 1.1 + y0 * (1 - y0) / (2 * kn / math.sqrt(math.pi))
    sc = c.train()
    assert abs(sc.sigma_p - sigma_cell) < 4 * math.sqrt(sc.boundary[1].S[0, 0])
    assert s.p_constitutive[0] < 1e-12 and s.p_constitutive[1] < 1e-6
    m2 = s.constitutive[2]
    sd = np.sqrt(np.diag(m2.S))
    assert np.all(np.abs(m2.m - [-0.05, 0.04]) < 4 * sd)


def test_posterior_draws_have_the_posterior_moments():
    kn, F = 1.0, 0.0374
    ux, pxy = synthetic_windows(kn, F, 100, 100, 9)
    t = sg.SurrogateTrainer(kn, F, 100)
    t.add(ux, pxy)
    p = t.train().constitutive[3]
    w = p.draw(200000, np.random.default_rng(0))
    assert w.shape == (200000, 3)
    se = np.sqrt(np.diag(p.S) / 200000)
    assert np.all(np.abs(w.mean(0) - p.m) < 5 * se)
    assert np.allclose(np.cov(w.T), p.S, rtol=0.03, atol=1e-3 * np.abs(p.S).max())
    assert t.history[-1].boundary[0].draw(3, np.random.default_rng(0)).shape == (3, 0)


def test_rejects_bad_windows():
    t = sg.SurrogateTrainer(0.1, 0.01, 50)
    with pytest.raises(ValueError):
        t.add(np.zeros(49), np.zeros(49))
    with pytest.raises(ValueError):
        t.add(np.full(50, np.nan), np.zeros(50))
    with pytest.raises(ValueError):
        t.train()
    with pytest.raises(ValueError):
        sg.SurrogateTrainer(0.1, 0.01, 2)
    with pytest.raises(ValueError):
        sg.SurrogateTrainer(0.1, 0.01, 50, max_order=4)
    with pytest.raises(ValueError):
        sg.SurrogateTrainer(0.1, 0.01, 50, wall="plate")


def test_table_lookup_matches_oracle():
    for kn in (0.01, 0.02, 0.03, 0.07, 0.1, 0.14, 0.15, 0.3, 0.7, 1.0, 2.2, 5.0, 40.0):
        assert sg.table_exponents(kn) == ref.exponents(kn)


def test_patch_training_matches_oracle():
    """A patch of the hybrid: 25 cells of width 0.004 next to the bottom
    plate, the last 5 a buffer left out of the constitutive targets, and
    the bottom plate's wall velocity alone."""
    kn, F, C, dy, ntr = 0.05, 0.0084, 25, 0.004, 20
    rng = np.random.default_rng(12)
    y = (np.arange(C) + 0.5) * dy
    c = 2 * kn / math.sqrt(math.pi)
    ux = 0.8 * F + F / c * y * (1 - y) + rng.normal(scale=0.004, size=(150, C))
    pxy = 2 * F * (y - 0.5) + rng.normal(scale=0.003, size=(150, C))
    t = sg.SurrogateTrainer(kn, F, C, cells=np.arange(ntr), dy=dy, plates=1)
    t.add(ux, pxy)
    step = t.train()
    us, Ps = list(ux), list(pxy)
    for k in range(4):
        r = ref.bayesian_ridge(*ref.constitutive_system(us, Ps, kn, k, dy=dy, n_train=ntr))
        assert_posterior_equal(step.constitutive[k], r, f"C_{k}")
    for slip in (False, True):
        r = ref.bayesian_ridge(*ref.slip_system(us, F, slip, plates=1))
        assert_posterior_equal(step.boundary[int(slip)], r, "slip" if slip else "no-slip")
    assert step.boundary[1].n_data == 150
