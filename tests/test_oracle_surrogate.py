"""Pins of the surrogate-model oracle (Sec. 2.2, Eqs. 11-17, Appendix A)
against what the mathematics and the library the paper names fix."""
import math

import numpy as np
import pytest
from sklearn.linear_model import BayesianRidge

from oracle import surrogate as S


@pytest.mark.parametrize("N,M,noise,seed", [(400, 1, 0.1, 1), (800, 2, 1.0, 2), (300, 3, 0.05, 3),
                                            (2000, 3, 2.0, 4)])
def test_bayesian_ridge_matches_the_library_the_paper_used(N, M, noise, seed):
    """The paper trains with scikit-learn's Bayesian ridge regression (Sec.
    2.2); the oracle, written from Tipping's Appendix A with MacKay's
    re-estimation, must reach the same weights and precisions."""
    rng = np.random.default_rng(seed)
    Phi = rng.normal(size=(N, M))
    w = rng.normal(size=M)
    t = Phi @ w + rng.normal(scale=noise, size=N)
    r = S.bayesian_ridge(Phi, t)
    br = BayesianRidge(fit_intercept=False, compute_score=True).fit(Phi, t)
    assert np.allclose(r["m"], br.coef_, rtol=1e-9, atol=1e-12)
    assert math.isclose(r["alpha"], br.lambda_, rel_tol=1e-9)
    assert math.isclose(r["beta"], br.alpha_, rel_tol=1e-9)
    assert np.allclose(r["S"], br.sigma_, rtol=1e-8, atol=1e-14)
    # the library's score adds the log hyperprior densities (rates 1e-6)
    assert abs(r["log_evidence"] - br.scores_[-1]) < 1e-3


def test_bayesian_ridge_fixed_point():
    """At convergence alpha = gamma / m.m and beta = (N - gamma) / |t - Phi m|^2
    with gamma = sum beta l / (alpha + beta l) over the eigenvalues l of Phi'Phi
    (without hyperprior terms, up to the stopping tolerance)."""
    rng = np.random.default_rng(7)
    Phi = rng.normal(size=(1000, 2))
    t = Phi @ np.array([0.3, -0.7]) + rng.normal(scale=0.5, size=1000)
    r = S.bayesian_ridge(Phi, t, tol=1e-12, max_iter=1000, h=0.0)
    lam = np.linalg.eigvalsh(Phi.T @ Phi)
    gamma = float(np.sum(r["beta"] * lam / (r["alpha"] + r["beta"] * lam)))
    res = t - Phi @ r["m"]
    assert math.isclose(r["alpha"], gamma / float(r["m"] @ r["m"]), rel_tol=1e-6)
    assert math.isclose(r["beta"], (1000 - gamma) / float(res @ res), rel_tol=1e-6)
    # posterior moments are the closed forms at those precisions
    A = r["alpha"] * np.eye(2) + r["beta"] * Phi.T @ Phi
    assert np.allclose(r["S"], np.linalg.inv(A))
    assert np.allclose(r["m"], r["beta"] * np.linalg.solve(A, Phi.T @ t))


def test_log_evidence_is_the_gaussian_marginal_likelihood():
    """Bishop Eq. 3.86 equals the log density of t under N(0, I/beta + Phi Phi'/alpha)."""
    rng = np.random.default_rng(11)
    Phi = rng.normal(size=(60, 2))
    t = Phi @ np.array([1.0, 0.5]) + rng.normal(scale=0.8, size=60)
    r = S.bayesian_ridge(Phi, t)
    C = np.eye(60) / r["beta"] + Phi @ Phi.T / r["alpha"]
    sign, logdet = np.linalg.slogdet(C)
    direct = -0.5 * (60 * math.log(2 * math.pi) + logdet + float(t @ np.linalg.solve(C, t)))
    assert math.isclose(r["log_evidence"], direct, rel_tol=1e-10)


def test_zero_order_model_evidence():
    """A model without weights (no-slip, C_0) is t ~ N(0, 1/beta): the
    evidence at the MAP noise precision, in closed form."""
    t = np.array([0.3, -0.1, 0.2, 0.05, -0.25])
    r = S.bayesian_ridge(np.zeros((5, 0)), t, h=0.0)
    beta = 5 / float(t @ t)
    want = 2.5 * math.log(beta) - 0.5 * beta * float(t @ t) - 2.5 * math.log(2 * math.pi)
    assert math.isclose(r["beta"], beta, rel_tol=1e-12)
    assert math.isclose(r["log_evidence"], want, rel_tol=1e-12)


def test_model_probabilities_are_normalised_bayes():
    p = S.model_probabilities([-10.0, -10.0, -10.0])
    assert np.allclose(p, [1 / 3] * 3)
    p = S.model_probabilities([0.0, math.log(3.0)])
    assert np.allclose(p, [0.25, 0.75])
    p = S.model_probabilities([-1e6, 0.0, -1e6])
    assert p[1] == 1.0 and sum(p) == 1.0


def test_velocity_gradient_exact_for_quadratics():
    """Second-order central and one-sided differences are exact on quadratics."""
    n = 40
    dy = 1.0 / n
    y = (np.arange(n) + 0.5) * dy
    u = 0.3 + 1.7 * y - 2.2 * y * y
    g = S.velocity_gradient(list(u), dy)
    assert np.allclose(g, 1.7 - 4.4 * y, atol=1e-12)


def test_newton_error_vanishes_for_newtons_law():
    """E = P + 2 Kn/sqrt(pi) du/dy is zero when the stress obeys Newton's law
    in the units of Eq. 6 (P = -2 Kn/sqrt(pi) du/dy, Eq. 7 with S = 0)."""
    n, kn, F = 50, 0.3, 0.01
    y = (np.arange(n) + 0.5) / n
    c = 2 * kn / math.sqrt(math.pi)
    u = F / c * y * (1 - y)        # parabola: du/dy = F/c (1 - 2y)
    P = -c * (F / c) * (1 - 2 * y)  # = 2F(y - 1/2), the Cauchy stress line
    assert np.allclose(S.newton_error(list(u), list(P), 1.0 / n, kn), 0.0, atol=1e-12)


def test_basis_is_antisymmetric_and_table_lookup():
    for b in (7.0, 20.0, 130.0):
        for y in (0.01, 0.2, 0.5, 0.73):
            assert math.isclose(S.basis(1 - y, 0.2, b), -S.basis(y, 0.2, b), abs_tol=1e-15)
    assert S.basis(0.5, 0.2, 10.0) == 0.0
    assert S.exponents(0.1) == (20.0, 40.0, 10.0)
    assert S.exponents(1.0) == (8.0, 6.0, 20.0)
    assert S.exponents(0.07) == (30.0, 40.0, 70.0)   # nearer 0.05 than 0.1 in log(Kn)
    assert S.exponents(50.0) == (7.0, 6.0, 5.0)


def test_selection_recovers_a_planted_stress_correction():
    """Samples whose Newton-law error is 2Kn/sqrt(pi) S_2(y) plus noise: the
    models with the planted terms win clearly over C_0 and C_1, and C_2's
    weights are recovered within their posterior uncertainty."""
    rng = np.random.default_rng(5)
    kn, n_p, n_s = 0.1, 60, 200
    b = S.exponents(kn)
    a = np.array([-0.04, 0.03])
    y = (np.arange(n_p) + 0.5) / n_p
    corr = sum(a[l] * np.array([S.basis(v, kn, b[l]) for v in y]) for l in range(2))
    # u with zero gradient in the interior and edges, so E = P exactly
    us = [np.zeros(n_p) for _ in range(n_s)]
    Ps = [corr + rng.normal(scale=0.002, size=n_p) for _ in range(n_s)]
    logs, fits = [], []
    for k in range(4):
        Phi, t = S.constitutive_system(us, Ps, kn, k)
        r = S.bayesian_ridge(Phi, t)
        logs.append(r["log_evidence"])
        fits.append(r)
    p = S.model_probabilities(logs)
    assert p[2] + p[3] > 0.999 and p[0] < 1e-100 and p[1] < 1e-10
    m, Sd = fits[2]["m"], np.sqrt(np.diag(fits[2]["S"]))
    assert np.all(np.abs(m - a) < 4 * Sd), (m, a, Sd)


def test_wall_velocity_extrapolation_is_exact_for_linear_profiles():
    """Half a cell beyond the first centre: exact for a profile linear near
    each plate; the cell reading returns the end cells."""
    n = 16
    y = (np.arange(n) + 0.5) / n
    u = np.where(y < 0.5, 0.2 + 3.0 * y, 0.2 + 3.0 * (1 - y))
    ub, ut = S.wall_velocities(list(u))
    assert math.isclose(ub, 0.2, abs_tol=1e-15) and math.isclose(ut, 0.2, abs_tol=1e-15)
    assert S.wall_velocities(list(u), "cell") == (u[0], u[-1])
    with pytest.raises(ValueError):
        S.wall_velocities(list(u), "centre")


def test_slip_model_recovers_the_slip_coefficient():
    """Wall velocities sigma F plus noise (Eq. 12 with P = -F, +F at the
    plates): the slip model wins and sigma is recovered."""
    rng = np.random.default_rng(9)
    F, sigma = 0.01, 1.3
    us = []
    for _ in range(300):
        u = np.zeros(20)
        u[0] = sigma * F + rng.normal(scale=0.004)
        u[-1] = sigma * F + rng.normal(scale=0.004)
        us.append(u)
    fits = [S.bayesian_ridge(*S.slip_system(us, F, slip, wall="cell")) for slip in (False, True)]
    p = S.model_probabilities([f["log_evidence"] for f in fits])
    assert p[1] > 0.999
    m, sd = fits[1]["m"][0], math.sqrt(fits[1]["S"][0, 0])
    assert abs(m - sigma) < 4 * sd
    # the same plates seen through the extrapolated reading: u_w = 1.5 u_1
    ext = S.bayesian_ridge(*S.slip_system(us, F, True))
    assert abs(ext["m"][0] - 1.5 * sigma) < 4 * 1.5 * sd
