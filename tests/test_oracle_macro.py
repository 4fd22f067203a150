"""Pins of the finite-difference macro-model oracle (Eqs. 7-10, 14) against
closed forms of plane Poiseuille flow, the momentum balance, symmetry and its
order of accuracy."""
import math

import numpy as np

from oracle import macro as om


def test_no_slip_poiseuille_is_exact():
    """S = 0, no-slip: the Stokes solution u = sqrt(pi) F / (2 Kn) y (1 - y)
    (Eq. 3 in the units of Eq. 6), which second differences reproduce exactly."""
    for kn, F in ((0.1, 0.014), (1.0, 0.037), (5.0, 0.04)):
        y, u, P = om.solve(kn, F, 0.0, [], [], 64)
        want = math.sqrt(math.pi) * F / (2 * kn) * y * (1 - y)
        assert np.allclose(u, want, rtol=0, atol=1e-13 * want.max())
        assert np.allclose(P, 2 * F * (y - 0.5), atol=1e-12 * F)


def test_slip_poiseuille_is_exact():
    """S = 0 with the slip condition u(0) = -sigma P(0), u(1) = sigma P(1):
    the parabola lifted by sigma F (the wall stress is -F and +F)."""
    for kn, F, sig in ((0.1, 0.014, 0.84), (1.0, 0.037, 1.3)):
        y, u, P = om.solve(kn, F, sig, [], [], 50)
        want = math.sqrt(math.pi) * F / (2 * kn) * y * (1 - y) + sig * F
        assert np.allclose(u, want, rtol=0, atol=1e-12 * want.max())
        assert math.isclose(u[0], -sig * P[0], rel_tol=1e-10)
        assert math.isclose(u[-1], sig * P[-1], rel_tol=1e-10)


def test_corrected_model_keeps_the_momentum_balance():
    """With any correction and slip the stress is 2F(y - 1/2) (Eqs. 5 and 7),
    to the scheme's second order."""
    kn, F, sig, a, b = 0.2, 0.02, 0.9, [0.05, -0.03], [20.0, 12.0]
    errs = []
    for n in (100, 200, 400):
        y, u, P = om.solve(kn, F, sig, a, b, n)
        errs.append(np.abs(P - 2 * F * (y - 0.5)).max())
    assert errs[-1] < 1e-3 * F
    assert 3.0 < errs[0] / errs[1] < 5.0 and 3.0 < errs[1] / errs[2] < 5.0


def test_second_order_convergence_and_symmetry():
    kn, F, sig, a, b = 1.0, 0.037, 1.05, [-0.27, 0.29, 0.12], [8.0, 6.0, 20.0]
    us = [om.solve(kn, F, sig, a, b, n)[1] for n in (100, 200, 400)]
    d1 = np.abs(us[1][::2] - us[0]).max()
    d2 = np.abs(us[2][::4] - us[1][::2]).max()
    assert 3.5 < d1 / d2 < 4.5
    for u in us:
        assert np.allclose(u, u[::-1], rtol=0, atol=1e-10 * np.abs(u).max())


def test_monte_carlo_std_closed_forms():
    """Equal draws give no spread; draws of the slip coefficient alone shift
    the whole profile by sigma F, so the spread is F times theirs (without a
    correction, so that the scheme's wall stress is exactly -F)."""
    kn, F, b = 0.5, 0.03, [10.0]
    _, sd = om.monte_carlo_std(kn, F, [0.9] * 5, np.full((5, 1), 0.02), b, 40)
    assert np.all(sd < 1e-15)
    sig = np.array([0.8, 0.9, 1.0, 1.2, 0.95])
    _, sd = om.monte_carlo_std(kn, F, sig, np.zeros((5, 1)), b, 40)
    assert np.allclose(sd, F * np.std(sig, ddof=1), rtol=1e-9)
