"""Plain reference solution of the corrected macroscopic model (Sec. 2.1:
Eq. 7 corrected Newton law, Eq. 8 macro equation, Eq. 9 no-slip and Eq. 10
slip boundary conditions, Eq. 14 stress correction) and of the Monte Carlo
uncertainty of Sec. 2.2.

TEST INFRASTRUCTURE: only tests/, the smoke entry point and the bench's CPU
baseline may import this module.  It solves the boundary-value problem
numerically, by second-order finite differences on a uniform grid of nodes
including the two plates, with no use of its closed-form solution, so that
it checks an exact solver independently:

  interior nodes   (u[i-1] - 2 u[i] + u[i+1]) / h^2 = -(sqrt(pi)/Kn) F + S'(y_i)
  slip at y = 0    u[0] = -sigma_P P(0),  P(0) = -c u'(0) + c S(0)
  slip at y = 1    u[n] =  sigma_P P(1),  P(1) = -c u'(1) + c S(1)
  no-slip          u[0] = u[n] = 0

with c = 2 Kn / sqrt(pi), S' the derivative of Eq. 14 and u' at the plates
by second-order one-sided differences.  The dense linear system is solved by
a library routine.  P along the gap follows from Eq. 7 with central
differences inside.
"""
from __future__ import annotations

import math

import numpy as np


def correction(y, a, b):
    """S(y) = sum_l a_l (exp(-b_l y) - exp(-b_l (1 - y))) (Eq. 14, plates at 0 and 1)."""
    s = 0.0
    for l in range(len(a)):
        s += a[l] * (math.exp(-b[l] * y) - math.exp(-b[l] * (1.0 - y)))
    return s


def correction_slope(y, a, b):
    """dS/dy of Eq. 14."""
    s = 0.0
    for l in range(len(a)):
        s += a[l] * (-b[l] * math.exp(-b[l] * y) - b[l] * math.exp(-b[l] * (1.0 - y)))
    return s


def solve(kn, force, sigma_p, a, b, n):
    """Nodes y_i = i / n and the finite-difference velocity u_i and shear
    stress P_i of Eqs. 7-8 with the slip condition of Eq. 10 (sigma_p = 0
    gives the no-slip condition of Eq. 9)."""
    h = 1.0 / n
    c = 2.0 * kn / math.sqrt(math.pi)
    y = [i * h for i in range(n + 1)]
    A = np.zeros((n + 1, n + 1))
    r = np.zeros(n + 1)
    for i in range(1, n):
        A[i, i - 1] = 1.0 / (h * h)
        A[i, i] = -2.0 / (h * h)
        A[i, i + 1] = 1.0 / (h * h)
        r[i] = -(math.sqrt(math.pi) / kn) * force + correction_slope(y[i], a, b)
    # u[0] = -sigma (-c u'(0) + c S(0)), i.e. u[0] - sigma c u'(0) = -sigma c S(0),
    # u'(0) = (-3u0 + 4u1 - u2) / 2h
    A[0, 0] = 1.0 - sigma_p * c * (-3.0) / (2.0 * h)
    A[0, 1] = -sigma_p * c * 4.0 / (2.0 * h)
    A[0, 2] = -sigma_p * c * (-1.0) / (2.0 * h)
    r[0] = -sigma_p * c * correction(0.0, a, b)
    # u[n] = sigma (-c u'(1) + c S(1)), i.e. u[n] + sigma c u'(1) = sigma c S(1),
    # u'(1) = (3un - 4un-1 + un-2) / 2h
    A[n, n] = 1.0 + sigma_p * c * 3.0 / (2.0 * h)
    A[n, n - 1] = sigma_p * c * (-4.0) / (2.0 * h)
    A[n, n - 2] = sigma_p * c * 1.0 / (2.0 * h)
    r[n] = sigma_p * c * correction(1.0, a, b)
    u = np.linalg.solve(A, r)
    P = np.zeros(n + 1)
    for i in range(n + 1):
        if i == 0:
            du = (-3.0 * u[0] + 4.0 * u[1] - u[2]) / (2.0 * h)
        elif i == n:
            du = (3.0 * u[n] - 4.0 * u[n - 1] + u[n - 2]) / (2.0 * h)
        else:
            du = (u[i + 1] - u[i - 1]) / (2.0 * h)
        P[i] = -c * du + c * correction(y[i], a, b)
    return np.array(y), u, P


def monte_carlo_std(kn, force, sigma_draws, a_draws, b, n):
    """Standard deviation over trials of the finite-difference velocity, one
    solve per drawn weight set (Sec. 2.2); the draws are inputs."""
    runs = []
    for t in range(len(a_draws)):
        _, u, _ = solve(kn, force, sigma_draws[t], list(a_draws[t]), b, n)
        runs.append(u)
    runs = np.array(runs)
    return runs.mean(axis=0), runs.std(axis=0, ddof=1)
