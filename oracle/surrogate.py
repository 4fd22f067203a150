"""Plain reference implementation of the paper's surrogate models (Sec. 2.2,
Eqs. 11-16 and Appendix A) and their Bayesian training and selection (Eq. 17).

TEST INFRASTRUCTURE: only tests/, the smoke entry point and the bench's CPU
baseline may import this module.  It is written step by step from the paper
and from the textbook algorithm it names (Bayesian ridge regression with the
evidence maximised by MacKay's re-estimation, as in Tipping's Appendix A),
with no vectorised shortcuts, so that it can be checked against the text.

Readings of points the paper leaves open (each one a choice of this
reference, stated where it is used):
  - du/dy of the Newton-law error E (Eq. 13): second-order central
    differences in the interior cells and second-order one-sided
    differences in the first and last cells, on cell-centred values.
  - The velocity "at the wall" of the slip models (Eqs. 11-12), u(y_bot)
    and u(y_top): the cell-centred profile extrapolated linearly to the
    plate from the two cells next to it, u_w = (3 u_1 - u_2) / 2, half a
    cell beyond the first centre.  (The value of the first cell itself,
    half a cell from the plate, is kept as an option.)
  - The wall shear stress P^CFD of the slip model: for the force-driven
    channel the momentum balance fixes P_xy = 2F(y - 1/2) whatever the
    constitutive law, so P = -F at the bottom plate and +F at the top (the
    units of Eq. 6).
  - Exponents b_l of the stress correction (Table 1): the column of the
    tabulated Kn nearest in log(Kn).
  - Bayesian ridge regression: initial noise precision 1/Var(t) and weight
    precision 1; Gamma hyperpriors with shape and rate 1e-6 on both
    precisions; stop when the weights change by less than 1e-3 in sum of
    absolute values, or after 300 updates (the defaults of the library the
    paper used).  The evidence of a model is the log marginal likelihood
    at the final precisions (Bishop Eq. 3.86); a model without weights has
    the noise precision as its only parameter.
"""
from __future__ import annotations

import math

import numpy as np

# Table 1: exponents of the stress-correction basis functions per Kn.
TABLE1_KN = (0.01, 0.05, 0.1, 0.2, 0.5, 1.0, 5.0)
TABLE1_B = ((130.0, 150.0, 200.0), (30.0, 40.0, 70.0), (20.0, 40.0, 10.0),
            (20.0, 12.0, 8.0), (10.0, 7.0, 6.0), (8.0, 6.0, 20.0), (7.0, 6.0, 5.0))


def exponents(kn):
    """Table 1 column for the tabulated Kn nearest to kn in log(Kn)."""
    best = 0
    for q in range(len(TABLE1_KN)):
        if abs(math.log(TABLE1_KN[q] / kn)) < abs(math.log(TABLE1_KN[best] / kn)):
            best = q
    return TABLE1_B[best]


def basis(y, kn, b):
    """phi(y) = 2 Kn / sqrt(pi) (exp(-b (y - y_bot)) - exp(-b (y_top - y))),
    plates at y_bot = 0 and y_top = 1 (Eq. 14 and Appendix A)."""
    c = 2.0 * kn / math.sqrt(math.pi)
    return c * (math.exp(-b * y) - math.exp(-b * (1.0 - y)))


def velocity_gradient(u, dy):
    """du/dy of a cell-centred profile: central differences inside,
    second-order one-sided at the two end cells."""
    n = len(u)
    g = [0.0] * n
    for i in range(1, n - 1):
        g[i] = (u[i + 1] - u[i - 1]) / (2.0 * dy)
    g[0] = (-3.0 * u[0] + 4.0 * u[1] - u[2]) / (2.0 * dy)
    g[n - 1] = (3.0 * u[n - 1] - 4.0 * u[n - 2] + u[n - 3]) / (2.0 * dy)
    return g


def newton_error(u, P, dy, kn):
    """E_i = P_i + 2 Kn / sqrt(pi) du/dy|_i (Eq. 13) for one sample."""
    c = 2.0 * kn / math.sqrt(math.pi)
    g = velocity_gradient(u, dy)
    return [P[i] + c * g[i] for i in range(len(u))]


def constitutive_system(us, Ps, kn, k, b=None, dy=None, n_train=None):
    """Target vector t_{i + j N_P} = E_{i,j} and design matrix of model C_k
    (Appendix A) from samples us[j][i], Ps[j][i] on cells of width dy from
    the bottom plate (default 1/len(us[j]): the whole gap).  n_train keeps
    the first n_train cells only (a patch of the hybrid, whose last cells
    are its buffer, Sec. 3.2); the gradient still uses every cell."""
    n_c = len(us[0])
    dy = 1.0 / n_c if dy is None else dy
    n_p = n_c if n_train is None else n_train
    b = exponents(kn) if b is None else b
    y = [(i + 0.5) * dy for i in range(n_c)]
    t = []
    rows = []
    for j in range(len(us)):
        e = newton_error(us[j], Ps[j], dy, kn)
        for i in range(n_p):
            t.append(e[i])
            rows.append([basis(y[i], kn, b[l]) for l in range(k)])
    return np.array(rows, dtype=np.float64).reshape(len(t), k), np.array(t, dtype=np.float64)


def wall_velocities(u, wall="extrapolated"):
    """u(y_bot), u(y_top) of one cell-centred profile: extrapolated to the
    plates from the two nearest cells, or the nearest cells' values."""
    n = len(u)
    if wall == "cell":
        return u[0], u[n - 1]
    if wall != "extrapolated":
        raise ValueError(wall)
    return 1.5 * u[0] - 0.5 * u[1], 1.5 * u[n - 1] - 0.5 * u[n - 2]


def slip_system(us, force, slip, wall="extrapolated", plates=2):
    """Targets u_j(y_bot), u_j(y_top) and the slip model's design column
    -P(y_bot) = F, P(y_top) = F (Eq. 12 and Appendix A); the no-slip model
    (Eq. 11) has no column.  plates = 1: the samples are patches at the
    bottom plate only (u_j(y_bot) alone)."""
    t = []
    rows = []
    for u in us:
        ub, ut = wall_velocities(u, wall)
        t.append(ub)
        rows.append([force] if slip else [])
        if plates == 2:
            t.append(ut)
            rows.append([force] if slip else [])
    return np.array(rows, dtype=np.float64).reshape(len(t), 1 if slip else 0), np.array(t, dtype=np.float64)


def bayesian_ridge(Phi, t, tol=1e-3, max_iter=300, h=1e-6):
    """Evidence-maximising Bayesian ridge regression.  Returns dict with the
    posterior mean m and covariance S of the weights, the weight precision
    alpha, the noise precision beta, the log evidence and the updates made."""
    N, M = Phi.shape
    beta = 1.0 / (float(np.var(t)) + np.finfo(np.float64).eps)
    alpha = 1.0
    if M == 0:
        # only the noise precision: its MAP value under the Gamma hyperprior
        rss = float(t @ t)
        beta = (N + 2.0 * h) / (rss + 2.0 * h)
        log_ev = 0.5 * N * math.log(beta) - 0.5 * beta * rss - 0.5 * N * math.log(2.0 * math.pi)
        return dict(m=np.zeros(0), S=np.zeros((0, 0)), alpha=float("nan"), beta=beta,
                    log_evidence=log_ev, n_iter=0)
    PtP = Phi.T @ Phi
    Ptt = Phi.T @ t
    m_old = None
    it = 0
    for it in range(1, max_iter + 1):
        A = alpha * np.eye(M) + beta * PtP
        S = np.linalg.inv(A)
        m = beta * (S @ Ptt)
        # effective number of well-determined parameters
        lam = np.linalg.eigvalsh(beta * PtP)
        gamma = sum(float(l) / (float(l) + alpha) for l in lam)
        r = t - Phi @ m
        rss = float(r @ r)
        alpha = (gamma + 2.0 * h) / (float(m @ m) + 2.0 * h)
        beta = (N - gamma + 2.0 * h) / (rss + 2.0 * h)
        if m_old is not None and float(np.sum(np.abs(m_old - m))) < tol:
            break
        m_old = m
    # posterior at the final precisions
    A = alpha * np.eye(M) + beta * PtP
    S = np.linalg.inv(A)
    m = beta * (S @ Ptt)
    r = t - Phi @ m
    E = 0.5 * beta * float(r @ r) + 0.5 * alpha * float(m @ m)
    sign, logdet = np.linalg.slogdet(A)
    log_ev = (0.5 * M * math.log(alpha) + 0.5 * N * math.log(beta) - E - 0.5 * logdet
              - 0.5 * N * math.log(2.0 * math.pi))
    return dict(m=m, S=S, alpha=alpha, beta=beta, log_evidence=log_ev, n_iter=it)


def model_probabilities(log_evidences):
    """p(M_i | D) = p(D | M_i) / sum_k p(D | M_k) with equal priors (Eq. 17)."""
    top = max(log_evidences)
    w = [math.exp(v - top) for v in log_evidences]
    s = sum(w)
    return [x / s for x in w]
