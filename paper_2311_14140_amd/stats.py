"""Host-side statistics of DSMC outputs.

The solver returns window averages (``dsmc_sample`` with reset gives one
window, e.g. the paper's 100-step training samples, Sec. 3).  Windows of one
run, or independent replicas, are combined here:

- batch means: the mean of B window averages and its standard error
  sd / sqrt(B), with the lag-1 autocorrelation of the window series as a check
  that windows are long enough to be nearly independent;
- Welch comparison of two sets of samples, per cell;
- the profile-agreement rule used for reduced-precision runs: the number of
  cells with |z| > 3 stays within the 99.9% binomial bound for the Student-t
  tail probability, and no |z| exceeds 5; the mass flow agrees within a
  relative tolerance (0.5% by default) when its standard error resolves it.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import stats as _st


def batch_means(samples):
    """samples: array [B, ...] of window averages.  Returns (mean, se, lag1)."""
    a = np.asarray(samples, dtype=np.float64)
    B = a.shape[0]
    if B < 2:
        raise ValueError("need at least two windows")
    mean = a.mean(0)
    se = a.std(0, ddof=1) / math.sqrt(B)
    d = a - mean
    denom = (d * d).sum(0)
    with np.errstate(invalid="ignore", divide="ignore"):
        lag1 = (d[1:] * d[:-1]).sum(0) / denom
    return mean, se, lag1


def welch(a, b):
    """Per-element Welch statistic of two sample sets [Ra, ...] and [Rb, ...].
    Returns (z, degrees of freedom, standard error of the difference)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    va = a.var(0, ddof=1) / a.shape[0]
    vb = b.var(0, ddof=1) / b.shape[0]
    se = np.sqrt(va + vb)
    z = (a.mean(0) - b.mean(0)) / se
    nu = (va + vb) ** 2 / (va**2 / (a.shape[0] - 1) + vb**2 / (b.shape[0] - 1))
    return z, nu, se


def profiles_agree(a: dict, b: dict, quantities, z_max: float = 5.0) -> dict:
    """Apply the agreement rule to profiles a[q], b[q] of shape [R, C]."""
    zs, nus = [], []
    for q in quantities:
        z, nu, _ = welch(a[q], b[q])
        zs.append(np.ravel(z))
        nus.append(np.ravel(nu))
    z = np.concatenate(zs)
    nu = float(np.median(np.concatenate(nus)))
    p3 = 2.0 * _st.t.sf(3.0, nu)
    bound = int(_st.binom.ppf(0.999, z.size, p3))
    n3 = int((np.abs(z) > 3.0).sum())
    zmax = float(np.abs(z).max())
    return {"ok": n3 <= bound and zmax < z_max, "n_over_3": n3, "bound": bound,
            "max_abs_z": zmax, "n_tests": int(z.size), "dof": nu}


def mass_flow_agree(qa, qb, rel_tol: float = 0.005) -> dict:
    """Relative mass-flow difference of two replica sets, with the 3-sigma
    resolution of the comparison."""
    qa = np.asarray(qa, dtype=np.float64)
    qb = np.asarray(qb, dtype=np.float64)
    ma, mb = qa.mean(), qb.mean()
    se = math.sqrt(qa.var(ddof=1) / qa.size + qb.var(ddof=1) / qb.size)
    rel = abs(ma - mb) / abs(mb)
    return {"ok": rel <= rel_tol and abs(ma - mb) < 3 * se, "rel": rel,
            "three_se_rel": 3 * se / abs(mb), "resolvable": 3 * se / abs(mb) <= rel_tol}


def percentile(values, p: float) -> float:
    v = np.sort(np.asarray(values, dtype=np.float64))
    if v.size == 0:
        return float("nan")
    return float(np.percentile(v, p, method="linear"))
