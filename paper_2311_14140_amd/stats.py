"""Host-side statistics of DSMC outputs.

The solver returns window averages (``dsmc_sample`` with reset gives one
window, e.g. the paper's 100-step training samples, Sec. 3).  Windows of one
run, or independent replicas, are combined here:

- batch means: the mean of B window averages and its standard error
  sd / sqrt(B), with the lag-1 autocorrelation of the window series as a check
  that windows are long enough to be nearly independent, for every profile
  and the mass flow of a run's windows;
- percentiles of the served requests' latencies.
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


def window_statistics(windows, keys=("n", "ux", "T", "pxy", "pxy_mid", "qx")) -> dict:
    """Batch means over the windows of one run: ``windows`` is a list of the
    dicts ``Solver.sample(reset=True)`` returns, one per window of equal
    length (the paper's 100-step samples, Sec. 3, or longer batches).  For
    each profile in ``keys`` and for the mass flow: the mean over the
    windows, its standard error and the lag-1 autocorrelation of the window
    series (near 0 when the windows are long enough to be independent)."""
    if len(windows) < 2:
        raise ValueError("need at least two windows")
    steps = {int(w["n_sampled_steps"]) for w in windows}
    if len(steps) != 1 or steps == {0}:
        raise ValueError("windows must hold the same, non-zero number of sampled steps")
    out = {}
    for k in tuple(keys) + ("mass_flow",):
        m, se, lag1 = batch_means([np.asarray(w[k], dtype=np.float64) for w in windows])
        out[k] = {"mean": m, "se": se, "lag1": lag1}
    out["windows"] = len(windows)
    out["steps_per_window"] = steps.pop()
    return out


def percentile(values, p: float) -> float:
    v = np.sort(np.asarray(values, dtype=np.float64))
    if v.size == 0:
        return float("nan")
    return float(np.percentile(v, p, method="linear"))
