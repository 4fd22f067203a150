"""Pins of the oracle's initial state.

The gas starts at rest between the plates at the wall temperature (Sec. 2.1),
with the DSMC resolution of Sec. 3 given as particles per cell: every sampling
cell holds exactly ppc particles, placed uniformly inside it, and every
velocity component is an independent normal with variance k T_w / m (the
Maxwellian at rest).  Slots start in nominal cell order: slot p belongs to
cell floor(p / ppc), the order the deterministic parity contract fixes.
"""
import math

import numpy as np
import pytest
from scipy import stats

import oracle
from synth import Params


def _initial(p):
    o = oracle.Oracle(p)
    assert o.step_index == 0
    y, vx, vy, vz, _ = o.particles()
    return o, y, np.stack([vx, vy, vz], 1)


@pytest.mark.parametrize("kw", [dict(n_cells=37, particles_per_cell=53),
                                dict(n_cells=200, particles_per_cell=50, n_sub=3),
                                dict(n_cells=45, particles_per_cell=40, domain_length=0.225)],
                         ids=["closed", "sub_cells", "open_patch"])
def test_every_cell_starts_with_ppc_particles_uniform_inside(kw):
    p = Params(kn=0.3, body_force=0.01, seed=77, **kw)
    o, y, _ = _initial(p)
    C, ppc = p.n_cells, p.particles_per_cell
    L = kw.get("domain_length") or 1.0
    assert o.N == C * ppc
    cell = np.floor(y * C / L).astype(np.int64)
    # exactly ppc per sampling cell ...
    assert np.array_equal(np.bincount(cell, minlength=C), np.full(C, ppc))
    # ... in nominal order: slot p in cell floor(p / ppc), inside its cell
    own = np.arange(o.N) // ppc
    assert np.array_equal(cell, own)
    assert np.all(y >= own * (L / C)) and np.all(y < (own + 1) * (L / C))
    # uniform inside the cell
    frac = y * C / L - own
    assert stats.kstest(frac, "uniform").pvalue > 1e-3
    # every collision cell starts with crmax at its initial value and no
    # carried remainder
    crmax, rem, _, _ = o.cells()
    assert np.all(crmax == crmax[0]) and np.all(rem == 0.0)


@pytest.mark.parametrize("tw", [2.5, 0.4])
def test_initial_velocities_are_the_wall_maxwellian_at_rest(tw):
    """Each component N(0, T_w): zero mean, variance T_w, kurtosis 3,
    normal by Kolmogorov-Smirnov, and the components uncorrelated."""
    p = Params(kn=0.5, body_force=0.01, wall_temperature=tw, n_cells=200,
               particles_per_cell=250, seed=91)
    _, _, v = _initial(p)
    N = len(v)
    for a in range(3):
        w = v[:, a]
        assert abs(w.mean()) < 4.5 * math.sqrt(tw / N), (a, w.mean())
        assert abs(w.var() - tw) < 4.5 * tw * math.sqrt(2.0 / N), (a, w.var())
        assert abs(stats.kurtosis(w, fisher=False) - 3.0) < 4.5 * math.sqrt(24.0 / N)
        assert stats.kstest(w / math.sqrt(tw), "norm").pvalue > 1e-3, a
    for a, b in ((0, 1), (0, 2), (1, 2)):
        assert abs(np.mean(v[:, a] * v[:, b])) < 4.5 * tw / math.sqrt(N), (a, b)
    # the energy per particle is 3/2 k T_w
    e = 0.5 * np.mean(np.sum(v * v, 1))
    assert abs(e - 1.5 * tw) < 4.5 * tw * math.sqrt(1.5 / N)


def test_initial_state_is_a_property_of_the_seed():
    """The same seed gives the same state; another seed, another one."""
    p = Params(kn=0.5, body_force=0.01, n_cells=20, particles_per_cell=30, seed=5)
    _, y1, v1 = _initial(p)
    _, y2, v2 = _initial(p)
    _, y3, v3 = _initial(p.with_(seed=6))
    assert np.array_equal(y1, y2) and np.array_equal(v1, v2)
    assert not np.array_equal(y1, y3) and not np.array_equal(v1, v3)
