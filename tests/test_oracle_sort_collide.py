"""Pins of the oracle's cell sort and collision step.

- The sort equals numpy's stable argsort by cell (brute force on random,
  degenerate and edge inputs) and the sort phase permutes the particle
  records by exactly that permutation.
- Each collision conserves momentum and energy (checked per cell from the
  states before and after a collide-only phase).
- The equilibrium hard-sphere collision frequency 4 n d^2 sqrt(pi kT/m) =
  <c>/lambda per particle is reproduced within 1%.
"""
import math

import numpy as np
import pytest

import oracle
from synth import Params


@pytest.mark.parametrize("n,k", [(0, 5), (1, 1), (7, 1), (1000, 1), (1000, 37), (5000, 300),
                                 (64, 2000), (3, 3)])
def test_stable_sort_matches_numpy(n, k):
    rng = np.random.default_rng(n * 31 + k)
    keys = rng.integers(0, k, n).astype(np.int32)
    perm, count, offset = oracle.stable_sort_perm(keys, k)
    assert np.array_equal(perm, np.argsort(keys, kind="stable"))
    assert np.array_equal(count, np.bincount(keys, minlength=k))
    assert np.array_equal(offset, np.concatenate([[0], np.cumsum(count)[:-1]]))


def test_stable_sort_degenerate_inputs():
    keys = np.full(513, 4, dtype=np.int32)  # all in one cell, other cells empty
    perm, count, offset = oracle.stable_sort_perm(keys, 9)
    assert np.array_equal(perm, np.arange(513))
    assert count[4] == 513 and count.sum() == 513
    keys = np.arange(100, dtype=np.int32)[::-1].copy()  # one per cell, reversed
    perm, _, _ = oracle.stable_sort_perm(keys, 100)
    assert np.array_equal(perm, np.arange(100)[::-1])


def test_sort_phase_permutes_records():
    p = Params(kn=0.5, body_force=0.01, n_cells=40, particles_per_cell=30, seed=9, n_sub=2)
    o = oracle.Oracle(p)
    o.step(3)
    o.step(1, oracle.PHASE_MOVE)
    y, vx, vy, vz, cell = o.particles()
    o.step(1, oracle.PHASE_SORT)
    y2, vx2, vy2, vz2, cell2 = o.particles()
    perm = np.argsort(cell, kind="stable")
    for a, b in ((y, y2), (vx, vx2), (vy, vy2), (vz, vz2), (cell, cell2)):
        assert np.array_equal(a[perm], b)
    _, _, count, offset = o.cells()
    assert np.array_equal(count, np.bincount(cell, minlength=o.Cc))
    # collision cell of a particle is floor(y * Cc) with y in [0, 1]
    assert np.array_equal(cell2, np.minimum((y2 * o.Cc).astype(np.int64), o.Cc - 1))


def test_collisions_conserve_momentum_and_energy():
    p = Params(kn=0.05, body_force=0.02, n_cells=20, particles_per_cell=200, seed=21)
    o = oracle.Oracle(p)
    o.step(5)
    checked = 0
    for _ in range(20):
        o.step(1, oracle.PHASE_MOVE | oracle.PHASE_SORT)
        _, vx, vy, vz, _ = o.particles()
        c0 = o.diagnostics()["n_coll"]
        o.step(1, oracle.PHASE_COLLIDE)
        _, wx, wy, wz, _ = o.particles()
        assert o.diagnostics()["n_coll"] > c0
        _, _, count, offset = o.cells()
        for c in range(o.Cc):
            s = slice(offset[c], offset[c] + count[c])
            v = np.stack([vx[s], vy[s], vz[s]], 1)
            w = np.stack([wx[s], wy[s], wz[s]], 1)
            scale_p = np.abs(v).sum()
            assert np.all(np.abs(v.sum(0) - w.sum(0)) <= 1e-12 * scale_p)
            e0, e1 = (v * v).sum(), (w * w).sum()
            assert abs(e0 - e1) <= 1e-12 * e0
            checked += 1
        # something actually changed
        assert not np.array_equal(vx, wx)
    assert checked == 20 * o.Cc


def test_collision_frequency_hard_sphere():
    """Measured 2 n_coll / (N K dt) equals <c>/lambda = 4 n d^2 sqrt(pi kT/m)
    (times 1 - 1/N for the N(N-1) pair count) within 1%."""
    p = Params(kn=1.0, body_force=0.0, n_cells=100, particles_per_cell=50, seed=5,
               n_transient=0)
    o = oracle.Oracle(p)
    o.step(100)
    o.reset_window()
    K = 1500
    o.step(K)
    c = o.constants()
    nc = o.diagnostics()["n_coll"]
    nu = 2.0 * nc / (o.N * K * c["dt"])
    mean_speed = math.sqrt(8.0 / math.pi)  # <c> at kT/m = 1
    want = mean_speed / c["lam"] * (1.0 - 1.0 / o.N)
    assert abs(nu / want - 1.0) < 0.01, (nu, want)


def test_collision_frequency_with_subcells():
    """Collision sub-cells change which pairs may collide, not the rate."""
    p = Params(kn=0.5, body_force=0.0, n_cells=20, particles_per_cell=120, seed=6,
               n_transient=0, n_sub=3)
    o = oracle.Oracle(p)
    o.step(50)
    o.reset_window()
    K = 800
    o.step(K)
    c = o.constants()
    nu = 2.0 * o.diagnostics()["n_coll"] / (o.N * K * c["dt"])
    want = math.sqrt(8.0 / math.pi) / c["lam"]
    assert abs(nu / want - 1.0) < 0.015, (nu, want)


def test_crmax_never_decreases_and_rem_in_unit_interval():
    p = Params(kn=0.2, body_force=0.05, n_cells=30, particles_per_cell=60, seed=8)
    o = oracle.Oracle(p)
    prev = o.cells()[0].copy()
    for _ in range(30):
        o.step(1)
        crmax, rem, _, _ = o.cells()
        assert np.all(crmax >= prev)
        assert np.all((rem >= 0) & (rem < 1))
        prev = crmax.copy()
    assert np.all(prev >= o.constants()["crmax0"])
