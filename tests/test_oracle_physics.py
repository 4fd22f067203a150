"""Pins of the oracle's sampling, estimators and whole-solver physics.

- Estimators on hand-built particle sets equal the plain central-moment
  definitions computed here with numpy.
- Exact momentum balance: gas momentum change = body-force impulse - wall
  absorption, to rounding.
- Relaxation to and preservation of the Maxwellian at zero force.
- The Cauchy momentum balance (Eq. 1, valid at any Kn): the shear stress is the
  straight line P_xy = 2F (y - 1/2) in the paper's units.
- Flow symmetry about the channel centre (the symmetry the paper builds into
  its stress correction, Eq. 14).
- Near-continuum bulk curvature from the Stokes equation (Eq. 3 / Eq. 8 with
  S = 0): u'' = -sqrt(pi) F / Kn_mu, with Kn_mu the viscosity-based Knudsen
  number of Eq. 7 (0.99749 times the hard-sphere Kn).
"""
import math
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest
from scipy import stats

import oracle
from synth import Params, CONFIG0


def test_estimators_match_central_moment_definitions():
    C, ppc = 6, 37
    p = Params(kn=1.0, body_force=0.0, n_cells=C, particles_per_cell=ppc, n_transient=0,
               seed=4, n_sub=2)
    o = oracle.Oracle(p)
    rng = np.random.default_rng(0)
    N = o.N
    y = rng.random(N)
    cell = np.minimum((y * o.Cc).astype(np.int32), o.Cc - 1)
    v = rng.normal(size=(N, 3)) * [1.0, 1.3, 0.7] + [0.3, -0.2, 0.1]
    v[:, 0] += y  # a shear flow, so P_xy and q are non-zero
    v[:, 1] += 0.5 * v[:, 0] ** 2 - 0.5
    o.set_particles(y=y, vx=v[:, 0], vy=v[:, 1], vz=v[:, 2], cell=cell)
    o.step(1, oracle.PHASE_SORT | oracle.PHASE_SAMPLE)
    e = o.estimators()
    assert e["n_sampled_steps"] == 1
    scell = cell // 2
    v0 = math.sqrt(2.0)
    for c in range(C):
        w = v[scell == c]
        nu = len(w) * C / N
        u = w.mean(0)
        cc = w - u
        M = cc.T @ cc / len(w)
        heat = 0.5 * nu * ((cc**2).sum(1)[:, None] * cc).mean(0)
        assert math.isclose(e["n"][c], nu, rel_tol=1e-14)
        assert np.allclose([e["ux"][c], e["uy"][c], e["uz"][c]], u / v0, rtol=1e-12, atol=1e-14)
        assert math.isclose(e["T"][c], np.trace(M) / 3, rel_tol=1e-12)
        assert math.isclose(e["pxy"][c], nu * M[0, 1], rel_tol=1e-10, abs_tol=1e-14)
        # no collide phase: the stresses before and after it coincide
        assert math.isclose(e["pxy_mid"][c], nu * M[0, 1], rel_tol=1e-10, abs_tol=1e-14)
        assert math.isclose(e["qx"][c], heat[0] / v0, rel_tol=1e-9, abs_tol=1e-13)
        assert math.isclose(e["qy"][c], heat[1] / v0, rel_tol=1e-9, abs_tol=1e-13)
    assert math.isclose(e["mass_flow"], v[:, 0].sum() / N / v0, rel_tol=1e-13)
    raw = o.acc()
    assert np.isclose(raw[:, 0].sum(), N)


def test_exact_momentum_balance():
    p = Params(kn=0.3, body_force=0.02, n_cells=40, particles_per_cell=50, seed=12)
    o = oracle.Oracle(p)
    o.step(20)
    P0 = o.particles()[1].sum()
    w0 = o.diagnostics()["wall_dpx"]
    K = 300
    o.step(K)
    P1 = o.particles()[1].sum()
    w1 = o.diagnostics()["wall_dpx"]
    c = o.constants()
    impulse = o.N * c["g"] * c["dt"] * K
    assert abs((P1 - P0) - (impulse - (w1 - w0))) < 1e-9 * (impulse + abs(w1 - w0) + 1.0)


def test_relaxation_to_maxwellian_at_zero_force():
    p = Params(kn=0.2, body_force=0.0, n_cells=20, particles_per_cell=500, seed=31)
    o = oracle.Oracle(p)
    rng = np.random.default_rng(1)
    # uniform velocities with unit variance: kurtosis 1.8, far from Maxwellian
    v = rng.uniform(-math.sqrt(3), math.sqrt(3), size=(o.N, 3))
    o.set_particles(vx=v[:, 0], vy=v[:, 1], vz=v[:, 2])
    o.step(300)
    _, vx, vy, vz, _ = o.particles()
    w = np.concatenate([vx, vy, vz])
    n = len(w)
    assert abs(w.var() - 1.0) < 0.03
    assert abs(stats.kurtosis(w, fisher=False) - 3.0) < 0.1
    assert stats.kstest(w / w.std(), "norm").pvalue > 1e-3
    assert abs(np.mean(vx * vy)) < 4 / math.sqrt(o.N)


def test_maxwellian_preserved_profiles_flat():
    p = Params(kn=1.0, body_force=0.0, n_cells=50, particles_per_cell=100, seed=41,
               n_transient=100)
    o = oracle.Oracle(p)
    o.step(1100)
    e = o.estimators()
    # 1000 sampled steps of 100 particles per cell: density and T within a few %
    assert np.all(np.abs(e["n"] - 1.0) < 0.03)
    assert np.all(np.abs(e["T"] - 1.0) < 0.03)
    assert np.all(np.abs(e["ux"]) < 0.03)
    assert abs(e["mass_flow"]) < 0.005


def _batch_run(params, transient, batches, batch_steps):
    o = oracle.Oracle(params)
    o.step(transient)
    out = []
    for _ in range(batches):
        o.reset_window()
        o.step(batch_steps)
        out.append(o.estimators())
    return out


@pytest.fixture(scope="module")
def cfg0_batches():
    """Config 0 (Kn = 1), 20 batches of 250 sampling steps on 4 replicas."""
    reps = [CONFIG0.with_(seed=CONFIG0.seed + r) for r in range(4)]
    with ThreadPoolExecutor(4) as ex:
        runs = list(ex.map(lambda p: _batch_run(p, 1000, 5, 250), reps))
    return [b for r in runs for b in r]


def _mean_se(batches, key):
    a = np.array([b[key] for b in batches])
    return a.mean(0), a.std(0, ddof=1) / math.sqrt(len(a))


def test_cauchy_stress_line_cell_by_cell(cfg0_batches):
    """Config 0 (Kn = 1, F = 0.01): in every cell the time-centred stress
    P_xy (the P^DSMC of Eq. 13) sits on the line 2F (y - 1/2) that the
    momentum balance of Eq. 1 gives, within its batch standard error.  The
    slope itself is pinned to 1% by the replica test below."""
    F = CONFIG0.body_force
    C = CONFIG0.n_cells
    yc = (np.arange(C) + 0.5) / C
    m, se = _mean_se(cfg0_batches, "pxy_mid")
    want = 2.0 * F * (yc - 0.5)
    z = (m - want) / se
    assert np.mean(z**2) < 1.6, np.mean(z**2)
    assert np.max(np.abs(z)) < 4.5


def test_profiles_symmetric_about_centre(cfg0_batches):
    for key, sign in (("ux", 1), ("T", 1), ("pxy", -1), ("qx", 1), ("n", 1)):
        a = np.array([b[key] for b in cfg0_batches])
        d = a - sign * a[:, ::-1]
        d = d[:, : a.shape[1] // 2]
        m = d.mean(0)
        se = d.std(0, ddof=1) / math.sqrt(len(d))
        z = m / se
        assert np.mean(z**2) < 1.8, (key, np.mean(z**2))
        assert np.max(np.abs(z)) < 4.5, key


def test_velocity_profile_has_slip_and_positive_flow(cfg0_batches):
    m, se = _mean_se(cfg0_batches, "ux")
    assert np.all(m > 0)
    # velocity at the wall cells is non-zero (rarefied slip) and below the centre
    assert m[0] > 5 * se[0] and m[0] < m[len(m) // 2]
    q = np.array([b["mass_flow"] for b in cfg0_batches])
    assert q.mean() > 10 * q.std(ddof=1) / math.sqrt(len(q))


@pytest.mark.slow
def test_near_continuum_bulk_curvature():
    """Kn = 0.1: in the bulk (more than two mean free paths from the walls) the
    profile is the Stokes parabola with u'' = -sqrt(pi) F / Kn_mu, in the
    paper's units (Eq. 8 with S = 0), Kn_mu = 0.99749 Kn."""
    F = 0.01
    kn = 0.1
    C = 100
    reps = [Params(kn=kn, body_force=F, n_cells=C, particles_per_cell=200, seed=2000 + r)
            for r in range(8)]
    with ThreadPoolExecutor(8) as ex:
        runs = list(ex.map(lambda p: _batch_run(p, 600, 5, 2000), reps))
    yc = (np.arange(C) + 0.5) / C
    sel = (yc > 2 * kn) & (yc < 1 - 2 * kn)
    curv = []
    for r in runs:
        for b in r:
            coef = np.polyfit(yc[sel] - 0.5, b["ux"][sel], 2)
            curv.append(2 * coef[0])
    curv = np.array(curv)
    m, se = curv.mean(), curv.std(ddof=1) / math.sqrt(len(curv))
    want = -math.sqrt(math.pi) * F / (0.99749 * kn)
    assert abs(m - want) < 3 * se + 0.02 * abs(want), (m, se, want)


def test_pre_collision_stress_sum_is_taken_before_the_collide_phase():
    """The thirteenth sum of a sampled step is sum vx vy over each collision
    cell of the state the collide phase starts from (recomputed here from
    the particles), and the collisions change it (they relax the stress)."""
    p = Params(kn=0.2, body_force=0.03, n_cells=20, particles_per_cell=40, n_transient=0,
               seed=21, n_sub=2)
    o = oracle.Oracle(p)
    o.step(30)
    o.step(1, oracle.PHASE_MOVE | oracle.PHASE_SORT)
    y, vx, vy, vz, cell = o.particles()
    _, _, count, offset = o.cells()
    want = np.array([np.sum(vx[offset[c]:offset[c] + count[c]] * vy[offset[c]:offset[c] + count[c]])
                     for c in range(o.Cc)])
    before = o.acc().copy()
    o.step(1, oracle.PHASE_COLLIDE | oracle.PHASE_SAMPLE)
    after = o.acc()
    assert np.allclose(after[:, 12] - before[:, 12], want, rtol=1e-12, atol=1e-12)
    post = after[:, 7] - before[:, 7]
    assert np.abs(post - want).max() > 1e-3       # the collisions did act
    assert np.allclose(after[:, 0] - before[:, 0], count)


def _stress_slopes(seed, kn):
    """Least-squares slope (over 2F) and centre value of the post-collision
    and time-centred stresses of a channel at ``kn`` with F = 0.05, 40 cells
    of 100 particles, sampled 30000 steps; cells within 0.1 of a plate are
    left out."""
    C, F = 40, 0.05
    p = Params(kn=kn, body_force=F, n_cells=C, particles_per_cell=100, n_transient=300,
               seed=seed)
    o = oracle.Oracle(p)
    o.step(30300)
    e = o.estimators()
    y = (np.arange(C) + 0.5) / C
    sel = (y > 0.1) & (y < 0.9)
    out = {}
    for k in ("pxy", "pxy_mid"):
        slope, centre = np.polyfit(y[sel] - 0.5, e[k][sel], 1)
        out[k] = (slope / (2 * F), centre)
    return out, o.constants()["dt"]


@pytest.mark.parametrize("kn", [1.0, 0.2])
def test_stress_slope_meets_the_momentum_balance_at_any_kn(kn):
    """Steady force-driven flow has dP/dy = 2F whatever the Knudsen number
    (Eq. 1, the balance the paper calls always correct, in the units of
    Eq. 6), and P = 0 at the centre by symmetry.  The time-centred stress
    meets the slope to 1%: its second-order residual is a few tenths of a
    percent at the default step.  The stress sampled after the collisions
    lies below the free-flight flux by half of the relaxation dt / tau_p the
    collisions apply, tau_p = mu / p = 1.016 (5/16) sqrt(2 pi) lambda for
    hard spheres (Chapman and Cowling, with the higher-order factor), so its
    slope is 1 - dt / (2 tau_p) = 0.911 at dt = 0.2 lambda / sqrt(2).  Eight
    independent replicas per Kn give the spread; the slope's standard error
    is below 0.001, so a 3% error in the stress fails by over 20 of them."""
    with ThreadPoolExecutor(8) as ex:
        runs = list(ex.map(lambda s: _stress_slopes(s, kn), range(300, 308)))
    dt = runs[0][1]
    tau_p = 1.016 * (5.0 / 16.0) * math.sqrt(2.0 * math.pi) * kn
    for k, want in (("pxy", 1.0 - 0.5 * dt / tau_p), ("pxy_mid", 1.0)):
        slopes = np.array([r[0][k][0] for r in runs])
        centres = np.array([r[0][k][1] for r in runs])
        se = slopes.std(ddof=1) / math.sqrt(len(slopes))
        assert se < 0.002, (k, se)
        assert abs(slopes.mean() - want) < 0.01, (k, slopes.mean(), want, se)
        se_c = centres.std(ddof=1) / math.sqrt(len(centres))
        assert abs(centres.mean()) < 5 * se_c + 1e-5, (k, centres.mean(), se_c)
