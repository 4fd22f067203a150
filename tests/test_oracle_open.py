"""Pins of the oracle's open boundary (a DSMC patch of the hybrid, Sec. 2 and
Sec. 3.2): particles leaving through it are removed, particles enter from a
Chapman-Enskog distribution at the imposed macro state, and a patch in
equilibrium with its reservoir stays in equilibrium."""
import math

import numpy as np
import pytest

import oracle
from synth import Params

SQRT2 = math.sqrt(2.0)


def _patch(**kw):
    base = dict(kn=0.05, body_force=0.0, n_cells=50, particles_per_cell=100, seed=5,
                n_transient=0, domain_length=0.5)
    base.update(kw)
    return oracle.Oracle(Params(**base))


def test_closed_domain_is_the_default():
    o = oracle.Oracle(Params(kn=0.5, body_force=0.0, n_cells=10, particles_per_cell=10, seed=1))
    assert o.capacity == o.N == 100
    o.step(5)
    assert o.N == 100 and o.open_diagnostics()["n_injected"] == 0


def test_invalid_domain_lengths_are_refused():
    for L in (-0.1, 1.5, float("nan")):
        with pytest.raises(ValueError):
            oracle.Oracle(Params(kn=0.5, body_force=0.0, n_cells=10, particles_per_cell=10,
                                 domain_length=L))


def test_injected_velocities_have_the_chapman_enskog_flux_moments():
    """Flux-weighted half-range moments of f0 (1 - a C_x C_y), C = (c - u)/sqrt(2T),
    T = 1: E[v_y] = -sqrt(pi/2); E[v_x - u] = (a/2) sqrt(pi/2); E[(v_x - u) v_y]
    = -a; E[v_y^2] = 2; E[v_z] = 0; E[v_z^2] = 1."""
    o = _patch()
    kn, dudy, u = 0.05, 2.0, 0.03
    a = 4 * kn / math.sqrt(math.pi) * dudy
    o.set_inflow(u=u, dudy=dudy)
    n = 60000
    st = np.array([o.inject_one(7 + k // 1000, k % 1000) for k in range(n)])
    c = o.constants()
    vx, vy, vz = st[:, 1], st[:, 2], st[:, 3]
    outside = (st[:, 0] - 0.5) / -vy           # dt minus the time inside
    assert np.all(vy < 0) and np.all(outside >= 0) and np.all(outside < c["dt"] * (1 + 1e-12))
    tx = vx - u * SQRT2 + c["g"] * outside       # the drawn thermal x velocity
    def close(x, want, what):
        se = x.std() / math.sqrt(n)
        assert abs(x.mean() - want) < 4.5 * se, (what, x.mean(), want, se)
    close(vy, -math.sqrt(math.pi / 2), "E[vy]")
    close(tx, 0.5 * a * math.sqrt(math.pi / 2), "E[tx]")
    close(tx * vy, -a, "E[tx vy]")
    close(vy * vy, 2.0, "E[vy^2]")
    close(vz, 0.0, "E[vz]")
    close(vz * vz, 1.0, "E[vz^2]")
    # entry times uniform over the step
    frac = 1 - outside / c["dt"]
    close(frac, 0.5, "entry time")


def test_injection_count_is_the_expected_flux_exactly():
    """Per step, floor(expected + carried remainder) particles enter, the
    expected number being n sqrt(T/(2 pi)) dt times the nominal line density."""
    o = _patch(n_cells=20, particles_per_cell=50, domain_length=0.3)
    o.set_inflow(T=1.3, n=0.9)
    c = o.constants()
    want_per_step = 0.9 * (1000 / 0.3) * math.sqrt(1.3 / (2 * math.pi)) * c["dt"]
    K = 137
    o.step(K)
    d = o.open_diagnostics()
    assert d["n_injected"] == math.floor(K * want_per_step + 1e-9)
    assert abs(d["inj_rem"] - (K * want_per_step - d["n_injected"])) < 1e-9
    assert d["n_live"] == 1000 + d["n_injected"] - d["n_deleted"]
    assert d["status"] == 0


def test_particles_leaving_through_the_open_boundary_are_removed():
    """With no inflow, exactly the particles whose straight flight crosses the
    open boundary within the step disappear, and the rest keep their order
    (the sort is stable)."""
    o = _patch(n_cells=10, particles_per_cell=20, domain_length=0.2)
    o.set_inflow(n=0.0)
    rng = np.random.default_rng(3)
    N = o.N
    y = rng.uniform(0.0, 0.2, N)
    vy = rng.normal(size=N) * 3.0
    vx = rng.normal(size=N)
    vz = rng.normal(size=N)
    cell = np.minimum((y / 0.02).astype(np.int32), 9)
    o.set_particles(y=y, vx=vx, vy=vy, vz=vz, cell=cell)
    dt = o.constants()["dt"]
    # only the phases that matter: move and sort
    o.step(1, oracle.PHASE_MOVE | oracle.PHASE_SORT)
    leave = y + vy * dt >= 0.2
    hits_wall = y + vy * dt < 0.0
    assert np.all(~(leave & hits_wall))
    assert o.N == N - leave.sum()
    assert o.open_diagnostics()["n_deleted"] == leave.sum()
    ny, nvx, nvy, nvz, ncell = o.particles()
    assert np.all((ny >= 0) & (ny <= 0.2)) and np.all(np.diff(ncell) >= 0)
    # the survivors that did not meet the wall keep their velocities
    keep = ~leave & ~hits_wall
    assert np.isin(vz[keep], nvz).all()


def test_patch_in_equilibrium_with_its_reservoir_stays_there():
    """Wall and reservoir at T = 1, no force, reservoir at rest: the patch
    keeps the nominal density on average, at rest, at T = 1, with the
    injected and removed fluxes in balance."""
    o = _patch(kn=0.2, n_cells=20, particles_per_cell=40, domain_length=0.4, n_transient=200,
               seed=11)
    counts = []
    o.step(200)
    for _ in range(40):
        o.step(50)
        counts.append(o.N)
    e = o.estimators()
    d = o.open_diagnostics()
    counts = np.array(counts, dtype=float)
    # the count wanders slowly; its mean over 2000 steps within 3%
    assert abs(counts.mean() / 800 - 1) < 0.03, counts.mean()
    assert abs(e["n"].mean() - 1) < 0.03
    assert np.all(np.abs(e["n"] - 1) < 0.15)
    assert abs(e["T"].mean() - 1) < 0.01 and np.all(np.abs(e["T"] - 1) < 0.06)
    assert np.all(np.abs(e["ux"]) < 0.05)
    assert d["status"] == 0
    assert abs(d["n_injected"] - d["n_deleted"]) < 0.1 * d["n_injected"]


def _sheared_patch(ce, seed, kn=0.05, L=0.3, dudy=0.4):
    c = 2 * kn / math.sqrt(math.pi)
    o = oracle.Oracle(Params(kn=kn, body_force=0.0, n_cells=30, particles_per_cell=60, seed=seed,
                             n_transient=2000, domain_length=L))
    o.set_inflow(u=0.9 * c * dudy + dudy * L, dudy=dudy if ce else 0.0)
    o.step(22000)
    return o.estimators()


def test_chapman_enskog_inflow_carries_the_imposed_gradient():
    """A force-free patch (Kn 0.05, 6 mean free paths thick) fed by a
    reservoir at velocity u and gradient du/dy: with the Chapman-Enskog
    inflow the interior velocity gradient is the imposed one and the stress
    is uniform; a Maxwellian inflow at the same u (du/dy = 0 in the weight)
    loses about a tenth of the gradient.  This is why the hybrid injects the
    Chapman-Enskog distribution (Sec. 2)."""
    from concurrent.futures import ThreadPoolExecutor
    dudy, L = 0.4, 0.3
    with ThreadPoolExecutor(4) as ex:
        res = list(ex.map(lambda a: _sheared_patch(*a), [(1, 21), (1, 22), (0, 21), (0, 22)]))
    y = (np.arange(30) + 0.5) / 30 * L
    slopes = {}
    for name, rs in (("ce", res[:2]), ("maxwell", res[2:])):
        u = np.mean([r["ux"] for r in rs], axis=0)
        slopes[name] = np.polyfit(y[8:22], u[8:22], 1)[0] / dudy
        P = np.mean([r["pxy_mid"] for r in rs], axis=0)
        # force-free: uniform stress (interior line slope small against its level)
        sl = np.polyfit(y, P, 1)[0] * L
        assert abs(sl) < 0.08 * abs(P.mean()), (name, sl, P.mean())
        assert P.mean() < 0                    # the wall at rest drags the sheared gas
    assert abs(slopes["ce"] - 1) < 0.05, slopes
    assert slopes["maxwell"] < 0.95, slopes
