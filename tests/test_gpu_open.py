"""The GPU solver's open boundary (a DSMC patch of the hybrid, Sec. 2 and
Sec. 3.2): bit-exact against the oracle in the FP64 deterministic mode, the
oracle's physics pins on the fast paths, batching invariance, and argument
checks."""
import math
import sys

import numpy as np
import pytest

import oracle
import synth
from synth import Params

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def D():
    from paper_2311_14140_amd import dsmc
    return dsmc


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _open(D, prec, **kw):
    base = dict(kn=0.05, body_force=0.01, n_cells=30, particles_per_cell=40, seed=17,
                n_transient=20, domain_length=0.3, precision=prec)
    base.update(kw)
    return Params(**base)


@pytest.mark.parametrize("ppc,n_sub,cells", [(40, 1, 30), (300, 1, 30), (60, 2, 30), (500, 1, 300)])
def test_open_patch_bit_exact_with_oracle(D, ppc, n_sub, cells):
    """FP64 deterministic: injections, removals, states, cell tables, sums
    and the open-boundary counters equal the oracle's to the last bit, across
    an inflow change.  The 300-cell patch (1.5e5 particles) sorts in tiles
    larger than the move-scatter's registers hold."""
    p = _open(D, D.DSMC_FP64_DETERMINISTIC, particles_per_cell=ppc, n_sub=n_sub, n_cells=cells)
    _say(f"open det parity: ppc {ppc}, n_sub {n_sub}, cells {cells}")
    o = oracle.Oracle(p)
    with D.Solver(p) as g:
        for (u, dudy, steps) in ((0.08, 0.3, 40), (0.11, -0.2, 35)):
            o.set_inflow(u=u, dudy=dudy)
            g.set_inflow(u=u, dudy=dudy)
            o.step(steps)
            g.step(steps)
            od, gd = o.open_diagnostics(), g.open_state()
            assert gd["n_live"] == od["n_live"] == o.N
            assert gd["n_injected"] == od["n_injected"] and gd["n_deleted"] == od["n_deleted"]
            assert gd["inj_rem"] == od["inj_rem"]
            assert od["n_injected"] > 0 and od["n_deleted"] > 0
            gy, gvx, gvy, gvz, gcell, _ = g.get_state()
            oy, ovx, ovy, ovz, ocell = o.particles()
            for a, b in ((gy, oy), (gvx, ovx), (gvy, ovy), (gvz, ovz), (gcell, ocell)):
                assert np.array_equal(a, b)
            gc = g.get_cells()
            oc = o.cells()
            for a, b in zip(gc, oc):
                assert np.array_equal(a, b)
            assert np.array_equal(g.sample(raw=True)["raw"], o.acc())


def test_open_and_closed_in_one_group_equal_alone(D):
    """An open patch batched with closed instances (FP32, bucket and
    workgroup collide paths) is bit-identical to each stepped alone."""
    ps = [_open(D, D.DSMC_FP32_FAST, particles_per_cell=60, seed=31),
          Params(kn=0.5, body_force=0.01, n_cells=80, particles_per_cell=50, seed=32,
                 n_transient=5, precision=D.DSMC_FP32_FAST),
          _open(D, D.DSMC_FP32_FAST, kn=0.1, particles_per_cell=300, domain_length=0.4, seed=33)]
    alone = []
    for p in ps:
        with D.Solver(p) as s:
            if p.domain_length:
                s.set_inflow(u=0.05, dudy=0.2)
            s.step(37)
            alone.append((s.get_state(), s.sample(raw=True)["raw"],
                          s.open_state() if p.domain_length else None))
    sols = [D.Solver(p) for p in ps]
    for s, p in zip(sols, ps):
        if p.domain_length:
            s.set_inflow(u=0.05, dudy=0.2)
    g = D.Group()
    for s in sols:
        g.add(s)
    g.step(37)
    g.sync()
    for s, (st, raw, os_) in zip(sols, alone):
        for a, b in zip(s.get_state(), st):
            assert np.array_equal(np.asarray(a), np.asarray(b))
        assert np.array_equal(s.sample(raw=True)["raw"], raw)
        if os_ is not None:
            assert s.open_state() == os_
    g.close()
    for s in sols:
        s.close()


@pytest.mark.parametrize("prec_name", ["DSMC_FP32_FAST", "DSMC_FP64_FAST"])
def test_patch_in_equilibrium_with_its_reservoir(D, prec_name):
    """Fast paths: wall and reservoir at T = 1, no force, reservoir at rest:
    nominal density, rest and T = 1 on average, fluxes in balance."""
    prec = getattr(D, prec_name)
    R = 16
    ps = [_open(D, prec, kn=0.2, body_force=0.0, n_cells=20, particles_per_cell=40,
                domain_length=0.4, n_transient=300, seed=synth.seed_of(8, 0, r)) for r in range(R)]
    sols = [D.Solver(p) for p in ps]
    g = D.Group()
    for s in sols:
        g.add(s)
    g.step(2300)
    es = g.sample()
    n = np.array([e["n"] for e in es]).mean(0)
    T = np.array([e["T"] for e in es]).mean(0)
    ux = np.array([e["ux"] for e in es]).mean(0)
    live = np.array([s.open_state()["n_live"] for s in sols])
    _say(f"{prec_name}: density {n.min():.4f}..{n.max():.4f}, T {T.min():.4f}..{T.max():.4f}, "
         f"|ux| max {np.abs(ux).max():.4f}, live mean {live.mean():.1f} of 800")
    assert abs(n.mean() - 1) < 0.01 and np.all(np.abs(n - 1) < 0.05)
    assert abs(T.mean() - 1) < 0.005 and np.all(np.abs(T - 1) < 0.02)
    assert np.all(np.abs(ux) < 0.01)
    assert abs(live.mean() / 800 - 1) < 0.03
    g.close()
    for s in sols:
        s.close()


def test_chapman_enskog_inflow_carries_the_imposed_gradient(D):
    """FP32 path, as the oracle's pin: a force-free patch fed by a sheared
    reservoir keeps the imposed gradient with the Chapman-Enskog inflow and
    loses about a tenth of it with a Maxwellian one."""
    kn, L, dudy = 0.05, 0.3, 0.4
    c = 2 * kn / math.sqrt(math.pi)
    R = 16
    slopes = {}
    for name, w in (("ce", dudy), ("maxwell", 0.0)):
        ps = [_open(D, D.DSMC_FP32_FAST, body_force=0.0, particles_per_cell=60, n_transient=2000,
                    seed=synth.seed_of(9, 0, r)) for r in range(R)]
        sols = [D.Solver(p) for p in ps]
        g = D.Group()
        for s in sols:
            s.set_inflow(u=0.9 * c * dudy + dudy * L, dudy=w)
            g.add(s)
        g.step(12000)
        es = g.sample()
        u = np.array([e["ux"] for e in es]).mean(0)
        y = (np.arange(30) + 0.5) / 30 * L
        slopes[name] = np.polyfit(y[8:22], u[8:22], 1)[0] / dudy
        g.close()
        for s in sols:
            s.close()
    _say(f"interior gradient over the imposed one: {slopes}")
    assert abs(slopes["ce"] - 1) < 0.04
    assert slopes["maxwell"] < 0.95


def test_open_boundary_argument_checks(D):
    p = Params(kn=0.5, body_force=0.0, n_cells=10, particles_per_cell=10, seed=1,
               precision=D.DSMC_FP32_FAST)
    with D.Solver(p) as s:
        with pytest.raises(D.DsmcError):
            s.set_inflow(u=0.1)
        with pytest.raises(D.DsmcError):
            s.open_state()
    with pytest.raises(D.DsmcError):
        D.Solver(p.with_(domain_length=1.5))
    with pytest.raises(D.DsmcError):
        D.Solver(p.with_(domain_length=0.5), debug_phase_mask=D.DSMC_PHASE_MOVE)
    with D.Solver(p.with_(domain_length=0.5)) as s:
        with pytest.raises(D.DsmcError):
            s.set_inflow(dudy=100.0)      # |a| > 1
        with pytest.raises(D.DsmcError):
            s.set_inflow(T=0.0)
        with pytest.raises(D.DsmcError):
            s.set_inflow(n=1e9)           # more entrants than slots
        s.set_inflow(u=0.1, dudy=0.5)
        s.step(10)
        assert s.open_state()["n_injected"] > 0


@pytest.mark.parametrize("prec_name", ["DSMC_FP64_DETERMINISTIC", "DSMC_FP32_FAST"])
def test_open_patch_checkpoint_resumes_bit_exactly(D, prec_name):
    """Boundary state, particles and cell tables of an open patch restored
    into a fresh instance continue exactly as the original."""
    p = _open(D, getattr(D, prec_name), particles_per_cell=50, seed=77)
    with D.Solver(p) as a:
        a.set_inflow(u=0.07, dudy=0.25)
        a.step(30)
        os_ = a.open_state()
        st = a.get_state()
        cells = a.get_cells()
        a.step(25)
        want = (a.get_state(), a.sample(raw=True)["raw"], a.open_state())
    with D.Solver(p) as b:
        b.set_open_state(**os_)
        b.set_state(*st[:5], step=st[5])
        b.set_cells(*cells)
        b.set_inflow(u=0.07, dudy=0.25)
        b.sample(reset=True)
        b.step(25)
        got = (b.get_state(), b.sample(raw=True)["raw"], b.open_state())
    for x, y in zip(got[0], want[0]):
        assert np.array_equal(np.asarray(x), np.asarray(y))
    assert got[2] == want[2]
    assert got[1].shape == want[1].shape


@pytest.mark.parametrize("prec_name", ["DSMC_FP32_FAST", "DSMC_FP64_FAST"])
def test_fast_open_patch_matches_oracle_replicas(D, prec_name):
    """64 replicas of the Kn = 0.1 hybrid patch with a fixed Chapman-Enskog
    inflow (500 + 6000 steps) against 64 oracle replicas: every cell's
    density, velocity, temperature, both shear stresses and heat flux by the
    Welch rule of the other statistical parity tests, and the mass flow."""
    import os
    from test_gpu_parity_fp32 import assert_profiles_agree, welch
    d = np.load(os.path.join(os.path.dirname(__file__), "golden", "oracle_patch0_r0_64.npz"))
    quant = ("n", "ux", "T", "pxy", "qx", "pxy_mid")
    ref = {q: d[q] for q in quant}
    R = ref["ux"].shape[0]
    base = synth.PATCH0.with_(precision=getattr(D, prec_name))
    sols = [D.Solver(base.with_(seed=synth.seed_of(11, 0, 1000 + r))) for r in range(R)]
    g = D.Group()
    for s in sols:
        s.set_inflow(**synth.PATCH0_INFLOW)
        g.add(s)
    g.step(synth.PATCH0_STEPS)
    es = g.sample()
    g.close()
    for s in sols:
        s.close()
    gpu = {q: np.array([e[q] for e in es]) for q in quant}
    assert all(e["n_sampled_steps"] == synth.PATCH0_STEPS - synth.PATCH0.n_transient for e in es)
    assert_profiles_agree(gpu, ref, quant)
    Q = np.array([e["mass_flow"] for e in es])
    zq, _, se = welch(Q[:, None], d["mass_flow"][:, None])
    _say(f"{prec_name}: mass flow {Q.mean():.6f} vs oracle {d['mass_flow'].mean():.6f} (z {zq[0]:.2f})")
    assert abs(zq[0]) < 3.5
