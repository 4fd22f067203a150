"""GPU parity of the FP64 deterministic path against the CPU oracle.

The deterministic mode follows the same recipe as the oracle with every
floating-point operation in the same IEEE order, so particle states, cell
state, raw moment sums and estimators must be bit-identical.  All calls go
through the C ABI (``paper_2311_14140_amd.dsmc``).
"""
import numpy as np
import pytest

import oracle
from synth import CONFIG0, CONFIG1, CONFIG2, Params, FP64_DETERMINISTIC

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def D():
    from paper_2311_14140_amd import dsmc
    return dsmc


def _det(p, **kw):
    return p.with_(precision=FP64_DETERMINISTIC, **kw)


def assert_same_state(g, o, what=""):
    gy, gvx, gvy, gvz, gcell, gstep = g.get_state()
    oy, ovx, ovy, ovz, ocell = o.particles()
    assert gstep == o.step_index, what
    for name, a, b in (("y", gy, oy), ("vx", gvx, ovx), ("vy", gvy, ovy), ("vz", gvz, ovz)):
        if not np.array_equal(a, b):
            bad = np.flatnonzero(a != b)
            raise AssertionError(f"{what}: {name} differs at {len(bad)} slots, first {bad[:5]}: "
                                 f"{a[bad[:3]]} vs {b[bad[:3]]}")
    assert np.array_equal(gcell, ocell), what


def assert_same_cells(g, o, what=""):
    for name, a, b in zip(("crmax", "rem", "count", "offset"), g.get_cells(), o.cells()):
        assert np.array_equal(a, b), f"{what}: {name}"


def test_initial_state_bit_exact(D):
    p = _det(CONFIG0)
    o = oracle.Oracle(p)
    with D.Solver(p) as g:
        gy, gvx, gvy, gvz, _, step = g.get_state()
        oy, ovx, ovy, ovz, _ = o.particles()
        assert step == 0
        for a, b in ((gy, oy), (gvx, ovx), (gvy, ovy), (gvz, ovz)):
            assert np.array_equal(a, b)
        assert g.constants == pytest.approx(o.constants(), rel=0, abs=0)


def test_move_only_bit_exact(D):
    p = _det(CONFIG0)
    o = oracle.Oracle(p)
    with D.Solver(p, debug_phase_mask=D.DSMC_PHASE_MOVE) as g:
        for k in range(12):
            g.step(1)
            o.step(1, oracle.PHASE_MOVE)
            assert_same_state(g, o, f"move step {k + 1}")


def test_move_and_sort_bit_exact(D):
    p = _det(CONFIG0, n_sub=2)
    o = oracle.Oracle(p)
    with D.Solver(p, debug_phase_mask=D.DSMC_PHASE_MOVE | D.DSMC_PHASE_SORT) as g:
        for k in range(12):
            g.step(1)
            o.step(1, oracle.PHASE_MOVE | oracle.PHASE_SORT)
            assert_same_state(g, o, f"move+sort step {k + 1}")
            _, _, gc, go = g.get_cells()
            _, _, oc, oo = o.cells()
            assert np.array_equal(gc, oc) and np.array_equal(go, oo)


def test_full_steps_bit_exact_config0(D):
    """100 steps of the Kn = 1 workload: particles, cells, raw sums and
    estimators identical to the oracle."""
    p = _det(CONFIG0, n_transient=40)
    o = oracle.Oracle(p)
    with D.Solver(p) as g:
        for k in range(10):
            g.step(1)
            o.step(1)
            assert_same_state(g, o, f"step {k + 1}")
            assert_same_cells(g, o, f"step {k + 1}")
        g.step(90)
        o.step(90)
        assert_same_state(g, o, "step 100")
        assert_same_cells(g, o, "step 100")
        e = g.sample(raw=True)
        assert np.array_equal(e["raw"], o.acc())
        oe = o.estimators()
        assert e["n_sampled_steps"] == oe["n_sampled_steps"] == 60
        assert e["n_collisions"] > 0
        for k in ("n", "ux", "uy", "uz", "T", "pxy", "qx", "qy"):
            assert np.array_equal(e[k], oe[k]), k
        assert e["mass_flow"] == oe["mass_flow"]


def test_graph_replay_equals_eager_steps(D):
    """dsmc_step replays captured graphs of 8, 4, 2 and 1 steps (37 = four
    8-step graphs, a 4-step and a 1-step one; or 37 one-step graphs); both
    must equal steps launched kernel by kernel (the profiling call)."""
    p = _det(CONFIG0, n_transient=0, seed=77)
    with D.Solver(p) as a, D.Solver(p) as b, D.Solver(p) as c:
        a.step(37)
        for _ in range(37):
            b.step(1)
        c.profile(37)
        sa, sb, sc = a.get_state(), b.get_state(), c.get_state()
        for x, y, z in zip(sa, sb, sc):
            assert np.array_equal(np.asarray(x), np.asarray(y))
            assert np.array_equal(np.asarray(x), np.asarray(z))
        ea, eb, ec = a.sample(raw=True), b.sample(raw=True), c.sample(raw=True)
        assert np.array_equal(ea["raw"], eb["raw"])
        assert np.array_equal(ea["raw"], ec["raw"])


def test_window_reset_and_resample(D):
    p = _det(CONFIG0, n_transient=0, seed=5)
    o = oracle.Oracle(p)
    with D.Solver(p) as g:
        g.step(30)
        o.step(30)
        g.sample(reset=True)
        o.reset_window()
        g.step(25)
        o.step(25)
        e = g.sample(raw=True)
        assert e["n_sampled_steps"] == 25
        assert np.array_equal(e["raw"], o.acc())
        assert e["n_collisions"] == o.diagnostics()["n_coll"]


def test_checkpoint_resume_bit_exact(D):
    p = _det(CONFIG0, n_transient=0, seed=9)
    with D.Solver(p) as a, D.Solver(p) as b:
        a.step(50)
        st = a.get_state()
        cells = a.get_cells()
        a.step(50)
        b.set_state(*st[:5], step=st[5])
        b.set_cells(*cells)
        b.step(50)
        for x, y in zip(a.get_state(), b.get_state()):
            assert np.array_equal(np.asarray(x), np.asarray(y))


def test_run_to_run_deterministic(D):
    p = _det(CONFIG0, kn=0.3, seed=1234)
    runs = []
    for _ in range(2):
        with D.Solver(p) as g:
            g.step(60)
            runs.append(g.get_state())
    for x, y in zip(*runs):
        assert np.array_equal(np.asarray(x), np.asarray(y))


@pytest.mark.parametrize("params", [
    Params(kn=0.05, body_force=0.02, n_cells=1, particles_per_cell=700, seed=3),   # one cell
    Params(kn=2.0, body_force=0.01, n_cells=7, particles_per_cell=3, seed=4),      # N < 256
    Params(kn=5.0, body_force=0.05, n_cells=33, particles_per_cell=1, seed=5),     # 1 per cell, high Kn
    Params(kn=0.5, body_force=0.0, n_cells=9, particles_per_cell=300, seed=6, n_sub=7),
    Params(kn=0.2, body_force=0.01, n_cells=257, particles_per_cell=13, seed=7),   # ragged tiles
])
def test_edge_shapes_bit_exact(D, params):
    p = params.with_(n_transient=3)
    o = oracle.Oracle(p)
    with D.Solver(p) as g:
        g.step(15)
        o.step(15)
        assert_same_state(g, o, str(p))
        assert_same_cells(g, o, str(p))
        assert np.array_equal(g.sample(raw=True)["raw"], o.acc())


def test_crafted_sort_inputs(D):
    """All particles crowded into a few cells with most cells empty: the sort
    must equal the oracle's (which equals numpy's stable argsort)."""
    p = Params(kn=1.0, body_force=0.0, n_cells=50, particles_per_cell=40, seed=8,
               dt=1e-300, n_transient=0)
    o = oracle.Oracle(p)
    rng = np.random.default_rng(3)
    y = np.where(rng.random(o.N) < 0.5, 0.1 + 0.0001 * rng.random(o.N), 0.83 + 0.01 * rng.random(o.N))
    y[::97] = 1.0
    y[::101] = 0.0
    vx, vy, vz = rng.normal(size=(3, o.N))
    o.set_particles(y=y, vx=vx, vy=vy, vz=vz)
    mask = D.DSMC_PHASE_MOVE | D.DSMC_PHASE_SORT
    with D.Solver(p, debug_phase_mask=mask) as g:
        g.set_state(y, vx, vy, vz, step=0)
        g.step(1)
        o.step(1, oracle.PHASE_MOVE | oracle.PHASE_SORT)
        assert_same_state(g, o, "crafted")
        _, _, cnt, off = g.get_cells()
        assert (cnt == 0).sum() > 40
        _, _, ocnt, ooff = o.cells()
        assert np.array_equal(cnt, ocnt) and np.array_equal(off, ooff)


@pytest.mark.parametrize("cells,ppc", [(300, 500), (1500, 600)])
def test_wide_tiles_from_unsorted_state_bit_exact(D, cells, ppc):
    """Tiles larger than the move-scatter holds in registers (300 cells of 500:
    1280-slot tiles, over the 1024 slots the FP64 registers hold; 1500 cells
    of 600: 6144-slot tiles) are walked in chunks ranked 64 keys per pass.
    From a state in random slot order every chunk spans all keys (5 and 24
    passes), a few cells are crowded and many empty; with 1500 keys a tile
    spans more keys than its LDS table holds (1024), and the rest keep their
    next destinations in global memory.  Two full steps must still equal the
    oracle bit for bit."""
    p = Params(kn=0.3, body_force=0.01, n_cells=cells, particles_per_cell=ppc, seed=27,
               n_transient=0, precision=FP64_DETERMINISTIC)
    o = oracle.Oracle(p)
    rng = np.random.default_rng(11)
    y = rng.random(o.N)
    crowd = rng.random(o.N) < 0.3
    y[crowd] = 0.4 + 0.002 * rng.random(int(crowd.sum()))
    y[(y > 0.6) & (y < 0.75)] = 0.9
    vx, vy, vz = rng.normal(size=(3, o.N))
    o.set_particles(y=y, vx=vx, vy=vy, vz=vz)
    with D.Solver(p) as g:
        g.set_state(y, vx, vy, vz, step=0)
        prof = g.profile(1)
        o.step(1)
        assert prof["move_scatter"] > 0
        g.step(1)
        o.step(1)
        assert_same_state(g, o, "unsorted")
        assert_same_cells(g, o, "unsorted")
        assert np.array_equal(g.sample(raw=True)["raw"], o.acc())


def test_torch_arena_and_stream(D):
    import torch
    p = _det(CONFIG0, n_transient=0, seed=21)
    s = torch.cuda.Stream()
    with D.Solver(p) as a, D.Solver(p, stream=s, arena="torch") as b:
        a.step(20)
        b.step(20)
        for x, y in zip(a.get_state(), b.get_state()):
            assert np.array_equal(np.asarray(x), np.asarray(y))


@pytest.mark.parametrize("base,steps", [(CONFIG1, 4), (CONFIG2, 2)])
def test_full_size_bit_exact(D, base, steps):
    """The full single-instance sizes (300k and 2e7 particles) in the FP64
    deterministic mode, a few steps, against the oracle."""
    p = _det(base, n_transient=0)
    o = oracle.Oracle(p)
    with D.Solver(p) as g:
        g.step(steps)
        o.step(steps)
        assert_same_state(g, o, f"N={o.N}")
        assert_same_cells(g, o, f"N={o.N}")
        assert np.array_equal(g.sample(raw=True)["raw"], o.acc())
