"""Resident stepping of small instances (one workgroup per instance, whole
steps in one launch, particles held in LDS) against the multi-kernel step:
the same state, cell tables, sums, collision counts and boundary state, bit
for bit, for closed and open instances in both fast modes, across launch
chunks and sampling windows."""
import sys

import numpy as np
import pytest

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


CASES = [
    # (name, params, inflow)
    ("closed_kn0.5_80x50", dict(kn=0.5, body_force=0.01, n_cells=80, particles_per_cell=50), None),
    ("closed_kn1_100x20_sub2", dict(kn=1.0, body_force=0.02, n_cells=100, particles_per_cell=20, n_sub=2), None),
    ("closed_kn0.05_255x16", dict(kn=0.05, body_force=0.005, n_cells=255, particles_per_cell=16), None),
    ("closed_kn5_20x200", dict(kn=5.0, body_force=0.01, n_cells=20, particles_per_cell=200), None),
    ("open_patch_kn0.1", dict(kn=0.1, body_force=synth.training_force(0.1), n_cells=45,
                              particles_per_cell=50, domain_length=0.225), dict(u=0.0333, dudy=0.069)),
    ("open_patch_kn0.01", dict(kn=0.01, body_force=synth.training_force(0.01), n_cells=9,
                               particles_per_cell=50, domain_length=0.045), dict(u=0.004, dudy=0.02)),
    ("open_patch_kn0.2", dict(kn=0.2, body_force=synth.training_force(0.2), n_cells=85,
                              particles_per_cell=50, domain_length=0.425), dict(u=0.05, dudy=0.015)),
    ("closed_kn0.2_60x48", dict(kn=0.2, body_force=0.01, n_cells=60, particles_per_cell=48), None),
    # at the limits: 256 keys and 6144 slots; 255 cells and the key of the
    # particles that left
    ("closed_limits_256x24", dict(kn=0.3, body_force=0.01, n_cells=256, particles_per_cell=24), None),
    ("open_limits_255x16", dict(kn=0.2, body_force=0.01, n_cells=255, particles_per_cell=16,
                                domain_length=0.5), dict(u=0.02, dudy=0.05)),
]


def _slots(p):
    """Particle slots of an instance: N, and for an open one room for a
    quarter more, at least 8 sqrt(N) + 64."""
    N = p.n_cells * p.particles_per_cell
    if not p.domain_length:
        return N
    return N + max(N // 4, int(8.0 * N ** 0.5) + 64)


def _snapshot(D, s, open_):
    st = s.get_state()
    return dict(state=[np.asarray(a).copy() for a in st[:5]], step=st[5],
                cells=[np.asarray(a).copy() for a in s.get_cells()],
                raw=s.sample(raw=True)["raw"].copy(),
                open=s.open_state() if open_ else None)


def _run(D, plist, inflow, resident, windows):
    sols = [D.Solver(p) for p in plist]
    g = D.Group()
    g.set_resident(resident)
    for s in sols:
        if inflow:
            s.set_inflow(**inflow)
        g.add(s)
    snaps = []
    for n in windows:
        g.step(n)
        g.sync()
        snaps.append([_snapshot(D, s, inflow is not None) for s in sols])
    prof = sols[0].profile(2)
    g.close()
    for s in sols:
        s.close()
    return snaps, prof


def _assert_same(a, b):
    for x, y in zip(a, b):
        for u, v in zip(x["state"], y["state"]):
            assert np.array_equal(u, v)
        assert x["step"] == y["step"]
        for u, v in zip(x["cells"], y["cells"]):
            assert np.array_equal(u, v)
        assert np.array_equal(x["raw"], y["raw"])
        assert x["open"] == y["open"]


@pytest.mark.parametrize("prec_name", ["DSMC_FP32_FAST", "DSMC_FP64_FAST"])
@pytest.mark.parametrize("name,kw,inflow", CASES, ids=[c[0] for c in CASES])
def test_resident_equals_multi_kernel(D, prec_name, name, kw, inflow):
    prec = getattr(D, prec_name)
    p = Params(seed=synth.seed_of(13, len(name)), n_transient=30, precision=prec, **kw)
    if _slots(p) > (6144 if prec == D.DSMC_FP32_FAST else 3072):
        pytest.skip("more slots than one workgroup holds: stepped by the multi-kernel path")
    _say(f"resident vs multi-kernel: {name} {prec_name}")
    windows = (1, 36, 100)
    res, prof = _run(D, [p], inflow, True, windows)
    ref, prof_ref = _run(D, [p], inflow, False, windows)
    # the resident lane's step is one kernel, timed in the collide slot
    assert prof["count"] == 0 and prof["move_scatter"] == 0 and prof["collide"] > 0
    assert prof_ref["count"] > 0 and prof_ref["move_scatter"] > 0
    for a, b in zip(res, ref):
        _assert_same(a, b)
    assert res[-1][0]["raw"].any()


def test_resident_group_of_patches_equals_multi_kernel(D):
    """64 replicas of the Kn = 0.1 hybrid patch with a fixed inflow, and a
    run longer than one resident launch (4096 steps)."""
    base = synth.PATCH0.with_(precision=D.DSMC_FP32_FAST, n_transient=100)
    plist = [base.with_(seed=synth.seed_of(13, 1, r)) for r in range(64)]
    _say("64 patch replicas, 4200 steps, resident and multi-kernel")
    res, _ = _run(D, plist, synth.PATCH0_INFLOW, True, (4200,))
    ref, _ = _run(D, plist, synth.PATCH0_INFLOW, False, (4200,))
    _assert_same(res[0], ref[0])
    assert all(x["open"]["n_injected"] > 0 for x in res[0])


def test_resident_mixed_group_falls_back(D):
    """A group with a member too large to be resident steps all members with
    the multi-kernel step, equal to each member stepped resident alone."""
    small = Params(kn=0.5, body_force=0.01, n_cells=40, particles_per_cell=30, seed=5,
                   n_transient=10, precision=D.DSMC_FP32_FAST)
    large = Params(kn=0.5, body_force=0.01, n_cells=400, particles_per_cell=30, seed=6,
                   n_transient=10, precision=D.DSMC_FP32_FAST)
    mixed, prof = _run(D, [small, large], None, True, (57,))
    assert prof["count"] > 0            # multi-kernel step
    alone, prof1 = _run(D, [small], None, True, (57,))
    assert prof1["count"] == 0          # resident
    _assert_same([mixed[0][0]], alone[0])


def test_set_resident_argument_check(D):
    g = D.Group()
    assert D.lib.dsmc_group_set_resident(g._g, 2) == D.DSMC_ERR_INVALID_ARG
    assert D.lib.dsmc_group_set_resident(None, 1) == D.DSMC_ERR_INVALID_ARG
    g.close()


def test_two_resident_lanes_equal_alone(D):
    """520 small instances (2.08e6 particles) run in two lanes, each of them
    resident; members equal themselves stepped alone, also after the group is
    autotuned (the autotune's steps use other tiles and bucket sizes, which
    change neither the states nor the window sums)."""
    ps = [Params(kn=0.5 + 0.01 * (r % 7), body_force=0.01, n_cells=80, particles_per_cell=50,
                 seed=synth.seed_of(15, r), n_transient=5, precision=D.DSMC_FP32_FAST)
          for r in range(520)]
    _say("520 small instances in two resident lanes")
    sols = [D.Solver(p) for p in ps]
    g = D.Group()
    for s in sols:
        g.add(s)
    g.step(23)
    g.sync()
    assert g.lanes() == 2
    prof = sols[0].profile(1)
    assert prof["count"] == 0 and prof["collide"] > 0
    picks = (0, 259, 519)
    before = [(sols[i].get_state(), sols[i].sample(raw=True)["raw"]) for i in picks]
    g.autotune()
    g.sync()
    after = [(sols[i].get_state(), sols[i].sample(raw=True)["raw"]) for i in picks]
    g.close()
    for s in sols:
        s.close()
    for i, (st, raw), (st2, raw2) in zip(picks, before, after):
        with D.Solver(ps[i]) as s:
            s.step(24)
            s.sync()
            for a, b in zip(s.get_state(), st):
                assert np.array_equal(np.asarray(a), np.asarray(b))
            assert np.array_equal(s.sample(raw=True)["raw"], raw)
            s.step(int(st2[5]) - 24)
            s.sync()
            for a, b in zip(s.get_state(), st2):
                assert np.array_equal(np.asarray(a), np.asarray(b))
            assert np.array_equal(s.sample(raw=True)["raw"], raw2)


@pytest.mark.parametrize("kw", [dict(n_cells=257, particles_per_cell=20),       # 257 keys
                                dict(n_cells=256, particles_per_cell=25),       # 6400 slots
                                dict(n_cells=256, particles_per_cell=16, domain_length=0.5)],  # 257 keys open
                         ids=["keys", "slots", "open_keys"])
def test_just_past_the_limits_is_multi_kernel(D, kw):
    """One key or one tile of slots past the limits the lane is stepped by
    the multi-kernel path, and the results are those of an explicit
    multi-kernel group."""
    p = Params(kn=0.3, body_force=0.01, seed=23, n_transient=5, precision=D.DSMC_FP32_FAST, **kw)
    inflow = dict(u=0.02, dudy=0.05) if kw.get("domain_length") else None
    res, prof = _run(D, [p], inflow, True, (19,))
    ref, _ = _run(D, [p], inflow, False, (19,))
    assert prof["count"] > 0 and prof["move_scatter"] > 0
    _assert_same(res[0], ref[0])


@pytest.mark.parametrize("big_lanes", [1, 2])
def test_small_members_of_a_mixed_group_run_in_a_resident_lane(D, big_lanes):
    """A group that mixes small members with larger ones steps the small ones
    resident in a lane of their own, beside the multi-kernel lanes of the
    larger ones (one of them, or two once those hold 2e6 particles); every
    member equals itself stepped alone, state, cell tables and window sums,
    and the sizes of the lanes show in the lane information."""
    small = [Params(kn=0.4 + 0.1 * r, body_force=0.01, n_cells=60 + 7 * r, particles_per_cell=40,
                    seed=synth.seed_of(16, r), n_transient=6, precision=D.DSMC_FP32_FAST)
             for r in range(5)]
    big_ppc = 150 if big_lanes == 1 else 1100
    big = [Params(kn=0.2 + 0.3 * r, body_force=0.01, n_cells=900 + 100 * r, particles_per_cell=big_ppc,
                  seed=synth.seed_of(16, 100 + r), n_transient=6, precision=D.DSMC_FP32_FAST)
           for r in range(2)]
    ps = small + big
    _say(f"{len(small)} small + {len(big)} larger members")
    sols = [D.Solver(p) for p in ps]
    g = D.Group()
    for s in sols:
        g.add(s)
    g.step(21)
    g.sync()
    li = g.lane_info()
    assert li["resident_lanes"] == 1 and li["lanes"] == big_lanes + 1, li
    assert li["resident_particles"] == sum(p.n_particles for p in small)
    assert li["resident_cells"] == sum(p.n_cells for p in small)
    prof = sols[0].profile(1)
    assert prof["count"] > 0 and prof["resident"] > 0 and prof["collide"] > prof["resident"]
    got = [_snapshot(D, s, False) for s in sols]
    g.close()
    for s in sols:
        s.close()
    for p, snap in zip(ps, got):
        with D.Solver(p) as s:
            s.step(22)   # 21 steps and the profiled one
            ref = _snapshot(D, s, False)
        for a, b in zip(snap["state"], ref["state"]):
            assert np.array_equal(a, b)
        for a, b in zip(snap["cells"], ref["cells"]):
            assert np.array_equal(a, b)
        assert np.array_equal(snap["raw"], ref["raw"])
