"""The allocation-free group sample (dsmc_group_sample_noalloc) against
dsmc_group_sample, called through the C ABI: two identical groups, one
sampled by each entry point, give the same estimators bit for bit on two
calls in a row (the second after members leave, so with a smaller input,
and with the windows reset), and sizes beyond the fixed scratch are refused."""
import ctypes as ct

import numpy as np
import pytest

import synth
from synth import Params

pytestmark = pytest.mark.gpu

KEYS = ("n", "ux", "uy", "uz", "T", "pxy", "qx", "qy", "pxy_mid")


@pytest.fixture(scope="module")
def D():
    from paper_2311_14140_amd import dsmc
    return dsmc


def _say(msg):
    print(f"[no_alloc] {msg}", flush=True)


def _outs(D, sols):
    ms = (D.dsmc_moments * len(sols))()
    arrs = []
    for i, s in enumerate(sols):
        a = {k: np.full(s.C, np.nan) for k in KEYS}
        ms[i].n_cells = s.C
        for k, v in a.items():
            setattr(ms[i], k, v.ctypes.data_as(ct.POINTER(ct.c_double)))
        arrs.append(a)
    return ms, arrs


def _sample(D, g, sols, fn, reset):
    ms, arrs = _outs(D, sols)
    rc = fn(g._g, ms, len(sols), 1 if reset else 0)
    assert rc == D.DSMC_OK, D.lib.dsmc_last_error(None)
    for i, a in enumerate(arrs):
        a["mass_flow"] = ms[i].mass_flow
        a["n_sampled_steps"] = ms[i].n_sampled_steps
        a["n_collisions"] = ms[i].n_collisions
    return arrs


def _same(got, ref):
    assert len(got) == len(ref)
    for a, b in zip(got, ref):
        for k in KEYS:
            assert np.array_equal(a[k], b[k]), k
        assert a["n_sampled_steps"] == b["n_sampled_steps"] > 0
        assert a["n_collisions"] == b["n_collisions"]
        assert a["mass_flow"] == b["mass_flow"]


def _group(D, ps):
    g = D.Group()
    sols = [D.Solver(p) for p in ps]
    for s in sols:
        g.add(s)
    return g, sols


def test_noalloc_sample_equals_group_sample_twice_second_smaller(D):
    ps = [p.with_(n_transient=20, seed=synth.seed_of(30, i))
          for i, p in enumerate(synth.config3_instances(7, seed=31, cells_range=(50, 900),
                                                        ppc_range=(20, 120)))]
    ps.append(Params(kn=0.2, body_force=0.01, n_cells=300, particles_per_cell=300, n_transient=20,
                     seed=synth.seed_of(30, 99), precision=synth.FP32_FAST))
    _say(f"{len(ps)} members, FP32")
    ga, sa = _group(D, ps)
    gb, sb = _group(D, ps)
    for g in (ga, gb):
        g.step(57)
    ref = _sample(D, ga, sa, D.lib.dsmc_group_sample, reset=True)
    got = _sample(D, gb, sb, D.lib.dsmc_group_sample_noalloc, reset=True)
    _same(got, ref)
    _say("first call equal; members leave")
    for g, sols in ((ga, sa), (gb, sb)):
        for s in sols[5:]:
            g.remove(s)
            s.close()
        del sols[5:]
        g.step(31)
    ref = _sample(D, ga, sa, D.lib.dsmc_group_sample, reset=False)
    got = _sample(D, gb, sb, D.lib.dsmc_group_sample_noalloc, reset=False)
    _same(got, ref)
    assert all(a["n_sampled_steps"] == 31 for a in got)  # the first call's reset took
    _say("second call (5 members) equal")
    # the no-alloc call on the first group sees the same windows again
    again = _sample(D, ga, sa, D.lib.dsmc_group_sample_noalloc, reset=False)
    _same(again, ref)
    for g, sols in ((ga, sa), (gb, sb)):
        g.close()
        for s in sols:
            s.close()


def test_noalloc_sample_refuses_more_than_its_scratch(D):
    # 46 members of 10240 cells need 46 * 92192 doubles of staging, more
    # than the 32 MiB scratch holds
    ps = [Params(kn=1.0, body_force=0.0, n_cells=10240, particles_per_cell=1, n_transient=0,
                 seed=synth.seed_of(32, i), precision=synth.FP32_FAST) for i in range(46)]
    g, sols = _group(D, ps)
    g.step(2)
    g.sync()
    ms, _ = _outs(D, sols)
    assert D.lib.dsmc_group_sample_noalloc(g._g, ms, len(sols), 0) == D.DSMC_ERR_INVALID_ARG
    assert b"32 MiB" in D.lib.dsmc_last_error(None)
    # the allocating entry point serves the same group
    assert D.lib.dsmc_group_sample(g._g, ms, len(sols), 0) == D.DSMC_OK
    g.close()
    for s in sols:
        s.close()
