"""The served path on the GPU: requests arriving over time are admitted by
footprint and batched; every result equals the same solve run alone."""
import numpy as np
import pytest

import synth
from synth import Params

pytestmark = pytest.mark.gpu


def test_served_results_equal_alone():
    from paper_2311_14140_amd import dsmc
    from paper_2311_14140_amd.serve import GpuExecutor, Request, Server
    ps = synth.config3_instances(10, seed=44, cells_range=(50, 300), ppc_range=(20, 60))
    reqs = [Request(i, 0.002 * i, p.with_(n_transient=30, seed=synth.seed_of(4, i)), steps=90 + 13 * i)
            for i, p in enumerate(ps)]
    budget = sum(dsmc.footprint_bytes(r.params) for r in reqs[:4])
    ex = GpuExecutor()
    res, summ = Server(ex, budget_bytes=budget, max_slots=8, quantum=40).run(reqs)
    ex.close()
    assert summ["served"] == len(reqs) and summ["rejected"] == 0
    assert summ["peak_bytes"] <= budget
    by = {r.rid: r for r in res}
    for q in reqs:
        with dsmc.Solver(q.params) as s:
            s.step(q.steps)
            alone = s.sample()
        got = by[q.rid].moments
        assert got["n_sampled_steps"] == q.steps - 30
        for k in ("n", "ux", "uy", "uz", "T", "pxy", "qx", "qy"):
            assert np.array_equal(got[k], alone[k]), (q.rid, k)
        assert got["mass_flow"] == alone["mass_flow"]
        assert got["n_collisions"] == alone["n_collisions"]


def test_served_fp64_deterministic_results_equal_the_oracle():
    """Requests in the FP64 deterministic mode served through the continuous-
    batching loop (admitted by footprint as memory frees up, batched in one
    group with the others running, removed when done) return the CPU
    oracle's estimators of the same solve bit for bit."""
    import oracle
    from paper_2311_14140_amd import dsmc
    from paper_2311_14140_amd.serve import GpuExecutor, Request, Server
    ps = synth.config3_instances(9, seed=46, cells_range=(50, 240), ppc_range=(20, 50),
                                 precision=synth.FP64_DETERMINISTIC)
    reqs = [Request(i, 0.002 * i, p.with_(n_transient=40, seed=synth.seed_of(4, i, 7)),
                    steps=110 + 17 * i) for i, p in enumerate(ps)]
    budget = sum(sorted(dsmc.footprint_bytes(r.params) for r in reqs)[-3:])
    ex = GpuExecutor()
    res, summ = Server(ex, budget_bytes=budget, max_slots=5, quantum=30).run(reqs)
    ex.close()
    assert summ["served"] == len(reqs) and summ["rejected"] == 0
    assert summ["peak_bytes"] <= budget
    by = {r.rid: r for r in res}
    for q in reqs:
        o = oracle.Oracle(q.params)
        o.step(q.steps)
        want = o.estimators()
        got = by[q.rid].moments
        assert got["n_sampled_steps"] == want["n_sampled_steps"] == q.steps - 40
        for k in ("n", "ux", "uy", "uz", "T", "pxy", "qx", "qy", "pxy_mid"):
            assert np.array_equal(got[k], want[k]), (q.rid, k)
        assert got["mass_flow"] == want["mass_flow"], q.rid
        assert got["n_collisions"] == o.diagnostics()["n_coll"], q.rid
