"""The three scans of the sort's count matrices give the same step: the
single-workgroup scan of lanes whose matrices all fit LDS, the
single-workgroup scan with the segment sums in LDS of lanes whose segment
sums all fit it, and the column-scan kernels of lanes with a larger member.
Instances stepped in a group of small instances equal themselves stepped
beside a medium and beside a large one, bit for bit, closed and open, FP32
and FP64-fast."""
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


def _run(D, plist, n_steps, inflow_for):
    sols = [D.Solver(p) for p in plist]
    g = D.Group()
    g.set_resident(False)
    for s, p in zip(sols, plist):
        if p.domain_length:
            s.set_inflow(**inflow_for)
        g.add(s)
    g.step(n_steps)
    g.sync()
    prof = sols[0].profile(1)
    out = [(s.get_state(), s.get_cells(), s.sample(raw=True)["raw"],
             s.open_state() if p.domain_length else None) for s, p in zip(sols, plist)]
    g.close()
    for s in sols:
        s.close()
    return out, prof


@pytest.mark.parametrize("prec_name", ["DSMC_FP32_FAST", "DSMC_FP64_FAST"])
def test_small_scan_equals_column_scans(D, prec_name):
    prec = getattr(D, prec_name)
    small = [Params(kn=1.0, body_force=0.01, n_cells=200, particles_per_cell=50, seed=41,
                    n_transient=10, precision=prec),
             synth.PATCH0.with_(seed=42, n_transient=10, precision=prec),
             Params(kn=0.1, body_force=0.005, n_cells=30, particles_per_cell=300, seed=43,
                    n_transient=10, precision=prec)]
    medium = Params(kn=0.05, body_force=0.005, n_cells=2000, particles_per_cell=100, seed=44,
                    n_transient=10, precision=prec)
    large = Params(kn=0.01, body_force=0.005, n_cells=4000, particles_per_cell=300, seed=45,
                   n_transient=10, precision=prec)
    print(f"small-matrix scan vs segment scan vs column scans: {prec_name}", flush=True)
    sys.stdout.flush()
    inflow = synth.PATCH0_INFLOW
    a, prof_a = _run(D, small, 41, inflow)
    b, prof_b = _run(D, small + [medium], 41, inflow)
    c, prof_c = _run(D, small + [large], 41, inflow)
    # the single-workgroup scans leave the column-sum and prefix slots empty
    assert prof_a["colsum"] == 0 and prof_a["colprefix"] == 0 and prof_a["scan"] > 0
    assert prof_b["colsum"] == 0 and prof_b["colprefix"] == 0 and prof_b["scan"] > 0
    assert prof_c["colsum"] > 0 and prof_c["colprefix"] > 0
    for other in (b, c):
        for x, y in zip(a, other[:len(small)]):
            for u, v in zip(x[0], y[0]):
                assert np.array_equal(np.asarray(u), np.asarray(v))
            for u, v in zip(x[1], y[1]):
                assert np.array_equal(np.asarray(u), np.asarray(v))
            assert np.array_equal(x[2], y[2])
            assert x[3] == y[3]
