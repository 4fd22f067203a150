"""One-way verification of the micro-macro coupling on the GPU (Sec. 3.1):
surrogates trained on windows of the 50-per-cell solver, the corrected macro
model solved with them, and its velocity compared with a benchmark run of
500 particles per cell."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_one_way_mms_matches_the_benchmark_at_kn1():
    from paper_2311_14140_amd import mms
    print("one-way MMS: Kn 1, 64 replicas x 200 windows; benchmark 8 x 25000 steps", flush=True)
    r = mms.one_way(1.0, training_steps=2, samples_per_step=100, replicas=64,
                    bench_steps=200000, bench_replicas=8, n_trials=1000)
    s = r.trainer.history[-1]
    c = r.compare()
    print({k: round(v, 5) if isinstance(v, float) else v for k, v in c.items()},
          f"sigma_P {s.sigma_p:.4f}", f"p(C_k) {np.round(s.p_constitutive, 4)}", flush=True)
    sys.stdout.flush()
    assert s.n_samples == 12800
    assert s.slip and s.p_boundary[1] > 0.999999
    assert s.p_constitutive[0] < 1e-6
    # the stress of the macro model is the momentum balance's
    assert np.allclose(r.solution.pxy, 2 * r.trainer.force * (r.solution.y - 0.5))
    assert c["max_rel_err"] < 0.015
    assert abs(c["mass_flow_rel_err"]) < 0.01
    assert np.all(r.solution.u_std > 0)
