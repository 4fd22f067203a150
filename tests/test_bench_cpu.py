"""bench.py refuses more than one GPU (the build has no multi-GPU path)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_rejects_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=60)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_all_core_oracle_rate_counts_every_thread():
    sys.path.insert(0, ROOT)
    import bench
    import synth
    ps = [synth.CONFIG0.with_(n_cells=20, particles_per_cell=10, seed=synth.seed_of(0, i))
          for i in range(3)]
    rate, done, el, used = bench.cpu_oracle_rate_all_cores(ps, 0.3, 2)
    assert used == 2 and done > 0 and el >= 0.3
    assert done % 2 == 0 and rate == done / el
    host = bench.host_identity()
    assert 1 <= host["usable_cores"] <= 16 and host["nproc"] >= 1
