"""Pins of the oracle's random-number machinery against references outside it.

- Philox4x32-10 against the generator's published known-answer vectors and
  against rocRAND's independent engine (compiled here for the host).
- The 53-bit uniform map: range (0,1], exact multiples of 2^-53, moments.
- The atanh-series logarithm against the C library's correctly rounded-ish
  ``log`` (within 4 ulp) and at edge values.
- Polar normal pairs and Marsaglia sphere points: their textbook moments and
  a Kolmogorov-Smirnov test.
"""
import math
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import stats

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


def test_philox_known_answers():
    path = os.path.join(HERE, "golden", "philox4x32_10_kat.txt")
    n = 0
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        w = [int(x, 16) for x in line.split()]
        ctr, key, want = w[0:4], w[4:6], w[6:10]
        got = oracle.philox(ctr, key)
        assert [int(x) for x in got] == want
        n += 1
    assert n == 3


@pytest.fixture(scope="module")
def rocrand_ref(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("philox") / "philox_ref")
    src = os.path.join(HERE, "golden", "philox_rocrand_ref.cpp")
    subprocess.run([hipcc, "-O1", "-o", exe, src], check=True, capture_output=True)
    return exe


def test_philox_matches_rocrand(rocrand_ref):
    rng = np.random.default_rng(12345)
    lines, want = [], []
    for _ in range(3000):
        k = rng.integers(0, 2**32, 2)
        c = rng.integers(0, 2**32, 4)
        c[1] %= 2**30  # rocRAND takes counter words 0-1 as offset/4 in 64 bits
        lines.append(" ".join("%x" % v for v in list(k) + list(c)))
        want.append(" ".join("%08x" % x for x in oracle.philox(c, k)))
    out = subprocess.run([rocrand_ref], input="\n".join(lines) + "\n", capture_output=True,
                         text=True, check=True).stdout.split("\n")
    assert out[:len(want)] == want


def test_philox_counter_words_all_matter():
    base = oracle.philox([1, 2, 3, 4], [5, 6])
    for i in range(4):
        c = [1, 2, 3, 4]
        c[i] ^= 1
        assert not np.array_equal(oracle.philox(c, [5, 6]), base)
    assert not np.array_equal(oracle.philox([1, 2, 3, 4], [5, 7]), base)


def test_uniform_range_and_grid():
    u = np.array([oracle.uniform2(7, s, e, 0, 3, 0) for s in range(50) for e in range(200)]).ravel()
    assert u.min() > 0.0 and u.max() <= 1.0
    k = u * 2.0**53
    assert np.all(k == np.round(k))
    # uniform moments: mean 1/2, variance 1/12; KS against U(0,1)
    n = len(u)
    assert abs(u.mean() - 0.5) < 4 * math.sqrt(1 / 12 / n)
    assert abs(u.var() - 1 / 12) < 4 * math.sqrt(1 / 180 / n)
    assert stats.kstest(u, "uniform").pvalue > 1e-3


def _ulp_diff(a, b):
    return abs(a - b) / math.ulp(b) if b != 0 else abs(a) / math.ulp(1.0)


def test_series_log_within_4ulp():
    rng = np.random.default_rng(2)
    xs = list(rng.random(20000) + 2.0**-53)
    xs += list(np.exp(-rng.random(5000) * 36.0))
    worst = 0.0
    for x in xs:
        x = float(x)
        got = oracle.series_log(x)
        want = math.log(x)
        worst = max(worst, _ulp_diff(got, want))
    assert worst <= 4.0


def test_series_log_edges():
    assert oracle.series_log(1.0) == 0.0
    assert oracle.series_log(0.5) == -math.log(2.0) or _ulp_diff(oracle.series_log(0.5), math.log(0.5)) <= 1
    sqrt2 = 1.4142135623730951
    for x in (2.0**-53, 2.0**-52, 1.0 - 2.0**-53, 0.5 + 2.0**-53, sqrt2 / 2,
              math.nextafter(sqrt2 / 2, 0), math.nextafter(sqrt2 / 2, 1), 0.75, 1e-16):
        assert _ulp_diff(oracle.series_log(x), math.log(x)) <= 4.0, x


def test_normal_pairs_moments():
    v = np.array([oracle.normal2(11, 3, e, s, 2, 1) for e in range(400) for s in range(50)]).ravel()
    n = len(v)
    assert abs(v.mean()) < 4 / math.sqrt(n)
    assert abs(v.var() - 1.0) < 4 * math.sqrt(2 / n)
    assert abs(stats.kurtosis(v, fisher=False) - 3.0) < 4 * math.sqrt(24 / n)
    assert stats.kstest(v, "norm").pvalue > 1e-3
    # variance scales with the requested sqrt_var
    w = np.array([oracle.normal2(11, 3, e, 0, 2, 1, sqrt_var=2.0) for e in range(400)]).ravel()
    u = np.array([oracle.normal2(11, 3, e, 0, 2, 1) for e in range(400)]).ravel()
    assert np.allclose(w, 2.0 * u, rtol=0, atol=1e-15)


def test_sphere_points_isotropic():
    d = np.array([oracle.sphere(5, 9, e, s, 3, 2) for e in range(400) for s in range(25)])
    n = len(d)
    assert np.allclose(np.linalg.norm(d, axis=1), 1.0, atol=1e-14)
    assert np.all(np.abs(d.mean(axis=0)) < 4 * math.sqrt(1 / 3 / n))
    sec = (d**2).mean(axis=0)
    assert np.all(np.abs(sec - 1 / 3) < 4 * math.sqrt(4 / 45 / n))
    # each coordinate of a uniform sphere point is uniform on [-1, 1] (Archimedes)
    assert stats.kstest(d[:, 2], "uniform", args=(-1, 2)).pvalue > 1e-3
    assert stats.kstest(d[:, 0], "uniform", args=(-1, 2)).pvalue > 1e-3


def test_uniform_all_53_bits_are_fair():
    """U = (k + 1) 2^-53 with k uniform on [0, 2^53): every bit of k is a fair
    coin, so no bit of the 53 is stuck or duplicated."""
    u = np.array([oracle.uniform2(19, s, e, 1, 2, 3) for s in range(40) for e in range(250)]).ravel()
    k = (u * 2.0**53).astype(np.uint64) - np.uint64(1)
    n = len(k)
    for b in range(53):
        frac = float(((k >> np.uint64(b)) & np.uint64(1)).mean())
        assert abs(frac - 0.5) < 4.5 * 0.5 / math.sqrt(n), (b, frac)
