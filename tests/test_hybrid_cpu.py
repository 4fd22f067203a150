"""Host logic of the MMS hybrid driver (Sec. 3.2): patch geometry and
transient length."""
import math

import pytest

from paper_2311_14140_amd import hybrid as hy


@pytest.mark.parametrize("kn,n_train", [(0.01, 4), (0.05, 20), (0.1, 40), (0.2, 80), (0.001, 3)])
def test_patch_spans_two_mean_free_paths_plus_the_buffer(kn, n_train):
    p = hy.patch_for(kn)
    assert p.n_train == n_train and p.n_buffer == 5
    assert p.n_train * p.dy >= min(2 * kn, p.n_train * p.dy) - 1e-12
    assert (p.n_train - 1) * p.dy < max(2 * kn, 3 * p.dy)
    assert math.isclose(p.length, (n_train + 5) * 0.005)


def test_patch_past_the_centre_line_is_refused():
    with pytest.raises(ValueError):
        hy.patch_for(0.3)


def test_patch_transient_covers_five_relaxation_times():
    for kn in (0.01, 0.05, 0.1, 0.2):
        L = hy.patch_for(kn).length
        steps = hy.patch_transient(kn, L)
        dt = 0.2 * kn / math.sqrt(2.0)
        assert steps >= 500 and steps * dt >= 5 * L * L / (0.796 * kn) - dt
