"""The oracle's pins catch plausible mistakes.

Each case below plants one mistake in a copy of the oracle's C source (a
wrong sign, a dropped term, a wrong index or bit count, a step out of
order, a wrong initial state ...), builds the copy, and runs the pins named
for it against that build (the oracle package loads it through
DSMC_ORACLE_LIB).  A pin that still passes with the mistake in place would
not be pinning anything, so every case must make at least one of its pins
fail.  The unmutated oracle passes the same pins in the ordinary run of the
suite.
"""
import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(ROOT, "oracle", "dsmc_oracle.c")

INIT = "test_oracle_init.py::"
RNG = "test_oracle_rng.py::"
MOVE = "test_oracle_move.py::"
SC = "test_oracle_sort_collide.py::"
PHYS = "test_oracle_physics.py::"

# (name, text in the oracle, replacement, pins expected to catch it)
MUTATIONS = [
    # initial state (Sec. 2.1 gas at rest between the plates, Sec. 3 particles per cell)
    ("init_all_in_cell_0", "int32_t c = p / ppc;", "int32_t c = 0;",
     [INIT + "test_every_cell_starts_with_ppc_particles_uniform_inside"]),
    ("init_cell_p_mod_C", "int32_t c = p / ppc;", "int32_t c = p % S->C;",
     [INIT + "test_every_cell_starts_with_ppc_particles_uniform_inside"]),
    ("init_lower_half_of_cell", "S->y[p] = ((double)c + (1.0 - ua)) * dy;",
     "S->y[p] = ((double)c + 0.5 * (1.0 - ua)) * dy;",
     [INIT + "test_every_cell_starts_with_ppc_particles_uniform_inside"]),
    ("init_vz_three_times_wide", "stream_normal2(&s, S->sqrt_tw, &S->vz[p], &dummy);",
     "stream_normal2(&s, 3.0 * S->sqrt_tw, &S->vz[p], &dummy);",
     [INIT + "test_initial_velocities_are_the_wall_maxwellian_at_rest"]),
    ("init_unit_temperature", "stream_normal2(&s, S->sqrt_tw, &S->vx[p], &S->vy[p]);",
     "stream_normal2(&s, 1.0, &S->vx[p], &S->vy[p]);",
     [INIT + "test_initial_velocities_are_the_wall_maxwellian_at_rest"]),
    ("init_vz_copies_vx", "stream_normal2(&s, S->sqrt_tw, &S->vz[p], &dummy);",
     "S->vz[p] = S->vx[p]; (void)dummy;",
     [INIT + "test_initial_velocities_are_the_wall_maxwellian_at_rest"]),
    # random numbers
    ("philox_wrong_multiplier", "PHILOX_M0 = 0xD2511F53u", "PHILOX_M0 = 0xD2511F55u",
     [RNG + "test_philox_known_answers"]),
    ("philox_nine_rounds", "for (int r = 0; r < 10; ++r)", "for (int r = 0; r < 9; ++r)",
     [RNG + "test_philox_known_answers"]),
    ("uniform_52_bits", "(uint64_t)(b >> 6)", "(uint64_t)(b >> 7)",
     [RNG + "test_uniform_range_and_grid", RNG + "test_uniform_all_53_bits_are_fair"]),
    ("log_series_dropped_term", "for (int i = 10; i >= 0; --i)", "for (int i = 10; i >= 1; --i)",
     [RNG + "test_series_log_within_4ulp"]),
    ("polar_missing_factor_2", "sqrt((-2.0 * or_log(q)) / q)", "sqrt((-1.0 * or_log(q)) / q)",
     [RNG + "test_normal_pairs_moments"]),
    ("sphere_wrong_axis", "d[2] = 1.0 - 2.0 * q;", "d[2] = 1.0 - q;",
     [RNG + "test_sphere_points_isotropic"]),
    # free flight, walls, cell index (Sec. 2.1; Eq. 6 force scaling)
    ("force_kick_whole_step", "            y = y + vy * t;\n            vx = vx + S->g * t;",
     "            y = y + vy * t;\n            vx = vx + S->g * S->dt;",
     [PHYS + "test_exact_momentum_balance"]),
    ("force_not_doubled", "S->g = 2.0 * p->body_force;", "S->g = p->body_force;",
     [MOVE + "test_no_hit_is_exact_constant_acceleration"]),
    ("wall_hit_not_strict", "if (tw >= t) {", "if (tw > t) {",
     [MOVE + "test_landing_exactly_on_wall_is_not_a_hit"]),
    ("wall_normal_speed_not_flux_weighted", "double vn = sqrt(-2.0 * or_log(ua)) * S->sqrt_tw;",
     "double vn = sqrt(-or_log(ua)) * S->sqrt_tw;",
     [MOVE + "test_wall_reemission_is_flux_weighted_maxwellian"]),
    ("wall_time_not_reduced", "        t = t - tw;\n", "",
     [MOVE + "test_single_top_hit_reemits_downwards"]),
    ("wall_keeps_tangential_velocity", "stream_normal2(&s, S->sqrt_tw, &vx, &vz);",
     "{ double t0_, t1_; stream_normal2(&s, S->sqrt_tw, &t0_, &t1_); }",
     [MOVE + "test_wall_reemission_is_flux_weighted_maxwellian"]),
    ("cell_index_rounded", "int32_t c = (int32_t)(y * S->inv_dy);",
     "int32_t c = (int32_t)(y * S->inv_dy + 0.5);",
     [MOVE + "test_cell_index_edges"]),
    # stable counting sort
    ("sort_unstable", "for (int32_t i = 0; i < n; ++i) perm[next[key[i]]++] = i;",
     "for (int32_t i = n - 1; i >= 0; --i) perm[next[key[i]]++] = i;",
     [SC + "test_stable_sort_matches_numpy"]),
    # NTC collisions
    ("ntc_n_squared_pairs", "((0.5 * (double)n) * (double)(n - 1))",
     "((0.5 * (double)n) * (double)n)", [SC + "test_collision_frequency_hard_sphere"]),
    ("ntc_remainder_dropped", "S->rem[c] = m_real - m_floor;", "S->rem[c] = 0.0;",
     [SC + "test_collision_frequency_hard_sphere"]),
    ("ntc_pair_may_repeat", "if (j >= i) j = j + 1;", "if (j > n - 1) j = n - 1;",
     [SC + "test_collision_frequency_hard_sphere"]),
    ("ntc_acceptance_by_cr_squared", "if (ua2 * S->crmax[c] < cr) {",
     "if (ua2 * S->crmax[c] * S->crmax[c] < cr * cr) {",
     [SC + "test_collision_frequency_hard_sphere"]),
    ("scatter_same_sign", "vx[j] = cmx - hh * d[0];", "vx[j] = cmx + hh * d[0];",
     [SC + "test_collisions_conserve_momentum_and_energy"]),
    ("scatter_half_relative_speed", "double hh = 0.5 * cr;", "double hh = 0.25 * cr;",
     [SC + "test_collisions_conserve_momentum_and_energy"]),
    # sampling and estimators (Eq. 13 stress, Eq. 6 normalisation)
    ("sample_v2_without_vz", "double v2 = (x * x + y * y) + z * z;", "double v2 = x * x + y * y;",
     [PHYS + "test_estimators_match_central_moment_definitions"]),
    ("estimator_temperature_over_2", "if (T) T[c] = ((mxx + myy) + mzz) / 3.0;",
     "if (T) T[c] = ((mxx + myy) + mzz) / 2.0;",
     [PHYS + "test_estimators_match_central_moment_definitions"]),
    ("estimator_mass_flow_per_cell", "if (Q) *Q = (qsum / (K * N)) / v0;",
     "if (Q) *Q = (qsum / (K * (double)C)) / v0;",
     [PHYS + "test_estimators_match_central_moment_definitions"]),
    ("estimator_heat_flux_sign", "double cx = ((s[10] / s[0] - u * (trace2 / s[0])) -",
     "double cx = ((s[10] / s[0] + u * (trace2 / s[0])) -",
     [PHYS + "test_estimators_match_central_moment_definitions"]),
    ("pre_collision_sum_after_collide",
     "        if (sampling) phase_sample_pre(S);\n        if (phase_mask & PHASE_COLLIDE) phase_collide(S, step);",
     "        if (phase_mask & PHASE_COLLIDE) phase_collide(S, step);\n        if (sampling) phase_sample_pre(S);",
     [PHYS + "test_pre_collision_stress_sum_is_taken_before_the_collide_phase"]),
    ("stress_mid_uses_post_twice", "pxy_mid[c] = n_c * ((0.5 * (s[7] + s[12])) / s[0] - u * v);",
     "pxy_mid[c] = n_c * ((0.5 * (s[7] + s[7])) / s[0] - u * v);",
     [PHYS + "test_stress_slope_meets_the_momentum_balance_at_any_kn[1.0]"]),
]


def _build(name, src, tmp):
    c = os.path.join(tmp, name + ".c")
    so = os.path.join(tmp, name + ".so")
    with open(c, "w") as fh:
        fh.write(src)
    subprocess.run(["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
                    "-shared", "-w", "-o", so, c, "-lm"], check=True)
    return so


def _run_pins(so, pins):
    env = dict(os.environ, DSMC_ORACLE_LIB=so)
    try:
        r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                            "-p", "no:xdist", "-m", "not gpu"] +
                           [os.path.join(HERE, t) for t in pins],
                           cwd=ROOT, env=env, capture_output=True, text=True, timeout=180)
    except subprocess.TimeoutExpired:
        return None, "pins did not finish within 180 s"
    return r.returncode, r.stdout[-2000:]


def test_every_planted_mistake_is_caught():
    with open(SRC) as fh:
        src = fh.read()
    for name, old, new, _ in MUTATIONS:
        assert src.count(old) == 1, f"{name}: the mutated text must occur once in the oracle"
    names = [m[0] for m in MUTATIONS]
    assert len(set(names)) == len(names)
    with tempfile.TemporaryDirectory() as tmp:
        def one(m):
            name, old, new, pins = m
            so = _build(name, src.replace(old, new), tmp)
            return name, _run_pins(so, pins)

        with ThreadPoolExecutor(min(8, os.cpu_count() or 1)) as ex:
            results = list(ex.map(one, MUTATIONS))
    missed = [(name, out) for name, (rc, out) in results if rc != 1]
    assert not missed, "mistakes not caught (or pins errored): " + "; ".join(
        f"{n}: {o[-400:]}" for n, o in missed)


@pytest.mark.parametrize("pins", sorted({p for m in MUTATIONS for p in m[3]}))
def test_pins_of_the_mutation_cases_exist(pins):
    path, _, name = pins.partition("::")
    with open(os.path.join(HERE, path)) as fh:
        assert "def " + name.split("[")[0] + "(" in fh.read()
