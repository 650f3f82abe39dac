"""The oracle's pins must catch plausible mistakes.

Each case plants one mistake in a private copy of oracle.c (a dropped term, a
wrong sign or index, a wrong coefficient, a missing rule), builds it on the CPU
and runs the pin that should catch it against the mutant in a subprocess.  The
pin must FAIL on the mutant.  Nothing here touches the GPU.
"""
import os
import subprocess
import sys

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.c")

MUTANTS = [
    ("jerk_drops_radial_term", "jx += m[j] * (wx * s_m32 - 3.0 * rw * rx * s_m52);",
     "jx += m[j] * (wx * s_m32);", "test_jerk_is_time_derivative_of_acceleration"),
    ("acc_wrong_sign", "ax += m[j] * rx * s_m32;", "ax -= m[j] * rx * s_m32;",
     "test_two_body_attraction_direction_and_symmetry"),
    ("transposed_index", "const double wy = v[3 * j + 1] - v[3 * i + 1];",
     "const double wy = v[3 * j + 1] - v[3 * i + 0];", "test_momentum_and_angular_momentum_rates_vanish"),
    ("acc_uses_wrong_power", "const double s_m32 = s_m12 / s;", "const double s_m32 = s_m12 / sqrt(s);",
     "test_shell_theorem_outside_fibonacci_sphere"),
    ("self_term_kept", "if (j == i)\n                continue;", "",
     "test_two_body_attraction_direction_and_symmetry"),
    ("softening_dropped", "rz * rz + eps2;", "rz * rz;",
     "test_two_body_attraction_direction_and_symmetry"),
    ("predictor_half_missing", "a[q] * d * d / 2.0 + jk[q]", "a[q] * d * d + jk[q]",
     "test_predictor_exact_for_cubic_motion"),
    ("corrector_a3_coefficient", "(12.0 * (a0[c] - a1[c])", "(6.0 * (a0[c] - a1[c])",
     "test_corrector_exact_for_quintic_trajectory"),
    ("corrector_x_term", "a3 * dt * dt * dt * dt * dt / 120.0", "a3 * dt * dt * dt * dt * dt / 24.0",
     "test_corrector_exact_for_quintic_trajectory"),
    ("aarseth_wrong_power", "const double num = na * na2 + nj * nj;",
     "const double num = na * na2 + nj;", "test_aarseth_step_on_circular_motion"),
    ("doubling_ignores_commensurability", "fmod(t_new, 2.0 * dt) == 0.0", "1",
     "test_block_dt_rules"),
    ("energy_counts_pairs_twice", "for (int64_t j = i + 1; j < N; j++) {",
     "for (int64_t j = 0; j < N; j++) { if (j == i) continue;",
     "test_potential_energy_matches_half_sum_of_potentials"),
]


@pytest.mark.parametrize("name,old,new,pin", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pin_catches_mutant(tmp_path, name, old, new, pin):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor for {name} not unique"
    mut = tmp_path / "oracle_mut.c"
    mut.write_text(src.replace(old, new))
    lib = str(tmp_path / "liboracle_mut.so")
    oracle.build(str(mut), lib)
    env = dict(os.environ, NBODY_ORACLE_LIB=lib)
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle.py") + "::" + pin],
                       env=env, cwd=ROOT, capture_output=True, text=True, timeout=300)
    assert r.returncode != 0, f"pin {pin} did not catch mutant {name}:\n{r.stdout[-2000:]}"
