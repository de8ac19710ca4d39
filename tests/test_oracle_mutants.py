"""Planted mistakes in a copy of the oracle must be caught by its pins (CPU).

Each case edits one line of a temporary copy of ``oracle/rewl_oracle.c`` (a
swapped operand, a wrong sign, a dropped term, an update at the wrong bin,
an off-by-one in the exchange shuffle), builds it, and runs one pin test against it in a subprocess.  The pin must
fail; if it passed, the pin would not be able to tell the oracle from a
plausible wrong implementation.
"""
import os
import subprocess
import sys

import pytest

from oracle import build

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

MUTANTS = [
    ("wl_accept_inverted",
     "double delta = s->lng[slot][b - lo] - s->lng[slot][bn - lo];",
     "double delta = s->lng[slot][bn - lo] - s->lng[slot][b - lo];",
     "tests/test_oracle_rewl.py::test_fixed_lng_stationary_distribution_with_exchanges"),
    ("exchange_eq1_sign",
     "double lnP = (s->lng[si][ix] - s->lng[si][iy]) + (s->lng[sj][jy] - s->lng[sj][jx]);",
     "double lnP = (s->lng[si][ix] - s->lng[si][iy]) + (s->lng[sj][jx] - s->lng[sj][jy]);",
     "tests/test_oracle_rewl.py::test_fixed_lng_stationary_distribution_with_exchanges"),
    ("histogram_not_reset_at_merge",
     "    for (int k = 0; k < m; ++k) s->H[w * m + k][j] = 0;\n",
     "",
     "tests/test_oracle_rewl.py::test_histogram_counts_attempts_and_merge_semantics"),
    ("lnf_not_halved",
     "double next = phase_b ? tinv : 0.5 * s->lnf[w];",
     "double next = phase_b ? tinv : 0.75 * s->lnf[w];",
     "tests/test_oracle_rewl.py::test_histogram_counts_attempts_and_merge_semantics"),
    ("merge_wrong_divisor",
     "double mean = tree_sum64(t64, m) / (double)m;",
     "double mean = tree_sum64(t64, m) / (double)(m + 1);",
     "tests/test_oracle_rewl.py::test_histogram_counts_attempts_and_merge_semantics"),
    ("stitch_shift_sign",
     "shift = (la[best - oa] + shift) - lb[best - ob];",
     "shift = (la[best - oa] - shift) - lb[best - ob];",
     "tests/test_oracle_rewl.py::test_stitch_recovers_exact_from_offset_pieces"),
    ("potts_dE_sign",
     "dE = eq_old - eq_new;",
     "dE = eq_new - eq_old;",
     "tests/test_oracle_rewl.py::test_energy_and_histogram_bookkeeping"),
    ("exp_dropped_term",
     "  p = fma(p, r, 1.0 / 6.0);\n",
     "",
     "tests/test_oracle_primitives.py::test_exp_spec_within_one_ulp_of_libm"),
    ("flatness_threshold_transposed",
     "if ((uint64_t)s->p.flat_den * cnt * mn < (uint64_t)s->p.flat_num * sum) ready = 0;",
     "if ((uint64_t)s->p.flat_num * cnt * mn < (uint64_t)s->p.flat_den * sum) ready = 0;",
     "tests/test_oracle_rewl.py::test_histogram_counts_attempts_and_merge_semantics"),
    ("one_over_t_value",
     "double tinv = (double)cnt / (double)s->att[w * m];",
     "double tinv = (double)(cnt + 1) / (double)s->att[w * m];",
     "tests/test_oracle_schedule.py::test_one_over_t_schedule_follows_its_definition"),
    ("one_over_t_late_switch",
     "int to_b = s->p.schedule == ORC_ONE_OVER_T && !phase_b && next <= tinv;",
     "int to_b = s->p.schedule == ORC_ONE_OVER_T && !phase_b && next <= 0.5 * tinv;",
     "tests/test_oracle_schedule.py::test_one_over_t_schedule_follows_its_definition"),
    ("jackknife_variance_factor",
     "err[b] = sqrt((double)(m - 1) / (double)m * v);",
     "err[b] = sqrt(v / (double)m);",
     "tests/test_oracle_schedule.py::test_jackknife_single_window_is_standard_error_of_mean"),
    ("pieces_wrong_walker",
     "s->pieces[w * m + k][j] = lng_at(s, w * m + k, j);",
     "s->pieces[w * m + k][j] = lng_at(s, w * m, j);",
     "tests/test_oracle_schedule.py::test_pieces_are_the_walkers_before_the_freezing_merge"),
    ("pairing_sattolo",
     "int j = (int)(((uint64_t)r[used++] * (uint32_t)(i + 1)) >> 32);",
     "int j = (int)(((uint64_t)r[used++] * (uint32_t)i) >> 32);",
     "tests/test_oracle_pairing.py::test_pairing_is_uniform_over_all_permutations"),
    ("pairing_last_swap_skipped",
     "for (int i = m - 1; i >= 1; --i) {\n    if (used == 4) {",
     "for (int i = m - 1; i >= 2; --i) {\n    if (used == 4) {",
     "tests/test_oracle_pairing.py::test_pairing_is_uniform_over_all_permutations"),
    ("exchange_partner_not_permuted",
     "int si = w * m + k, sj = (w + 1) * m + pi[k];",
     "int si = w * m + k, sj = (w + 1) * m + k;",
     "tests/test_oracle_pairing.py::test_exchange_round_pairs_walkers_by_the_pairing"),
    ("energy_neighbour_index",
     "int sd = sp[((y + 1) % L) * L + x];",
     "int sd = sp[((y + 1) % L) * L + (x + 1) % L];",
     "tests/test_oracle_primitives.py::test_energy_matches_independent_formula"),
]


@pytest.mark.parametrize("name,old,new,pin", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pin_catches_planted_mistake(tmp_path, name, old, new, pin):
    src = open(build.SRC).read()
    assert src.count(old) == 1, f"mutation site for {name} not unique"
    mutated = tmp_path / "rewl_oracle.c"
    mutated.write_text(src.replace(old, new))
    (tmp_path / "rewl_oracle.h").write_text(open(os.path.join(os.path.dirname(build.SRC),
                                                              "rewl_oracle.h")).read())
    lib = tmp_path / "libmutant.so"
    subprocess.check_call(["gcc", *build.CFLAGS, str(mutated), "-o", str(lib), "-lm"])
    env = dict(os.environ, REWL_ORACLE_LIB=str(lib))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, pin)], cwd=ROOT, env=env,
                       capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"pin {pin} did not detect mutant {name}:\n{r.stdout[-2000:]}"
