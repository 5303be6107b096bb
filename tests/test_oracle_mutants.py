"""The oracle's pins must catch plausible mistakes.  Each mutant below is a
copy of the oracle source with one planted error (a sign, an index, a
threshold, a tie-break, a dropped term); it is compiled into a temporary
library and the pin checks are re-run against it: every mutant must fail at
least one of them.  Mistakes are planted in the oracle on the CPU only."""
import os
import subprocess

import numpy as np
import pytest

import oracle
import test_oracle as pins
import test_oracle_scaled as cpins
import test_oracle_shifted as spins
from golden_io import decode_cases

MUTANTS = {
    "residual_sign": ("r[i] = y[i] - s[i];", "r[i] = y[i] + s[i];"),
    "update_sign": ("x_out[j] = x_out[j] + (w ?", "x_out[j] = x_out[j] - (w ?"),
    "scaled_update_multiplies": ("(w ? omega[j] / w[j] : omega[j])", "(w ? omega[j] * w[j] : omega[j])"),
    "scaled_residual_unweighted": ("const double term = w ? w[j] * x[j] : x[j];", "const double term = x[j];"),
    "scaled_residual_weight_index": ("const double term = w ? w[j] * x[j] : x[j];",
                                     "const double term = w ? w[(j + 1) % n] * x[j] : x[j];"),
    "tie_break_largest": ("(score == top && v[t] < w)", "(score == top && v[t] > w)"),
    "drop_zero_count": ("(rule == ORC_RULE_MODE) ? freq : before - after;", "(rule == ORC_RULE_MODE) ? freq : d - after;"),
    "shift_drop_zero_count": ("(shifted_rule == ORC_RULE_SHIFTED_MODE) ? freq : before - after;",
                              "(shifted_rule == ORC_RULE_SHIFTED_MODE) ? freq : d - after;"),
    "threshold_floor": ("const int32_t a = (int32_t)ceil(alpha);\n    const double tau = zero_threshold(m, y, tol, tol_mode);",
                        "const int32_t a = (int32_t)floor(alpha);\n    const double tau = zero_threshold(m, y, tol, tol_mode);"),
    "strict_threshold": ("return top != INT_MIN && top >= a;", "return top != INT_MIN && top > a;"),
    "zero_test_nonstrict": ("return fabs(v) > tau;", "return fabs(v) >= tau;"),
    "gather_index": ("for (int32_t t = 0; t < d; ++t) vt[t] = r[col_idx[j * d + t]];",
                     "for (int32_t t = 0; t < d; ++t) vt[t] = r[col_idx[j * d]];"),
    "residual_skips_last_row": ("for (int32_t i = 0; i < m; ++i) r[i] = y[i] - s[i];",
                                "for (int32_t i = 0; i + 1 < m; ++i) r[i] = y[i] - s[i];"),
    "serial_row_recompute_missing": ("r[i] = y[i] - s;", "r[i] = y[i] - s * (t == 0);"),
    "tau_absolute": ("return tol * s;", "return tol;"),
    "shift_offset": ("score_column_shifted(d, vt, p % d,", "score_column_shifted(d, vt, (p + 1) % d,"),
    "shift_position_by_update": ("score_column_shifted(d, vt, p % d,", "score_column_shifted(d, vt, l % d,"),
    "shift_no_retry": ("if (shifted && ++empty < d) continue;", "if (shifted && ++empty < 1) continue;"),
    "repeated_row_accepted": ("if (rows[u] == rows[t]) return 0;", "if (rows[u] == rows[t] && m < 0) return 0;"),
    "repeated_row_first_only": ("for (int32_t u = 0; u < t; ++u)", "for (int32_t u = 0; u < t && u < 1; ++u)"),
    "absolute_mode_ignored": ("    if (tol_mode == ORC_TOL_ABSOLUTE) return tol;\n", ""),
    "shift_zero_candidate": ("    *omega = 0.0;\n    if (!is_nonzero(v[t], tau)) return 0;\n", "    *omega = 0.0;\n"),
}


def _run_pins():
    """Run the pin checks; return the names of those that fail."""
    failed = []
    checks = [("scorer", pins.test_scorer_cases)]
    for c in decode_cases():
        checks.append((f"worked-{c[0]}-{c[4]['algo']}-{c[4]['rule']}-{c[4]['alpha']}",
                       lambda c=c: pins.test_worked_decodes(c)))
    checks += [
        ("closed_form_count", lambda: [pins.test_score_equals_count_closed_form(t, r)
                                       for t in (0.0, 1e-10) for r in (0, 1)]),
        ("disjoint", pins.test_disjoint_columns_one_iteration),
        ("k1", lambda: pins.test_k1_recovers_in_one_iteration(0)),
        ("true_updates", lambda: pins.test_updates_are_true_values_and_trace_decreases(0)),
        ("scaling", lambda: [pins.test_power_of_two_scaling_bitwise(e) for e in (-40, 5)]),
        ("serial_parallel", pins.test_serial_and_parallel_agree),
        ("shift_literal", lambda: [spins.test_shifted_selection_is_the_literal_score_of_one_candidate(t, r)
                                   for t in (0.0, 1e-9) for r in (oracle.RULE_L0DEC, oracle.RULE_MODE)]),
        ("shift_subset", spins.test_shifted_selects_a_subset_of_the_full_vote),
        ("shift_closed", spins.test_shifted_k0_and_disjoint_columns),
        ("shift_theorem", lambda: spins.test_theorem_4_8_on_dissociated_signals(0)),
        ("scaled_unit", lambda: cpins.test_unit_weights_are_the_unscaled_decoder(oracle.RULE_L0DEC)),
        ("scaled_pow2", lambda: cpins.test_power_of_two_weights_decode_the_weighted_signal(oracle.RULE_L0DEC)),
        ("scaled_literal", lambda: cpins.test_scaled_selection_is_the_literal_decrease(oracle.RULE_L0DEC)),
        ("scaled_residual", cpins.test_scaled_residual_against_a_dense_product),
        ("scaled_pm1", lambda: cpins.test_pm1_signals_recovered_only_with_scaled_columns(0)),
        ("repeated_row", pins.test_repeated_row_in_a_column_is_rejected),
        ("absolute_tau", pins.test_absolute_tolerance_is_tau_itself),
    ]
    for name, fn in checks:
        try:
            fn()
        except (AssertionError, ValueError, pytest.fail.Exception):
            failed.append(name)
    return failed


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path, monkeypatch):
    with open(oracle._SRC) as f:
        src = f.read()
    old, new = MUTANTS[name]
    assert src.count(old) == 1, f"mutation site for {name} not found exactly once"
    path = os.path.join(tmp_path, "mut.c")
    with open(path, "w") as f:
        f.write(src.replace(old, new))
    lib = os.path.join(tmp_path, "libmut.so")
    subprocess.run(["gcc", "-O2", "-fPIC", "-shared", "-ffp-contract=off", "-std=c11", "-o", lib, path,
                    "-lm"], check=True)
    monkeypatch.setattr(oracle, "_LIB", lib)
    monkeypatch.setattr(oracle, "_lib", None)
    failed = _run_pins()
    assert failed, f"mutant {name} passed every pin"


def test_unmutated_oracle_passes_all_pins():
    assert _run_pins() == []
