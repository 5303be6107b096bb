"""Pins of the oracle's shifted Parallel-l0 (Section 4.3.1: Algorithm 3 and
Theorem 4.8) against what the paper and the definitions fix: the literal
l0-decrease of eq. (selection_l0) at the one candidate each column tries,
the relation to the full vote, closed forms and Theorem 4.8's behaviour on
dissociated signals.  The hand-derived worked decodes WS1, WS3 and W3 are
checked by test_oracle.test_worked_decodes."""
import numpy as np
import pytest

import gen
import oracle

SHIFTED = {oracle.RULE_L0DEC: oracle.RULE_SHIFTED_L0DEC, oracle.RULE_MODE: oracle.RULE_SHIFTED_MODE}


def _planted(rng, m, tau):
    base = rng.standard_normal(6)
    r = base[rng.integers(0, 6, m)].copy()
    r[rng.random(m) < 0.25] = 0.0
    if tau > 0:
        noisy = rng.random(m) < 0.3
        r[noisy] += rng.uniform(-0.4, 0.4, noisy.sum()) * tau
    return r


@pytest.mark.parametrize("tau", [0.0, 1e-9])
@pytest.mark.parametrize("rule", [oracle.RULE_L0DEC, oracle.RULE_MODE])
def test_shifted_selection_is_the_literal_score_of_one_candidate(tau, rule):
    """Column selected at position t <=> r at its t-th row is nonzero and
    ||r||_0 - ||r - v_t a_j||_0 (formed over the whole vector) reaches a, or,
    for the frequency rule, v_t occurs at least a times in r_N(j)."""
    rng = np.random.default_rng(7)
    m, d, ncols = 60, 7, 400
    for trial in range(4):
        r = _planted(rng, m, tau)
        rows = np.concatenate([rng.choice(m, d, replace=False) for _ in range(ncols)]).astype(np.int32)
        for a in (2, 4):
            for t in range(d):
                sel, om = oracle.score_columns_shifted(rows, d, r, tau, a, t, rule=SHIFTED[rule])
                for c in range(ncols):
                    rc = rows[c * d:(c + 1) * d]
                    v = r[rc]
                    cand = v[t]
                    if not abs(cand) > tau:
                        assert not sel[c]
                        continue
                    if rule == oracle.RULE_L0DEC:
                        score = oracle.literal_decrease(rc, r, cand, tau)
                    else:
                        score = int(np.sum(np.abs(v - cand) <= tau))
                    assert bool(sel[c]) == (score >= a), (trial, a, t, c)
                    if sel[c]:
                        assert om[c] == cand


def test_shifted_selects_a_subset_of_the_full_vote():
    """Exact equality (tau = 0) and a > d/2: at most one value can qualify in
    a column, so whatever a shifted pass selects the full vote selects too,
    with the same omega."""
    rng = np.random.default_rng(11)
    m, d, ncols = 40, 7, 600
    for trial in range(5):
        r = _planted(rng, m, 0.0)
        rows = np.concatenate([rng.choice(m, d, replace=False) for _ in range(ncols)]).astype(np.int32)
        for rule in (oracle.RULE_L0DEC, oracle.RULE_MODE):
            fsel, fom, _ = oracle.score_columns(rows, d, r, 0.0, 4, rule=rule)
            for t in range(d):
                sel, om = oracle.score_columns_shifted(rows, d, r, 0.0, 4, t, rule=SHIFTED[rule])
                assert np.all(fsel[sel.astype(bool)]), (trial, rule, t)
                assert np.array_equal(om[sel.astype(bool)], fom[sel.astype(bool)])


def test_shifted_k0_and_disjoint_columns():
    inst = gen.make_instance(3, 500, 60, 5, 0)
    o = oracle.parallel_l0(inst.n, inst.m, inst.d, inst.col_idx, inst.y, 3, rule=oracle.RULE_SHIFTED_L0DEC)
    assert o["outcome"] == oracle.CONVERGED and o["iters"] == 0 and o["passes"] == 0
    # disjoint columns: every support column's rows all hold its value, so
    # position 0 already identifies every one of them
    n, d, k = 40, 4, 9
    col = np.arange(n * d, dtype=np.int32)
    rng = np.random.default_rng(5)
    x = np.zeros(n)
    x[rng.choice(n, k, replace=False)] = rng.standard_normal(k)
    y = np.repeat(x, d)
    o = oracle.parallel_l0(n, n * d, d, col, y, 3, rule=oracle.RULE_SHIFTED_L0DEC)
    assert o["trace"].tolist() == [k * d, 0] and o["iters"] == 1 and o["passes"] == 1
    assert np.array_equal(o["x"], x)


@pytest.mark.parametrize("seed", range(4))
def test_theorem_4_8_on_dissociated_signals(seed):
    """Dissociated small-rho instances: the shifted decoder recovers x, every
    update it applies is a true entry of x, and ||r||_0 never increases; it
    needs at least as many vote passes as the full vote needs iterations."""
    inst = gen.make_instance(900 + seed, 3000, 600, 7, 30)
    alpha = 4
    full = oracle.parallel_l0(inst.n, inst.m, inst.d, inst.col_idx, inst.y, alpha)
    o = oracle.parallel_l0(inst.n, inst.m, inst.d, inst.col_idx, inst.y, alpha,
                           rule=oracle.RULE_SHIFTED_L0DEC)
    assert o["outcome"] == oracle.CONVERGED and full["outcome"] == oracle.CONVERGED
    assert np.max(np.abs(o["x"] - inst.x)) <= 1e-12 * np.max(np.abs(inst.x))
    assert np.all(np.diff(o["trace"]) <= 0)
    assert o["passes"] >= full["iters"]
    # stepwise: every column updated so far is a true support column and holds
    # its value (read off a partly peeled residual, so up to rounding)
    scale = np.max(np.abs(inst.x))
    for it in range(1, o["iters"] + 1):
        part = oracle.parallel_l0(inst.n, inst.m, inst.d, inst.col_idx, inst.y, alpha, max_iter=it,
                                  rule=oracle.RULE_SHIFTED_L0DEC)
        nz = part["x"] != 0
        assert np.all(inst.x[nz] != 0), it
        assert np.max(np.abs(part["x"][nz] - inst.x[nz]), initial=0.0) <= 1e-12 * scale, it


def test_shifted_serial_is_rejected():
    inst = gen.make_instance(3, 200, 40, 5, 4)
    with pytest.raises(ValueError):
        oracle.serial_l0(inst.n, inst.m, inst.d, inst.col_idx, inst.y, 3, rule=oracle.RULE_SHIFTED_L0DEC)
