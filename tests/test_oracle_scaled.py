"""Pins of the oracle's column-scaled mode (Section 4.3.3: scaling each column
of A by an i.i.d. continuous draw makes non-dissociated signals, such as +-1
values, identifiable) against what the definitions fix: the unit-weight
special case, an exact metamorphic relation for power-of-two weights, the
literal l0-decrease of eq. (selection_l0) with a scaled a_j, a dense scaled
product for the residual, and the recovery the section describes.  The
hand-derived decodes WC0 (unit columns, stalls) and WC1 (scaled, recovers)
are checked by test_oracle.test_worked_decodes."""
import math

import numpy as np
import pytest

import gen
import oracle
from oracle import brute

ALL_RULES = [oracle.RULE_L0DEC, oracle.RULE_MODE, oracle.RULE_SHIFTED_L0DEC, oracle.RULE_SHIFTED_MODE]


def _decode(inst, y, rule, w, **kw):
    return oracle.parallel_l0(inst.n, inst.m, inst.d, inst.col_idx, y, inst.alpha, rule=rule, w=w, **kw)


def _same(a, b):
    assert a["outcome"] == b["outcome"] and a["iters"] == b["iters"] and a["passes"] == b["passes"]
    assert np.array_equal(a["trace"], b["trace"]) and np.array_equal(a["tsize"], b["tsize"])


@pytest.mark.parametrize("rule", ALL_RULES)
def test_unit_weights_are_the_unscaled_decoder(rule):
    """w = 1 divides and multiplies by one: bit for bit the unit-column run,
    converging or not."""
    for seed, kind, k in ((1, gen.VALUES_NORMAL, 50), (2, gen.VALUES_PM1, 60), (3, gen.VALUES_NORMAL, 200)):
        inst = gen.make_instance(seed, 4096, 512, 7, k, kind=kind)
        a = _decode(inst, inst.y, rule, None)
        b = _decode(inst, inst.y, rule, np.ones(inst.n))
        _same(a, b)
        assert np.array_equal(a["x"], b["x"])


@pytest.mark.parametrize("rule", ALL_RULES)
def test_power_of_two_weights_decode_the_weighted_signal(rule):
    """With w_j = 2^e_j every product and quotient is exact, so decoding
    y = A_w x with the weights and decoding the same y on unit columns (where
    it measures z = w x) take the same steps: x_hat_w * w == x_hat_unit bit for
    bit, with the same trace.  A weight dropped from the residual, or an
    update multiplied instead of divided, breaks it."""
    rng = np.random.default_rng(31)
    for seed, kind in ((410, gen.VALUES_NORMAL), (411, gen.VALUES_PM1), (412, gen.VALUES_NORMAL)):
        inst = gen.make_instance(seed, 3000, 600, 7, 60, kind=kind)
        w = np.ldexp(1.0, rng.integers(-4, 5, inst.n))
        y = gen.measure(inst.n, inst.m, inst.d, inst.col_idx, inst.supp, inst.vals, w)
        s = _decode(inst, y, rule, w)
        u = _decode(inst, y, rule, None)
        _same(s, u)
        assert np.array_equal(s["x"] * w, u["x"])
        assert s["iters"] > 0


@pytest.mark.parametrize("rule", [oracle.RULE_L0DEC, oracle.RULE_MODE])
def test_scaled_selection_is_the_literal_decrease(rule):
    """One vote step on a scaled A against eq. (selection_l0) written out: for
    each column j and each nonzero r_t on N(j), omega = r_t / w_j, and the
    decrease ||r||_0 - ||r - omega a_j||_0 is formed over the whole vector
    with a_j = w_j on N(j) (each entry r_u - fl(omega w_j)).  The column is
    selected iff the best decrease reaches a, and its update is the smallest
    best-scoring omega."""
    inst = gen.make_instance(77, 2000, 400, 7, 40, kind=gen.VALUES_PM1, scaled=True)
    w, r = inst.w, inst.y
    tol = 1e-10
    tau = oracle.zero_threshold(r, tol)
    a = math.ceil(inst.alpha)
    one = _decode(inst, r, rule, w, max_iter=1, tol=tol)
    selected = 0
    for j in range(inst.n):
        rows = inst.col_idx[j * inst.d:(j + 1) * inst.d]
        best, best_om = None, None
        for t in range(inst.d):
            rt = r[rows[t]]
            if not abs(rt) > tau:
                continue
            om = rt / w[j]
            if rule == oracle.RULE_L0DEC:
                score = oracle.literal_decrease(rows, r, om * w[j], tau)
            else:
                score = int(np.sum(np.abs(r[rows] - om * w[j]) <= tau))
            if best is None or score > best or (score == best and om < best_om):
                best, best_om = score, om
        if best is not None and best >= a:
            selected += 1
            assert one["x"][j] == best_om, j
        else:
            assert one["x"][j] == 0.0, j
    assert selected == one["tsize"][0] > 0


def test_scaled_residual_against_a_dense_product():
    """r = y - A_w x: with dyadic weights and integer x every sum is exact and
    equals the dense product; with continuous weights it agrees with the
    dense product to rounding."""
    n, m, d = 300, 80, 5
    col = gen.columns(5, n, m, d)
    dense = brute.dense_matrix(n, m, d, col)
    rng = np.random.default_rng(3)
    y = rng.standard_normal(m)
    x = np.zeros(n)
    nz = rng.choice(n, 40, replace=False)
    x[nz] = rng.integers(-3, 4, 40)
    w = np.ldexp(1.0, rng.integers(-3, 4, n))
    yd = np.round(y * 64) / 64
    assert np.array_equal(oracle.residual(n, m, d, col, yd, x, w), yd - (dense * w[None, :]) @ x)
    w = gen.weights(9, n)
    x[nz] = rng.standard_normal(40)
    r = oracle.residual(n, m, d, col, y, x, w)
    ref = y - (dense * w[None, :]) @ x
    assert np.max(np.abs(r - ref)) <= 1e-13 * (1 + np.max(np.abs(ref)))
    # and it is not the unit-column residual
    assert not np.allclose(r, oracle.residual(n, m, d, col, y, x))


@pytest.mark.parametrize("seed", range(4))
def test_pm1_signals_recovered_only_with_scaled_columns(seed):
    """Section 4.3.3: +-1 nonzeros are not dissociated, and on unit columns
    the decoder stops short of x; with columns scaled by weights uniform on
    [1/2, 3/2] it recovers x, every update so far being a true entry of x and
    ||r||_0 never increasing."""
    unit = gen.make_instance(700 + seed, 3000, 600, 7, 60, kind=gen.VALUES_PM1)
    u = _decode(unit, unit.y, oracle.RULE_L0DEC, None)
    assert u["outcome"] != oracle.CONVERGED
    inst = gen.make_instance(700 + seed, 3000, 600, 7, 60, kind=gen.VALUES_PM1, scaled=True)
    assert np.array_equal(inst.supp, unit.supp) and np.array_equal(inst.vals, unit.vals)
    s = _decode(inst, inst.y, oracle.RULE_L0DEC, inst.w)
    assert s["outcome"] == oracle.CONVERGED
    assert np.max(np.abs(s["x"] - inst.x)) <= 1e-12
    assert np.all(np.diff(s["trace"]) <= 0)
    for it in range(1, s["iters"] + 1):
        part = _decode(inst, inst.y, oracle.RULE_L0DEC, inst.w, max_iter=it)
        nz = part["x"] != 0
        assert np.all(inst.x[nz] != 0), it
        assert np.max(np.abs(part["x"][nz] - inst.x[nz]), initial=0.0) <= 1e-12, it


def test_scaled_shifted_recovers_pm1():
    inst = gen.make_instance(720, 3000, 600, 7, 60, kind=gen.VALUES_PM1, scaled=True)
    s = _decode(inst, inst.y, oracle.RULE_SHIFTED_L0DEC, inst.w)
    assert s["outcome"] == oracle.CONVERGED
    assert np.max(np.abs(s["x"] - inst.x)) <= 1e-12
    assert s["passes"] >= s["iters"]


@pytest.mark.parametrize("bad", [0.0, -1.0, np.nan, np.inf])
def test_invalid_weights_are_rejected(bad):
    inst = gen.make_instance(3, 200, 40, 5, 4, scaled=True)
    w = inst.w.copy()
    w[17] = bad
    with pytest.raises(ValueError):
        _decode(inst, inst.y, oracle.RULE_L0DEC, w)
    with pytest.raises(ValueError):
        _decode(inst, inst.y, oracle.RULE_L0DEC, inst.w[:-1])
