"""Pins of the CPU oracle against things other than itself: hand-derived
worked cases (tests/golden/), closed forms, brute force over supports on
tiny systems, the paper's lemmas and theorems as invariants, and metamorphic
relations.  All of these run on the CPU."""
import math

import numpy as np
import pytest

import gen
import oracle
from golden_io import decode_cases, graph_arrays, load, num
from oracle import brute

RULES = {"L0DEC": oracle.RULE_L0DEC, "MODE": oracle.RULE_MODE, "SHIFTED_L0DEC": oracle.RULE_SHIFTED_L0DEC,
         "SHIFTED_MODE": oracle.RULE_SHIFTED_MODE}
OUT = {"CONVERGED": oracle.CONVERGED, "STALLED": oracle.STALLED, "MAX_ITER": oracle.MAX_ITER}


# --------------------------------------------------------------------------
# worked cases (hand-derived from Algorithms 1-2 and eq. (selection_l0))
# --------------------------------------------------------------------------

def test_scorer_cases():
    fx = load("scorer.json")
    for c in fx["cases"]:
        v = np.array([num(e) for e in c["v"]])
        d = v.size
        rows = np.arange(d, dtype=np.int32)
        sel, omega, best = oracle.score_columns(rows, d, v, num(c["tau"]), c["a"])
        assert bool(sel[0]) == c["selected"], c
        assert best[0] == c["best"], c
        if c["selected"]:
            assert omega[0] == num(c["omega"]), c


@pytest.mark.parametrize("case", decode_cases(), ids=lambda c: f"{c[0]}-{c[4]['algo']}-{c[4]['rule']}-a{c[4]['alpha']}")
def test_worked_decodes(case):
    name, g, y, x, c = case
    n, m, d, col = graph_arrays(g)
    w = np.array(g["w"], float) if "w" in g else None
    # the fixture's y is the measurement of its x (column-scaled when w is given)
    dense = brute.dense_matrix(n, m, d, col)
    if w is not None:
        dense = dense * w[None, :]
    assert np.array_equal(dense @ x, y)
    assert c.get("weights", False) == (w is not None)
    if c["algo"] == "parallel":
        res = oracle.parallel_l0(n, m, d, col, y, c["alpha"], max_iter=c["max_iter"], tol=c["tol"],
                                 rule=RULES[c["rule"]], w=w)
        assert res["trace"].tolist() == c["trace"]
        assert res["tsize"].tolist() == c["tsize"]
        assert res["iters"] == c["iters"]
        if "passes" in c:
            assert res["passes"] == c["passes"]
    else:
        res = oracle.serial_l0(n, m, d, col, y, c["alpha"], max_sweeps=c["max_iter"], tol=c["tol"],
                               rule=RULES[c["rule"]])
        assert res["updates"] == c["updates"] and res["sweeps"] == c["sweeps"]
    assert res["outcome"] == OUT[c["outcome"]]
    assert np.array_equal(res["x"], np.array(c["x_hat"], float))


# --------------------------------------------------------------------------
# the score: closed form c - z, literal decrease, candidate restriction
# --------------------------------------------------------------------------

def _planted_residual(rng, m, tau):
    """A residual with exact zeros, noise-level zeros, and clusters of equal
    values (some perturbed inside tau) so that columns see repeated values."""
    base = rng.standard_normal(8)
    r = base[rng.integers(0, 8, m)].copy()
    noisy = rng.random(m) < 0.3
    r[noisy] += rng.uniform(-0.4, 0.4, noisy.sum()) * tau
    r[rng.random(m) < 0.2] = 0.0
    tiny = rng.random(m) < 0.05
    r[tiny] = rng.uniform(-0.9, 0.9, tiny.sum()) * tau
    return r


@pytest.mark.parametrize("tau", [0.0, 1e-10, 1e-3])
@pytest.mark.parametrize("rule", [oracle.RULE_L0DEC, oracle.RULE_MODE])
def test_score_equals_count_closed_form(tau, rule):
    """Under the threshold reading, ||r||_0 - ||r - v_t a_j||_0 restricted to
    N(j) equals c_t - z, with c_t the number of entries within tau of v_t and z
    the number of zeros; MODE scores c_t.  Best over nonzero candidates,
    smallest value on ties."""
    rng = np.random.default_rng(7)
    m, d = 40, 7
    r = _planted_residual(rng, m, tau if tau > 0 else 1e-12)
    rows = np.concatenate([np.sort(rng.choice(m, d, replace=False)) for _ in range(400)]).astype(np.int32)
    a = 3
    sel, omega, best = oracle.score_columns(rows, d, r, tau, a, rule)
    for c in range(400):
        v = r[rows[c * d:(c + 1) * d]]
        nzmask = np.abs(v) > tau
        z = int(d - nzmask.sum())
        cand = []
        for t in np.nonzero(nzmask)[0]:
            ct = int(np.sum(~(np.abs(v - v[t]) > tau)))
            cand.append((ct - z if rule == oracle.RULE_L0DEC else ct, v[t]))
        if not cand:
            assert not sel[c]
            continue
        top = max(s for s, _ in cand)
        w = min(val for s, val in cand if s == top)
        assert best[c] == top
        assert bool(sel[c]) == (top >= a)
        if top >= a:
            assert omega[c] == w


def test_score_matches_literal_full_vector_decrease():
    """eq. (selection_l0) computed on the whole m-vector (numpy, independent of
    the oracle's per-column loop) agrees with the oracle's best score, and no
    real omega outside the candidates does better when tau = 0."""
    rng = np.random.default_rng(3)
    m, d = 30, 5
    r = _planted_residual(rng, m, 1e-12)
    r[np.abs(r) < 1e-9] = 0.0  # exact zeros only: tau = 0 regime
    for _ in range(300):
        rows = np.sort(rng.choice(m, d, replace=False)).astype(np.int32)
        def dec(w):
            q = r.copy()
            q[rows] = r[rows] - w
            return int(np.count_nonzero(r)) - int(np.count_nonzero(q))
        cands = [r[i] for i in rows if r[i] != 0.0]
        sel, omega, best = oracle.score_columns(rows, d, r, 0.0, 2)
        if not cands:
            continue
        lit = max(dec(w) for w in cands)
        assert best[0] == lit
        # also matches the oracle's own literal routine
        assert oracle.literal_decrease(rows, r, omega[0] if sel[0] else cands[0], 0.0) <= lit
        for w in rng.standard_normal(20):  # non-candidate omegas never beat the best
            assert dec(w) <= max(lit, 0)


# --------------------------------------------------------------------------
# closed forms
# --------------------------------------------------------------------------

def test_k0_converges_immediately():
    inst = gen.make_instance(1, 2000, 200, 7, 0)
    res = oracle.parallel_l0(inst.n, inst.m, inst.d, inst.col_idx, inst.y, 4)
    assert res["iters"] == 0 and res["outcome"] == oracle.CONVERGED
    assert res["trace"].tolist() == [0] and not np.any(res["x"])


@pytest.mark.parametrize("seed", range(6))
def test_k1_recovers_in_one_iteration(seed):
    """One nonzero: y has d copies of x_j; column j decreases ||r||_0 by d and
    no other column can reach ceil(alpha) unless it shares >= (a+d)/2 rows."""
    n, m, d = 3000, 300, 7
    inst = gen.make_instance(100 + seed, n, m, d, 1)
    cols = inst.col_idx.reshape(n, d)
    j = int(inst.supp[0])
    overlap = np.array([len(np.intersect1d(cols[q], cols[j])) for q in range(n)])
    overlap[j] = 0
    a = 4
    assert overlap.max() < a  # no competitor can collect a copies
    res = oracle.parallel_l0(n, m, d, inst.col_idx, inst.y, a)
    assert res["trace"].tolist() == [d, 0] and res["iters"] == 1
    assert np.array_equal(res["x"], inst.x)


def test_disjoint_columns_one_iteration():
    """N(j) = {jd, ..., jd+d-1}: every row holds at most one column, so one
    iteration recovers x exactly: trace [k d, 0]."""
    n, d, k = 50, 5, 9
    m = n * d
    col = np.arange(n * d, dtype=np.int32)
    supp = gen.support(8, n, k)
    vals = gen.values(8, supp)
    y = gen.measure(n, m, d, col, supp, vals)
    res = oracle.parallel_l0(n, m, d, col, y, 3)
    x = np.zeros(n)
    x[supp] = vals
    assert res["trace"].tolist() == [k * d, 0] and res["iters"] == 1
    assert np.array_equal(res["x"], x)


# --------------------------------------------------------------------------
# brute force over supports (n <= 20)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(12))
def test_converged_output_is_sparsest_solution(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(10, 17))
    m = int(rng.integers(8, 13))
    d = 3
    k = int(rng.integers(1, 4))
    inst = gen.make_instance(500 + seed, n, m, d, k)
    A = brute.dense_matrix(n, m, d, inst.col_idx)
    size, sols = brute.sparsest_solutions(A, inst.y, max_size=k)
    for rule in (oracle.RULE_L0DEC, oracle.RULE_MODE):
        res = oracle.parallel_l0(n, m, d, inst.col_idx, inst.y, 2, tol=1e-10, rule=rule)
        if res["outcome"] == oracle.CONVERGED:
            assert size is not None and size <= k
            assert any(np.max(np.abs(res["x"] - s)) <= 1e-12 * max(1, np.max(np.abs(s))) for s in sols)
            # a false update later undone can leave rounding noise behind
            scale = max(1.0, float(np.max(np.abs(inst.y))))
            assert np.count_nonzero(np.abs(res["x"]) > 1e-12 * scale) == size
    if size == k and len(sols) == 1:
        assert np.max(np.abs(sols[0] - inst.x)) < 1e-9


# --------------------------------------------------------------------------
# invariants from the paper's lemmas and theorems
# --------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(4))
def test_updates_are_true_values_and_trace_decreases(seed):
    """Lemma 4.5 / Theorem 4.6: with a dissociated x in the theorem's regime
    (alpha > d/2, few nonzeros) each applied update is x_j at a true index,
    so x_hat's support stays inside x's and ||r||_0 never increases."""
    n, m, d = 20000, 2000, 7
    inst = gen.make_instance(900 + seed, n, m, d, 60)
    x = inst.x
    full = oracle.parallel_l0(n, m, d, inst.col_idx, inst.y, 4)
    assert full["outcome"] == oracle.CONVERGED
    assert np.all(np.diff(full["trace"]) <= 0)
    for it in range(1, full["iters"] + 1):
        part = oracle.parallel_l0(n, m, d, inst.col_idx, inst.y, 4, max_iter=it)
        xh = part["x"]
        on = np.nonzero(xh)[0]
        assert set(on.tolist()) <= set(inst.supp.tolist())
        assert np.max(np.abs(xh[on] - x[on]) / np.abs(x[on])) <= 1e-12
    assert np.max(np.abs(full["x"] - x)) / np.max(np.abs(x)) <= 1e-12


@pytest.mark.parametrize("rho", [0.05, 0.075, 0.1])
def test_iterations_bounded_by_log_k(rho):
    """Theorem 4.6: |S_{l+1}| <= 2 eps d / (1 + floor(2 eps d)) |S_l|; with
    alpha = (1 - 2 eps) d = 4, d = 7 the factor is 3/4, so convergence takes at
    most log k / log(4/3) + 1 iterations (Section 5 observes <= log k)."""
    n = 1 << 15
    m = gen.mk_m(n, 0.1)
    k = gen.mk_k(m, rho)
    inst = gen.make_instance(77, n, m, 7, k)
    res = oracle.parallel_l0(n, m, 7, inst.col_idx, inst.y, 4)
    assert res["outcome"] == oracle.CONVERGED
    assert res["iters"] <= math.log(k) / math.log(4 / 3) + 1
    assert res["iters"] <= math.log(k) + 1


def test_serial_and_parallel_agree():
    inst = gen.single_workload("small")
    par = oracle.parallel_l0(inst.n, inst.m, inst.d, inst.col_idx, inst.y, inst.alpha)
    ser = oracle.serial_l0(inst.n, inst.m, inst.d, inst.col_idx, inst.y, inst.alpha)
    assert par["outcome"] == ser["outcome"] == oracle.CONVERGED
    scale = np.max(np.abs(inst.vals))
    assert np.max(np.abs(par["x"] - inst.x)) <= 1e-12 * scale
    assert np.max(np.abs(ser["x"] - inst.x)) <= 1e-12 * scale
    # Serial-l0 needs at most as many sweeps as Parallel-l0 needs iterations
    assert ser["sweeps"] <= par["iters"] + 1


def test_mode_rule_false_updates_grow_residual():
    """Section 3.5.3 (the mode does not minimise ||r||_0): zeros in r_N(j) matter.  On W1 the frequency score adds
    wrong values and raises ||r||_0 where the l0-decrease does not."""
    fx = load("W1.json")
    n, m, d, col = graph_arrays(fx["graph"])
    y = np.array(fx["y"], float)
    l0 = oracle.parallel_l0(n, m, d, col, y, 2, max_iter=6, tol=0)
    md = oracle.parallel_l0(n, m, d, col, y, 2, max_iter=6, tol=0, rule=oracle.RULE_MODE)
    assert np.all(np.diff(l0["trace"]) <= 0)
    assert np.any(np.diff(md["trace"]) > 0)


# --------------------------------------------------------------------------
# metamorphic relations and resume
# --------------------------------------------------------------------------

def _run(n, m, d, col, y, **kw):
    return oracle.parallel_l0(n, m, d, col, y, 4, **kw)


def test_row_relabel_and_column_reorder_bitwise():
    inst = gen.make_instance(31, 6000, 600, 7, 90)
    n, m, d = inst.n, inst.m, inst.d
    base = _run(n, m, d, inst.col_idx, inst.y)
    perm = np.random.default_rng(1).permutation(m).astype(np.int32)
    col2 = perm[inst.col_idx]
    y2 = np.empty(m)
    y2[perm] = inst.y
    rel = _run(n, m, d, col2, y2)
    assert np.array_equal(rel["x"], base["x"]) and rel["trace"].tolist() == base["trace"].tolist()
    shuf = inst.col_idx.reshape(n, d)[:, ::-1].copy().reshape(-1)
    re2 = _run(n, m, d, shuf, inst.y)
    assert np.array_equal(re2["x"], base["x"]) and re2["iters"] == base["iters"]


@pytest.mark.parametrize("e", [-40, -3, 5, 40])
def test_power_of_two_scaling_bitwise(e):
    inst = gen.make_instance(32, 6000, 600, 7, 90)
    base = _run(inst.n, inst.m, inst.d, inst.col_idx, inst.y)
    sc = _run(inst.n, inst.m, inst.d, inst.col_idx, inst.y * 2.0 ** e)
    assert np.array_equal(sc["x"], base["x"] * 2.0 ** e)
    assert sc["trace"].tolist() == base["trace"].tolist()


def test_resume_is_bitwise():
    inst = gen.make_instance(33, 8000, 800, 7, 100)
    full = _run(inst.n, inst.m, inst.d, inst.col_idx, inst.y, max_iter=20)
    assert full["iters"] >= 5
    K = 3
    first = _run(inst.n, inst.m, inst.d, inst.col_idx, inst.y, max_iter=K)
    rest = _run(inst.n, inst.m, inst.d, inst.col_idx, inst.y, max_iter=20 - K, x_init=first["x"])
    assert np.array_equal(rest["x"], full["x"])
    assert rest["trace"].tolist() == full["trace"][K:].tolist()
    assert first["iters"] + rest["iters"] == full["iters"]


def test_argument_checks():
    inst = gen.make_instance(1, 100, 20, 3, 2)
    for alpha in (1.0, 0.5, 3.5):
        with pytest.raises(ValueError):
            oracle.parallel_l0(inst.n, inst.m, inst.d, inst.col_idx, inst.y, alpha)
    bad = inst.col_idx.copy()
    bad[5] = inst.m
    with pytest.raises(ValueError):
        oracle.parallel_l0(inst.n, inst.m, inst.d, bad, inst.y, 2)
    with pytest.raises(ValueError):
        oracle.parallel_l0(inst.n, inst.m, inst.d, inst.col_idx, inst.y, 2, tol=-1.0)


# --------------------------------------------------------------------------
# input of the decoders: A is binary with d distinct rows per column
# --------------------------------------------------------------------------

def test_repeated_row_in_a_column_is_rejected():
    """Definition 2.2: A is the binary adjacency matrix of a left d-regular
    graph, exactly d ones per column, so a column listing one row twice is no
    such matrix.  The case of rows (0, 0, 1) with r = (2, 5) shows why it
    cannot be decoded as if it were one: counted as two unit entries, omega = 2
    zeroes both copies (decrease 2 >= alpha = 2 at tau = 0); read as an entry
    A_00 = 2, the decrease of omega = 2 is 0.  The oracle refuses it, both
    decoders, whatever position the copy is in."""
    y = np.array([2.0, 5.0, 0.0, 0.0])
    good = np.array([0, 2, 1, 1, 2, 3], dtype=np.int32)
    oracle.parallel_l0(2, 4, 3, good, y, 2, tol=0.0)   # a valid graph runs
    oracle.serial_l0(2, 4, 3, good, y, 2, tol=0.0)
    for bad in ([0, 0, 1, 1, 2, 3], [0, 1, 0, 1, 2, 3], [0, 2, 1, 3, 2, 3], [0, 2, 1, 1, 3, 3]):
        col = np.array(bad, dtype=np.int32)
        with pytest.raises(ValueError):
            oracle.parallel_l0(2, 4, 3, col, y, 2, tol=0.0)
        with pytest.raises(ValueError):
            oracle.serial_l0(2, 4, 3, col, y, 2, tol=0.0)
    # the last column of a generated instance, and every rule
    inst = gen.make_instance(2, 300, 40, 5, 4)
    col = inst.col_idx.copy()
    col[-1] = col[-3]
    for rule in RULES.values():
        with pytest.raises(ValueError):
            oracle.parallel_l0(inst.n, inst.m, inst.d, col, inst.y, 2, rule=rule)


def test_absolute_tolerance_is_tau_itself():
    """In the absolute mode tau = tol: a run at tol = fl(t * max|y|) makes
    the same zero/equality decisions as the relative run at t (the same
    double tau), bit for bit; and tol >= max|y| makes every entry of y zero,
    so the run converges at once with x_hat = 0."""
    inst = gen.make_instance(5, 20000, 2000, 7, 120)
    s = float(np.max(np.abs(inst.y)))
    for t in (1e-10, 1e-3, 0.0):
        rel = oracle.parallel_l0(inst.n, inst.m, inst.d, inst.col_idx, inst.y, 4, tol=t)
        ab = oracle.parallel_l0(inst.n, inst.m, inst.d, inst.col_idx, inst.y, 4, tol=t * s,
                                tol_mode=oracle.TOL_ABSOLUTE)
        assert ab["outcome"] == rel["outcome"] and ab["trace"].tolist() == rel["trace"].tolist()
        assert np.array_equal(ab["x"].view(np.int64), rel["x"].view(np.int64))
    top = oracle.parallel_l0(inst.n, inst.m, inst.d, inst.col_idx, inst.y, 4, tol=s,
                             tol_mode=oracle.TOL_ABSOLUTE)
    assert top["outcome"] == oracle.CONVERGED and top["iters"] == 0 and top["trace"].tolist() == [0]
    assert not np.any(top["x"])
    # just below max|y|: the largest entry stays nonzero
    below = oracle.parallel_l0(inst.n, inst.m, inst.d, inst.col_idx, inst.y, 4,
                               tol=np.nextafter(s, 0.0), tol_mode=oracle.TOL_ABSOLUTE)
    assert below["trace"][0] == int(np.sum(np.abs(inst.y) == s))
