"""Seeded input generator: matrix model (Definition 2.2, footnote of Section
1.1), support/values (Section 5 preamble) and y = A x."""
import math

import numpy as np
import pytest

import gen
from oracle import brute


def test_columns_distinct_sorted_in_range():
    n, m, d = 3000, 97, 7
    col = gen.columns(11, n, m, d).reshape(n, d)
    assert col.min() >= 0 and col.max() < m
    assert np.all(np.diff(col, axis=1) > 0)  # strictly ascending => distinct


def test_columns_deterministic_and_seeded():
    a = gen.columns(5, 500, 50, 5)
    b = gen.columns(5, 500, 50, 5)
    c = gen.columns(6, 500, 50, 5)
    assert np.array_equal(a, b) and not np.array_equal(a, c)
    # a column's rows depend only on (seed, j): a longer draw extends a shorter one
    longer = gen.columns(5, 800, 50, 5)
    assert np.array_equal(longer[: a.size], a)


def test_columns_uniform_rows():
    # each row should be hit d*n/m times on average (uniform d-subsets)
    n, m, d = 200000, 64, 5
    col = gen.columns(3, n, m, d)
    counts = np.bincount(col, minlength=m)
    expect = n * d / m
    chi2 = float(np.sum((counts - expect) ** 2 / expect))
    # 63 degrees of freedom; 120 is far in the tail
    assert chi2 < 120, chi2


def test_columns_pair_frequency_uniform_subsets():
    # for m=6, d=3 every one of the C(6,3)=20 subsets should be about equally likely
    n = 60000
    col = gen.columns(9, n, 6, 3).reshape(n, 3)
    keys = col[:, 0] * 36 + col[:, 1] * 6 + col[:, 2]
    _, counts = np.unique(keys, return_counts=True)
    assert counts.size == 20
    assert np.all(np.abs(counts - n / 20) < 6 * math.sqrt(n / 20))


def test_support_and_values():
    s = gen.support(1, 1000, 100)
    assert s.size == 100 and np.all(np.diff(s) > 0) and s[0] >= 0 and s[-1] < 1000
    assert gen.support(1, 10, 10).tolist() == list(range(10))
    assert gen.support(1, 10, 0).size == 0
    v = gen.values(1, np.arange(20000), gen.VALUES_NORMAL)
    assert abs(v.mean()) < 0.05 and abs(v.std() - 1) < 0.05
    pm = gen.values(1, np.arange(2000), gen.VALUES_PM1)
    assert set(np.unique(pm).tolist()) == {-1.0, 1.0}


def test_measure_equals_dense_ascending_product():
    """y = A x from row lists equals the dense 0/1 product summed over all
    columns in ascending order (adding 0*x_j is exact), bitwise."""
    inst = gen.make_instance(21, 60, 20, 4, 12)
    A = brute.dense_matrix(inst.n, inst.m, inst.d, inst.col_idx)
    x = inst.x
    for i in range(inst.m):
        s = 0.0
        for j in range(inst.n):
            s = s + A[i, j] * x[j]
        assert s == inst.y[i] or (s == 0.0 and inst.y[i] == 0.0)


def test_normal_draws_are_dissociated_pm1_are_not():
    """Definition 1.1; continuous draws are dissociated with probability 1."""
    for seed in range(5):
        v = gen.values(seed, np.arange(16), gen.VALUES_NORMAL)
        assert brute.is_dissociated(v)
    assert not brute.is_dissociated(gen.values(0, np.arange(8), gen.VALUES_PM1))


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_bounded_frequency_lemma(seed):
    """Lemma 4.2: for dissociated x each nonzero value occurs in y = A x at
    most d times."""
    inst = gen.make_instance(seed, 5000, 400, 7, 80)
    y = inst.y[inst.y != 0.0]
    _, counts = np.unique(y, return_counts=True)
    assert counts.max() <= inst.d


def test_information_preserving_unique_neighbours():
    """Lemma 2.4 (information preservation): on generated instances most of the
    support's edges land on rows with exactly one support neighbour, and each
    such row carries that column's value."""
    inst = gen.make_instance(4, 20000, 2000, 7, 100)
    cols = inst.col_idx.reshape(inst.n, inst.d)
    deg = np.zeros(inst.m, dtype=np.int64)
    for j in inst.supp:
        deg[cols[j]] += 1
    n1 = 0
    for j, v in zip(inst.supp, inst.vals):
        for i in cols[j]:
            if deg[i] == 1:
                n1 += 1
                assert inst.y[i] == v
    # an edge is a unique-neighbour edge with probability (1 - d/m)^(k-1) in
    # this random model; |N1(S)| = (1 - 2 eps) d |S| then sits near that
    expect = inst.d * inst.k * (1 - inst.d / inst.m) ** (inst.k - 1)
    assert abs(n1 - expect) < 0.1 * expect


def test_workload_shapes():
    assert gen.SINGLE["small"] == (4096, 512, 7, 50)
    assert gen.SINGLE["n2^20"] == (1 << 20, 104858, 7, 20971)
    assert gen.SINGLE["n2^24"] == (1 << 24, 16777, 7, 4194)
    p = gen.sweep_params(4096)
    assert len(p) == 4096
    ns = np.array([q["n"] for q in p])
    assert ns.min() >= 1024 and ns.max() <= 1 << 18
    assert all(q["m"] >= q["d"] for q in p)
    assert {q["d"] for q in p} == {5, 7, 9}
    s = gen.serve_params(2000)
    assert all(q["k"] == math.floor(0.15 * q["m"] + 1e-9) for q in s)


def test_weights_and_scaled_measure():
    w = gen.weights(3, 5000)
    assert w.min() >= 0.5 and w.max() <= 1.5 and abs(w.mean() - 1.0) < 0.02
    assert np.array_equal(w, gen.weights(3, 5000)) and not np.array_equal(w, gen.weights(4, 5000))
    assert np.array_equal(gen.weights(3, 7000)[:5000], w)  # per-column streams
    n, m, d = 200, 40, 5
    col = gen.columns(1, n, m, d)
    supp = gen.support(1, n, 12)
    vals = gen.values(1, supp)
    w = gen.weights(1, n)
    y = gen.measure(n, m, d, col, supp, vals, w)
    A = brute.dense_matrix(n, m, d, col) * w[None, :]
    x = np.zeros(n)
    x[supp] = vals
    assert np.max(np.abs(y - A @ x)) <= 1e-14
    assert np.array_equal(gen.measure(n, m, d, col, supp, vals, np.ones(n)), gen.measure(n, m, d, col, supp, vals))


@pytest.mark.parametrize("band", [0.0, 0.3, 0.9, 1.0])
def test_banded_values(band):
    supp = gen.support(9, 100000, 2000)
    v = gen.banded_values(9, supp, band)
    _, counts = np.unique(v, return_counts=True)
    kb = int(round(band * supp.size))
    assert counts.max() == max(kb, 1)
    if band == 0.0:
        assert np.array_equal(v, gen.values(9, supp))
    assert np.array_equal(v, gen.banded_values(9, supp, band))
