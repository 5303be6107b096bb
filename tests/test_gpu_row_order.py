"""A's columns as the caller lists them: rows in any order, each row once.

Definition 2.2 makes A binary with exactly d ones per column, so a column
that lists a row twice is invalid input: the oracle refuses it and every GPU
path (one-shot decode, prepared matrix, batched decoder, server) ends that
solve with L0_DEV_REPEATED_ROW and leaves x_hat zero.  The order of a
column's rows is the caller's: the ordinary rules do not depend on it (their
score and tie-break look at values only), the shifted rules of Algorithm 3
try the rows in col_idx order.  Every rule is run on per-column permuted
rows, alone and batched, against the oracle on the same permuted input."""
import numpy as np
import pytest
import torch

import gen
import oracle
import paper_1508_01256_amd as l0
from parity import assert_batched_parity, assert_parity, batched_run, gpu_run, oracle_run, run_both, say, to_dev

pytestmark = pytest.mark.gpu

RULES = [l0.L0_RULE_L0DEC, l0.L0_RULE_MODE, l0.L0_RULE_SHIFTED_L0DEC, l0.L0_RULE_SHIFTED_MODE]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    l0.lib()


def _with_repeat(inst, j, t, u):
    """col_idx of inst with column j's row t replaced by its row u."""
    col = inst.col_idx.copy()
    col[j * inst.d + t] = col[j * inst.d + u]
    return col


@pytest.mark.parametrize("n,m,d", [(5000, 500, 7), (70000, 40000, 5), (3000, 60, 20), (257, 60, 4)])
def test_repeated_row_rejected_alone(n, m, d):
    """One-shot decode, l0_decode and a prepared matrix, for 16-bit and
    32-bit row stores, a repeat at the first, a middle and the last column."""
    inst = gen.make_instance(31 + n, n, m, d, max(1, n // 100))
    for j, t, u in ((0, 1, 0), (n // 2, d - 1, 1), (n - 1, d - 1, d - 2)):
        col = _with_repeat(inst, j, t, u)
        say("repeated row", n, m, d, j, t, u)
        with pytest.raises(ValueError):
            oracle_run(n, m, d, col, inst.y, inst.alpha)
        for rule in (l0.L0_RULE_L0DEC, l0.L0_RULE_SHIFTED_L0DEC):
            g = gpu_run(n, m, d, col, inst.y, inst.alpha, rule=rule)
            assert g["outcome"] == l0.L0_DEV_REPEATED_ROW, (j, t, u, g["outcome"])
            assert not np.any(g["x"])
        colt = to_dev(col, torch.int32)
        y = to_dev(inst.y, torch.float64)
        x = torch.empty(n, dtype=torch.float64, device="cuda")
        it = torch.zeros(1, dtype=torch.int32, device="cuda")
        assert l0.l0_decode(colt, n, m, d, y, inst.alpha, 100, 1e-10, x, it) == l0.L0_OK
        torch.cuda.synchronize()
        assert int(it.item()) == -l0.L0_DEV_REPEATED_ROW and not torch.any(x)
        with l0.Matrix(colt, n, m, d) as A:
            r = A.solve(y, inst.alpha)
            assert r["outcome"] == l0.L0_DEV_REPEATED_ROW
    # an out-of-range index takes precedence over a repeat elsewhere
    col = _with_repeat(inst, 1, 1, 0)
    col[5 * d] = m
    assert gpu_run(n, m, d, col, inst.y, inst.alpha)["outcome"] == l0.L0_DEV_BAD_INDEX


def test_repeated_row_rejected_batched_and_served():
    """A repeat fails only its own instance of a batch (also inside a team of
    several workgroups) and its own server request."""
    insts = [gen.make_instance(900 + q, n, m, d, k) for q, (n, m, d, k) in enumerate(
        [(3000, 300, 7, 20), (40000, 4000, 5, 300), (300000, 30000, 7, 2000), (2000, 200, 9, 10),
         (5000, 500, 3, 30)])]
    arrs = [(i.n, i.m, i.d, i.col_idx, i.y, i.alpha) for i in insts]
    bad = {1: _with_repeat(insts[1], 17, 4, 2), 2: _with_repeat(insts[2], insts[2].n - 1, 6, 0)}
    for q, col in bad.items():
        i = insts[q]
        arrs[q] = (i.n, i.m, i.d, col, i.y, i.alpha)
    res = batched_run(arrs)
    for q, i in enumerate(insts):
        if q in bad:
            assert res[q]["outcome"] == l0.L0_DEV_REPEATED_ROW, (q, res[q])
            assert not np.any(res[q]["x"])
        else:
            o = oracle_run(i.n, i.m, i.d, i.col_idx, i.y, i.alpha)
            assert_batched_parity(res[q], o, label=f"batch/{q}")
    # the large instance again, alone in its batch (a team of workgroups)
    res = batched_run([arrs[2]])
    assert res[0]["outcome"] == l0.L0_DEV_REPEATED_ROW
    # server: the bad requests complete with the outcome, the rest decode
    dev = "cuda"
    with l0.Server(1 << 30) as srv:
        xs = []
        for q, (n, m, d, col, y, a) in enumerate(arrs):
            x = torch.empty(n, dtype=torch.float64, device=dev)
            xs.append(x)
            assert srv.submit(q, to_dev(col, torch.int32), to_dev(y, torch.float64), n, m, d, x, a) == l0.L0_OK
        done = {c["id"]: c for c in srv.drain()}
    for q in range(len(arrs)):
        assert done[q]["status"] == l0.L0_OK
        if q in bad:
            assert done[q]["outcome"] == l0.L0_DEV_REPEATED_ROW
        else:
            assert done[q]["outcome"] == res_outcome(insts[q])


def res_outcome(i):
    return oracle_run(i.n, i.m, i.d, i.col_idx, i.y, i.alpha)["outcome"]


@pytest.mark.parametrize("rule", RULES)
@pytest.mark.parametrize("n,m,d,k", [
    (4096, 512, 7, 50),        # the small workload's shape
    (100003, 10007, 7, 700),   # 16-bit rows, ragged tail
    (400000, 40000, 5, 3000),  # 32-bit rows, words from L2
    (20000, 4000, 20, 60),     # largest d
])
def test_permuted_rows_alone(rule, n, m, d, k):
    inst = gen.make_instance(4100 + n + d, n, m, d, k)
    col = gen.permute_rows(inst.col_idx, d, 77 + n)
    assert not np.array_equal(col, inst.col_idx)
    for alpha in ((2.0, inst.alpha) if rule >= l0.L0_RULE_SHIFTED_L0DEC else (inst.alpha,)):
        say("permuted rows", rule, n, m, d, k, alpha)
        g, o = run_both((n, m, d, col, inst.y, alpha), rule=rule)
        assert_parity(g, o, label=f"perm {rule} {n}/{m}/{d} a{alpha}")
        if rule in (l0.L0_RULE_L0DEC, l0.L0_RULE_MODE):
            # order-free rules: bitwise the run on ascending rows
            s = gpu_run(n, m, d, inst.col_idx, inst.y, alpha, rule=rule)
            assert np.array_equal(s["x"].view(np.int64), g["x"].view(np.int64))
            assert s["trace"].tolist() == g["trace"].tolist()


@pytest.mark.parametrize("rule", RULES)
def test_permuted_rows_batched(rule):
    shapes = [(4096, 512, 7, 50), (30000, 3000, 5, 400), (20000, 300, 9, 30), (300000, 30000, 7, 3000),
              (5000, 40000, 3, 40), (1000, 100, 20, 5), (70000, 70000, 7, 5000)]
    insts = [gen.make_instance(5300 + q, n, m, d, k) for q, (n, m, d, k) in enumerate(shapes)]
    arrs = [(i.n, i.m, i.d, gen.permute_rows(i.col_idx, i.d, 91 + q), i.y,
             2.0 if rule >= l0.L0_RULE_SHIFTED_L0DEC else i.alpha) for q, i in enumerate(insts)]
    say("permuted rows batched", rule)
    res = batched_run(arrs, rule=rule)
    for q, (a, b) in enumerate(zip(arrs, res)):
        o = oracle_run(*a, rule=rule)
        assert_batched_parity(b, o, label=f"perm-batch {rule}/{q}")
