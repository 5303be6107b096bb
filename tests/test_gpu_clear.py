"""A solve from x_hat = 0 leaves no value of the caller's output buffer
behind.  The solve kernel zeroes x_hat during its start-up, each member a
contiguous run of it by 16-byte stores (a leading double when the buffer is
8 but not 16 bytes past an aligned address, an odd last one);
these tests fill the output with NaN first and compare every entry with the
oracle, bitwise, across ragged sizes, both row widths, both alignments, and
the paths that end before any vote (y = 0, max_iter = 0, a device-detected
input error)."""
import numpy as np
import pytest
import torch

import gen
import paper_1508_01256_amd as l0
from parity import oracle_run, say, to_dev

pytestmark = pytest.mark.gpu


def nan_buffer(n, offset):
    """A float64 device view of n entries at `offset` elements into a NaN
    buffer (offset 1 is 8 but not 16 bytes past an aligned start)."""
    buf = torch.full((n + 2,), float("nan"), dtype=torch.float64, device="cuda")
    x = buf[offset:offset + n]
    assert (x.data_ptr() % 16 == 0) == (offset % 2 == 0)
    return x


def solve_into(A, y, alpha, x, **kw):
    res = l0.new_result()
    A.solve_async(y, alpha, x=x, res=res, **kw)
    torch.cuda.synchronize()
    return l0.results_list(res.view(1, 3))[0]


# (n, m, k): 16-bit rows (m <= 65536) with odd n, n below one chunk, n one
# past a chunk boundary, whole chunks; 32-bit rows (m > 65536)
SHAPES = [(4097, 410, 40), (37, 20, 2), (128 * 41 + 1, 600, 50), (128 * 64, 900, 80),
          (65535, 6554, 600), (700001, 70001, 3000)]


@pytest.mark.parametrize("offset", [0, 1])
@pytest.mark.parametrize("n,m,k", SHAPES)
def test_output_fully_written(n, m, k, offset):
    inst = gen.make_instance(4100 + n % 97, n, m, 7, k)
    say("clear", n, m, k, "offset", offset)
    col = to_dev(inst.col_idx, torch.int32)
    y = to_dev(inst.y, torch.float64)
    o = oracle_run(n, m, 7, inst.col_idx, inst.y, 4)
    with l0.Matrix(col, n, m, 7) as A:
        for rep in range(2):  # the second solve reuses the workspace
            x = nan_buffer(n, offset)
            r = solve_into(A, y, 4, x)
            xh = x.cpu().numpy()
            assert not np.isnan(xh).any(), (n, offset, rep)
            assert r["outcome"] == o["outcome"] and r["iters"] == o["iters"], (n, offset, rep)
            assert np.array_equal(xh.view(np.int64), o["x"].view(np.int64)), (n, offset, rep)


@pytest.mark.parametrize("offset", [0, 1])
def test_paths_that_end_before_a_vote(offset):
    n, m = 128 * 33 + 1, 500
    inst = gen.make_instance(4300, n, m, 7, 30)
    col = to_dev(inst.col_idx, torch.int32)
    with l0.Matrix(col, n, m, 7) as A:
        # y = 0: converged at the start
        x = nan_buffer(n, offset)
        r = solve_into(A, torch.zeros(m, dtype=torch.float64, device="cuda"), 4, x)
        assert r["outcome"] == l0.L0_CONVERGED and r["iters"] == 0
        assert not torch.any(x != 0).item()
        # max_iter = 0
        x = nan_buffer(n, offset)
        r = solve_into(A, to_dev(inst.y, torch.float64), 4, x, max_iter=0)
        assert r["outcome"] == l0.L0_MAX_ITER and r["iters"] == 0
        assert not torch.any(x != 0).item()
        # non-finite y: a device-detected input error
        yb = inst.y.copy()
        yb[7] = np.inf
        x = nan_buffer(n, offset)
        r = solve_into(A, to_dev(yb, torch.float64), 4, x)
        assert r["outcome"] == l0.L0_DEV_NONFINITE_Y
        assert not torch.any(x != 0).item()
    # an index out of range, found while preparing the matrix
    bad = inst.col_idx.copy()
    bad[5] = m
    with l0.Matrix(to_dev(bad, torch.int32), n, m, 7) as A:
        x = nan_buffer(n, offset)
        r = solve_into(A, to_dev(inst.y, torch.float64), 4, x)
        assert r["outcome"] == l0.L0_DEV_BAD_INDEX
        assert not torch.any(x != 0).item()


def test_shifted_rules():
    """Shifted rules (Algorithm 3), whose passes may select nothing before
    the next position is tried: x_hat is still written in full."""
    inst = gen.make_instance(4400, 20001, 2000, 7, 150)
    col = to_dev(inst.col_idx, torch.int32)
    y = to_dev(inst.y, torch.float64)
    for rule in (l0.L0_RULE_SHIFTED_L0DEC, l0.L0_RULE_SHIFTED_MODE):
        o = oracle_run(inst.n, inst.m, 7, inst.col_idx, inst.y, 4, rule=rule)
        with l0.Matrix(col, inst.n, inst.m, 7) as A:
            x = nan_buffer(inst.n, 0)
            r = solve_into(A, y, 4, x, rule=rule)
        assert r["outcome"] == o["outcome"] and r["iters"] == o["iters"]
        assert np.array_equal(x.cpu().numpy().view(np.int64), o["x"].view(np.int64))


def one_shot_into(inst, col, y, x, max_iter=100):
    """l0_decode_ex into x (the one-shot decode); returns the result record."""
    res = l0.new_result()
    ws = torch.empty(l0.l0_workspace_bytes(inst.n, inst.m, inst.d, max_iter), dtype=torch.uint8, device="cuda")
    assert l0.l0_decode_ex(col, inst.n, inst.m, inst.d, y, 4, max_iter, 1e-10, x, None, res, ws) == l0.L0_OK
    torch.cuda.synchronize()
    return l0.results_list(res.view(1, 3))[0]


@pytest.mark.parametrize("offset", [0, 1])
@pytest.mark.parametrize("n,m,k", SHAPES[:5])
def test_one_shot_output_fully_written(n, m, k, offset):
    """The one-shot decode over NaN-filled outputs, both alignments."""
    inst = gen.make_instance(4500 + n % 89, n, m, 7, k)
    say("one-shot clear", n, m, k, "offset", offset)
    col = to_dev(inst.col_idx, torch.int32)
    y = to_dev(inst.y, torch.float64)
    o = oracle_run(n, m, 7, inst.col_idx, inst.y, 4)
    for rep in range(2):
        x = nan_buffer(n, offset)
        r = one_shot_into(inst, col, y, x)
        xh = x.cpu().numpy()
        assert r["outcome"] == o["outcome"] and r["iters"] == o["iters"], (n, offset, rep)
        assert np.array_equal(xh.view(np.int64), o["x"].view(np.int64)), (n, offset, rep)


def test_one_shot_paths_that_end_before_a_vote():
    """y = 0 and max_iter = 0 through the one-shot decode: x_hat all zero;
    with an index out of range or a repeated row the input error wins."""
    n, m = 128 * 33 + 1, 500
    inst = gen.make_instance(4600, n, m, 7, 30)
    col = to_dev(inst.col_idx, torch.int32)
    zero_y = torch.zeros(m, dtype=torch.float64, device="cuda")
    x = nan_buffer(n, 0)
    r = one_shot_into(inst, col, zero_y, x)
    assert r["outcome"] == l0.L0_CONVERGED and r["iters"] == 0 and not torch.any(x != 0).item()
    x = nan_buffer(n, 0)
    r = one_shot_into(inst, col, to_dev(inst.y, torch.float64), x, max_iter=0)
    assert r["outcome"] == l0.L0_MAX_ITER and r["iters"] == 0 and not torch.any(x != 0).item()
    bad = inst.col_idx.copy()
    bad[11] = m
    for yy in (zero_y, to_dev(inst.y, torch.float64)):
        x = nan_buffer(n, 0)
        r = one_shot_into(inst, to_dev(bad, torch.int32), yy, x)
        assert r["outcome"] == l0.L0_DEV_BAD_INDEX and not torch.any(x != 0).item()
    rep = inst.col_idx.copy()
    rep[7 * 5 + 3] = rep[7 * 5 + 1]
    x = nan_buffer(n, 0)
    r = one_shot_into(inst, to_dev(rep, torch.int32), to_dev(inst.y, torch.float64), x)
    assert r["outcome"] == l0.L0_DEV_REPEATED_ROW and not torch.any(x != 0).item()


@pytest.mark.parametrize("cap", [1, 3, 7, 100])
@pytest.mark.parametrize("offset", [0, 1])
def test_output_fully_written_with_few_members(cap, offset):
    """The members split the clear into contiguous runs by their count: with
    admission capped at 1, 3, 7 or 100 members (145 tiles: 10 workgroups
    launched) every entry is still written."""
    n, m, k = 256 * 144 + 77, 3700, 300
    inst = gen.make_instance(4700 + cap, n, m, 7, k)
    say("clear with members", cap, "offset", offset)
    col = to_dev(inst.col_idx, torch.int32)
    y = to_dev(inst.y, torch.float64)
    o = oracle_run(n, m, 7, inst.col_idx, inst.y, 4)
    l0.l0_set_solve_admission(cap, 0)
    try:
        with l0.Matrix(col, n, m, 7) as A:
            x = nan_buffer(n, offset)
            r = solve_into(A, y, 4, x)
    finally:
        l0.l0_set_solve_admission(0, 0)
    xh = x.cpu().numpy()
    assert r["outcome"] == o["outcome"] and r["iters"] == o["iters"], (cap, offset)
    assert np.array_equal(xh.view(np.int64), o["x"].view(np.int64)), (cap, offset)
