"""l0_decode_noalloc: the plain decode working in the library's fixed device
array instead of an allocation.  Through the C-ABI, against l0_decode (the
allocating entry point) and the oracle, bit for bit; two calls in a row, the
second on a smaller problem (the array keeps the first call's contents, so
the second must clear what it needs); sizes past the array refused."""
import numpy as np
import pytest
import torch

import gen
import paper_1508_01256_amd as l0
from parity import oracle_run, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    l0.lib()


def _both(inst, col=None):
    """The same decode through l0_decode and l0_decode_noalloc."""
    col = inst.col_idx if col is None else col
    c = to_dev(col, torch.int32)
    y = to_dev(inst.y, torch.float64)
    out = []
    for fn in (l0.l0_decode, l0.l0_decode_noalloc):
        x = torch.full((inst.n,), 7.0, dtype=torch.float64, device="cuda")
        it = torch.full((1,), -99, dtype=torch.int32, device="cuda")
        assert fn(c, inst.n, inst.m, inst.d, y, inst.alpha, 100, 1e-10, x, it) == l0.L0_OK
        torch.cuda.synchronize()
        out.append((x.cpu().numpy(), int(it.item())))
    return out


@pytest.mark.parametrize("order", ["large_then_small", "small_then_large"])
def test_noalloc_equals_l0_decode_twice_in_a_row(order):
    big = gen.make_instance(7100, 1 << 20, 104858, 7, 20971)    # 32-bit rows, ~60 MiB of the array
    small = gen.make_instance(7101, 100003, 10007, 5, 700)        # 16-bit rows
    assert l0.l0_noalloc_workspace_bytes(big.n, big.m, big.d, 100) <= l0.L0_NOALLOC_SCRATCH_BYTES
    seq = [big, small] if order == "large_then_small" else [small, big]
    for inst in seq:
        say("noalloc", inst.n, inst.m, inst.d)
        (xa, ia), (xb, ib) = _both(inst)
        assert ia == ib
        assert np.array_equal(xa.view(np.int64), xb.view(np.int64))
        o = oracle_run(inst.n, inst.m, inst.d, inst.col_idx, inst.y, inst.alpha)
        assert ib == o["iters"] and np.array_equal(xb, o["x"])


def test_noalloc_device_errors_then_a_good_call():
    inst = gen.make_instance(7102, 5000, 500, 7, 30)
    col = inst.col_idx.copy()
    col[3 * 7 + 2] = col[3 * 7]
    (xa, ia), (xb, ib) = _both(inst, col)
    assert ia == ib == -l0.L0_DEV_REPEATED_ROW and not np.any(xb)
    # the next call on the same array starts clean
    (xa, ia), (xb, ib) = _both(inst)
    assert ia == ib and np.array_equal(xa, xb) and ib >= 1


def test_noalloc_refuses_problems_past_the_array():
    n, m, d = 1 << 23, 16777, 7
    need = l0.l0_noalloc_workspace_bytes(n, m, d, 100)
    assert need > l0.L0_NOALLOC_SCRATCH_BYTES
    col = torch.zeros(n * d, dtype=torch.int32, device="cuda")
    y = torch.zeros(m, dtype=torch.float64, device="cuda")
    x = torch.empty(n, dtype=torch.float64, device="cuda")
    it = torch.zeros(1, dtype=torch.int32, device="cuda")
    assert l0.l0_decode_noalloc(col, n, m, d, y, 4, 100, 1e-10, x, it) == l0.L0_ERR_WORKSPACE
