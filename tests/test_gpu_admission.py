"""The single-instance solve kernel is an ordinary launch whose workgroups
admit themselves at start; the members split the columns and rows among
them.  A decode's result must not depend on how many workgroups become
members: caps force 1 to 100 members of the up to 256 launched, and a 1 us
window makes the first member close admission while others are still
starting (a member count that varies from run to run).  Every run is checked
against the oracle (support, iterations, outcome, ||r||_0 trace and x_hat
bitwise), over both scoring rules, the shifted rules, a column-scaled A and a
resumed run."""
import numpy as np
import pytest
import torch

import gen
import paper_1508_01256_amd as l0
from parity import assert_parity, gpu_run, oracle_run, run_both, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    l0.lib()
    yield
    l0.l0_set_solve_admission(0, 0)


@pytest.fixture(autouse=True)
def _defaults():
    yield
    l0.l0_set_solve_admission(0, 0)


SETTINGS = [(1, 0), (3, 0), (17, 0), (100, 0), (0, 1), (5, 1)]


@pytest.mark.parametrize("cap,window", SETTINGS)
def test_member_count_does_not_change_the_result(cap, window):
    # many tiles, a ragged tail, r and the bucket words in LDS
    inst = gen.make_instance(9100, 100003, 10007, 7, 700)
    say("admission", cap, window)
    l0.l0_set_solve_admission(cap, window)
    g, o = run_both(inst)
    assert_parity(g, o, label=f"cap {cap} window {window}")
    assert o["outcome"] == l0.L0_CONVERGED


@pytest.mark.parametrize("cap,window", [(1, 0), (7, 0), (0, 1)])
@pytest.mark.parametrize("rule", [l0.L0_RULE_MODE, l0.L0_RULE_SHIFTED_L0DEC, l0.L0_RULE_SHIFTED_MODE])
def test_rules_with_few_members(cap, window, rule):
    inst = gen.make_instance(9200 + rule, 40000, 4000, 7, 300)
    l0.l0_set_solve_admission(cap, window)
    g, o = run_both(inst, alpha=2.0, rule=rule)
    assert_parity(g, o, label=f"rule {rule} cap {cap} window {window}")


@pytest.mark.parametrize("cap,window", [(2, 0), (0, 1)])
def test_scaled_and_wide_rows_with_few_members(cap, window):
    """A column-scaled A with +-1 values, and m past the LDS word capacity
    (32-bit rows, words read from L2)."""
    l0.l0_set_solve_admission(cap, window)
    inst = gen.make_instance(9300, 60000, 6000, 7, 400, kind=gen.VALUES_PM1, scaled=True)
    g, o = run_both(inst)
    assert_parity(g, o, label=f"scaled cap {cap} window {window}")
    inst = gen.make_instance(9301, 400000, 40000, 7, 3000)
    g, o = run_both(inst)
    assert_parity(g, o, label=f"wide cap {cap} window {window}")


def test_resume_with_few_members():
    inst = gen.make_instance(9400, 8000, 800, 7, 100)
    first = gpu_run(inst.n, inst.m, inst.d, inst.col_idx, inst.y, 4, max_iter=2)
    l0.l0_set_solve_admission(3, 0)
    rest = gpu_run(inst.n, inst.m, inst.d, inst.col_idx, inst.y, 4, x_init=first["x"])
    o = oracle_run(inst.n, inst.m, inst.d, inst.col_idx, inst.y, 4, x_init=first["x"])
    assert_parity(rest, o, label="resume cap 3")


def test_full_size_with_a_short_window():
    """The n = 2^24 workload with admission closed after 1 us: however many
    workgroups got in, the decode is the oracle's."""
    inst = gen.single_workload("n2^24", 0)
    say("full size, window 1 us")
    l0.l0_set_solve_admission(0, 1)
    g, o = run_both(inst)
    assert_parity(g, o, label="n2^24 window 1 us")
    l0.l0_set_solve_admission(0, 0)
    u = gpu_run(inst.n, inst.m, inst.d, inst.col_idx, inst.y, inst.alpha)
    assert np.array_equal(u["x"], g["x"]) and u["trace"].tolist() == g["trace"].tolist()


def test_concurrent_solves_on_two_streams():
    """Two one-shot decodes enqueued on two streams at once, eight times over.
    Each solve takes every compute unit, so the second one's workgroups start
    only as the first one's leave (the solves do not execute side by side,
    which is not supported); a solve may close admission with only the
    workgroups that got one.  Every result equals the same decode run alone."""
    a = gen.make_instance(9500, 1 << 20, 10486, 7, 1000)
    b = gen.make_instance(9501, 1 << 20, 30000, 5, 2500)  # 4096 tiles: a grid of one workgroup per CU
    dev = "cuda"

    def upload(i):
        return (torch.from_numpy(i.col_idx).to(dev), torch.from_numpy(i.y).to(dev),
                torch.empty(l0.l0_workspace_bytes(i.n, i.m, i.d, 100), dtype=torch.uint8, device=dev))

    (ca, ya, wa), (cb, yb, wb) = upload(a), upload(b)
    ref = {}
    for name, i, c, y, w in (("a", a, ca, ya, wa), ("b", b, cb, yb, wb)):
        x = torch.empty(i.n, dtype=torch.float64, device=dev)
        r = l0.new_result(dev)
        assert l0.l0_decode_ex(c, i.n, i.m, i.d, y, i.alpha, 100, 1e-10, x, None, r, w) == l0.L0_OK
        torch.cuda.synchronize()
        ref[name] = (x.cpu(), r.cpu())
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    outs = []
    torch.cuda.synchronize()
    for rep in range(8):
        xa, ra = torch.empty(a.n, dtype=torch.float64, device=dev), l0.new_result(dev)
        xb, rb = torch.empty(b.n, dtype=torch.float64, device=dev), l0.new_result(dev)
        with torch.cuda.stream(s1):
            assert l0.l0_decode_ex(ca, a.n, a.m, a.d, ya, a.alpha, 100, 1e-10, xa, None, ra, wa) == l0.L0_OK
        with torch.cuda.stream(s2):
            assert l0.l0_decode_ex(cb, b.n, b.m, b.d, yb, b.alpha, 100, 1e-10, xb, None, rb, wb) == l0.L0_OK
        outs.append((xa, ra, xb, rb))
    torch.cuda.synchronize()
    say("concurrent solves done")
    for xa, ra, xb, rb in outs:
        assert torch.equal(ra.cpu(), ref["a"][1]) and torch.equal(xa.cpu(), ref["a"][0])
        assert torch.equal(rb.cpu(), ref["b"][1]) and torch.equal(xb.cpu(), ref["b"][0])
    o = oracle_run(a.n, a.m, a.d, a.col_idx, a.y, a.alpha)
    assert np.array_equal(ref["a"][0].numpy(), o["x"])
