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
