"""GPU parity: the HIP decoder, called through the C-ABI, against the CPU
oracle on the same seeded inputs (support, iterations, outcome and ||r||_0
trace bitwise; x_hat bitwise, hence within 1e-12 relative)."""
import numpy as np
import pytest
import torch

import gen
import paper_1508_01256_amd as l0
from golden_io import decode_cases, graph_arrays
from parity import assert_parity, gpu_run, oracle_run, run_both, say, to_dev

pytestmark = pytest.mark.gpu

RULES = {"L0DEC": l0.L0_RULE_L0DEC, "MODE": l0.L0_RULE_MODE, "SHIFTED_L0DEC": l0.L0_RULE_SHIFTED_L0DEC,
         "SHIFTED_MODE": l0.L0_RULE_SHIFTED_MODE}
OUT = {"CONVERGED": l0.L0_CONVERGED, "STALLED": l0.L0_STALLED, "MAX_ITER": l0.L0_MAX_ITER}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    l0.lib()


@pytest.mark.parametrize("case", [c for c in decode_cases() if c[4]["algo"] == "parallel"],
                         ids=lambda c: f"{c[0]}-{c[4]['rule']}-a{c[4]['alpha']}")
def test_worked_cases(case):
    name, g_, y, x, c = case
    n, m, d, col = graph_arrays(g_)
    w = np.array(g_["w"], float) if "w" in g_ else None
    say("worked", name, c)
    g = gpu_run(n, m, d, col, y, c["alpha"], max_iter=c["max_iter"], tol=c["tol"], rule=RULES[c["rule"]],
                w=w)
    assert g["outcome"] == OUT[c["outcome"]] and g["iters"] == c["iters"]
    assert g["trace"].tolist() == c["trace"] and g["tsize"].tolist() == c["tsize"]
    assert np.array_equal(g["x"], np.array(c["x_hat"], float))


@pytest.mark.parametrize("seed", range(100))
def test_small_workload(seed):
    """The small workload (n = 4096, m = 512, d = 7, k = 50) over 100 seeds."""
    inst = gen.single_workload("small", seed)
    say("small seed", seed)
    g, o = run_both(inst)
    assert_parity(g, o, label=f"small/{seed}")
    if o["outcome"] == 0:  # success criterion: ||x_hat - x||_inf / ||x||_inf <= 1e-12
        assert np.max(np.abs(g["x"] - inst.x)) <= 1e-12 * np.max(np.abs(inst.x))


@pytest.mark.parametrize("seed", range(4))
def test_small_workload_mode_rule(seed):
    inst = gen.single_workload("small", seed)
    g, o = run_both(inst, rule=l0.L0_RULE_MODE)
    assert_parity(g, o, label=f"small-mode/{seed}")


@pytest.mark.parametrize("rule", [l0.L0_RULE_SHIFTED_L0DEC, l0.L0_RULE_SHIFTED_MODE])
@pytest.mark.parametrize("seed", range(4))
def test_small_workload_shifted_rules(seed, rule):
    """Shifted Parallel-l0 (Algorithm 3): one candidate per column per pass."""
    inst = gen.make_instance(700 + seed, 4096, 512, 7, 20 + 10 * seed)
    for alpha in (2.0, 4.0):
        g, o = run_both(inst, alpha=alpha, rule=rule)
        assert_parity(g, o, label=f"shifted-{rule}-{seed}-{alpha}")


@pytest.mark.parametrize("n,m,d,k", [
    (400000, 40000, 7, 3000),   # 32-bit rows, words from L2
    (262144, 26215, 7, 2621),   # 16-bit rows
    (50000, 5000, 9, 300),
    (3000, 60, 3, 8),           # tiny m: many overflowing passes
])
def test_shapes_shifted(n, m, d, k):
    inst = gen.make_instance(5151 + n + d, n, m, d, k)
    say("shifted shape", n, m, d, k)
    g, o = run_both(inst, rule=l0.L0_RULE_SHIFTED_L0DEC)
    assert_parity(g, o, label=f"shifted {n}/{m}/{d}/{k}")


@pytest.mark.parametrize("n,m,d,k", [
    (100003, 10007, 7, 700),    # many tiles, ragged tail, r in LDS
    (100003, 10007, 7, 2500),   # stalls (dense for alpha = 4)
    (262144, 26215, 7, 2621),   # 16-bit rows, 32-bit bucket words in LDS
    (300000, 36864, 9, 2000),   # largest m with 32-bit words in LDS
    (300000, 36865, 5, 2000),   # smallest m with 16-bit folded words in LDS
    (400000, 40000, 7, 3000),   # 16-bit folded words
    (300000, 65536, 7, 2500),   # largest m with 16-bit rows and words
    (300000, 65537, 7, 2500),   # smallest m with 32-bit rows, 8-bit folded words
    (400000, 147456, 5, 4000),  # largest m with 8-bit words in LDS
    (400000, 147457, 5, 4000),  # smallest m with words gathered from global memory
    (600000, 400000, 7, 9000),  # global words
    (50000, 5000, 5, 400),
    (50000, 5000, 9, 300),
    (30000, 3000, 3, 150),
    (20000, 4000, 20, 60),      # largest supported d
    (1, 3, 2, 1),               # one column
    (300, 40, 2, 5),
    (257, 60, 4, 10),           # one column past a tile
])
def test_shapes(n, m, d, k):
    inst = gen.make_instance(4242 + n + d, n, m, d, k)
    say("shape", n, m, d, k)
    g, o = run_both(inst)
    assert_parity(g, o, label=f"{n}/{m}/{d}/{k}")


@pytest.mark.parametrize("alpha", [2.0, 2.5, 3.0, 5.0, 7.0])
def test_alpha_values(alpha):
    inst = gen.make_instance(77, 20000, 2000, 7, 150)
    g, o = run_both(inst, alpha=alpha)
    assert_parity(g, o, label=f"alpha={alpha}")


def test_pm1_signals():
    inst = gen.make_instance(88, 40000, 4000, 7, 600, kind=gen.VALUES_PM1)
    g, o = run_both(inst)
    assert_parity(g, o, label="pm1")


@pytest.mark.parametrize("tol", [0.0, 1e-14, 1e-6, 1e-3])
def test_tolerances(tol):
    inst = gen.make_instance(99, 20000, 2000, 7, 120)
    g, o = run_both(inst, tol=tol)
    assert_parity(g, o, label=f"tol={tol}")


def test_absolute_tolerance():
    """tau = tol itself (L0_TOL_ABSOLUTE), against the oracle's absolute mode,
    at a tolerance that decides the run (one far below the rounding noise of
    the residual, one above it)."""
    inst = gen.make_instance(5, 20000, 2000, 7, 120)
    y = inst.y * 2.0 ** -3
    for tol in (2.0 ** -30, 1e-20, 0.0):
        g, o = run_both((inst.n, inst.m, inst.d, inst.col_idx, y, 4), tol=tol,
                        tol_mode=l0.L0_TOL_ABSOLUTE)
        assert_parity(g, o, label=f"tol-abs {tol}")
    assert g["outcome"] == o["outcome"]


def test_edge_k0_and_max_iter0():
    inst = gen.make_instance(6, 5000, 500, 7, 0)
    g, o = run_both(inst)
    assert_parity(g, o, label="k0")
    assert g["iters"] == 0 and g["outcome"] == l0.L0_CONVERGED and not np.any(g["x"])
    inst = gen.make_instance(6, 5000, 500, 7, 30)
    g, o = run_both(inst, max_iter=0)
    assert_parity(g, o, label="max_iter0")
    assert g["outcome"] == l0.L0_MAX_ITER and g["iters"] == 0
    g, o = run_both(inst, max_iter=1)
    assert_parity(g, o, label="max_iter1")


def test_resume_matches_uninterrupted_run():
    inst = gen.make_instance(33, 8000, 800, 7, 100)
    full = gpu_run(inst.n, inst.m, inst.d, inst.col_idx, inst.y, 4, max_iter=20)
    assert full["iters"] >= 5
    K = 3
    first = gpu_run(inst.n, inst.m, inst.d, inst.col_idx, inst.y, 4, max_iter=K)
    rest = gpu_run(inst.n, inst.m, inst.d, inst.col_idx, inst.y, 4, max_iter=20 - K, x_init=first["x"])
    assert np.array_equal(rest["x"], full["x"])
    assert rest["trace"].tolist() == full["trace"][K:].tolist()
    o = oracle_run(inst.n, inst.m, inst.d, inst.col_idx, inst.y, 4, max_iter=20 - K, x_init=first["x"])
    assert_parity(rest, o, label="resume")


def test_repeated_runs_are_bitwise_identical():
    inst = gen.make_instance(12, 200000, 20000, 7, 1800)
    runs = [gpu_run(inst.n, inst.m, inst.d, inst.col_idx, inst.y, 4) for _ in range(3)]
    for r in runs[1:]:
        assert np.array_equal(r["x"].view(np.int64), runs[0]["x"].view(np.int64))
        assert r["trace"].tolist() == runs[0]["trace"].tolist()


def test_device_detected_errors():
    inst = gen.make_instance(3, 5000, 500, 7, 30)
    y = inst.y.copy()
    y[17] = np.nan
    g = gpu_run(inst.n, inst.m, inst.d, inst.col_idx, y, 4)
    assert g["outcome"] == l0.L0_DEV_NONFINITE_Y and not np.any(g["x"])
    col = inst.col_idx.copy()
    col[123] = inst.m  # out of range: clamped during repacking and reported
    g = gpu_run(inst.n, inst.m, inst.d, col, inst.y, 4)
    assert g["outcome"] == l0.L0_DEV_BAD_INDEX
    col[123] = -5
    g = gpu_run(inst.n, inst.m, inst.d, col, inst.y, 4)
    assert g["outcome"] == l0.L0_DEV_BAD_INDEX


def test_host_rejects_bad_buffers():
    inst = gen.make_instance(3, 5000, 500, 7, 30)
    col = to_dev(inst.col_idx, torch.int32)
    y = to_dev(inst.y, torch.float64)
    x = torch.empty(inst.n, dtype=torch.float64, device="cuda")
    res = l0.new_result()
    ws = torch.empty(l0.l0_workspace_bytes(inst.n, inst.m, inst.d, 10), dtype=torch.uint8, device="cuda")
    ok = l0.l0_decode_ex(col, inst.n, inst.m, inst.d, y, 4, 10, 1e-10, x, None, res, ws)
    assert ok == l0.L0_OK
    torch.cuda.synchronize()
    # workspace too small
    assert l0.l0_decode_ex(col, inst.n, inst.m, inst.d, y, 4, 10, 1e-10, x, None, res, ws[:-4096]) \
        == l0.L0_ERR_WORKSPACE
    # host memory instead of device memory
    xh = torch.empty(inst.n, dtype=torch.float64)
    assert l0.l0_decode_ex(col, inst.n, inst.m, inst.d, y, 4, 10, 1e-10, xh, None, res, ws) == l0.L0_ERR_ARG
    # buffer too short for n
    assert l0.l0_decode_ex(col, inst.n + 100000, inst.m, inst.d, y, 4, 10, 1e-10, x, None, res, ws) \
        in (l0.L0_ERR_ARG, l0.L0_ERR_WORKSPACE)
    torch.cuda.synchronize()


def test_plain_decode_and_prepared_matrix_agree():
    inst = gen.make_instance(21, 60000, 6000, 7, 400)
    col = to_dev(inst.col_idx, torch.int32)
    y = to_dev(inst.y, torch.float64)
    x = torch.empty(inst.n, dtype=torch.float64, device="cuda")
    it = torch.zeros(1, dtype=torch.int32, device="cuda")
    assert l0.l0_decode(col, inst.n, inst.m, inst.d, y, 4, 100, 1e-10, x, it) == l0.L0_OK
    torch.cuda.synchronize()
    o = oracle_run(inst.n, inst.m, inst.d, inst.col_idx, inst.y, 4)
    assert int(it.item()) == o["iters"]
    assert np.array_equal(x.cpu().numpy(), o["x"])
    with l0.Matrix(col, inst.n, inst.m, inst.d) as A:
        for rep in range(3):
            r = A.solve(y, 4)
            assert r["iters"] == o["iters"] and r["trace"].tolist() == o["trace"].tolist()
            assert np.array_equal(r["x"].cpu().numpy(), o["x"])
        # a different y on the same prepared matrix
        inst2 = gen.make_instance(22, 60000, 6000, 7, 300)
        inst2.col_idx = inst.col_idx
        y2 = gen.measure(inst.n, inst.m, inst.d, inst.col_idx, inst2.supp, inst2.vals)
        r2 = A.solve(to_dev(y2, torch.float64), 4)
        o2 = oracle_run(inst.n, inst.m, inst.d, inst.col_idx, y2, 4)
        assert r2["trace"].tolist() == o2["trace"].tolist()
        assert np.array_equal(r2["x"].cpu().numpy(), o2["x"])


@pytest.mark.parametrize("name,kind", [("n2^20", gen.VALUES_NORMAL), ("n2^24", gen.VALUES_NORMAL),
                                       ("n2^24", gen.VALUES_PM1)])
def test_full_size_workloads(name, kind):
    inst = gen.single_workload(name, 0, kind=kind)
    say("full", name, kind)
    g, o = run_both(inst)
    assert_parity(g, o, label=f"{name}/{kind}")


def test_index_store_past_two_gigabytes():
    """n = 2^27 columns of degree 5: 2.7 GB of 32-bit column indices (byte
    offsets past 2^31) and m = 2^20 rows (32-bit repacked rows, bucket words
    read from global memory), decoded bitwise as the oracle does."""
    inst = gen.make_instance(9700, 1 << 27, 1 << 20, 5, 20000)
    say("index store past 2 GB", inst.n, inst.m, inst.d)
    g, o = run_both(inst)
    assert_parity(g, o, label="n2^27 d5")
    assert o["outcome"] == l0.L0_CONVERGED


@pytest.mark.parametrize("max_iter", [100, 40000])
def test_one_shot_control_reset_paths(max_iter):
    """A one-shot decode has its preparation clear the solve's control block
    and counters when they form a short run; with max_iter = 40000 the
    counters are too long for that and the solve fills them itself.  Both
    paths, twice in a row on one workspace (the second call must not see the
    first one's counters), against the oracle."""
    inst = gen.make_instance(9900, 50000, 5000, 7, 300)
    col = to_dev(inst.col_idx, torch.int32)
    y = to_dev(inst.y, torch.float64)
    ws = torch.empty(l0.l0_workspace_bytes(inst.n, inst.m, inst.d, max_iter), dtype=torch.uint8, device="cuda")
    o = oracle_run(inst.n, inst.m, inst.d, inst.col_idx, inst.y, inst.alpha, max_iter=max_iter)
    for rep in range(2):
        x = torch.empty(inst.n, dtype=torch.float64, device="cuda")
        res = l0.new_result()
        assert l0.l0_decode_ex(col, inst.n, inst.m, inst.d, y, inst.alpha, max_iter, 1e-10, x, None, res, ws) == l0.L0_OK
        torch.cuda.synchronize()
        r = l0.results_list(res.view(1, 3))[0]
        assert r["outcome"] == o["outcome"] and r["iters"] == o["iters"], (max_iter, rep, r)
        assert np.array_equal(x.cpu().numpy(), o["x"]), (max_iter, rep)
