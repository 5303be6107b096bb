"""GPU parity of the batched decoder (l0_decode_batched), called through the
C-ABI: every instance of a batch against the CPU oracle (outcome, iterations,
final ||r||_0, update count, x_hat bitwise) and against its own solo run."""
import numpy as np
import pytest
import torch

import gen
import paper_1508_01256_amd as l0
from parity import assert_batched_parity, batched_run, gpu_run, oracle_run, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    l0.lib()


def sweep_like(count, seed, n_max_log2=14, scaled=None):
    """Instances shaped like the phase-transition sweep (mixed n, delta, d
    in {5, 7, 9}, rho), with n capped so the oracle finishes in seconds.
    scaled: None (unit columns), "all" or "half" (every other instance draws
    +-1 nonzeros on a column-scaled A)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(count):
        n = int(round(2.0 ** rng.uniform(6.0, n_max_log2)))
        delta = float(rng.choice([0.01, 0.03, 0.1, 0.3]))
        d = int(rng.choice([5, 7, 9]))
        m = max(gen.mk_m(n, delta), d)
        k = gen.mk_k(m, float(rng.uniform(0.05, 0.5)))
        sc = scaled == "all" or (scaled == "half" and i % 2 == 0)
        out.append(gen.make_instance(seed * 7919 + i, n, m, d, k, scaled=sc,
                                     kind=gen.VALUES_PM1 if sc else gen.VALUES_NORMAL))
    return out


def check_all(insts, res, label, **kw):
    for q, (i, b) in enumerate(zip(insts, res)):
        o = oracle_run(i.n, i.m, i.d, i.col_idx, i.y, kw.get("alphas", [i.alpha] * len(insts))[q],
                       max_iter=kw.get("max_iters", [100] * len(insts))[q],
                       rule=kw.get("rule", l0.L0_RULE_L0DEC), w=i.w)
        assert_batched_parity(b, o, label=f"{label}/{q} n={i.n} m={i.m} d={i.d} k={i.k}")


@pytest.mark.parametrize("bt,wc", [(0, 0), (512, 16384), (256, 64)])
def test_mixed_batch_against_oracle(bt, wc):
    insts = sweep_like(160, 11)
    say("batched mixed", bt, wc, len(insts))
    res = batched_run(insts, block_threads=bt, words_cap=wc)
    check_all(insts, res, f"mixed-{bt}-{wc}")


def test_batch_matches_solo_runs():
    insts = sweep_like(40, 12)
    res = batched_run(insts)
    for q, (i, b) in enumerate(zip(insts, res)):
        g = gpu_run(i.n, i.m, i.d, i.col_idx, i.y, i.alpha)
        for key in ("iters", "outcome", "final_nnz", "support_size", "updates"):
            assert b[key] == g[key], (q, key, b[key], g[key])
        assert np.array_equal(b["x"].view(np.int64), g["x"].view(np.int64)), q


def test_edge_instances():
    """k = 0, one column, m = d, tiny m with d = 9, largest and smallest d,
    a column past a 64-column group, and instances whose m exceeds the LDS
    word capacity, all in one batch (several degree groups)."""
    insts = [
        gen.make_instance(1, 4096, 512, 7, 0),
        gen.make_instance(2, 1, 3, 2, 1),
        gen.make_instance(3, 50, 9, 9, 2),
        gen.make_instance(4, 200, 10, 9, 1),
        gen.make_instance(5, 3000, 600, 20, 20),
        gen.make_instance(6, 3000, 300, 2, 10),
        gen.make_instance(7, 65, 30, 3, 3),
        gen.make_instance(8, 60000, 12000, 7, 900),   # m above an 8192-word capacity
        gen.make_instance(9, 40000, 36000, 5, 900),
        gen.make_instance(10, 64, 20, 4, 2),
    ]
    res = batched_run(insts, words_cap=8192)
    check_all(insts, res, "edge")
    assert res[0]["outcome"] == l0.L0_CONVERGED and res[0]["iters"] == 0


def test_rules_alpha_and_max_iter():
    insts = sweep_like(48, 13, n_max_log2=13)
    alphas = [float(2 + (q % 3)) if i.d >= 4 else 2.0 for q, i in enumerate(insts)]
    alphas = [min(a, float(i.d)) for a, i in zip(alphas, insts)]
    iters = [q % 4 for q in range(len(insts))]  # 0..3: many stop at MAX_ITER
    for rule in (l0.L0_RULE_L0DEC, l0.L0_RULE_MODE):
        res = batched_run(insts, alphas=alphas, max_iters=iters, rule=rule)
        check_all(insts, res, f"rule{rule}", alphas=alphas, max_iters=iters, rule=rule)


def test_absolute_tolerance():
    insts = sweep_like(24, 14, n_max_log2=12)
    tol = 2.0 ** -30
    res = batched_run(insts, tol=tol, tol_mode=l0.L0_TOL_ABSOLUTE)
    for q, (i, b) in enumerate(zip(insts, res)):
        g = gpu_run(i.n, i.m, i.d, i.col_idx, i.y, i.alpha, tol=tol, tol_mode=l0.L0_TOL_ABSOLUTE)
        for key in ("iters", "outcome", "final_nnz", "support_size", "updates"):
            assert b[key] == g[key], (q, key)
        assert np.array_equal(b["x"].view(np.int64), g["x"].view(np.int64)), q
        o = oracle_run(i.n, i.m, i.d, i.col_idx, i.y, i.alpha, tol=tol, tol_mode=l0.L0_TOL_ABSOLUTE)
        assert_batched_parity(b, o, label=f"abs/{q}")


def test_per_instance_device_errors():
    """A bad row index or a non-finite y fails only its own instance."""
    insts = sweep_like(12, 15, n_max_log2=12)
    bad_col = insts[3].col_idx.copy()
    bad_col[5] = insts[3].m          # one row index out of range
    bad_y = insts[7].y.copy()
    bad_y[0] = np.nan
    arrs = [(i.n, i.m, i.d, i.col_idx, i.y, i.alpha) for i in insts]
    arrs[3] = (insts[3].n, insts[3].m, insts[3].d, bad_col, insts[3].y, insts[3].alpha)
    arrs[7] = (insts[7].n, insts[7].m, insts[7].d, insts[7].col_idx, bad_y, insts[7].alpha)
    res = batched_run(arrs)
    assert res[3]["outcome"] == l0.L0_DEV_BAD_INDEX
    assert res[7]["outcome"] == l0.L0_DEV_NONFINITE_Y
    for q, i in enumerate(insts):
        if q in (3, 7):
            continue
        o = oracle_run(i.n, i.m, i.d, i.col_idx, i.y, i.alpha)
        assert_batched_parity(res[q], o, label=f"err/{q}")


def test_autotune_then_decode():
    insts = sweep_like(64, 16, n_max_log2=13)
    res = batched_run(insts, autotune=True)
    check_all(insts, res, "autotuned")


def test_two_batches_in_a_row_reuse_nothing_stale():
    """A second, smaller batch after a first (same process, fresh workspace
    contents left by the first) gives its own oracle results."""
    a = sweep_like(30, 17, n_max_log2=13)
    b = sweep_like(9, 18, n_max_log2=11)
    batched_run(a)
    res = batched_run(b)
    check_all(b, res, "second")


def test_sweep_workload_full_size_sampled():
    """The full phase-transition sweep's instance mix at its real sizes
    (n up to 2^18) in one batched call; a spread sample is checked against the
    oracle, every instance against the invariants of its outcome."""
    params = gen.sweep_params(4096)
    idx = list(range(0, 4096, 8))   # 512 instances, every size class
    insts = [gen.make_instance(params[i]["seed"], params[i]["n"], params[i]["m"], params[i]["d"],
                               params[i]["k"]) for i in idx]
    say("sweep sample", len(insts))
    res = batched_run(insts)
    for q in range(0, len(insts), 4):   # 128 oracle runs
        i = insts[q]
        o = oracle_run(i.n, i.m, i.d, i.col_idx, i.y, i.alpha)
        assert_batched_parity(res[q], o, label=f"sweep/{idx[q]}")
    for b in res:
        assert b["outcome"] in (l0.L0_CONVERGED, l0.L0_STALLED, l0.L0_MAX_ITER)
        assert (b["final_nnz"] == 0) == (b["outcome"] == l0.L0_CONVERGED)


def test_long_support_lists():
    """Tiny m with d = 9: a first iteration selects most columns, so row
    support lists grow to hundreds of entries (sorted in LDS) and, at
    n = 4000, past the LDS sort's capacity (the one-thread path)."""
    insts = [gen.make_instance(31, 1030, 10, 9, 3), gen.make_instance(32, 1046, 10, 9, 4),
             gen.make_instance(33, 4000, 10, 9, 3), gen.make_instance(34, 2000, 20, 9, 5),
             gen.make_instance(35, 6931, 69, 7, 15)]
    res = batched_run(insts)
    check_all(insts, res, "long-lists")
    g = gpu_run(insts[2].n, insts[2].m, insts[2].d, insts[2].col_idx, insts[2].y, insts[2].alpha)
    assert res[2]["support_size"] == g["support_size"]


def test_long_lists_growing_over_many_iterations():
    """Instances of the sweep workload with m of 11 to 94 that run to
    max_iter: columns keep entering the support, so long row lists get a few
    new entries after their sorted prefix in most iterations (merged by rank
    into the prefix)."""
    params = gen.sweep_params(4096)
    insts = [gen.make_instance(params[q]["seed"], params[q]["n"], params[q]["m"], params[q]["d"],
                               params[q]["k"]) for q in (1734, 118, 2425, 3803, 1482, 3481)]
    res = batched_run(insts)
    check_all(insts, res, "growing-lists")
    assert sum(r["outcome"] == l0.L0_MAX_ITER for r in res) >= 4


def test_teams_on_large_instances():
    """Instances with more than 2^19 column indices are decoded by teams of
    workgroups (here 14, 6 and the cap of 32, one with bucket words in global
    memory), mixed with single-workgroup ones; each result against the
    oracle and against its solo run."""
    big = [gen.make_instance(41, 1 << 20, 104858, 7, 9000),     # team of 14, words in global memory
           gen.make_instance(42, 400000, 8000, 7, 1500),        # team of 6, words in LDS
           gen.make_instance(43, 1 << 22, 41943, 7, 6000),      # team of 32 (cap)
           gen.make_instance(44, 600000, 60000, 5, 3000)]       # team of 6, words in global memory
    small = sweep_like(24, 19, n_max_log2=12)
    insts = big + small
    say("teams", [(i.n, i.m, i.d) for i in big])
    res = batched_run(insts, block_threads=512, words_cap=32768)
    check_all(insts, res, "teams")
    for q, i in enumerate(big):
        g = gpu_run(i.n, i.m, i.d, i.col_idx, i.y, i.alpha)
        assert res[q]["support_size"] == g["support_size"], q
        assert res[q]["updates"] == g["updates"], q


def test_teams_with_small_grid_schedule():
    """The same large instances with 256-thread workgroups and an 8192-word
    capacity (more passes, other team sizes)."""
    insts = [gen.make_instance(45, 1 << 20, 10486, 9, 1000), gen.make_instance(46, 300000, 30000, 5, 2500)]
    res = batched_run(insts, block_threads=256, words_cap=8192)
    check_all(insts, res, "teams-256")


@pytest.mark.parametrize("rule", [l0.L0_RULE_SHIFTED_L0DEC, l0.L0_RULE_SHIFTED_MODE])
def test_shifted_rules_in_a_batch(rule):
    """Shifted Parallel-l0 on a mixed batch, including a team-decoded
    instance; each against the oracle's shifted run."""
    insts = sweep_like(60, 31, n_max_log2=13) + [gen.make_instance(47, 1 << 20, 10486, 7, 900)]
    alphas = [2.0 if q % 2 else float(i.alpha) for q, i in enumerate(insts)]
    res = batched_run(insts, alphas=alphas, rule=rule)
    check_all(insts, res, f"shifted{rule}", alphas=alphas, rule=rule)


@pytest.mark.parametrize("rule", [l0.L0_RULE_L0DEC, l0.L0_RULE_SHIFTED_L0DEC])
def test_column_scaled_instances_in_a_batch(rule):
    """Column-scaled A (Section 4.3.3) per instance: a batch mixing +-1
    signals on scaled columns with unit-column instances, including
    team-decoded ones with words in LDS and in global memory; each against
    the oracle and against its solo run."""
    big = [gen.make_instance(48, 1 << 20, 104858, 7, 9000, kind=gen.VALUES_PM1, scaled=True),
           gen.make_instance(49, 400000, 8000, 7, 1500, kind=gen.VALUES_PM1, scaled=True)]
    insts = big + sweep_like(50, 33, n_max_log2=13, scaled="half")
    say("scaled batch", rule)
    res = batched_run(insts, rule=rule, block_threads=512, words_cap=32768)
    check_all(insts, res, f"scaled{rule}", rule=rule)
    for q, i in enumerate(insts[:6]):
        g = gpu_run(i.n, i.m, i.d, i.col_idx, i.y, i.alpha, rule=rule, w=i.w)
        for key in ("iters", "outcome", "final_nnz", "support_size", "updates"):
            assert res[q][key] == g[key], (q, key)
        assert np.array_equal(res[q]["x"].view(np.int64), g["x"].view(np.int64)), q
    # the scaled +-1 instances the oracle recovers are recovered exactly
    assert res[0]["outcome"] == l0.L0_CONVERGED


def test_bad_weight_fails_only_its_instance():
    insts = sweep_like(10, 34, n_max_log2=12, scaled="all")
    w3, w6 = insts[3].w.copy(), insts[6].w.copy()
    w3[2] = 0.0
    w6[insts[6].n - 1] = np.inf
    probs = []
    for q, i in enumerate(insts):
        w = w3 if q == 3 else w6 if q == 6 else i.w
        probs.append(dict(col_idx=to_dev(i.col_idx, torch.int32), n=i.n, m=i.m, d=i.d,
                          y=to_dev(i.y, torch.float64), alpha=i.alpha, max_iter=100, tol=1e-10,
                          weights=to_dev(w, torch.float64)))
    xs, res = l0.decode_batched(probs)
    assert res[3]["outcome"] == l0.L0_DEV_BAD_WEIGHT and not torch.any(xs[3])
    assert res[6]["outcome"] == l0.L0_DEV_BAD_WEIGHT
    for q, i in enumerate(insts):
        if q in (3, 6):
            continue
        o = oracle_run(i.n, i.m, i.d, i.col_idx, i.y, i.alpha, w=i.w)
        res[q]["x"] = xs[q].cpu().numpy()
        assert_batched_parity(res[q], o, label=f"badw/{q}")
