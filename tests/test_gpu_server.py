"""GPU tests of the decoding server (l0_server_*), called through the C-ABI:
every request's result equals its solo decode and the oracle, whatever
batch it lands in, under budget-limited admission."""
import numpy as np
import pytest
import torch

import gen
import paper_1508_01256_amd as l0
from parity import gpu_run, oracle_run, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    l0.lib()


def serve_like(count, seed, lo=10.0, hi=16.0):
    """Requests shaped like the serving mix (d = 7, delta in {0.01, 0.1},
    k = 0.15 m, a tenth with +-1 nonzeros), with n capped for the oracle."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(count):
        n = int(round(2.0 ** rng.uniform(lo, hi)))
        delta = float(rng.choice([0.01, 0.1]))
        m = max(gen.mk_m(n, delta), 7)
        kind = gen.VALUES_PM1 if rng.uniform() < 0.1 else gen.VALUES_NORMAL
        out.append(gen.make_instance(seed * 10007 + i, n, m, 7, gen.mk_k(m, 0.15), kind=kind))
    return out


def upload(insts):
    return [dict(col=to_dev(i.col_idx, torch.int32), y=to_dev(i.y, torch.float64),
                 x=torch.empty(i.n, dtype=torch.float64, device="cuda"),
                 w=None if i.w is None else to_dev(i.w, torch.float64)) for i in insts]


def run_server(insts, bufs, *, budget=1 << 30, order=None, **kw):
    done = {}
    with l0.Server(budget, **kw) as srv:
        for q in (order if order is not None else range(len(insts))):
            i, b = insts[q], bufs[q]
            assert srv.submit(q, b["col"], b["y"], i.n, i.m, i.d, b["x"], i.alpha, weights=b["w"]) == l0.L0_OK
            for c in srv.poll():
                done[c["id"]] = c
        for c in srv.drain():
            done[c["id"]] = c
        assert srv.outstanding() == 0
    return done


def check_against_oracle(insts, bufs, done, label):
    assert sorted(done) == list(range(len(insts)))
    for q, i in enumerate(insts):
        c = done[q]
        assert c["status"] == l0.L0_OK, (label, q)
        assert c["submit_s"] <= c["launch_s"] <= c["done_s"], (label, q)
        o = oracle_run(i.n, i.m, i.d, i.col_idx, i.y, i.alpha, w=i.w)
        x = bufs[q]["x"].cpu().numpy()
        assert c["outcome"] == o["outcome"] and c["iters"] == o["iters"], (label, q)
        assert c["final_nnz"] == int(o["trace"][-1]) and c["updates"] == int(np.sum(o["tsize"])), (label, q)
        assert np.array_equal(x.view(np.int64), o["x"].view(np.int64)), (label, q, "x_hat differs")


@pytest.mark.parametrize("inflight", [1, 2, 4])
def test_requests_against_oracle(inflight):
    insts = serve_like(60, 21)
    bufs = upload(insts)
    say("server", inflight)
    done = run_server(insts, bufs, max_inflight=inflight)
    check_against_oracle(insts, bufs, done, f"inflight{inflight}")


def test_budget_limits_batches():
    """A budget that holds only a few requests at a time: every request still
    completes with its oracle result, over several batches."""
    insts = serve_like(40, 22, lo=12.0, hi=15.0)
    bufs = upload(insts)
    need = max(l0.l0_batch_workspace_bytes(l0.problem_table([dict(col_idx=b["col"], n=i.n, m=i.m, d=i.d,
                                                                  y=b["y"], alpha=i.alpha, max_iter=100,
                                                                  tol=1e-10, x_out=b["x"])]))
               for i, b in zip(insts, bufs))
    done = run_server(insts, bufs, budget=3 * need + (1 << 16), max_inflight=2)
    check_against_oracle(insts, bufs, done, "budget")
    launches = sorted({c["launch_s"] for c in done.values()})
    assert len(launches) >= 5, launches


def test_request_larger_than_budget_is_refused():
    i = gen.make_instance(5, 200000, 20000, 7, 300)
    b = upload([i])[0]
    with l0.Server(1 << 20) as srv:
        assert srv.submit(0, b["col"], b["y"], i.n, i.m, i.d, b["x"], i.alpha) == l0.L0_ERR_WORKSPACE
        assert srv.submit(1, b["col"], b["y"], i.n, i.m, i.d, b["x"], 0.5) == l0.L0_ERR_ARG
        assert srv.outstanding() == 0


def test_alone_and_in_a_mix_give_the_same_result():
    insts = serve_like(30, 23)
    bufs = upload(insts)
    alone = run_server([insts[7]], [bufs[7]])
    x_alone = bufs[7]["x"].clone()
    mixed = run_server(insts, bufs, order=list(range(29, -1, -1)))
    assert torch.equal(x_alone, bufs[7]["x"])
    for key in ("iters", "outcome", "final_nnz", "support_size", "updates"):
        assert alone[0][key] == mixed[7][key], key
    g = gpu_run(insts[7].n, insts[7].m, insts[7].d, insts[7].col_idx, insts[7].y, insts[7].alpha)
    assert np.array_equal(g["x"], x_alone.cpu().numpy())


def test_large_requests_use_teams():
    """Requests large enough for workgroup teams, among small ones."""
    insts = serve_like(12, 24, lo=10.0, hi=13.0) + [gen.make_instance(77, 1 << 20, 10486, 7, 1500),
                                                    gen.make_instance(78, 1 << 21, 209715, 7, 30000)]
    bufs = upload(insts)
    done = run_server(insts, bufs, budget=4 << 30)
    check_against_oracle(insts, bufs, done, "teams")


def test_column_scaled_requests():
    """Requests on column-scaled matrices (+-1 signals), mixed with unit-column
    ones: each against the oracle."""
    plain = serve_like(16, 25)
    scaled = [gen.make_instance(9000 + q, i.n, i.m, i.d, i.k, kind=gen.VALUES_PM1, scaled=True)
              for q, i in enumerate(serve_like(16, 26))]
    insts = [x for pair in zip(plain, scaled) for x in pair]
    bufs = upload(insts)
    done = run_server(insts, bufs, max_inflight=2)
    check_against_oracle(insts, bufs, done, "scaled")


def test_concurrent_batches_share_the_device():
    """Requests just below the size that goes to the single-instance decoder,
    through four slots at once: batches in flight together are planned within
    a share of the device each, so none of their teams waits for members
    that cannot be scheduled (every result completes and equals the oracle's,
    none is aborted)."""
    rng = np.random.Generator(np.random.PCG64(27))
    insts = []
    for q in range(16):
        n = int(rng.choice([1 << 17, 3 << 16, 1 << 18]))
        m = int(0.01 * n) if q % 2 else int(0.1 * n)
        insts.append(gen.make_instance(27000 + q, n, m, 7, gen.mk_k(m, 0.1)))
    bufs = upload(insts)
    say("concurrent batches", len(insts))
    done = run_server(insts, bufs, budget=8 << 30, max_inflight=4, max_batch=3)
    check_against_oracle(insts, bufs, done, "concurrent")
    assert all(c["outcome"] != l0.L0_DEV_ABORTED for c in done.values())


def test_large_and_small_requests_mixed():
    """Large requests (decoded alone by the single-instance decoder) between
    small batched ones, each result equal to the oracle's."""
    insts = []
    for q in range(10):
        if q % 3 == 0:
            insts.append(gen.make_instance(28000 + q, 1 << 19, 5243, 7, 500))   # 3.7 M indices
        else:
            insts.append(gen.make_instance(28000 + q, 3000 + 500 * q, 300 + 50 * q, 7, 20))
    bufs = upload(insts)
    done = run_server(insts, bufs, budget=4 << 30, max_inflight=2)
    check_against_oracle(insts, bufs, done, "mixed-large")


def test_large_requests_queued_on_the_device():
    """Several large requests in a row, then small ones, through four slots:
    each large request is queued behind the work in flight (stream order, no
    host wait) and runs alone; small batches queued behind a large request
    wait for it.  Every result equals the oracle's."""
    insts = []
    for q in range(12):
        if q < 4 or q % 4 == 0:
            insts.append(gen.make_instance(29000 + q, 1 << 19, 5243 if q % 2 else 52429, 7, 400))
        else:
            insts.append(gen.make_instance(29000 + q, 4000 + 700 * q, 400 + 70 * q, 7, 25))
    bufs = upload(insts)
    say("queued large requests", len(insts))
    done = run_server(insts, bufs, budget=6 << 30, max_inflight=4)
    check_against_oracle(insts, bufs, done, "queued-large")
