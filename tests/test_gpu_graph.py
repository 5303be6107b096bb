"""A solve on a prepared matrix enqueues only kernels (the control-block fill
and the persistent solve), so a caller can capture it in a HIP graph and
replay it.  Each replay is checked against the eager solve, with eager work
and synchronisations between replays, and a replay on a new y (copied into
the captured buffer) against the oracle."""
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


def test_solve_replays_in_a_hip_graph():
    inst = gen.make_instance(9800, 200000, 20000, 7, 1500)
    other = gen.make_instance(9801, 200000, 20000, 7, 1200)
    y_other = gen.measure(inst.n, inst.m, inst.d, inst.col_idx, other.supp, other.vals)
    col = to_dev(inst.col_idx, torch.int32)
    y = to_dev(inst.y, torch.float64)
    with l0.Matrix(col, inst.n, inst.m, inst.d) as A:
        ws = A.workspace(100)
        x = torch.empty(inst.n, dtype=torch.float64, device="cuda")
        res = l0.new_result()
        A.solve_async(y, 4, x=x, res=res, workspace=ws)
        torch.cuda.synchronize()
        x_ref, res_ref = x.clone(), res.clone()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            A.solve_async(y, 4, x=x, res=res, workspace=ws)
        torch.cuda.synchronize()
        say("graph captured")
        for rep in range(4):
            x.fill_(7.0)
            res.zero_()
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            assert torch.equal(res, res_ref), rep
            assert torch.equal(x, x_ref), rep
        y.copy_(torch.from_numpy(y_other))
        g.replay()
        torch.cuda.synchronize()
        o = oracle_run(inst.n, inst.m, inst.d, inst.col_idx, y_other, 4)
        r = l0.results_list(res.view(1, 3))[0]
        assert r["iters"] == o["iters"] and r["outcome"] == o["outcome"]
        assert np.array_equal(x.cpu().numpy(), o["x"])
        del g
