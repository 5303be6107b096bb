"""Single-instance decodes whose rows sit in hundreds of support lists: tiny
instances of the phase-transition sweep with m = 10-13 rows and d = 9 (every
row in most columns), where the residual of a touched row merges hundreds of
new list entries per iteration.  Such rows are merged by the whole workgroup
(an entry's rank among the list's distinct column ids) instead of one thread;
the decode must stay bitwise equal to the oracle, also with the list merged
over many iterations and on a column-scaled A."""
import numpy as np
import pytest
import torch

import gen
import paper_1508_01256_amd as l0
from parity import assert_parity, oracle_run, run_both, say

pytestmark = pytest.mark.gpu


def tiny_sweep_instances():
    ps = [p for p in gen.sweep_params(4096) if p["m"] <= 13 and p["d"] == 9]
    return ps[:12]


def one_shot(inst, ws, res):
    col = torch.from_numpy(inst.col_idx).cuda()
    y = torch.from_numpy(inst.y).cuda()
    x = torch.empty(inst.n, dtype=torch.float64, device="cuda")
    assert l0.l0_decode_ex(col, inst.n, inst.m, inst.d, y, inst.alpha, 100, 1e-10, x, None, res, ws) == l0.L0_OK
    torch.cuda.synchronize()
    return x.cpu().numpy(), l0.results_list(res.view(1, 3))[0]


def test_tiny_instances_with_long_lists():
    ps = tiny_sweep_instances()
    assert len(ps) >= 6
    insts = [gen.make_instance(p["seed"], p["n"], p["m"], p["d"], p["k"]) for p in ps]
    ws = torch.empty(max(l0.l0_workspace_bytes(i.n, i.m, i.d, 100) for i in insts), dtype=torch.uint8,
                     device="cuda")
    res = l0.new_result()
    for i in insts:
        say("long lists", i.n, i.m, i.d, i.k)
        o = oracle_run(i.n, i.m, i.d, i.col_idx, i.y, i.alpha)
        x, r = one_shot(i, ws, res)
        assert (r["outcome"], r["iters"]) == (o["outcome"], o["iters"]), (i.n, i.m)
        assert np.array_equal(x.view(np.int64), o["x"].view(np.int64)), (i.n, i.m)


@pytest.mark.parametrize("q", [0, 3])
def test_tiny_instance_with_long_lists_scaled(q):
    p = tiny_sweep_instances()[q]
    inst = gen.make_instance(p["seed"], p["n"], p["m"], p["d"], p["k"], scaled=True)
    say("long lists, scaled", inst.n, inst.m)
    g, o = run_both(inst)
    assert_parity(g, o, label=f"scaled tiny {inst.n} {inst.m}")
