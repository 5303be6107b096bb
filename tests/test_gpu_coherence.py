"""Back-to-back one-shot decodes of many small instances, one workspace
reused, each bitwise against the oracle.  The persistent solve kernel's
grid barrier must make every store before it visible to every load after it
across the XCDs' separate L2 caches and the CUs' L1 caches; a barrier whose
L1 invalidation did not take effect decoded about 0.2% of such instances
wrongly (a few x_hat entries off, or another iteration count), and only
instances small enough for their index loads to be cached showed it.  The
instances are those of the phase-transition sweep with d = 5 and
n >= 40000, run three times over."""
import numpy as np
import pytest
import torch

import gen
import paper_1508_01256_amd as l0
from parity import oracle_run, say

pytestmark = pytest.mark.gpu


def test_small_decodes_back_to_back_match_the_oracle():
    params = [p for p in gen.sweep_params(4096) if p["d"] == 5 and p["n"] >= 40000][:160]
    insts = [gen.make_instance(p["seed"], p["n"], p["m"], p["d"], p["k"]) for p in params]
    say("coherence: instances", len(insts))
    oracles = [oracle_run(i.n, i.m, i.d, i.col_idx, i.y, i.alpha) for i in insts]
    cols = [torch.from_numpy(i.col_idx).cuda() for i in insts]
    ys = [torch.from_numpy(i.y).cuda() for i in insts]
    ws = torch.empty(max(l0.l0_workspace_bytes(i.n, i.m, i.d, 100) for i in insts), dtype=torch.uint8,
                     device="cuda")
    res = l0.new_result()
    wrong = []
    for rep in range(3):
        for q, (i, o) in enumerate(zip(insts, oracles)):
            x = torch.empty(i.n, dtype=torch.float64, device="cuda")
            assert l0.l0_decode_ex(cols[q], i.n, i.m, i.d, ys[q], i.alpha, 100, 1e-10, x, None, res, ws) == l0.L0_OK
            torch.cuda.synchronize()
            r = l0.results_list(res.view(1, 3))[0]
            same = (r["outcome"] == o["outcome"] and r["iters"] == o["iters"]
                    and np.array_equal(x.cpu().numpy().view(np.int64), o["x"].view(np.int64)))
            if not same:
                wrong.append((rep, q, i.n, i.m))
    assert not wrong, f"{len(wrong)} decodes differ from the oracle: {wrong[:8]}"
