"""The phase-transition protocol (Section 5.1's adaptive rho steps over the
24-value delta grid) driven through the GPU's batched decoder for every
curve of the experiments (alpha = 2 and ceil(d/2), the frequency rule at
alpha = 2 and at d/2 (parallel-LDDSR), the shifted rule, banded signals,
the odd degrees 5 to 19, +-1 signals on unit and scaled columns), at a small
n; every decode of the protocol is checked against the oracle bit for bit
(outcome, iterations, x_hat)."""
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest
import torch

import bench
import oracle
import paper_1508_01256_amd as l0
from parity import say

pytestmark = pytest.mark.gpu

GPU_RULES = {"L0DEC": l0.L0_RULE_L0DEC, "MODE": l0.L0_RULE_MODE, "SHIFTED_L0DEC": l0.L0_RULE_SHIFTED_L0DEC}
ORC_RULES = {"L0DEC": oracle.RULE_L0DEC, "MODE": oracle.RULE_MODE, "SHIFTED_L0DEC": oracle.RULE_SHIFTED_L0DEC}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    l0.lib()


def _gpu_decode(insts, alpha, rule, keep):
    dev = "cuda"
    probs = [dict(col_idx=torch.from_numpy(i.col_idx).to(dev), n=i.n, m=i.m, d=i.d,
                  y=torch.from_numpy(i.y).to(dev), alpha=alpha, max_iter=100, tol=1e-10,
                  weights=None if i.w is None else torch.from_numpy(i.w).to(dev)) for i in insts]
    xs, res = l0.decode_batched(probs, rule=GPU_RULES[rule], block_threads=512, words_cap=16384)
    out = []
    for i, x, r in zip(insts, xs, res):
        xh = x.cpu().numpy()
        sc = float(np.max(np.abs(i.vals))) if i.k else 1.0
        out.append((r["outcome"], r["iters"], float(np.max(np.abs(xh - i.x), initial=0.0)) / sc, xh))
    return out


@pytest.mark.parametrize("curve", list(bench.PHASE_CURVES))
def test_protocol_through_the_gpu(curve):
    d, alpha, rule, kind, scaled, band = bench.PHASE_CURVES[curve]
    say("phase protocol on the GPU", curve)
    deltas, points, records, count = bench.phase_protocol(curve, 1024, 2, _gpu_decode, lambda m: None,
                                                          check_every=1, start=0)
    assert len(records) == count > 0

    def check(rec):
        _, di, rho, inst, oc, it, x = rec
        o = oracle.parallel_l0(inst.n, inst.m, inst.d, inst.col_idx, inst.y, alpha, max_iter=100, tol=1e-10,
                               rule=ORC_RULES[rule], w=inst.w)
        same = (o["outcome"], o["iters"]) == (oc, it) and np.array_equal(o["x"].view(np.int64), x.view(np.int64))
        return None if same else (di, rho, oc, it, o["outcome"], o["iters"])

    # the single-threaded oracle releases the interpreter lock: check on a pool
    with ThreadPoolExecutor(8) as pool:
        bad = [b for b in pool.map(check, records) if b is not None]
    assert not bad, (curve, bad[:5])
