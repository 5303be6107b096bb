"""Seeded random configurations against the oracle: n, m, d, k, alpha, the
scoring rule, tol, max_iter, the value kind and column scaling are drawn per
case, so shapes no hand-written case chose (tile and chunk tails, both index
widths and word modes, any degree from 2 to 20, alpha anywhere in (1, d],
tol 0) meet the GPU path.  Each case is decoded alone (l0_decode_ex) and, per
rule, all cases of a chunk in one l0_decode_batched call; every result is
compared with the oracle bit for bit."""
import numpy as np
import pytest
import torch

import gen
import paper_1508_01256_amd as l0
from parity import assert_batched_parity, assert_parity, batched_run, oracle_run, run_both, say

pytestmark = pytest.mark.gpu

TOLS = (0.0, 1e-12, 1e-10, 1e-6)
CHUNKS, PER_CHUNK = 8, 16


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    l0.lib()


def draw(q):
    rng = np.random.default_rng(70000 + q)
    d = int(rng.integers(2, 21))
    m = int(rng.integers(max(d, 8), 100000))
    n = int(rng.integers(1, 200000))
    k = int(rng.integers(0, max(1, min(n, m // 3))))
    return dict(seed=71000 + q, n=n, m=m, d=d, k=k, alpha=float(rng.uniform(1.0, d)) or float(d),
                rule=int(rng.integers(0, 4)), tol=TOLS[int(rng.integers(0, len(TOLS)))],
                max_iter=int(rng.integers(0, 40)),
                kind=gen.VALUES_PM1 if rng.random() < 0.25 else gen.VALUES_NORMAL,
                scaled=bool(rng.random() < 0.25))


def instance(c):
    alpha = c["alpha"] if c["alpha"] > 1.0 else float(c["d"])
    return gen.make_instance(c["seed"], c["n"], c["m"], c["d"], c["k"], alpha=alpha, kind=c["kind"],
                             scaled=c["scaled"])


@pytest.mark.parametrize("chunk", range(CHUNKS))
def test_random_configurations_alone(chunk):
    for q in range(chunk * PER_CHUNK, (chunk + 1) * PER_CHUNK):
        c = draw(q)
        inst = instance(c)
        say("random", q, c)
        g, o = run_both(inst, rule=c["rule"], tol=c["tol"], max_iter=c["max_iter"])
        assert_parity(g, o, label=f"random {q} {c}")


@pytest.mark.parametrize("chunk", range(CHUNKS))
def test_random_configurations_batched(chunk):
    cases = [draw(q) for q in range(chunk * PER_CHUNK, (chunk + 1) * PER_CHUNK)]
    for rule in range(4):
        group = [c for c in cases if c["rule"] == rule]
        if not group:
            continue
        insts = [instance(c) for c in group]
        say("random batched", chunk, rule, len(insts))
        res = batched_run(insts, max_iters=[c["max_iter"] for c in group], rule=rule)
        for c, i, b in zip(group, insts, res):
            o = oracle_run(i.n, i.m, i.d, i.col_idx, i.y, i.alpha, max_iter=c["max_iter"], rule=rule, w=i.w)
            assert_batched_parity(b, o, label=f"random batched {c}")
