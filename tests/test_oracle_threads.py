"""The oracle's OpenMP build (the vote's columns split over threads) against
its plain single-threaded build: the same source, so every output must be
the same bit for bit, for every rule, with and without column weights."""
import numpy as np
import pytest

import gen
import oracle


@pytest.mark.parametrize("rule", [oracle.RULE_L0DEC, oracle.RULE_MODE, oracle.RULE_SHIFTED_L0DEC,
                                  oracle.RULE_SHIFTED_MODE])
@pytest.mark.parametrize("n,m,d,k,scaled", [(20000, 2000, 7, 150, False), (30001, 3000, 5, 500, True),
                                            (4096, 512, 9, 60, False)])
def test_threaded_oracle_is_bitwise_the_plain_one(rule, n, m, d, k, scaled):
    inst = gen.make_instance(6100 + n + rule, n, m, d, k, scaled=scaled)
    for alpha in (2.0, inst.alpha):
        a = oracle.parallel_l0(inst.n, inst.m, inst.d, inst.col_idx, inst.y, alpha, rule=rule, w=inst.w)
        b = oracle.parallel_l0(inst.n, inst.m, inst.d, inst.col_idx, inst.y, alpha, rule=rule, w=inst.w,
                               threads=True)
        for key in ("iters", "outcome", "passes"):
            assert a[key] == b[key], key
        assert a["trace"].tolist() == b["trace"].tolist()
        assert a["tsize"].tolist() == b["tsize"].tolist()
        assert np.array_equal(a["x"].view(np.int64), b["x"].view(np.int64))


def test_threaded_oracle_rejects_what_the_plain_one_rejects():
    inst = gen.make_instance(6200, 300, 40, 5, 4)
    col = inst.col_idx.copy()
    col[7] = col[6]
    with pytest.raises(ValueError):
        oracle.parallel_l0(inst.n, inst.m, inst.d, col, inst.y, 3, threads=True)
