"""Host logic of the phase-transition workload (the adaptive protocol of the
paper's experiments, Section 5.1, and the logistic 50% point), run on the
CPU with the oracle standing in for the GPU decoder."""
import numpy as np
import pytest

import bench
import oracle

RULES = {"L0DEC": oracle.RULE_L0DEC, "MODE": oracle.RULE_MODE, "SHIFTED_L0DEC": oracle.RULE_SHIFTED_L0DEC}


def test_delta_grid():
    d = bench.phase_deltas()
    assert len(d) == 24
    assert np.allclose(d[:4], [0.02, 0.04, 0.06, 0.08])
    assert d[4] == 0.1 and abs(d[-1] - 0.99) < 1e-12
    assert np.allclose(np.diff(d[4:]), 89 / 1900)


def test_logistic_midpoint():
    rng = np.random.default_rng(1)
    rhos = np.round(np.arange(0.01, 0.61, 0.01), 2)
    p = 1.0 / (1.0 + np.exp((rhos - 0.3) / 0.02))
    succ = rng.binomial(200, p)
    assert abs(bench.logistic_50(rhos, succ, [200] * rhos.size) - 0.3) < 0.005
    # perfect separation: the midpoint between the last success and the first all-fail point
    r = [0.01, 0.02, 0.03, 0.04]
    assert abs(bench.logistic_50(r, [10, 10, 10, 0], [10] * 4) - 0.035) < 0.002
    assert bench.logistic_50(r, [0, 0, 0, 0], [10] * 4) is None


def _oracle_decode(insts, alpha, rule, keep):
    out = []
    for i, kp in zip(insts, keep):
        o = oracle.parallel_l0(i.n, i.m, i.d, i.col_idx, i.y, alpha, rule=RULES[rule], w=i.w)
        sc = float(np.max(np.abs(i.vals))) if i.k else 1.0
        out.append((o["outcome"], o["iters"], float(np.max(np.abs(o["x"] - i.x), initial=0.0)) / sc,
                    o["x"] if kp else None))
    return out


@pytest.mark.parametrize("curve", ["l0dec-a2", "pm1-a2", "pm1-scaled-a2"])
def test_protocol_small(curve):
    """n = 512: every delta starts at rho = 0.01 and stops after the first
    step with no recovery; points, kept records and counts are consistent."""
    deltas, points, records, count = bench.phase_protocol(curve, 512, 2, _oracle_decode, lambda m: None,
                                                          check_every=7, start=0)
    assert len(points) == 24
    total = 0
    for di, pts in points.items():
        rhos = [r for r, _ in pts]
        assert np.allclose(rhos, 0.01 * np.arange(1, len(rhos) + 1))
        assert all(k > 0 for _, k in pts[:-1])
        assert pts[-1][1] == 0 or pts[-1][0] >= 1.0 - 1e-9
        total += 2 * len(pts)
    assert count == total
    assert len(records) == len(range(0, count, 7))


def test_scaled_pm1_recovers_like_dissociated_signals():
    """The same supports on a scaled A reach higher rho than on unit columns."""
    def star(curve):
        deltas, points, _, _ = bench.phase_protocol(curve, 1024, 2, _oracle_decode, lambda m: None)
        return np.mean([max(r for r, k in pts if k) if any(k for _, k in pts) else 0.0
                        for pts in points.values()])
    assert star("pm1-scaled-a2") > star("pm1-a2") + 0.05
