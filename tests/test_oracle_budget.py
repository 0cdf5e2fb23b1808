"""The oracle's budget planner and concentrations (closing remark of Section 4.1.2 with
Theorem 1; the concentrations of Section 6.2).

Pins: the two-sided normal quantile against scipy's; the planned budget reaches the
requested failure probability when the estimator is run many times on a graph with
exact counts by enumeration (and a quarter of it does not); closed forms on graphs
where every sample has one class."""
import numpy as np
import pytest
from scipy import stats

import graphgen as gg
import oracle
import pins


@pytest.mark.parametrize("delta", [0.5, 0.2, 0.1, 0.05, 0.01, 1e-4, 1e-9])
def test_normal_quantile_matches_scipy(delta):
    z = oracle.normal_two_sided(delta)
    assert abs(z - stats.norm.isf(delta / 2)) <= 1e-12 * z


def _failure_rate(og, k, K, truth, motif, eps, R, seed0, with_min=False):
    fails = 0
    for s in range(seed0, seed0 + R):
        r = og.estimate4min(K, s) if with_min else og.estimate(k, K, s, threads=4)
        if abs(r.estimate[motif - 1] - truth) > eps * truth:
            fails += 1
    return fails / R


@pytest.mark.parametrize("k,motif,with_min", [(4, 1, False), (4, 5, False), (5, 1, False), (4, 3, True)])
def test_planned_budget_reaches_target(k, motif, with_min):
    """P(|est - n| > eps n) at the planned budget is delta within sampling error (R runs),
    and clearly above delta at a quarter of the budget."""
    g = gg.gnp(12, 0.45, 31)
    og = oracle.Graph(g)
    truth = pins.brute_counts(g, k)[motif]
    assert truth > 0
    eps, delta, R = 0.05, 0.1, 400
    pilot = og.estimate4min(2_000_000, 77) if with_min else og.estimate(k, 2_000_000, 77, threads=8)
    budget, K = oracle.plan_budget(pilot, eps, delta, 1 << (motif - 1))
    assert K == budget[motif - 1] > 0
    rate = _failure_rate(og, k, K, truth, motif, eps, R, 1000, with_min)
    sd = np.sqrt(delta * (1 - delta) / R)
    assert abs(rate - delta) <= 4 * sd + 0.02, (K, rate)
    low = _failure_rate(og, k, max(2, K // 4), truth, motif, eps, R // 2, 5000, with_min)
    assert low >= 2.5 * delta, (K, low)


def test_budget_scales_with_precision():
    """Halving eps quadruples each budget (up to the rounding up); a smaller delta needs
    more samples."""
    og = oracle.Graph(gg.chung_lu(400, 3000, 2.3, 60, 5))
    pilot = og.estimate(4, 200_000, 3, threads=4)
    b1, _ = oracle.plan_budget(pilot, 0.1, 0.05)
    b2, _ = oracle.plan_budget(pilot, 0.05, 0.05)
    b3, _ = oracle.plan_budget(pilot, 0.1, 0.001)
    for i in range(6):
        if b1[i] > 10:
            assert 4 * b1[i] - 4 <= b2[i] <= 4 * b1[i]
            assert b3[i] > b1[i]


def test_zero_variance_and_unplannable():
    """The 4-cycle's only motif has zero variance: budget 1; motifs estimated at 0 get 0,
    and a mask of only such motifs leaves the pilot's size as the final budget."""
    og = oracle.Graph(gg.cycle(4))
    pilot = og.estimate(4, 1000, 1)
    b, K = oracle.plan_budget(pilot, 0.01, 0.01)
    assert list(b) == [0, 0, 1, 0, 0, 0] and K == 1
    r, Kf = og.estimate_to_precision(4, 0.01, 0.01, 1 << 5, 1234, 1, 10**9, 2)
    assert Kf == 1234 and r.K[0] == 1234
    r, Kf = og.estimate_to_precision(4, 0.01, 0.01, 1 << 2, 1234, 1, 10**9, 2)
    assert Kf == 1 and r.K[0] == 1 and r.estimate[2] == 1.0


def test_estimate_to_precision_is_pilot_then_plan():
    og = oracle.Graph(gg.chung_lu(400, 3000, 2.3, 60, 5))
    for k, with_min in ((4, False), (5, False), (4, True)):
        pilot = og.estimate4min(50_000, 9) if with_min else og.estimate(k, 50_000, 9)
        _, K = oracle.plan_budget(pilot, 0.02, 0.05, 0b101)
        r, Kf = og.estimate_to_precision(k, 0.02, 0.05, 0b101, 50_000, 9, 10**12, 4, with_min)
        assert Kf == K
        want = og.estimate4min(K, 4) if with_min else og.estimate(k, K, 4)
        np.testing.assert_array_equal(r.hits, want.hits)
        _, Kc = og.estimate_to_precision(k, 0.02, 0.05, 0b101, 50_000, 9, K // 3, 4, with_min)
        assert Kc == K // 3


def _result(estimates):
    r = oracle._Result()
    r.k = 5 if len(estimates) == 21 else 4
    r.n_motifs = len(estimates)
    for i, e in enumerate(estimates):
        r.estimate[i] = e
    return oracle.Result(r)


def test_concentrations():
    """omega_i = eta_i / sum_j eta_j: exact 4-node counts of the C1 graph, exact 5-node
    counts of a small graph, and graphs whose CISes are all of one class."""
    import json
    import os
    d = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "exact_c1.json")))
    eta = pins.brute_counts(gg.gnp(10, 0.5, 4), 5)[1:22]
    for counts in (d["n4"], eta):
        om = oracle.concentrations(_result([float(c) for c in counts]))
        np.testing.assert_allclose(om, np.array(counts, float) / sum(counts), rtol=1e-15)
        assert abs(om.sum() - 1.0) <= 1e-12
    for g, k, i in ((gg.cycle(9), 5, 1), (gg.star(7), 5, 2), (gg.cycle(4), 4, 3)):
        om = oracle.concentrations(oracle.Graph(g).estimate(k, 10_000, 1))
        want = np.zeros(len(om))
        want[i - 1] = 1.0
        np.testing.assert_array_equal(om, want)
    assert not oracle.concentrations(_result([0.0] * 6)).any()
