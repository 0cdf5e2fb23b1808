"""The oracle's samplers and estimators against exact rational enumeration.

For tiny graphs every outcome (v, u, w, r[, t]) of MOSS-4 (Algorithm 1), T-5
(Algorithm 3) and Path-5 (Algorithm 4) is enumerated with its exact probability,
written from the sampler descriptions.  That enumeration checks Theorems 2, 6
and 8 directly; the oracle's seeded samples must then follow the enumerated
distribution (chi-square), its estimates must be unbiased over many seeds, and
its variance formulas must reproduce the exact single-sample variance / K."""
from fractions import Fraction

import numpy as np
import pytest
from scipy import stats

import graphgen as gg
import oracle
import pins
from pins import choose

SAMPLERS = {"moss4": (oracle.MOSS4, 4, pins.PHI4_1), "t5": (oracle.T5, 5, pins.PHI5_1),
            "path5": (oracle.PATH5, 5, pins.PHI5_2)}


@pytest.mark.parametrize("sampler", ["moss4", "t5", "path5"])
@pytest.mark.parametrize("g", [gg.gnp(9, 0.5, 21), gg.gnp(10, 0.4, 22), gg.wheel(6)], ids=lambda g: g.name)
def test_sampling_weight_theorems(sampler, g):
    """Theorems 2, 6, 8: a CIS of class i is drawn with probability 2 phi_i / Gamma,
    and the outcome probabilities sum to one."""
    _, k, phi = SAMPLERS[sampler]
    by_class, by_set, G, dist = pins.class_distribution(g, sampler)
    assert sum(dist.values()) == 1
    adjsets = g.adjacency_sets()
    reachable = set()
    for s, p in by_set.items():
        c = pins.class_of_nodes(adjsets, tuple(s))
        assert p == Fraction(2 * phi[c], G), (s, c, p)
        reachable.add(s)
    # every CIS whose class has phi > 0 is reachable
    import itertools
    for nodes in itertools.combinations(range(g.n), k):
        c = pins.class_of_nodes(adjsets, nodes)
        if c and phi[c] > 0:
            assert frozenset(nodes) in reachable


@pytest.mark.parametrize("sampler,g,n", [
    ("moss4", gg.gnp(7, 0.5, 5), 200_000),
    ("t5", gg.gnp(6, 0.6, 6), 300_000),
    ("path5", gg.gnp(6, 0.55, 7), 300_000),
])
def test_contract_sampler_follows_exact_distribution(sampler, g, n):
    """The oracle's Philox-driven draws (bounded map, inverse-CDF pick, skip rules)
    realise the paper's distribution: chi-square over all outcomes."""
    sid, k, _ = SAMPLERS[sampler]
    _, _, _, dist = pins.class_distribution(g, sampler)
    og = oracle.Graph(g)
    counts = {}
    for i in range(n):
        _, nodes = og.sample(sid, 99, i)
        key = tuple(nodes[:k])
        counts[key] = counts.get(key, 0) + 1
    assert set(counts) <= set(dist)
    keys = sorted(dist)
    obs = np.array([counts.get(t, 0) for t in keys], dtype=np.float64)
    exp = np.array([float(dist[t]) * n for t in keys])
    assert exp.min() >= 5.0
    chi2 = float(((obs - exp) ** 2 / exp).sum())
    p = stats.chi2.sf(chi2, len(keys) - 1)
    assert p > 1e-4, (chi2, len(keys), p)


def test_class_returned_by_sample_matches_nodes():
    g = gg.gnp(12, 0.4, 8)
    og = oracle.Graph(g)
    adjsets = g.adjacency_sets()
    for sid, k in ((oracle.MOSS4, 4), (oracle.T5, 5), (oracle.PATH5, 5)):
        for i in range(300):
            c, nodes = og.sample(sid, 3, i)
            nd = nodes[:k]
            if c == 0:
                assert len(set(nd)) < k
            else:
                assert len(set(nd)) == k
                assert c == pins.class_of_nodes(adjsets, tuple(nd))


@pytest.mark.parametrize("threads", [2, 3, 8])
def test_threads_and_ranges_do_not_change_hits(threads):
    g = gg.gnp(40, 0.2, 10)
    og = oracle.Graph(g)
    for sid in (oracle.MOSS4, oracle.T5, oracle.PATH5):
        a = og.run(sid, 5, 0, 20_000, 1)
        b = og.run(sid, 5, 0, 20_000, threads)
        c = og.run(sid, 5, 0, 7_777, 1) + og.run(sid, 5, 7_777, 20_000, 1)
        np.testing.assert_array_equal(a, b)
        np.testing.assert_array_equal(a, c)
        assert int(a.sum()) == 20_000


def test_per_run_invariants():
    """sum m = K; sum_i phi^(1)_i n_i = (K - m_0) Gamma / (2K) for MOSS-4 (every
    accepted sample contributes Gamma / (2 phi_i) * phi_i / K)."""
    g = gg.chung_lu(500, 3000, 2.3, 60, 3)
    og = oracle.Graph(g)
    t = og.totals()
    for seed in (1, 2, 3):
        r = og.estimate(4, 50_000, seed)
        m = r.hits[0]
        assert int(m[:7].sum()) == 50_000
        lhs = sum(pins.PHI4_1[i] * r.estimate[i - 1] for i in range(1, 7))
        rhs = (50_000 - int(m[0])) * t["gamma"] / (2 * 50_000)
        assert abs(lhs - rhs) <= 1e-12 * rhs
        r5 = og.estimate(5, 40_001, seed)
        assert r5.K == [20_001, 20_000]
        assert int(r5.hits[0].sum()) == 20_001 and int(r5.hits[1].sum()) == 20_000


def _x_moments(by_class, phi, G, weights):
    """Mean and variance of one sample of sum_i weights_i 1{class i} / p_i."""
    mean = Fraction(0)
    sq = Fraction(0)
    for c, p in by_class.items():
        if c == 0 or phi[c] == 0 or c not in weights:
            continue
        x = weights[c] / Fraction(2 * phi[c], G)
        mean += p * x
        sq += p * x * x
    return mean, sq - mean * mean


def _close(a, b, rel=1e-12, abs_=1e-9):
    return abs(float(a) - float(b)) <= rel * max(abs(float(b)), abs(float(a))) + abs_


@pytest.mark.parametrize("g", [gg.gnp(11, 0.45, 2), gg.gnp(9, 0.6, 3)], ids=lambda g: g.name)
def test_moss4_variances_match_enumeration(g):
    """Theorem 3 as the oracle evaluates it, at hits equal to their expectations,
    against Var(one sample)/K from the exact enumeration."""
    by_class, _, G, _ = pins.class_distribution(g, "moss4")
    n = pins.brute_counts(g, 4)
    K = G * 3
    hits = [int(by_class.get(c, 0) * K) for c in range(7)]
    assert all(by_class.get(c, 0) * K == hits[c] for c in range(7))
    t = oracle.Graph(g).totals()
    est, var = oracle.finals4(K, hits, t["gamma"], t["lambda3"])
    for i in (1, 3, 4, 5, 6):
        assert _close(est[i - 1], n[i])
        _, v1 = _x_moments(by_class, pins.PHI4_1, G, {i: 1})
        assert _close(var[i - 1], v1 / K), (i, var[i - 1], float(v1 / K))
    assert _close(est[1], n[2])
    _, v2 = _x_moments(by_class, pins.PHI4_1, G, {4: 1, 5: 2, 6: 4})
    assert _close(var[1], v2 / K, rel=1e-9, abs_=1e-6 * float(t["lambda3"]))


@pytest.mark.parametrize("mix", [oracle.MIX_POOLED, oracle.MIX_PAPER])
def test_moss5_variances_match_enumeration(mix):
    """Theorems 7, 9 and 10 (and the pooled reading of the mix weights) at hits equal
    to their expectations, against exact single-sample moments / K_l."""
    g = gg.gnp(10, 0.5, 12)
    d1, _, G1, _ = pins.class_distribution(g, "t5")
    d2, _, G2, _ = pins.class_distribution(g, "path5")
    eta = pins.brute_counts(g, 5)
    K1, K2 = G1 * 2, G2 * 3
    h1 = [int(d1.get(c, 0) * K1) for c in range(22)]
    h2 = [int(d2.get(c, 0) * K2) for c in range(22)]
    assert all(d1.get(c, 0) * K1 == h1[c] and d2.get(c, 0) * K2 == h2[c] for c in range(22))
    t = oracle.Graph(g).totals()
    est, var, cov = oracle.finals5(K1, K2, h1, h2, t["gamma1"], t["gamma2"], t["lambda4"], mix)
    lam = {}
    for i in range(1, 22):
        if i == 2:
            continue
        p1 = Fraction(2 * pins.PHI5_1[i], G1)
        p2 = Fraction(2 * pins.PHI5_2[i], G2)
        _, v1 = _x_moments(d1, pins.PHI5_1, G1, {i: 1})
        _, v2 = _x_moments(d2, pins.PHI5_2, G2, {i: 1})
        V1, V2 = v1 / K1, v2 / K2
        if mix == oracle.MIX_POOLED or p1 == 0 or p2 == 0 or V1 + V2 == 0:
            l1 = K1 * p1 / (K1 * p1 + K2 * p2)
            want = l1 * l1 * V1 + (1 - l1) ** 2 * V2
        else:
            l1 = V2 / (V1 + V2)
            want = V1 * V2 / (V1 + V2)
        lam[i] = l1
        assert _close(est[i - 1], eta[i]), (i, est[i - 1], eta[i])
        assert _close(var[i - 1], want), (i, var[i - 1], float(want))
    # eta_2 and its variance: Var(sum_{Omega3*} phi3_i eta_i) from the two samplers
    assert _close(est[1], eta[2], abs_=1e-6)
    w1 = {i: pins.PHI5_3[i] * lam[i] for i in lam if pins.PHI5_3[i]}
    w2 = {i: pins.PHI5_3[i] * (1 - lam[i]) for i in lam if pins.PHI5_3[i]}
    _, a = _x_moments(d1, pins.PHI5_1, G1, w1)
    _, b = _x_moments(d2, pins.PHI5_2, G2, w2)
    assert _close(var[1], a / K1 + b / K2, rel=1e-9, abs_=1e-6)


def test_moss4_unbiased_over_seeds():
    """Mean of 300 independent estimates within 5 standard errors of the truth,
    the standard error taken from Theorem 3 at the true counts."""
    g = gg.gnp(12, 0.4, 31)
    og = oracle.Graph(g)
    n = pins.brute_counts(g, 4)
    t = og.totals()
    K, R = 3000, 300
    est = np.array([og.estimate(4, K, s).estimate for s in range(1, R + 1)])
    for i in (1, 3, 4, 5, 6):
        p = 2 * pins.PHI4_1[i] / t["gamma"]
        sd = np.sqrt(n[i] / K * (1 / p - n[i]) / R)
        assert abs(est[:, i - 1].mean() - n[i]) <= 5 * sd + 1e-9, (i, est[:, i - 1].mean(), n[i], sd)
    s = n[4] + 2 * n[5] + 4 * n[6]
    p4, p5, p6 = (2 * pins.PHI4_1[j] / t["gamma"] for j in (4, 5, 6))
    sd2 = np.sqrt((n[4] / p4 + 4 * n[5] / p5 + 16 * n[6] / p6 - s * s) / K / R)
    assert abs(est[:, 1].mean() - n[2]) <= 5 * sd2


def test_moss5_unbiased_over_seeds():
    g = gg.gnp(11, 0.45, 32)
    og = oracle.Graph(g)
    eta = pins.brute_counts(g, 5)
    R, K = 200, 6000
    res = [og.estimate(5, K, s) for s in range(1, R + 1)]
    est = np.array([r.estimate for r in res])
    var = np.array([r.variance for r in res])
    for i in range(1, 22):
        if eta[i] == 0:
            assert np.all(est[:, i - 1] == 0) or i == 2
            continue
        sd = np.sqrt(var[:, i - 1].mean() / R)
        assert abs(est[:, i - 1].mean() - eta[i]) <= 5 * sd + 1e-6 * eta[i], (i, est[:, i - 1].mean(), eta[i])


@pytest.mark.parametrize("seed", [1, 2, 77])
def test_zero_variance_closed_forms(seed):
    """Graphs on which every accepted sample has the same class: the estimate is the
    closed form for every seed."""
    K = 5000
    cases4 = [(gg.path(9), {1: 6}), (gg.cycle(9), {1: 9}), (gg.cycle(5), {1: 5}), (gg.cycle(4), {3: 1}),
              (gg.complete_bipartite(3, 4), {3: 18, 2: 16}), (gg.star(6), {2: 20})]
    for g, want in cases4:
        r = oracle.Graph(g).estimate(4, K, seed)
        for i in range(1, 7):
            assert _close(r.estimate[i - 1], want.get(i, 0)), (g.name, i, r.estimate)
    cases5 = [(gg.cycle(9), {1: 9}), (gg.path(10), {1: 6}), (gg.cycle(5), {6: 1}), (gg.star(7), {2: choose(7, 4)})]
    for g, want in cases5:
        r = oracle.Graph(g).estimate(5, K, seed)
        for i in range(1, 22):
            assert _close(r.estimate[i - 1], want.get(i, 0)), (g.name, i, r.estimate)
