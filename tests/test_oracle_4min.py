"""The oracle's MOSS-4Min (Section 4.2, Algorithm 2) against exact enumeration.

The pins here are written from the sampler's five steps and Table 1's definitions in
pure Python (tests/pins.py), not from the oracle: the rank tables counted pair by pair,
every outcome (v, u, w, r) with its exact probability, the number of ordered draws
c(s) that reach a node set by permutations, and exact counts by trying every 4-subset.

They also fix the reading this code takes of Theorem 4: a 4-cycle is reached by exactly
2 ordered draws and a 4-clique by 6, as the theorem states, but a diamond by 2, 4 or 6
depending on how its nodes are ordered, so the estimate weights each sample by its own
c(s); with the theorem's constant 2 the diamond estimate is biased (shown exactly below).
"""
import itertools
from fractions import Fraction

import numpy as np
import pytest
from scipy import stats

import graphgen as gg
import oracle
import pins

GRAPHS = [gg.gnp(9, 0.55, 9), gg.gnp(9, 0.55, 8), gg.gnp(10, 0.5, 3), gg.wheel(6), gg.complete(6),
          gg.cycle(7), gg.complete_bipartite(3, 4)]


def _class_and_ways(g):
    """{frozenset: (class, c(s))} over all 4-subsets of classes 3, 5, 6."""
    adj = g.adjacency_sets()
    d = [len(a) for a in adj]
    out = {}
    for s in itertools.combinations(range(g.n), 4):
        c = pins.class_of_nodes(adj, s)
        if c in (3, 5, 6):
            out[frozenset(s)] = (c, pins.ways(adj, d, s))
    return out


@pytest.mark.parametrize("g", GRAPHS, ids=lambda g: g.name)
def test_min_tables_match_definitions(g):
    """d_{v,x}, d_{x,v}, the descending rows, check-Gamma_v, its prefix and the row
    prefixes of d_{v,x} d_{x,v} (Section 4.2.1, Table 1)."""
    A, d, dvx, gmin, desc = pins.moss4min_weights(g)
    og = oracle.Graph(g)
    rank = og.table(oracle.TAB_RANK)
    mirror = og.table(oracle.TAB_RANK_MIRROR)
    col_rank = og.table(oracle.TAB_COL_RANK)
    acc_check = og.table(oracle.TAB_ACC_CHECK)
    rp = g.row_ptr
    for v in range(g.n):
        run = 0
        for j, x in enumerate(A[v]):
            e = rp[v] + j
            assert rank[e] == dvx[(v, x)] and mirror[e] == dvx[(x, v)]
            run += dvx[(v, x)] * dvx[(x, v)]
            assert acc_check[e] == run
        assert list(col_rank[rp[v]:rp[v + 1]]) == desc[v]
    assert list(og.table(oracle.TAB_GAMMA_MIN)) == gmin
    assert list(og.table(oracle.TAB_ACC_GAMMA_MIN)) == list(itertools.accumulate(gmin))
    assert og.totals()["gamma_min"] == sum(gmin)


@pytest.mark.parametrize("g", GRAPHS[:4], ids=lambda g: g.name)
def test_gamma_min_counts_ordered_walks(g):
    """check-Gamma is the number of node walks w-v-u-r with w in N_v above u and r in N_u
    above v (w = r allowed): the product form of Table 1 against a direct count."""
    adj = g.adjacency_sets()
    d = [len(a) for a in adj]
    walks = sum(1 for v in range(g.n) for u in adj[v] for w in adj[v] for r in adj[u]
                if pins.above(d, w, u) and pins.above(d, r, v))
    assert oracle.Graph(g).totals()["gamma_min"] == walks


@pytest.mark.parametrize("g", GRAPHS[:4], ids=lambda g: g.name)
def test_every_draw_has_probability_one_over_gamma_min(g):
    """The five steps multiply to 1/check-Gamma for every possible (v, u, w, r)."""
    dist, G = pins.moss4min_distribution(g)
    assert sum(dist.values()) == 1
    assert set(dist.values()) == {Fraction(1, G)}


def test_reach_counts_by_motif():
    """Over every order of four nodes: a 4-cycle is reached by 2 ordered draws and a
    4-clique by 6 (Theorem 4); a diamond by 2, 4 or 6; the oracle's count agrees with a
    count by permutations."""
    shapes = {3: [(0, 1), (1, 2), (2, 3), (3, 0)], 6: [(a, b) for a in range(4) for b in range(a + 1, 4)],
              5: [(0, 1), (0, 2), (0, 3), (1, 2), (2, 3)]}
    for cls, edges in shapes.items():
        adj = np.zeros((4, 4), np.uint8)
        for a, b in edges:
            adj[a, b] = adj[b, a] = 1
        adjsets = [set(np.nonzero(adj[i])[0].tolist()) for i in range(4)]
        seen = set()
        for perm in itertools.permutations(range(4)):
            keys = [10 + perm[i] for i in range(4)]  # any strict order of the four nodes
            c = oracle.ways_of(adj, keys)
            d_fake = {i: keys[i] for i in range(4)}  # above() compares d first: keys as degrees
            assert c == pins.ways(adjsets, d_fake, range(4))
            seen.add(c)
        want = {3: {2}, 6: {6}, 5: {2, 4, 6}}[cls]
        assert seen == want, (cls, seen)


@pytest.mark.parametrize("g", GRAPHS[:3], ids=lambda g: g.name)
def test_cis_probability_is_reach_over_gamma_min(g):
    """Summing the exact outcome probabilities per node set gives c(s)/check-Gamma for
    every CIS of classes 3, 5 and 6, and every such CIS is reachable."""
    dist, G = pins.moss4min_distribution(g)
    adj = g.adjacency_sets()
    by_set = {}
    for (v, u, w, r), p in dist.items():
        if r != w:
            s = frozenset((v, u, w, r))
            by_set[s] = by_set.get(s, 0) + p
    for s, (c, ways) in _class_and_ways(g).items():
        assert by_set.get(s, 0) == Fraction(ways, G), (sorted(s), c, ways)
        assert ways >= 2
    for s, p in by_set.items():
        if pins.class_of_nodes(adj, tuple(s)) in (3, 5, 6):
            assert s in _class_and_ways(g)


def test_theorem4_diamond_constant_is_biased():
    """With p_5 = 2/check-Gamma (Theorem 4 as printed) the expected diamond estimate
    exceeds n_5 on a graph whose diamonds are reached 4 or 6 ways; with each sample's
    own c(s) it equals n_5 exactly, and the 4-cycle and 4-clique constants are exact."""
    g = gg.gnp(9, 0.55, 9)
    dist, G = pins.moss4min_distribution(g)
    adj = g.adjacency_sets()
    d = [len(a) for a in adj]
    n = pins.brute_counts(g, 4)
    printed = {3: Fraction(2, G), 5: Fraction(2, G), 6: Fraction(6, G)}
    e_printed = {3: 0, 5: 0, 6: 0}
    e_ways = {3: 0, 5: 0, 6: 0}
    for (v, u, w, r), p in dist.items():
        if r == w:
            continue
        c = pins.class_of_nodes(adj, (v, u, w, r))
        if c in e_ways:
            e_printed[c] += p / printed[c]
            e_ways[c] += p * Fraction(G, pins.ways(adj, d, (v, u, w, r)))
    for c in (3, 5, 6):
        assert e_ways[c] == n[c]
    assert e_printed[3] == n[3] and e_printed[6] == n[6]
    assert e_printed[5] > n[5]


@pytest.mark.parametrize("g,n", [(gg.gnp(9, 0.55, 9), 300_000), (gg.wheel(6), 100_000)], ids=["gnp9", "wheel6"])
def test_oracle_draws_follow_exact_distribution(g, n):
    """The oracle's Philox-driven MOSS-4Min draws realise the five steps' distribution
    (chi-square over every outcome)."""
    dist, _ = pins.moss4min_distribution(g)
    og = oracle.Graph(g)
    counts = {}
    for i in range(n):
        _, nodes = og.sample(oracle.MOSS4MIN, 41, i)
        t = tuple(nodes[:4])
        counts[t] = counts.get(t, 0) + 1
    assert set(counts) <= set(dist)
    keys = sorted(dist)
    obs = np.array([counts.get(t, 0) for t in keys], np.float64)
    exp = np.array([float(dist[t]) * n for t in keys])
    assert exp.min() >= 5.0
    chi2 = float(((obs - exp) ** 2 / exp).sum())
    assert stats.chi2.sf(chi2, len(keys) - 1) > 1e-4


def test_hits_and_reach_counters_match_samples():
    """hits[1..6] count the classes of the drawn samples, hits[7..9] their diamonds by
    c(s) = 2, 4, 6, recounted from each sample's nodes."""
    g = gg.gnp(9, 0.55, 9)
    og = oracle.Graph(g)
    adj = g.adjacency_sets()
    d = [len(a) for a in adj]
    want = np.zeros(22, np.uint64)
    for i in range(4000):
        c, nodes = og.sample(oracle.MOSS4MIN, 5, i)
        nd = nodes[:4]
        assert c == (0 if nd[3] == nd[2] else pins.class_of_nodes(adj, nd))
        want[c] += 1
        if c == 5:
            want[6 + pins.ways(adj, d, nd) // 2] += 1
    assert np.array_equal(og.run(oracle.MOSS4MIN, 5, 0, 4000), want)
    assert np.array_equal(og.run(oracle.MOSS4MIN, 5, 0, 4000, threads=3), want)
    assert want[8] > 0 and want[9] > 0


def _min_class_moments(g, weights):
    """Mean and variance of one MOSS-4Min sample of sum_i weights_i 1{class i} G / c(s)."""
    dist, G = pins.moss4min_distribution(g)
    adj = g.adjacency_sets()
    d = [len(a) for a in adj]
    mean = Fraction(0)
    sq = Fraction(0)
    for t, p in dist.items():
        if t[3] == t[2]:
            continue
        c = pins.class_of_nodes(adj, t)
        if c not in weights:
            continue
        x = weights[c] * Fraction(G, pins.ways(adj, d, t))
        mean += p * x
        sq += p * x * x
    return mean, sq - mean * mean


def _close(a, b, rel=1e-12, abs_=1e-9):
    return abs(float(a) - float(b)) <= rel * max(abs(float(a)), abs(float(b))) + abs_


@pytest.mark.parametrize("mix", [oracle.MIX_POOLED, oracle.MIX_PAPER])
def test_mixed_finals_at_expected_hits(mix):
    """At hits equal to their expectations both samplers' estimates are exact; the
    variances of the mix are the exact single-sample moments / K combined with the
    weights of the chosen reading, and Var(n_2) is the variance of the two samplers'
    shares of n_4 + 2 n_5 + 4 n_6."""
    g = gg.gnp(9, 0.55, 9)
    by4, _, G4, _ = pins.class_distribution(g, "moss4")
    dist, Gc = pins.moss4min_distribution(g)
    adj = g.adjacency_sets()
    d = [len(a) for a in adj]
    n = pins.brute_counts(g, 4)
    K, Kc = G4 * 2, Gc * 3
    h4 = [int(by4.get(c, 0) * K) for c in range(7)]
    assert all(by4.get(c, 0) * K == h4[c] for c in range(7))
    hm = [Fraction(0)] * 10
    for t, p in dist.items():
        c = 0 if t[3] == t[2] else pins.class_of_nodes(adj, t)
        hm[c] += p * Kc
        if c == 5:
            hm[6 + pins.ways(adj, d, t) // 2] += p * Kc
    assert all(x.denominator == 1 for x in hm)
    hm = [int(x) for x in hm]
    t = oracle.Graph(g).totals()
    est, var = oracle.finals4min(K, h4, t["gamma"], t["lambda3"], Kc, hm, t["gamma_min"], mix)
    for i in range(1, 7):
        assert _close(est[i - 1], n[i], abs_=1e-8), (i, est[i - 1], n[i])
    lam = {}
    for i in (3, 5, 6):
        p = Fraction(2 * pins.PHI4_1[i], G4)
        q = Fraction({3: 2, 5: 2, 6: 6}[i], Gc)
        _, v1 = _moss4_moments(by4, G4, {i: 1})
        _, v2 = _min_class_moments(g, {i: 1})
        V1, V2 = v1 / K, v2 / Kc
        if mix == oracle.MIX_POOLED or V1 + V2 == 0:
            lam[i] = K * p / (K * p + Kc * q)
            want = lam[i] ** 2 * V1 + (1 - lam[i]) ** 2 * V2
        else:
            lam[i] = V2 / (V1 + V2)
            want = V1 * V2 / (V1 + V2)
        assert _close(var[i - 1], want), (i, var[i - 1], float(want))
    for i in (1, 4):
        _, v1 = _moss4_moments(by4, G4, {i: 1})
        assert _close(var[i - 1], v1 / K)
    _, a = _moss4_moments(by4, G4, {4: 1, 5: 2 * lam[5], 6: 4 * lam[6]})
    _, b = _min_class_moments(g, {5: 2 * (1 - lam[5]), 6: 4 * (1 - lam[6])})
    assert _close(var[1], a / K + b / Kc, rel=1e-9, abs_=1e-6)


def _moss4_moments(by_class, G, weights):
    mean = Fraction(0)
    sq = Fraction(0)
    for c, p in by_class.items():
        if c == 0 or c not in weights:
            continue
        x = weights[c] / Fraction(2 * pins.PHI4_1[c], G)
        mean += p * x
        sq += p * x * x
    return mean, sq - mean * mean


def test_finals_reduce_to_moss4_without_min_samples():
    """With no MOSS-4Min samples the mix is MOSS-4's estimate and Theorem 3."""
    g = gg.chung_lu(300, 2000, 2.3, 40, 4)
    og = oracle.Graph(g)
    t = og.totals()
    h = og.run(oracle.MOSS4, 7, 0, 20_000)
    e4, v4 = oracle.finals4(20_000, h, t["gamma"], t["lambda3"])
    for mix in (oracle.MIX_POOLED, oracle.MIX_PAPER):
        e, v = oracle.finals4min(20_000, h, t["gamma"], t["lambda3"], 0, np.zeros(10), t["gamma_min"], mix)
        assert np.allclose(e, e4, rtol=1e-14, atol=0) and np.allclose(v, v4, rtol=1e-14, atol=0)


def test_min_estimate_unbiased_over_seeds():
    """Mean of independent mixed estimates (and of MOSS-4Min alone) within 5 standard
    errors of the exact counts."""
    g = gg.gnp(9, 0.55, 9)
    og = oracle.Graph(g)
    n = pins.brute_counts(g, 4)
    t = og.totals()
    R, N = 300, 4000
    res = [og.estimate4min(N, s) for s in range(1, R + 1)]
    est = np.array([r.estimate for r in res])
    var = np.array([r.variance for r in res])
    for i in range(1, 7):
        sd = np.sqrt(var[:, i - 1].mean() / R)
        assert abs(est[:, i - 1].mean() - n[i]) <= 5 * sd + 1e-9, (i, est[:, i - 1].mean(), n[i], sd)
    Kc = res[0].K[1]
    alone = np.array([oracle.finals4min(0, np.zeros(7), t["gamma"], t["lambda3"], Kc, r.hits[1][:10],
                                        t["gamma_min"])[0] for r in res])
    for i in (3, 5, 6):
        _, v = _min_class_moments(g, {i: 1})
        sd = np.sqrt(float(v) / Kc / R)
        assert abs(alone[:, i - 1].mean() - n[i]) <= 5 * sd + 1e-9, (i, alone[:, i - 1].mean(), n[i])


@pytest.mark.parametrize("seed", [1, 5])
def test_zero_variance_cases(seed):
    """Graphs where every sample of both samplers is a 4-cycle (K_{a,b}, the 4-cycle
    itself): the mixed estimate is exact, with zero variance."""
    for g, want in ((gg.complete_bipartite(3, 4), {3: 18, 2: 16}), (gg.complete_bipartite(2, 5), {3: 10, 2: 20}),
                    (gg.cycle(4), {3: 1})):
        r = oracle.Graph(g).estimate4min(3000, seed)
        for i in range(1, 7):
            assert abs(r.estimate[i - 1] - want.get(i, 0)) <= 1e-9 * max(1, want.get(i, 0)), (g.name, i)
        assert np.all(r.variance <= 1e-9 * max(want.values()) ** 2)


def test_gamma_min_zero_draws_nothing():
    """A star has check-Gamma = 0 (no leaf is above the centre): MOSS-4Min draws
    nothing and the mix is MOSS-4 alone."""
    for g in (gg.star(6), gg.path(2)):
        og = oracle.Graph(g)
        assert og.totals()["gamma_min"] == 0
        assert not og.run(oracle.MOSS4MIN, 1, 0, 100).any()
    og = oracle.Graph(gg.star(6))
    r = og.estimate4min(1000, 3)
    assert r.estimate[1] == 20 and not r.hits[1].any()
