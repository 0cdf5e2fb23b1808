"""Oracle exact counts and weight tables against brute force and closed forms."""
import numpy as np
import pytest

import graphgen as gg
import oracle
import pins
from pins import choose

TINY = [
    gg.gnp(9, 0.45, 1), gg.gnp(11, 0.45, 2), gg.gnp(10, 0.6, 3), gg.gnp(12, 0.3, 4),
    gg.complete(6), gg.wheel(6), gg.complete_bipartite(3, 4), gg.path(8), gg.cycle(7),
    gg.star(6),
]


@pytest.mark.parametrize("g", TINY, ids=lambda g: g.name)
@pytest.mark.parametrize("k", [4, 5])
def test_enumeration_matches_brute_force(g, k):
    got = oracle.Graph(g).count_cis(k)
    want = pins.brute_counts(g, k)
    assert [int(x) for x in got] == want
    for threads in (2, 3, 16):  # start vertices dealt to several workers: the same counts
        assert [int(x) for x in oracle.Graph(g).count_cis(k, threads)] == want


@pytest.mark.parametrize("n", [5, 6, 8])
def test_complete_graph_counts(n):
    og = oracle.Graph(gg.complete(n))
    c4, c5 = og.count_cis(4), og.count_cis(5)
    assert int(c4[6]) == choose(n, 4) and int(c4.sum()) == choose(n, 4)
    assert int(c5[21]) == choose(n, 5) and int(c5.sum()) == choose(n, 5)


@pytest.mark.parametrize("a,b", [(2, 3), (3, 4), (4, 4), (2, 6)])
def test_complete_bipartite_counts(a, b):
    c4 = oracle.Graph(gg.complete_bipartite(a, b)).count_cis(4)
    assert int(c4[3]) == choose(a, 2) * choose(b, 2)
    assert int(c4[2]) == a * choose(b, 3) + b * choose(a, 3)
    assert int(c4.sum()) == int(c4[2] + c4[3])


def test_path_cycle_star_counts():
    for n in (6, 9, 13):
        c4 = oracle.Graph(gg.path(n)).count_cis(4)
        c5 = oracle.Graph(gg.path(n)).count_cis(5)
        assert int(c4[1]) == n - 3 and int(c4.sum()) == n - 3
        assert int(c5[1]) == n - 4 and int(c5.sum()) == n - 4
    for n in (6, 9):
        og = oracle.Graph(gg.cycle(n))
        assert int(og.count_cis(4)[1]) == n
        assert int(og.count_cis(5)[1]) == n
    assert int(oracle.Graph(gg.cycle(5)).count_cis(5)[6]) == 1
    assert int(oracle.Graph(gg.cycle(4)).count_cis(4)[3]) == 1
    for s in (3, 5, 8):
        og = oracle.Graph(gg.star(s))
        assert int(og.count_cis(4)[2]) == choose(s, 3)
        assert int(og.count_cis(5)[2]) == choose(s, 4)


def _tuple_counts_per_node(g):
    """Brute-force numbers of sampler tuples rooted at each node: MOSS-4 tuples
    (u, w, r) with u != w in N_v, r in N_u - {v}; T-5 tuples with two ordered extra
    neighbours of v; Path-5 tuples (u, w, r, t) with u != w in N_v, r in N_u - {v},
    t in N_w - {v}.  Their totals are Gamma_v, Gamma^(1)_v and Gamma^(2)_v."""
    A = g.adjacency_sets()
    c4, c5t, c5p = [], [], []
    for v in range(g.n):
        a = b = c = 0
        for u in A[v]:
            for w in A[v]:
                if w == u:
                    continue
                ru = len(A[u]) - 1
                a += ru
                b += (len(A[v]) - 2) * ru
                c += ru * (len(A[w]) - 1)
        c4.append(a)
        c5t.append(b)
        c5p.append(c)
    return c4, c5t, c5p


@pytest.mark.parametrize("g", TINY[:6], ids=lambda g: g.name)
def test_node_weights_count_sampler_tuples(g):
    og = oracle.Graph(g)
    c4, c5t, c5p = _tuple_counts_per_node(g)
    assert og.table(oracle.TAB_GAMMA).tolist() == c4
    assert og.table(oracle.TAB_GAMMA1).tolist() == c5t
    assert og.table(oracle.TAB_GAMMA2).tolist() == c5p
    t = og.totals()
    assert t["gamma"] == sum(c4) and t["gamma1"] == sum(c5t) and t["gamma2"] == sum(c5p)
    for which, tot in ((oracle.TAB_ACC_GAMMA, c4), (oracle.TAB_ACC_GAMMA1, c5t), (oracle.TAB_ACC_GAMMA2, c5p)):
        assert og.table(which).tolist() == np.cumsum(tot).tolist()


@pytest.mark.parametrize("g", TINY, ids=lambda g: g.name)
def test_identities(g):
    """Lambda_3 = n_2 + n_4 + 2 n_5 + 4 n_6 (Eq. n2); sum_i phi^(3)_i eta_i = Lambda_4
    (Section 5.1.3); Gamma = 2 sum_i phi^(1)_i n_i + 6 T (every MOSS-4 tuple is a
    3-path counted from both middle-edge directions, or a triangle with r = w);
    Gamma^(1) = 2 sum_i phi^(1)_i eta_i + 4 sum_v T_v (d_v - 2)."""
    og = oracle.Graph(g)
    t = og.totals()
    n = pins.brute_counts(g, 4)
    eta = pins.brute_counts(g, 5)
    deg = g.degrees()
    assert t["lambda3"] == sum(choose(int(d), 3) for d in deg)
    assert t["lambda4"] == sum(choose(int(d), 4) for d in deg)
    assert t["lambda3"] == n[2] + n[4] + 2 * n[5] + 4 * n[6]
    assert t["lambda4"] == sum(pins.PHI5_3[i] * eta[i] for i in range(1, 22))
    tv = pins.triangles_per_node(g)
    T = sum(tv) // 3
    assert t["gamma"] == 2 * sum(pins.PHI4_1[i] * n[i] for i in range(1, 7)) + 6 * T
    assert t["gamma1"] == 2 * sum(pins.PHI5_1[i] * eta[i] for i in range(1, 22)) + \
        4 * sum(tv[v] * (int(deg[v]) - 2) for v in range(g.n) if deg[v] >= 2)


def test_row_prefix_tables():
    g = gg.gnp(30, 0.2, 9)
    og = oracle.Graph(g)
    deg = g.degrees()
    sig = og.table(oracle.TAB_ACC_SIGMA)
    tau = og.table(oracle.TAB_ACC_TAU)
    S = og.table(oracle.TAB_S)
    Q = og.table(oracle.TAB_Q)
    for v in range(g.n):
        nb = g.neighbors(v)
        if len(nb) == 0:
            continue
        w = deg[nb] - 1
        assert sig[g.row_ptr[v]:g.row_ptr[v + 1]].tolist() == np.cumsum(w).tolist()
        assert int(S[v]) == int(w.sum()) and int(Q[v]) == int((w * w).sum())
        tw = w * (int(S[v]) - w)
        assert tau[g.row_ptr[v]:g.row_ptr[v + 1]].tolist() == np.cumsum(tw).tolist()
        assert int(tau[g.row_ptr[v + 1] - 1]) == int(S[v]) ** 2 - int(Q[v])


def test_validation_errors():
    good = gg.gnp(8, 0.5, 1)
    oracle.Graph(good)
    rp, col = good.row_ptr.copy(), good.col.copy()
    bad = gg.CSR(rp, col[::-1].copy())
    with pytest.raises(oracle.OracleError):
        oracle.Graph(bad)
    loop = gg.CSR(np.array([0, 1, 2], np.int32), np.array([0, 0], np.int32))
    with pytest.raises(oracle.OracleError) as e:
        oracle.Graph(loop)
    assert e.value.status == oracle.E_SELF_LOOP
    asym = gg.CSR(np.array([0, 1, 1], np.int32), np.array([1], np.int32))
    with pytest.raises(oracle.OracleError) as e:
        oracle.Graph(asym)
    assert e.value.status == oracle.E_ASYMMETRIC
    dup = gg.CSR(np.array([0, 2, 4], np.int32), np.array([1, 1, 0, 0], np.int32))
    with pytest.raises(oracle.OracleError) as e:
        oracle.Graph(dup)
    assert e.value.status == oracle.E_DUPLICATE


def test_overflow_is_reported():
    """Lambda_4 of the star K_{1,s} is C(s, 4): it fits 64 bits at s = 100,000 and
    does not at s = 150,000; the oracle must refuse rather than wrap."""
    og = oracle.Graph(gg.star(100_000))
    assert og.totals()["lambda4"] == choose(100_000, 4)
    with pytest.raises(oracle.OracleError) as e:
        oracle.Graph(gg.star(150_000))
    assert e.value.status == oracle.E_OVERFLOW


@pytest.mark.parametrize("g", TINY + [gg.chung_lu(300, 2000, 2.2, 60, 7), gg.complete(9), gg.wheel(12)],
                         ids=lambda g: g.name)
def test_pattern_conversion_counts_match_enumeration(g):
    """The non-induced-pattern route to n_1..n_6 agrees with ESU enumeration."""
    og = oracle.Graph(g)
    np.testing.assert_array_equal(og.count4_exact()[1:7], og.count_cis(4)[1:7])


def test_pattern_conversion_on_c1():
    g = gg.config_graph("C1")
    og = oracle.Graph(g)
    import json, os
    want = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "exact_c1.json")))
    assert want["graph_sha256"] == g.sha256()
    assert og.count4_exact()[1:7].tolist() == want["n4"]


def test_stored_c1_counts_meet_the_identities():
    """tests/golden/exact_c1.json (written by make_golden.py from the oracle's enumeration)
    must describe the C1 graph and satisfy Eq. n2 (Lambda_3 = n_2 + n_4 + 2 n_5 + 4 n_6)
    and its 5-node twin Lambda_4 = sum_i phi^(3)_i eta_i (Section 5.1.3), with Lambda
    counted here from the degrees."""
    import json
    import os
    d = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "exact_c1.json")))
    g = gg.config_graph("C1")
    assert d["graph_sha256"] == g.sha256()
    deg = [int(x) for x in g.degrees()]
    lam3, lam4 = sum(choose(x, 3) for x in deg), sum(choose(x, 4) for x in deg)
    n = dict(enumerate(d["n4"], 1))
    assert n[2] + n[4] + 2 * n[5] + 4 * n[6] == lam3
    eta = dict(enumerate(d["eta5"], 1))
    assert len(eta) == 21 and sum(pins.PHI5_3[i] * eta[i] for i in eta) == lam4
