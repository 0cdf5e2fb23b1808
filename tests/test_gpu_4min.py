"""MOSS-4Min on the GPU against the oracle (calls through the C ABI).

Rank tables, check-Gamma prefixes, per-sample classes and nodes, and the reach-count
bins of the diamonds must be identical to the oracle's; the mixed 4-node finals within
1e-12 relative.  Graphs include rows of every rank pass (short rows ranked per span, long rows sorted
per block in LDS or in their own scratch, degrees of 2^16 and more ranked per piece),
rows past the row-guide threshold, many equal degrees (ties broken by id), CSRs created
without the checks (searched mirrors) and graphs with check-Gamma = 0."""
import numpy as np
import pytest
import torch

import graphgen as gg
import oracle
from graphgen.csr import CSR
from gpu_util import assert_result_matches
from paper_1509_08089_amd import moss

pytestmark = pytest.mark.gpu

MIN = moss.MOSS_SAMPLER_MOSS4MIN


def _ties():
    # three hubs joined to the same 700 nodes (hub rows of three 256-entry pieces whose
    # entries mostly tie on degree), plus a few chords between those nodes
    edges = [(a, 3 + j) for a in range(3) for j in range(700)]
    edges += [(3 + j, 3 + j + 1) for j in range(0, 690, 7)]
    return gg.from_edges(703, edges, "ties")


GRAPHS = [
    gg.gnp(9, 0.55, 9), gg.gnp(40, 0.2, 5), gg.wheel(9), gg.complete(7), gg.complete_bipartite(4, 6),
    gg.chung_lu(600, 4000, 2.3, 80, 11), gg.chung_lu(5000, 40000, 2.1, 900, 12), gg.wheel(300),
    gg.complete_bipartite(3, 700), gg.complete(70), _ties(),
]


def ids(g):
    return g.name[:40]


@pytest.fixture(scope="module")
def c1():
    return gg.config_graph("C1")


@pytest.mark.parametrize("g", GRAPHS, ids=ids)
def test_min_tables_match_oracle(g):
    G = moss.Graph(g)
    G.build_tables(moss.MOSS_TABLES_K4MIN)
    og = oracle.Graph(g)
    assert G.info().gamma_min == og.totals()["gamma_min"]
    assert G.info().built_mask == moss.MOSS_TABLES_K4MIN
    np.testing.assert_array_equal(G.table(moss.MOSS_TAB_ACC_GAMMA_MIN), og.table(oracle.TAB_ACC_GAMMA_MIN))
    np.testing.assert_array_equal(G.table(moss.MOSS_TAB_ACC_CHECK), og.table(oracle.TAB_ACC_CHECK))
    rank = G.table(moss.MOSS_TAB_RANK)
    np.testing.assert_array_equal(rank[:, 0], og.table(oracle.TAB_RANK))
    np.testing.assert_array_equal(rank[:, 1], og.table(oracle.TAB_RANK_MIRROR))
    np.testing.assert_array_equal(G.table(moss.MOSS_TAB_COL_RANK), og.table(oracle.TAB_COL_RANK))


@pytest.mark.parametrize("g", GRAPHS, ids=ids)
@pytest.mark.parametrize("K,seed,mix", [(2, 3, 0), (1001, 1, 0), (200_001, 2, 0), (50_000, 4, 1)])
def test_mixed_estimate_matches_oracle(g, K, seed, mix):
    G, og = moss.Graph(g), oracle.Graph(g)
    r = G.estimate(4, K, seed, mix | moss.MOSS_K4_MIN)
    assert r.gamma[1] == og.totals()["gamma_min"]
    assert_result_matches(r, og.estimate4min(K, seed, mix, threads=8), float(og.totals()["lambda3"]))


def _hub_graph(leaves, extra=600, seed=3):
    # node 0 joined to `leaves` nodes, with a sprinkle of edges among them (so that the
    # hub's neighbours have different degrees) and a second, smaller hub
    rng = np.random.default_rng(seed)
    n = leaves + 1
    edges = {(0, j) for j in range(1, n)}
    edges |= {(1, j) for j in range(2, min(n, 3000))}
    while len(edges) < leaves + min(n, 3000) - 2 + extra:
        a, b = sorted(int(x) for x in rng.integers(1, n, 2))
        if a != b:
            edges.add((a, b))
    return gg.from_edges(n, sorted(edges), f"hub {leaves}")


def _check_min_tables(g, flags=0):
    G = moss.Graph(g, flags=flags)
    G.build_tables(moss.MOSS_TABLES_K4MIN)
    og = oracle.Graph(g)
    assert G.info().gamma_min == og.totals()["gamma_min"]
    rank = G.table(moss.MOSS_TAB_RANK)
    np.testing.assert_array_equal(rank[:, 0], og.table(oracle.TAB_RANK))
    np.testing.assert_array_equal(rank[:, 1], og.table(oracle.TAB_RANK_MIRROR))
    np.testing.assert_array_equal(G.table(moss.MOSS_TAB_COL_RANK), og.table(oracle.TAB_COL_RANK))
    np.testing.assert_array_equal(G.table(moss.MOSS_TAB_ACC_CHECK), og.table(oracle.TAB_ACC_CHECK))
    np.testing.assert_array_equal(G.table(moss.MOSS_TAB_ACC_GAMMA_MIN), og.table(oracle.TAB_ACC_GAMMA_MIN))


@pytest.mark.parametrize("leaves", [5000, 40000, 70000], ids=["lds-block", "row-scratch", "degree-2^16"])
def test_min_tables_hub_rows(leaves):
    """A hub row sorted by the full block in LDS (d = 5000), in its own scratch (d = 40000,
    beyond the LDS sort), and a degree of 2^16 or more (70000), where the per-piece rank
    passes and the searched mirrors take over."""
    _check_min_tables(_hub_graph(leaves))


def _boundary_graph(n, seed=5):
    # 3000 nodes at the top of the id range (a hub among them) plus 50 low ids joined to
    # them, in an otherwise empty graph of n nodes; the CSR is assembled with numpy
    rng = np.random.default_rng(seed)
    hi = np.arange(n - 3000, n)
    e = {(int(x), n - 1) for x in hi[:2900]}
    while len(e) < 2900 + 15000:
        a, b = rng.choice(hi, 2)
        if a != b:
            e.add((int(min(a, b)), int(max(a, b))))
    e |= {(lo, int(hi[lo * 7])) for lo in range(50)}
    E = np.array(sorted(e), dtype=np.int64)
    src, dst = np.concatenate([E[:, 0], E[:, 1]]), np.concatenate([E[:, 1], E[:, 0]])
    o = np.lexsort((dst, src))
    rp = np.zeros(n + 1, np.int64)
    np.add.at(rp, src[o] + 1, 1)
    return CSR(np.cumsum(rp).astype(np.int32), dst[o].astype(np.int32), f"ids up to {n - 1}")


@pytest.mark.timeout(300)
@pytest.mark.parametrize("n", [2**24, 2**24 + 1], ids=["ids-below-2^24", "ids-to-2^24"])
def test_min_tables_id_boundary(n):
    """Ids up to 2^24 - 1: the mirror sort's three 8-bit passes, the words holding the
    column's top 16 bits; one more id: the searched mirrors take over."""
    _check_min_tables(_boundary_graph(n))


@pytest.mark.parametrize("g", [gg.chung_lu(5000, 40000, 2.1, 900, 12), _ties(), gg.complete(70)], ids=ids)
def test_min_tables_trusted_csr(g):
    """A CSR created without the checks takes the searched mirror pass; same tables."""
    _check_min_tables(g, moss.MOSS_TRUST_CSR)


def test_min_tables_after_other_sets():
    """Building the 4-node, 5-node and MOSS-4Min sets in any order gives the same tables."""
    g = gg.chung_lu(5000, 40000, 2.1, 900, 12)
    og = oracle.Graph(g)
    for order in ([moss.MOSS_TABLES_K5, moss.MOSS_TABLES_K4MIN, moss.MOSS_TABLES_K4],
                  [moss.MOSS_TABLES_K4MIN | moss.MOSS_TABLES_K4 | moss.MOSS_TABLES_K5]):
        G = moss.Graph(g)
        for m in order:
            G.build_tables(m)
        np.testing.assert_array_equal(G.table(moss.MOSS_TAB_ACC_CHECK), og.table(oracle.TAB_ACC_CHECK))
        np.testing.assert_array_equal(G.table(moss.MOSS_TAB_ACC_SIGMA), og.table(oracle.TAB_ACC_SIGMA))
        np.testing.assert_array_equal(G.table(moss.MOSS_TAB_ACC_GAMMA), og.table(oracle.TAB_ACC_GAMMA))


def test_per_sample_classes_and_reach_bins(c1):
    G, og = moss.Graph(c1), oracle.Graph(c1)
    k0, k1 = 4321, 4321 + 70_001
    cls = torch.zeros(k1 - k0, dtype=torch.uint8, device="cuda")
    hits = G.sample_range(MIN, 7, k0, k1, cls)
    c = cls.cpu().numpy()
    np.testing.assert_array_equal(np.bincount(c, minlength=7)[:7], hits[:7])
    want = np.array([og.sample(oracle.MOSS4MIN, 7, k)[0] for k in range(k0, k1)], dtype=np.uint8)
    np.testing.assert_array_equal(c, want)
    np.testing.assert_array_equal(hits, og.run(oracle.MOSS4MIN, 7, k0, k1, 8))
    assert int(hits[7:10].sum()) == int(hits[5])
    a = G.sample_range(MIN, 7, k0, k0 + 33_333) + G.sample_range(MIN, 7, k0 + 33_333, k1)
    np.testing.assert_array_equal(a, hits)


def test_reach_bins_cover_all_counts():
    """A graph whose diamonds are reached 2, 4 and 6 ways: all three bins fill, as the
    oracle's."""
    g = gg.gnp(9, 0.55, 9)
    G, og = moss.Graph(g), oracle.Graph(g)
    hits = G.sample_range(MIN, 5, 0, 400_000)
    np.testing.assert_array_equal(hits, og.run(oracle.MOSS4MIN, 5, 0, 400_000, 8))
    assert hits[7] > 0 and hits[8] > 0 and hits[9] > 0


def test_sampled_nodes_match_oracle(c1):
    G, og = moss.Graph(c1), oracle.Graph(c1)
    idx = np.concatenate([np.arange(0, 300, dtype=np.uint64),
                          np.array([2**40 + 5, 2**63 - 1, 2**64 - 1], dtype=np.uint64),
                          np.random.Generator(np.random.PCG64(1)).integers(0, 2**62, 500, dtype=np.uint64)])
    nodes, cls = G.sample_nodes(MIN, 11, idx)
    for i, k in enumerate(idx):
        c, nd = og.sample(oracle.MOSS4MIN, 11, int(k))
        assert int(cls[i]) == c
        assert nodes[i].tolist() == nd[:4] + [-1], (int(k), nodes[i].tolist(), nd)


@pytest.fixture
def schedule():
    def set_(sch):
        moss.moss_set_tuning(0, 0, 0, sch)
    yield set_
    moss.moss_set_tuning(0, 0, 0, 0)


def test_grouped_schedule_same_samples(c1, schedule):
    """The XCD-grouped launch gives every MOSS-4Min sample the plain launch's outcome."""
    G = moss.Graph(c1)
    K = 300_007
    a = torch.zeros(K, dtype=torch.uint8, device="cuda")
    b = torch.zeros(K, dtype=torch.uint8, device="cuda")
    schedule(moss.MOSS_SCHEDULE_PLAIN)
    ha = G.sample_range(MIN, 3, 11, 11 + K, a)
    ra = G.estimate(4, 2 * K, 3, moss.MOSS_K4_MIN)
    schedule(moss.MOSS_SCHEDULE_XCD)
    hb = G.sample_range(MIN, 3, 11, 11 + K, b)
    rb = G.estimate(4, 2 * K, 3, moss.MOSS_K4_MIN)
    np.testing.assert_array_equal(ha, hb)
    assert torch.equal(a, b)
    np.testing.assert_array_equal(ra.hits_np, rb.hits_np)
    np.testing.assert_array_equal(ra.estimate_np, rb.estimate_np)


def test_batch_and_server_match_single_requests(c1):
    gs = [c1, gg.gnp(9, 0.55, 9), gg.star(9), gg.chung_lu(5000, 40000, 2.1, 900, 12)]
    hs = [moss.Graph(g) for g in gs]
    reqs = []
    for i in range(24):
        h = hs[i % len(hs)]
        flags = moss.MOSS_K4_MIN | (i // 4) % 2
        reqs.append((h.h, 4, 1000 + 7919 * i, i + 1, flags))
    reqs.append((hs[0].h, 4, 50_000, 99, 0))
    reqs.append((hs[3].h, 5, 50_000, 98, 0))
    alone = [moss.moss_estimate(*q) for q in reqs]
    for _ in range(2):
        got = moss.moss_estimate_batch(reqs)
        for a, b in zip(alone, got):
            np.testing.assert_array_equal(a.hits_np, b.hits_np)
            np.testing.assert_array_equal(a.estimate_np, b.estimate_np)
    srv = moss.moss_server_create(0, 8, 3_000)
    try:
        gid = {h.h.value: moss.moss_server_add_graph(srv, h.h) for h in hs}
        tickets = [moss.moss_server_submit(srv, gid[g.value], k, ns, seed, fl) for (g, k, ns, seed, fl) in reqs]
        for a, t in zip(alone, tickets):
            r = moss.moss_server_wait(srv, t, 60_000)
            np.testing.assert_array_equal(a.hits_np, r.hits_np)
            np.testing.assert_array_equal(a.estimate_np, r.estimate_np)
    finally:
        moss.moss_server_destroy(srv)


def test_gamma_min_zero_and_bad_arguments():
    """A star has check-Gamma = 0: MOSS-4Min draws nothing and the mix is MOSS-4's;
    the flag needs k = 4 and at least two samples."""
    G = moss.Graph(gg.star(9))
    r = G.estimate(4, 1000, 1, moss.MOSS_K4_MIN)
    assert r.gamma[1] == 0 and not r.hits_np[1].any()
    assert r.estimate[1] == 84.0  # C(9, 3) stars, exactly
    cls = torch.full((50,), 7, dtype=torch.uint8, device="cuda")
    assert not G.sample_range(MIN, 1, 0, 50, cls).any()
    assert not cls.any()
    with pytest.raises(moss.MossError):
        G.sample_nodes(MIN, 1, [0])
    H = moss.Graph(gg.gnp(12, 0.4, 1))
    for k, n, fl in ((5, 1000, moss.MOSS_K4_MIN), (4, 1, moss.MOSS_K4_MIN), (4, 100, 0x4)):
        with pytest.raises(moss.MossError):
            H.estimate(k, n, 1, fl)
