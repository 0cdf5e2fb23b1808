"""Row prefixes and row guides on the GPU.  The prefixes (ACC_sigma, ACC_tau,
ACC_check) must equal the oracle's; each row guide must follow its definition from the
prefix read back: for a row with d >= 64, g = floor(log2 d) - 1, total T and
s = max(0, bitlength(T) - g), entry b is the first i with A[i] > b * 2^s, else d - 1.
Graphs have rows crossing several 256-entry spans (hubs, one over 234 spans), rows
starting exactly at span boundaries, runs of rows without entries (also after the last
row with entries), rows whose weights are all zero and rows of one or two entries
between hubs."""
import numpy as np
import pytest

import graphgen as gg
import oracle
from paper_1509_08089_amd import moss

pytestmark = pytest.mark.gpu


def _hubs_and_gaps():
    rng = np.random.Generator(np.random.PCG64(11))
    n = 6000
    edges = set()
    hubs = [17, 18, 900, 3001, 5990]
    for h, dg in zip(hubs, (2500, 700, 257, 64, 1200)):
        for x in rng.choice(n, dg, replace=False):
            if x != h:
                edges.add((min(h, x), max(h, x)))
    for _ in range(3000):
        a, b = rng.integers(0, 4000, 2)
        if a != b:
            edges.add((min(a, b), max(a, b)))
    return gg.from_edges(n, sorted(edges), "hubs+gaps")


def _big_hub():
    """A hub joined to 60,000 of 70,000 nodes (a row over 234 spans, past the size at
    which rows add up their span sums by groups of 64 spans), plus random edges so
    that its neighbours' weights differ."""
    rng = np.random.Generator(np.random.PCG64(13))
    n = 70_000
    leaves = rng.choice(np.arange(1, n), 60_000, replace=False)
    edges = [(0, int(x)) for x in leaves]
    a = rng.integers(1, n, 40_000)
    b = rng.integers(1, n, 40_000)
    edges += [(int(x), int(y)) for x, y in zip(a, b) if x != y]
    return gg.from_edges(n, edges, "big hub")


def _trailing_empty():
    """Edges only among the first 2,500 of 9,000 nodes (a hub among them): 6,500 rows
    without entries after the last one with entries."""
    rng = np.random.Generator(np.random.PCG64(17))
    edges = [(0, int(x)) for x in rng.choice(np.arange(1, 2500), 900, replace=False)]
    a, b = rng.integers(1, 2500, 6000), rng.integers(1, 2500, 6000)
    edges += [(int(x), int(y)) for x, y in zip(a, b) if x != y]
    return gg.from_edges(9000, edges, "trailing empty rows")


GRAPHS = [_hubs_and_gaps(), gg.chung_lu(5000, 40000, 2.1, 900, 12), gg.star(3000), gg.wheel(700),
          gg.complete_bipartite(3, 900), gg.complete(90), _big_hub(), _trailing_empty()]


def expected_guides(rp, acc):
    out = []
    for v in range(len(rp) - 1):
        d = int(rp[v + 1] - rp[v])
        if d < 64:
            continue
        a = acc[rp[v]:rp[v + 1]].astype(np.uint64)
        g = d.bit_length() - 2
        total = int(a[-1])
        s = max(0, total.bit_length() - g)
        bounds = (np.arange((1 << g) + 1, dtype=object) << s)
        idx = np.searchsorted(a.astype(object), bounds, side="right")
        out.append(np.minimum(idx, d - 1).astype(np.uint32))
    return np.concatenate(out) if out else np.zeros(0, np.uint32)


@pytest.mark.parametrize("g", GRAPHS, ids=lambda g: g.name[:30])
def test_row_prefixes_and_guides(g):
    rp = np.asarray(g.row_ptr, np.int64)
    G, og = moss.Graph(g), oracle.Graph(g)
    G.build_tables(moss.MOSS_TABLES_K4 | moss.MOSS_TABLES_K5 | moss.MOSS_TABLES_K4MIN)
    glen = sum((1 << (int(d).bit_length() - 2)) + 1 for d in np.diff(rp) if d >= 64)
    for tab, otab, guide in ((moss.MOSS_TAB_ACC_SIGMA, oracle.TAB_ACC_SIGMA, moss.MOSS_TAB_SIGMA_GUIDE),
                             (moss.MOSS_TAB_ACC_TAU, oracle.TAB_ACC_TAU, moss.MOSS_TAB_TAU_GUIDE),
                             (moss.MOSS_TAB_ACC_CHECK, oracle.TAB_ACC_CHECK, moss.MOSS_TAB_CHECK_GUIDE)):
        acc = G.table(tab)
        np.testing.assert_array_equal(acc, og.table(otab))
        got = moss.moss_table_read(G.h, guide, glen)
        np.testing.assert_array_equal(got, expected_guides(rp, acc))
    # S_v (the sigma row totals) through the node weights: Gamma_v = (d_v - 1) S_v
    np.testing.assert_array_equal(G.table(moss.MOSS_TAB_ACC_GAMMA), og.table(oracle.TAB_ACC_GAMMA))
