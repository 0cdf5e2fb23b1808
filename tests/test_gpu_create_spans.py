"""Graph creation checks on the GPU walk the CSR in spans of 256 entries, finding each
entry's row from the row starts inside its span.  These cases put defects at the
places where that bookkeeping could go wrong: the first and last entries of spans,
rows that start exactly at a span boundary, runs of rows without entries, and a hub
row covering several spans.  The expected status comes from a plain validator written
here from the rules (column range, no self-loops, strictly ascending rows,
symmetry), taking the highest-priority defect as the library does."""
import numpy as np
import pytest

import graphgen as gg
import oracle
from paper_1509_08089_amd import moss

pytestmark = pytest.mark.gpu

PRIORITY = [moss.MOSS_E_ARG, moss.MOSS_E_SELF_LOOP, moss.MOSS_E_DUPLICATE, moss.MOSS_E_UNSORTED,
            moss.MOSS_E_ASYMMETRIC]


def expected_status(rp, col):
    n, nnz = len(rp) - 1, len(col)
    found = set()
    upper, lower = set(), []
    n_upper = 0
    for v in range(n):
        for e in range(rp[v], rp[v + 1]):
            c = int(col[e])
            if c < 0 or c >= n:
                found.add(moss.MOSS_E_ARG)
                continue
            if c == v:
                found.add(moss.MOSS_E_SELF_LOOP)
            if e > rp[v]:
                if col[e - 1] == c:
                    found.add(moss.MOSS_E_DUPLICATE)
                elif col[e - 1] > c:
                    found.add(moss.MOSS_E_UNSORTED)
            if c > v:
                upper.add((v, c))
                n_upper += 1
            elif c < v:
                lower.append((c, v))
    if any(x not in upper for x in lower) or 2 * n_upper != nnz:
        found.add(moss.MOSS_E_ASYMMETRIC)
    for s in PRIORITY:
        if s in found:
            return s
    return moss.MOSS_OK


def _graph():
    """3,000 nodes, runs of them without edges, one hub of degree about 700; with this
    seed several rows start exactly at multiples of 256."""
    rng = np.random.Generator(np.random.PCG64(7))
    n = 3000
    active = np.ones(n, bool)
    for start in rng.integers(0, n - 60, 25):
        active[start:start + rng.integers(5, 60)] = False
    ids = np.flatnonzero(active)
    edges = set()
    for _ in range(4000):
        a, b = rng.choice(ids, 2, replace=False)
        edges.add((min(a, b), max(a, b)))
    hub = int(ids[len(ids) // 2])
    for x in rng.choice(ids, 700, replace=False):
        if x != hub:
            edges.add((min(hub, x), max(hub, x)))
    return gg.from_edges(n, sorted(edges), "spans")


@pytest.fixture(scope="module")
def base():
    g = _graph()
    return np.asarray(g.row_ptr, np.int32), np.asarray(g.col, np.int32), g


def _create_status(rp, col):
    try:
        moss.moss_graph_destroy(moss.moss_graph_create(len(rp) - 1, len(col), rp, col, 0, 0))
        return moss.MOSS_OK
    except moss.MossError as e:
        return e.status


def _positions(rp, nnz):
    """Entries at span edges and row heads at or next to span boundaries."""
    pos = {e for e in range(nnz) if e % 256 in (0, 1, 63, 64, 127, 128, 255)}
    heads = set(int(x) for x in rp[:-1][np.diff(rp) > 0])
    pos |= {h for h in heads if h % 256 in (0, 1, 255)}
    return sorted(pos)


def test_valid_graph_creates_and_samples_like_the_oracle(base):
    rp, col, g = base
    assert expected_status(rp, col) == moss.MOSS_OK
    assert len(col) > 20 * 256
    heads = rp[:-1][np.diff(rp) > 0]
    assert (np.diff(rp) == 0).sum() > 500
    G, og = moss.Graph(g), oracle.Graph(g)
    for k in (4, 5):
        r = G.estimate(k, 300_000, 3)
        np.testing.assert_array_equal(r.hits_np, og.estimate(k, 300_000, 3, threads=8).hits)
    assert (heads % 256 == 0).any()


def _cases(rp, col, positions=None):
    nnz = len(col)
    heads = set(int(x) for x in rp[:-1][np.diff(rp) > 0])
    row_of = np.repeat(np.arange(len(rp) - 1), np.diff(rp))
    for e in (_positions(rp, nnz)[::3] if positions is None else positions):
        v = int(row_of[e])
        c = col.copy()
        if e not in heads:
            c[e] = c[e - 1]
            yield f"dup@{e}", rp, c
            c = col.copy()
            c[e - 1], c[e] = c[e], c[e - 1]
            yield f"swap@{e}", rp, c
        elif c[e] > 0:
            # a row's first entry is not compared with the previous row's last
            c[e] -= 1
            yield f"head@{e}", rp, c
        c = col.copy()
        c[e] = v
        yield f"self@{e}", rp, c
        c = col.copy()
        c[e] = len(rp) - 1
        yield f"range@{e}", rp, c
        # drop the entry: its mirror is left unmatched
        r2 = rp.copy()
        r2[v + 1:] -= 1
        yield f"drop@{e}", r2, np.delete(col, e)


def test_defects_at_span_edges(base):
    rp, col, _ = base
    n_cases = 0
    for name, r, c in _cases(rp, col):
        want = expected_status(r, c)
        assert want != moss.MOSS_OK, name
        assert _create_status(r, c) == want, (name, moss.STATUS[want])
        n_cases += 1
    assert n_cases > 150


def test_trailing_rows_without_entries(base):
    """The same graph with 5,000 more nodes that have no edges, after the last row with
    entries: valid as it is, and defects in its last span are still found."""
    rp, col, _ = base
    rp2 = np.concatenate([rp, np.full(5000, rp[-1], np.int32)])
    assert _create_status(rp2, col) == moss.MOSS_OK
    nnz = len(col)
    n_cases = 0
    for name, r, c in _cases(rp2, col, [nnz - 1, nnz - 2, (nnz - 1) // 256 * 256, (nnz - 1) // 256 * 256 + 1]):
        want = expected_status(r, c)
        assert want != moss.MOSS_OK, name
        assert _create_status(r, c) == want, (name, moss.STATUS[want])
        n_cases += 1
    assert n_cases >= 16
