"""Graph creation checks on the GPU walk the CSR in spans of 256 entries, finding each
entry's row from the row starts inside its span.  These cases put defects at the
places where that bookkeeping could go wrong: the first and last entries of spans,
rows that start exactly at a span boundary, runs of rows without entries, and a hub
row covering several spans.  The expected status comes from a plain validator written
here from the rules (column range, no self-loops, strictly ascending rows,
symmetry), taking the highest-priority defect as the library does (tests/defects.py;
checked against the oracle's validator on the CPU in tests/test_oracle_validation.py)."""
import numpy as np
import pytest

import defects
import graphgen as gg
import oracle
from paper_1509_08089_amd import moss

pytestmark = pytest.mark.gpu



def expected_status(rp, col):
    return defects.expected_status(rp, col)


@pytest.fixture(scope="module")
def base():
    g = defects.span_graph()
    return np.asarray(g.row_ptr, np.int32), np.asarray(g.col, np.int32), g


def _create_status(rp, col):
    try:
        moss.moss_graph_destroy(moss.moss_graph_create(len(rp) - 1, len(col), rp, col, 0, 0))
        return moss.MOSS_OK
    except moss.MossError as e:
        return e.status


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


def test_defects_at_span_edges(base):
    rp, col, _ = base
    n_cases = 0
    for name, r, c in defects.cases(rp, col):
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
    for name, r, c in defects.cases(rp2, col, [nnz - 1, nnz - 2, (nnz - 1) // 256 * 256, (nnz - 1) // 256 * 256 + 1]):
        want = expected_status(r, c)
        assert want != moss.MOSS_OK, name
        assert _create_status(r, c) == want, (name, moss.STATUS[want])
        n_cases += 1
    assert n_cases >= 16
