"""The oracle's motif classifier against the paper's constants.

The motif drawings of the paper are not available; the ids are fixed by the
constants it prints: phi^(1) and phi^(2) of Section 4.1.2 for 4 nodes and the
three rows of Table 2 for 5 nodes.  Here every labelled graph on 4 and 5 nodes is
enumerated, isomorphism classes are formed by brute-force canonical labelling,
the constants are recomputed by counting pattern embeddings over permutations,
and the oracle must return exactly the id whose printed constants match."""
import pytest

import oracle
import pins


@pytest.mark.parametrize("k,n_connected,n_classes", [(4, 38, 6), (5, 728, 21)])
def test_classifier_matches_printed_constants(k, n_connected, n_classes):
    pairs = k * (k - 1) // 2
    seen_conn = 0
    class_of_canon = {}
    ids = set()
    for mask in range(1 << pairs):
        adj = pins.adj_of_mask(k, mask)
        got = oracle.classify(k, adj)
        if not pins.connected(k, adj):
            assert got == -1
            continue
        seen_conn += 1
        canon = pins.canonical(k, adj)
        if canon not in class_of_canon:
            class_of_canon[canon] = pins.class_by_constants(k, adj)
        assert got == class_of_canon[canon], (mask, got, class_of_canon[canon])
        ids.add(got)
    # textbook counts: connected labelled graphs (1, 1, 4, 38, 728, ...) and
    # connected unlabelled graphs (1, 1, 2, 6, 21, ...)
    assert seen_conn == n_connected
    assert len(class_of_canon) == n_classes
    assert ids == set(range(1, n_classes + 1))


def test_pattern_automorphisms():
    assert pins.automorphisms(4, pins.P4_PATH) == 2
    assert pins.automorphisms(4, pins.P4_STAR) == 6
    assert pins.automorphisms(5, pins.P5_PATH) == 2
    assert pins.automorphisms(5, pins.P5_FORK) == 2
    assert pins.automorphisms(5, pins.P5_STAR) == 24


def test_named_motifs():
    """Ids that the text fixes in words: M_1^(4) is the 3-path whose copies MOSS-4
    counts, M_2^(4) the 3-star counted by Lambda_3, M_1^(5) the 4-path (Path-5),
    M_2^(5) the 4-star (Lambda_4), M_3^(5) the T shape sampled by T-5."""
    def adj_from_edges(k, edges):
        a = [[0] * k for _ in range(k)]
        for x, y in edges:
            a[x][y] = a[y][x] = 1
        return a
    assert oracle.classify(4, adj_from_edges(4, pins.P4_PATH)) == 1
    assert oracle.classify(4, adj_from_edges(4, pins.P4_STAR)) == 2
    assert oracle.classify(4, adj_from_edges(4, [(0, 1), (1, 2), (2, 3), (3, 0), (0, 2), (1, 3)])) == 6
    assert oracle.classify(5, adj_from_edges(5, pins.P5_PATH)) == 1
    assert oracle.classify(5, adj_from_edges(5, pins.P5_STAR)) == 2
    assert oracle.classify(5, adj_from_edges(5, pins.P5_FORK)) == 3
    k5 = [(i, j) for i in range(5) for j in range(i + 1, 5)]
    assert oracle.classify(5, adj_from_edges(5, k5)) == 21
    c5 = [(0, 1), (1, 2), (2, 3), (3, 4), (4, 0)]
    assert oracle.classify(5, adj_from_edges(5, c5)) == 6
