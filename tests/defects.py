"""CSR defects for the creation checks: a graph whose rows exercise the 256-entry span
bookkeeping of the GPU checks, single-edit defects placed at span edges and row heads,
and a plain validator written from the rules (column range, no self-loops, strictly
ascending rows, symmetry) that reports the highest-priority defect found, as the
library does.  Used by the GPU creation tests and, against the oracle's own validator,
by a CPU test."""
import numpy as np

import graphgen as gg

ARG, UNSORTED, SELF_LOOP, DUPLICATE, ASYMMETRIC = -1, -2, -3, -4, -5
PRIORITY = [ARG, SELF_LOOP, DUPLICATE, UNSORTED, ASYMMETRIC]


def expected_status(rp, col):
    n, nnz = len(rp) - 1, len(col)
    found = set()
    upper, lower = set(), []
    n_upper = 0
    for v in range(n):
        for e in range(rp[v], rp[v + 1]):
            c = int(col[e])
            if c < 0 or c >= n:
                found.add(ARG)
                continue
            if c == v:
                found.add(SELF_LOOP)
            if e > rp[v]:
                if col[e - 1] == c:
                    found.add(DUPLICATE)
                elif col[e - 1] > c:
                    found.add(UNSORTED)
            if c > v:
                upper.add((v, c))
                n_upper += 1
            elif c < v:
                lower.append((c, v))
    if any(x not in upper for x in lower) or 2 * n_upper != nnz:
        found.add(ASYMMETRIC)
    for s in PRIORITY:
        if s in found:
            return s
    return 0


def span_graph():
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


def edge_positions(rp, nnz):
    """Entries at span edges and row heads at or next to span boundaries."""
    pos = {e for e in range(nnz) if e % 256 in (0, 1, 63, 64, 127, 128, 255)}
    heads = set(int(x) for x in rp[:-1][np.diff(rp) > 0])
    pos |= {h for h in heads if h % 256 in (0, 1, 255)}
    return sorted(pos)


def cases(rp, col, positions=None):
    nnz = len(col)
    heads = set(int(x) for x in rp[:-1][np.diff(rp) > 0])
    row_of = np.repeat(np.arange(len(rp) - 1), np.diff(rp))
    for e in (edge_positions(rp, nnz)[::3] if positions is None else positions):
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
