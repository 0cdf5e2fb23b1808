"""Pin of the oracle's line-count mode (the algorithmic-bytes figure of the roofline).

The quantity: the mean, over the samples of one seed, of the number of distinct 64-byte
lines a sample reads when it follows the sampling contract with plain binary searches
and shares nothing with other samples.  Every table starts on a 64-byte boundary and
entry i of a table of w-byte elements lives in line floor(i * w / 64).

This file recomputes that count in pure Python, from the steps of the samplers as the
paper states them (MOSS-4: Section 4.1.1 with the initialization of Section 4.1.3;
MOSS-4Min: Section 4.2.1; T-5: Section 5.1.1; Path-5: Sections 5.1.2 and 5.1.5), with
its own tables built from their definitions (Table 1), numpy's Philox for the random
words, and Python's `bisect` run over instrumented sequences that note every element
it looks at.  Read rules of the count:
  - a weighted pick over an inclusive prefix of L entries (smallest i with A[i] > x)
    is a binary search over the first L - 1 entries (the last one is the answer when
    no earlier entry qualifies), plus one read of the last entry, which is the total
    the random word is scaled by (the node picks are scaled by a global total and read
    no table entry for it);
  - a row is found from row_ptr[v] and row_ptr[v + 1] (two i32 reads);
  - a neighbour at index j of a row is one read of col; a uniform neighbour other than
    a given one reads the entry at j and, when it is at or above the excluded node, the
    next one;
  - the induced-edge test of a pair {a, b} reads both rows' bounds and binary-searches
    the shorter row (the row of the node drawn first on a tie) for the other node,
    stopping at the first probe that finds it; only the pairs whose adjacency the
    sampled structure leaves open are tested, and a rejected sample tests none.
The test requires exact equality with the oracle's mean, so a wrong element width, a
known pair that is probed, a missing row_ptr read or a search over the wrong range
fails it.
"""
from __future__ import annotations

import bisect

import numpy as np
import pytest

import graphgen as gg
import oracle

M64 = (1 << 64) - 1
LINE = 64


def words(seed: int, tag: int, k: int, j: int):
    """Philox4x64-10 block with counter (k, j, 0, 0) and key (seed, tag), via numpy
    (numpy increments its counter once before each block)."""
    c = ((j << 64) | k) - 1
    ctr = np.array([(c >> (64 * i)) & M64 for i in range(4)], dtype=np.uint64)
    bg = np.random.Philox(key=np.array([seed, tag], dtype=np.uint64), counter=ctr)
    return [int(x) for x in bg.random_raw(4)]


def bounded(x: int, n: int) -> int:
    return (x * n) >> 64


class Noted:
    """A table whose element reads are noted as (table, line) pairs."""

    def __init__(self, name: str, data, width: int, lines: set):
        self.name, self.data, self.width, self.lines = name, data, width, lines
        self.trace = []

    def __len__(self):
        return len(self.data)

    def __getitem__(self, i):
        self.lines.add((self.name, (i * self.width) // LINE))
        self.trace.append(i)
        return self.data[i]


class Tables:
    """The sampling tables of Section 4.1.3 (and Table 1 for MOSS-4Min) from their
    definitions, as plain Python integers."""

    def __init__(self, csr):
        rp = [int(x) for x in csr.row_ptr]
        col = [int(x) for x in csr.col]
        n = len(rp) - 1
        d = [rp[v + 1] - rp[v] for v in range(n)]
        self.rp, self.col, self.n, self.d = rp, col, n, d
        S = [sum(d[x] - 1 for x in col[rp[v]:rp[v + 1]]) for v in range(n)]
        Q = [sum((d[x] - 1) ** 2 for x in col[rp[v]:rp[v + 1]]) for v in range(n)]
        gam = [(d[v] - 1) * S[v] if d[v] else 0 for v in range(n)]
        gam1 = [(d[v] - 1) * (d[v] - 2) * S[v] if d[v] >= 2 else 0 for v in range(n)]
        gam2 = [S[v] * S[v] - Q[v] for v in range(n)]
        self.acc_node = {"moss4": _acc(gam), "t5": _acc(gam1), "path5": _acc(gam2)}
        self.acc_sigma, self.acc_tau = [], []
        for v in range(n):
            row = col[rp[v]:rp[v + 1]]
            self.acc_sigma += _acc([d[u] - 1 for u in row])
            self.acc_tau += _acc([(d[u] - 1) * (S[v] - (d[u] - 1)) for u in row])
        # MOSS-4Min: a above b when (d_a, a) > (d_b, b); d_{v,x} = |{y in N_v above x}|
        key = [(d[x], x) for x in range(n)]
        self.rank, self.rank_mirror, self.col_rank, self.acc_check = [], [], [], []
        gmin = []
        for v in range(n):
            row = col[rp[v]:rp[v + 1]]
            dvx = [sum(1 for y in row if key[y] > key[x]) for x in row]
            dxv = [sum(1 for y in col[rp[x]:rp[x + 1]] if key[y] > key[v]) for x in row]
            self.rank += dvx
            self.rank_mirror += dxv
            self.col_rank += sorted(row, key=lambda y: key[y], reverse=True)
            prods = [a * b for a, b in zip(dvx, dxv)]
            self.acc_check += _acc(prods)
            gmin.append(sum(prods))
        self.acc_node["moss4min"] = _acc(gmin)


def _acc(xs):
    out, s = [], 0
    for x in xs:
        s += x
        out.append(s)
    return out


# pairs of the node order (v, u, w, r[, t]) that the sampled structure leaves open
OPEN = {
    "moss4": [(0, 3), (1, 2), (2, 3)],
    "moss4min": [(0, 3), (1, 2), (2, 3)],
    "t5": [(0, 4), (1, 2), (1, 3), (2, 3), (2, 4), (3, 4)],
    "path5": [(0, 3), (0, 4), (1, 2), (1, 4), (2, 3), (3, 4)],
}
TAG = {"moss4": oracle.MOSS4, "moss4min": oracle.MOSS4MIN, "t5": oracle.T5, "path5": oracle.PATH5}


def lines_of_sample(tb: Tables, sampler: str, seed: int, k: int) -> int:
    lines: set = set()
    rp = Noted("row_ptr", tb.rp, 4, lines)
    col = Noted("col", tb.col, 4, lines)
    acc_node = Noted("acc_node", tb.acc_node[sampler], 8, lines)
    sig = Noted("acc_sigma", tb.acc_sigma, 4, lines)
    tau = Noted("acc_tau", tb.acc_tau, 8, lines)
    chk = Noted("acc_check", tb.acc_check, 8, lines)
    rank = Noted("rank", tb.rank, 4, lines)
    rank_m = Noted("rank_mirror", tb.rank_mirror, 4, lines)
    col_rank = Noted("col_rank", tb.col_rank, 4, lines)

    def pick(table, base, length, word):
        total = table[base + length - 1]
        return bisect.bisect_right(table, bounded(word, total), base, base + length - 1) - base

    def pick_node(word):
        total = tb.acc_node[sampler][-1]  # the global total, no table read
        return bisect.bisect_right(acc_node, bounded(word, total), 0, tb.n - 1)

    def other_neighbour(a, excluded, word):
        base, end = rp[a], rp[a + 1]
        j = bounded(word, end - base - 1)
        x = col[base + j]
        return col[base + j + 1] if x >= excluded else x

    def adjacent(a, b):
        ra, ra1, rb, rb1 = rp[a], rp[a + 1], rp[b], rp[b + 1]
        lo, hi, key = (ra, ra1, b) if ra1 - ra <= rb1 - rb else (rb, rb1, a)
        probe = Noted("col", tb.col, 4, set())
        bisect.bisect_left(probe, key, lo, hi)
        for i in probe.trace:  # the search stops at the probe that finds the key
            col[i]
            if tb.col[i] == key:
                return True
        return False

    W = words(seed, TAG[sampler], k, 0)
    if sampler == "moss4":
        v = pick_node(W[0])
        base, dv = rp[v], rp[v + 1] - rp[v]
        iu = pick(sig, base, dv, W[1])
        u = col[base + iu]
        j = bounded(W[2], dv - 1)
        w = col[base + j + (j >= iu)]
        r = other_neighbour(u, v, W[3])
        nodes = [v, u, w, r]
        rejected = r == w
    elif sampler == "moss4min":
        v = pick_node(W[0])
        base, dv = rp[v], rp[v + 1] - rp[v]
        iu = pick(chk, base, dv, W[1])
        u = col[base + iu]
        dvu, duv = rank[base + iu], rank_m[base + iu]
        w = col_rank[base + bounded(W[2], dvu)]
        r = col_rank[rp[u] + bounded(W[3], duv)]
        nodes = [v, u, w, r]
        rejected = r == w
    elif sampler == "t5":
        W2 = words(seed, TAG[sampler], k, 1)
        v = pick_node(W[0])
        base, dv = rp[v], rp[v + 1] - rp[v]
        iu = pick(sig, base, dv, W[1])
        u = col[base + iu]
        iw = bounded(W[2], dv - 1)
        iw += iw >= iu
        w = col[base + iw]
        ir = bounded(W[3], dv - 2)
        for s in sorted((iu, iw)):
            ir += ir >= s
        r = col[base + ir]
        t = other_neighbour(u, v, W2[0])
        nodes = [v, u, w, r, t]
        rejected = t in (w, r)
    else:  # path5
        W2 = words(seed, TAG[sampler], k, 1)
        v = pick_node(W[0])
        base, dv = rp[v], rp[v + 1] - rp[v]
        iu = pick(tau, base, dv, W[1])
        u = col[base + iu]
        # mu draw over N_v - {u}: the row's sigma prefix with u's block cut out
        sv = sig[base + dv - 1]
        lo = sig[base + iu - 1] if iu else 0
        blk = sig[base + iu] - lo
        x = bounded(W[2], sv - blk)
        x += blk if x >= lo else 0
        iw = bisect.bisect_right(sig, x, base, base + dv - 1) - base
        w = col[base + iw]
        r = other_neighbour(u, v, W[3])
        t = other_neighbour(w, v, W2[0])
        nodes = [v, u, w, r, t]
        rejected = t == u or r == w or t == r
    if not rejected:
        for a, b in OPEN[sampler]:
            adjacent(nodes[a], nodes[b])
    return len(lines)


def mean_lines(csr, sampler: str, seed: int, k0: int, k1: int) -> float:
    tb = Tables(csr)
    total = sum(lines_of_sample(tb, sampler, seed, k) for k in range(k0, k1))
    return total / (k1 - k0)


GRAPHS = {
    "path": lambda: gg.path(40),
    "wheel": lambda: gg.wheel(60),
    "spider": lambda: gg.from_edges(  # a star with a path hanging off every leaf
        1 + 2 * 70, [(0, i) for i in range(1, 71)] + [(i, 70 + i) for i in range(1, 71)], "spider"),
    "gnp": lambda: gg.gnp(90, 0.12, 7),
    "chung_lu": lambda: gg.chung_lu(400, 2400, 2.3, 120, 9),
}


def _valid(csr, sampler):
    tb = Tables(csr)
    return tb.acc_node[sampler][-1] > 0


@pytest.mark.parametrize("name", sorted(GRAPHS))
@pytest.mark.parametrize("sampler", ["moss4", "moss4min", "t5", "path5"])
def test_line_count_matches_definition(name, sampler):
    csr = GRAPHS[name]()
    if not _valid(csr, sampler):
        pytest.skip(f"{sampler} has zero total weight on {name}")
    og = oracle.Graph(csr)
    for seed, k0, k1 in ((1, 0, 300), (12345, 2**40, 2**40 + 200)):
        want = mean_lines(csr, sampler, seed, k0, k1)
        got = og.line_count(TAG[sampler], seed, k0, k1)
        assert got == want, (name, sampler, seed, got, want)


def test_line_count_sees_every_read_rule():
    """The count must move with each read rule: a hub row searched by many samples has
    more lines than a path, and a sample that is rejected probes no pair."""
    hub = gg.wheel(60)
    path = gg.path(40)
    assert mean_lines(hub, "moss4", 1, 0, 200) > mean_lines(path, "moss4", 1, 0, 200)
    tb = Tables(hub)
    counts = [lines_of_sample(tb, "moss4", 1, k) for k in range(200)]
    assert min(counts) >= 6  # node pick, row_ptr, sigma total, u, w, r's row
