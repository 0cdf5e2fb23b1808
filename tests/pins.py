"""Independent checks for the oracle: small exact computations in pure Python.

Nothing here shares code with the oracle.  Motif ids are tied to the paper's
printed constants (Section 4.1.2 for 4 nodes, Table 2 for 5 nodes) by counting
pattern embeddings with permutations, a different method from the oracle's
spanning-tree enumeration.  Sampling distributions are written from the
sampler descriptions of Sections 4.1.1, 5.1.1 and 5.1.2 in exact rationals.
"""
from __future__ import annotations

import itertools
from fractions import Fraction
from math import comb

# --- the paper's printed constants (Section 4.1.2 and Table 2) -------------
PHI4_1 = {1: 1, 2: 0, 3: 4, 4: 2, 5: 6, 6: 12}          # 3-paths in M_i^(4)
PHI4_2 = {1: 0, 2: 1, 3: 0, 4: 1, 5: 2, 6: 4}           # 3-stars in M_i^(4)
_T2 = {
    1: (0, 1, 0), 2: (0, 0, 1), 3: (1, 0, 0), 4: (1, 2, 0), 5: (2, 2, 0), 6: (0, 5, 0),
    7: (2, 1, 0), 8: (2, 0, 1), 9: (4, 4, 0), 10: (4, 7, 0), 11: (5, 2, 1), 12: (4, 4, 1),
    13: (6, 6, 0), 14: (10, 10, 1), 15: (9, 6, 1), 16: (12, 6, 2), 17: (10, 14, 0),
    18: (20, 24, 1), 19: (20, 18, 2), 20: (36, 36, 3), 21: (60, 60, 5),
}
PHI5_1 = {i: t[0] for i, t in _T2.items()}   # forks (M_3^(5)) in M_i^(5)
PHI5_2 = {i: t[1] for i, t in _T2.items()}   # 4-paths (M_1^(5))
PHI5_3 = {i: t[2] for i, t in _T2.items()}   # 4-stars (M_2^(5))

# patterns as edge lists on labelled nodes
P4_PATH = [(0, 1), (1, 2), (2, 3)]
P4_STAR = [(0, 1), (0, 2), (0, 3)]
P5_PATH = [(0, 1), (1, 2), (2, 3), (3, 4)]
P5_FORK = [(0, 1), (0, 2), (0, 3), (3, 4)]
P5_STAR = [(0, 1), (0, 2), (0, 3), (0, 4)]


def _edge_set(edges):
    return {frozenset(e) for e in edges}


def automorphisms(k, edges) -> int:
    es = _edge_set(edges)
    return sum(1 for p in itertools.permutations(range(k))
               if {frozenset((p[a], p[b])) for a, b in edges} == es)


def embeddings(k, pattern, adj) -> int:
    """Number of (not necessarily induced) copies of `pattern` spanning the k nodes."""
    cnt = 0
    for p in itertools.permutations(range(k)):
        if all(adj[p[a]][p[b]] for a, b in pattern):
            cnt += 1
    return cnt // automorphisms(k, pattern)


def connected(k, adj) -> bool:
    seen = {0}
    stack = [0]
    while stack:
        a = stack.pop()
        for b in range(k):
            if adj[a][b] and b not in seen:
                seen.add(b)
                stack.append(b)
    return len(seen) == k


def canonical(k, adj) -> int:
    best = None
    for p in itertools.permutations(range(k)):
        code = 0
        bit = 0
        for i in range(k):
            for j in range(i + 1, k):
                if adj[p[i]][p[j]]:
                    code |= 1 << bit
                bit += 1
        if best is None or code < best:
            best = code
    return best


def class_by_constants(k, adj) -> int:
    """Motif id of a connected k-node graph from the paper's constants."""
    if k == 4:
        key = (embeddings(4, P4_PATH, adj), embeddings(4, P4_STAR, adj))
        hits = [i for i in PHI4_1 if (PHI4_1[i], PHI4_2[i]) == key]
    else:
        key = (embeddings(5, P5_FORK, adj), embeddings(5, P5_PATH, adj), embeddings(5, P5_STAR, adj))
        hits = [i for i in _T2 if _T2[i] == key]
    if len(hits) != 1:
        raise ValueError(f"no unique class for constants {key}")
    return hits[0]


def adj_of_mask(k, mask):
    adj = [[0] * k for _ in range(k)]
    bit = 0
    for i in range(k):
        for j in range(i + 1, k):
            if mask >> bit & 1:
                adj[i][j] = adj[j][i] = 1
            bit += 1
    return adj


_CLASS_CACHE = {}


def class_of_nodes(adjsets, nodes) -> int:
    k = len(nodes)
    adj = [[1 if nodes[j] in adjsets[nodes[i]] else 0 for j in range(k)] for i in range(k)]
    if not connected(k, adj):
        return 0
    c = canonical(k, adj)
    key = (k, c)
    if key not in _CLASS_CACHE:
        _CLASS_CACHE[key] = class_by_constants(k, adj)
    return _CLASS_CACHE[key]


def brute_counts(csr, k):
    """n_i or eta_i by trying every k-subset (Section 2's definition)."""
    adjsets = csr.adjacency_sets()
    counts = [0] * 22
    for nodes in itertools.combinations(range(csr.n), k):
        c = class_of_nodes(adjsets, nodes)
        if c:
            counts[c] += 1
    return counts


def triangles_per_node(csr):
    adjsets = csr.adjacency_sets()
    t = [0] * csr.n
    for a in range(csr.n):
        for b in adjsets[a]:
            if b > a:
                for c in adjsets[a] & adjsets[b]:
                    if c > b:
                        t[a] += 1
                        t[b] += 1
                        t[c] += 1
    return t


# --- exact sampler distributions (rationals), from the sampler descriptions ---
def _deg(adjsets):
    return [len(s) for s in adjsets]


def moss4_distribution(csr):
    """{tuple (v,u,w,r): probability} for MOSS-4 (Section 4.1.1)."""
    A = [sorted(s) for s in csr.adjacency_sets()]
    d = [len(a) for a in A]
    gam_v = [(d[v] - 1) * sum(d[x] - 1 for x in A[v]) if d[v] else 0 for v in range(csr.n)]
    G = sum(gam_v)
    out = {}
    for v in range(csr.n):
        if gam_v[v] == 0:
            continue
        S = sum(d[x] - 1 for x in A[v])
        for u in A[v]:
            if d[u] < 2:
                continue
            pu = Fraction(gam_v[v], G) * Fraction(d[u] - 1, S)
            for w in A[v]:
                if w == u:
                    continue
                for r in A[u]:
                    if r == v:
                        continue
                    out[(v, u, w, r)] = pu / (d[v] - 1) / (d[u] - 1)
    return out, G


def t5_distribution(csr):
    A = [sorted(s) for s in csr.adjacency_sets()]
    d = [len(a) for a in A]
    g1 = [(d[v] - 1) * (d[v] - 2) * sum(d[x] - 1 for x in A[v]) if d[v] >= 2 else 0 for v in range(csr.n)]
    G = sum(g1)
    out = {}
    for v in range(csr.n):
        if g1[v] == 0:
            continue
        S = sum(d[x] - 1 for x in A[v])
        for u in A[v]:
            if d[u] < 2:
                continue
            pu = Fraction(g1[v], G) * Fraction(d[u] - 1, S)
            for w in A[v]:
                if w == u:
                    continue
                for r in A[v]:
                    if r in (u, w):
                        continue
                    for t in A[u]:
                        if t == v:
                            continue
                        out[(v, u, w, r, t)] = pu / (d[v] - 1) / (d[v] - 2) / (d[u] - 1)
    return out, G


def path5_distribution(csr):
    A = [sorted(s) for s in csr.adjacency_sets()]
    d = [len(a) for a in A]
    S = [sum(d[x] - 1 for x in A[v]) for v in range(csr.n)]
    Q = [sum((d[x] - 1) ** 2 for x in A[v]) for v in range(csr.n)]
    g2 = [S[v] ** 2 - Q[v] for v in range(csr.n)]
    G = sum(g2)
    out = {}
    for v in range(csr.n):
        if g2[v] == 0:
            continue
        for u in A[v]:
            rest = S[v] - (d[u] - 1)
            tau = Fraction((d[u] - 1) * rest, g2[v])
            if tau == 0:
                continue
            for w in A[v]:
                if w == u or d[w] < 2:
                    continue
                mu = Fraction(d[w] - 1, rest)
                for r in A[u]:
                    if r == v:
                        continue
                    for t in A[w]:
                        if t == v:
                            continue
                        out[(v, u, w, r, t)] = Fraction(g2[v], G) * tau * mu / (d[u] - 1) / (d[w] - 1)
    return out, G


def rejected(sampler, tup):
    if sampler == "moss4":
        v, u, w, r = tup
        return r == w
    if sampler == "t5":
        v, u, w, r, t = tup
        return t in (w, r)
    v, u, w, r, t = tup
    return t == u or r == w or t == r


def class_distribution(csr, sampler):
    """P(class i) for one sample, {class: Fraction} with class 0 = rejected, and the
    probability of each sampled node set."""
    dist, G = {"moss4": moss4_distribution, "t5": t5_distribution, "path5": path5_distribution}[sampler](csr)
    adjsets = csr.adjacency_sets()
    by_class = {}
    by_set = {}
    for tup, p in dist.items():
        if rejected(sampler, tup):
            c = 0
        else:
            c = class_of_nodes(adjsets, tup)
            key = frozenset(tup)
            by_set[key] = by_set.get(key, 0) + p
        by_class[c] = by_class.get(c, 0) + p
    return by_class, by_set, G, dist


def choose(n, r):
    return comb(n, r) if n >= r >= 0 else 0


# --- MOSS-4Min (Section 4.2.1), exact rationals ------------------------------
# The order of Section 3.2's example: a above b when d_a > d_b, or d_a = d_b and a > b.
def above(d, a, b) -> bool:
    return d[a] > d[b] or (d[a] == d[b] and a > b)


def moss4min_weights(csr):
    """d_{v,x} = |{y in N_v : y above x}| for every entry, check-Gamma_v and each row in
    descending order, counted pair by pair from Table 1's definitions."""
    A = [sorted(s) for s in csr.adjacency_sets()]
    d = [len(a) for a in A]
    dvx = {}
    for v in range(csr.n):
        for x in A[v]:
            dvx[(v, x)] = sum(1 for y in A[v] if above(d, y, x))
    gmin = [sum(dvx[(v, x)] * dvx[(x, v)] for x in A[v]) for v in range(csr.n)]
    desc = []
    for v in range(csr.n):
        row = list(A[v])
        # insertion by pairwise comparison: y goes before every x it is above
        ordered = []
        for y in row:
            pos = 0
            while pos < len(ordered) and above(d, ordered[pos], y):
                pos += 1
            ordered.insert(pos, y)
        desc.append(ordered)
    return A, d, dvx, gmin, desc


def moss4min_distribution(csr):
    """{(v, u, w, r): probability} of the five steps of Section 4.2.1: v with weight
    check-Gamma_v, u in N_v with weight d_{u,v} d_{v,u}, w uniform in N_{v,u}, r uniform
    in N_{u,v}."""
    A, d, dvx, gmin, _ = moss4min_weights(csr)
    G = sum(gmin)
    out = {}
    for v in range(csr.n):
        if gmin[v] == 0:
            continue
        for u in A[v]:
            wu = dvx[(u, v)] * dvx[(v, u)]
            if wu == 0:
                continue
            pu = Fraction(gmin[v], G) * Fraction(wu, gmin[v])
            Nvu = [x for x in A[v] if above(d, x, u)]
            Nuv = [x for x in A[u] if above(d, x, v)]
            for w in Nvu:
                for r in Nuv:
                    out[(v, u, w, r)] = pu / len(Nvu) / len(Nuv)
    return out, G


def ways(adjsets, d, nodes) -> int:
    """c(s): ordered tuples (w, v, u, r) of the set with edges w-v, v-u, u-r, w above u and
    r above v (by permutations)."""
    c = 0
    for w, v, u, r in itertools.permutations(nodes):
        if v in adjsets[w] and u in adjsets[v] and r in adjsets[u] and above(d, w, u) and above(d, r, v):
            c += 1
    return c
