"""Small deterministic graphs with textbook motif counts, plus seeded G(n, p)."""
from __future__ import annotations

import numpy as np

from .csr import CSR, from_edges


def path(n: int) -> CSR:
    return from_edges(n, [(i, i + 1) for i in range(n - 1)], f"P{n}")


def cycle(n: int) -> CSR:
    return from_edges(n, [(i, (i + 1) % n) for i in range(n)], f"C{n}")


def star(s: int) -> CSR:
    """K_{1,s}: node 0 is the centre."""
    return from_edges(s + 1, [(0, i) for i in range(1, s + 1)], f"K1,{s}")


def complete(n: int) -> CSR:
    return from_edges(n, [(i, j) for i in range(n) for j in range(i + 1, n)], f"K{n}")


def complete_bipartite(a: int, b: int) -> CSR:
    return from_edges(a + b, [(i, a + j) for i in range(a) for j in range(b)], f"K{a},{b}")


def wheel(s: int) -> CSR:
    """Hub 0 joined to every node of the cycle 1..s."""
    e = [(0, i) for i in range(1, s + 1)]
    e += [(i, i % s + 1) for i in range(1, s + 1)]
    return from_edges(s + 1, e, f"W{s}")


def gnp(n: int, p: float, seed: int) -> CSR:
    rng = np.random.Generator(np.random.PCG64(seed))
    iu, ju = np.triu_indices(n, 1)
    keep = rng.random(iu.shape[0]) < p
    return from_edges(n, np.stack([iu[keep], ju[keep]], 1), f"G({n},{p},{seed})")
