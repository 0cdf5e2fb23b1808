"""Power-law Chung-Lu graphs ("erased" edge variant) standing in for the SNAP graphs.

Expected-degree weights follow Chung & Lu (2002): w_i proportional to (i + i0)^(-1/(beta-1)),
scaled so that sum(w) = 2m, with i0 solved numerically so that the largest weight is
dmax (this form also covers beta = 2, where the closed-form parametrisation breaks
down).  Endpoint pairs are drawn i.i.d. with probability proportional to w from a
PCG64 stream; self-loops and repeated pairs are dropped and the first m distinct
pairs (in draw order) are kept, so the graph has exactly m edges.  A seeded random
relabelling then scatters hubs over the id range, as in real graphs.
"""
from __future__ import annotations

import numpy as np

from .csr import CSR, from_edges


def chung_lu_weights(n: int, m: int, beta: float, dmax: float) -> np.ndarray:
    alpha = 1.0 / (beta - 1.0)
    idx = np.arange(n, dtype=np.float64)
    target = dmax / (2.0 * m)

    def top_share(log_i0: float) -> float:
        w = np.exp(-alpha * np.log(idx + np.exp(log_i0)))
        return w[0] / w.sum()

    lo, hi = np.log(1e-9), np.log(1e13)
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if top_share(mid) > target:
            lo = mid          # too concentrated: shift the curve right
        else:
            hi = mid
    i0 = np.exp(0.5 * (lo + hi))
    w = np.exp(-alpha * np.log(idx + i0))
    return w * (2.0 * m / w.sum())


def chung_lu(n: int, m: int, beta: float, dmax: float, seed: int, name: str = "") -> CSR:
    if m > n * (n - 1) // 2:
        raise ValueError("more edges than a simple graph on n nodes can hold")
    rng = np.random.Generator(np.random.PCG64(seed))
    w = chung_lu_weights(n, m, beta, dmax)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    keys = np.zeros(0, np.int64)
    batch = int(m * 1.2) + 16
    while True:
        a = np.searchsorted(cdf, rng.random(batch), side="right")
        b = np.searchsorted(cdf, rng.random(batch), side="right")
        np.minimum(a, n - 1, out=a)
        np.minimum(b, n - 1, out=b)
        lo = np.minimum(a, b).astype(np.int64)
        hi = np.maximum(a, b).astype(np.int64)
        k = lo * n + hi
        keys = np.concatenate([keys, k[lo != hi]])
        uniq, first = np.unique(keys, return_index=True)
        if uniq.shape[0] >= m:
            first.sort()
            keys = keys[first[:m]]
            break
        batch = int((m - uniq.shape[0]) * 1.5) + 1024
    perm = rng.permutation(n).astype(np.int64)
    e = np.stack([perm[keys // n], perm[keys % n]], axis=1)
    return from_edges(n, e, name or f"chung_lu(n={n},m={m},beta={beta},dmax={dmax},seed={seed})")
