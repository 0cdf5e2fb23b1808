"""Symmetric sorted CSR container and conversion from undirected edge lists."""
from __future__ import annotations

import dataclasses
import hashlib

import numpy as np


@dataclasses.dataclass(frozen=True)
class CSR:
    """Undirected simple graph as CSR.

    row_ptr: int32[n+1], col: int32[2m].  Row v lists N_v in ascending order,
    every edge appears in both endpoint rows, no self-loops, no duplicates.
    """
    row_ptr: np.ndarray
    col: np.ndarray
    name: str = ""

    @property
    def n(self) -> int:
        return int(self.row_ptr.shape[0] - 1)

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])

    @property
    def m(self) -> int:
        return self.nnz // 2

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr.astype(np.int64))

    def neighbors(self, v: int) -> np.ndarray:
        return self.col[self.row_ptr[v]:self.row_ptr[v + 1]]

    def sha256(self) -> str:
        h = hashlib.sha256()
        h.update(np.ascontiguousarray(self.row_ptr).tobytes())
        h.update(np.ascontiguousarray(self.col).tobytes())
        return h.hexdigest()

    def adjacency_sets(self):
        return [set(int(x) for x in self.neighbors(v)) for v in range(self.n)]


def from_edges(n: int, edges, name: str = "") -> CSR:
    """Build a symmetric sorted CSR from undirected pairs (self-loops and repeats dropped)."""
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    if e.size:
        if e.min() < 0 or e.max() >= n:
            raise ValueError("edge endpoint out of range")
        a = np.minimum(e[:, 0], e[:, 1])
        b = np.maximum(e[:, 0], e[:, 1])
        keep = a != b
        a, b = a[keep], b[keep]
        key = np.unique(a * n + b)
        a, b = key // n, key % n
        src = np.concatenate([a, b])
        dst = np.concatenate([b, a])
    else:
        src = np.zeros(0, np.int64)
        dst = np.zeros(0, np.int64)
    order = np.lexsort((dst, src))
    src, dst = src[order], dst[order]
    counts = np.bincount(src, minlength=n) if n else np.zeros(0, np.int64)
    row_ptr = np.zeros(n + 1, np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    if row_ptr[-1] >= 2**31:
        raise ValueError("graph too large for int32 CSR")
    return CSR(row_ptr.astype(np.int32), dst.astype(np.int32), name)


def edges_of(g: CSR) -> np.ndarray:
    """Undirected edge list (a < b) of a CSR graph."""
    deg = g.degrees()
    src = np.repeat(np.arange(g.n, dtype=np.int64), deg)
    dst = g.col.astype(np.int64)
    keep = src < dst
    return np.stack([src[keep], dst[keep]], axis=1)
