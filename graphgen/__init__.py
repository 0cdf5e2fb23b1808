"""Seeded synthetic graph inputs shared by the oracle tests, the GPU tests and the
benchmark.

This module only builds graphs: undirected, simple, symmetric CSR with every row
sorted ascending (the input form of the problem statement, Section 2; edge labels
and directions are dropped as in Table 3's preprocessing).  It holds none of the
estimator's arithmetic.

Contents
  chung_lu_device(...)               the same recipe generated on a torch device
  chung_lu(n, m, beta, dmax, seed)   power-law "erased" Chung-Lu graph with exactly
                                     m distinct edges and a seeded node relabelling
  gnp(n, p, seed), path(n), cycle(n), star(s), complete(n), complete_bipartite(a, b),
  wheel(s)                           small special graphs for closed-form checks
  from_edges(n, edges)               CSR from an undirected edge list
  workload_*                         request mixes for the batched / serving runs
"""
from .csr import CSR, from_edges, edges_of
from .special import path, cycle, star, complete, complete_bipartite, wheel, gnp
from .chung_lu import chung_lu, chung_lu_weights
from .chung_lu_device import chung_lu_device
from .workloads import (CONFIGS, config_graph, batch_workload, serving_workload,
                        graph_family)

__all__ = [
    "CSR", "from_edges", "edges_of", "path", "cycle", "star", "complete",
    "complete_bipartite", "wheel", "gnp", "chung_lu", "chung_lu_weights", "chung_lu_device",
    "CONFIGS", "config_graph", "batch_workload", "serving_workload", "graph_family",
]
