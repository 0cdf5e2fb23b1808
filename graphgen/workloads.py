"""The benchmark graphs and request mixes.

Graph recipe (all synthetic; they stand in for the SNAP graphs of the paper's
Table 3, which are not reproduced): power-law Chung-Lu, seeded by the config id.

  C1  n=2,000      m=10,000      beta=2.5  dmax=200     k=4, 1e5 samples, seed 1
  C2  n=100,000    m=1,000,000   beta=2.2  dmax=3,000   k=4, 1e7 samples, seed 1
  C3  n=1,000,000  m=10,000,000  beta=2.1  dmax=20,000  k=5, 1e8 samples, seed 1
  C4  32 graphs, m log-uniform in [1e3, 5e6], n=max(100, m/10), beta=2.2,
      dmax=min(3000, n/4); 256 requests: graph uniform, k in {4,5}, budget
      log-uniform in [1e4, 1e7], seed = request index + 1
  C5  64 graphs, m log-uniform in [1e3, 3.5e7] (the largest fixed at n=4e6,
      m=3.5e7, beta=2.0, dmax=2e4); Poisson arrivals at 500 req/s, k in {4,5},
      budget log-uniform in [1e4, 1e8]
"""
from __future__ import annotations

import dataclasses
import math
import os

import numpy as np

from .chung_lu import chung_lu
from .csr import CSR


@dataclasses.dataclass(frozen=True)
class GraphSpec:
    n: int
    m: int
    beta: float
    dmax: float
    seed: int

    def build(self):
        """The graph on the host.  With MOSS_GRAPH_CACHE naming a directory, the CSR is
        kept there as an .npz after the first build and read back by later builds."""
        name = f"CL(n={self.n},m={self.m},beta={self.beta},dmax={self.dmax},seed={self.seed})"
        cache = os.environ.get("MOSS_GRAPH_CACHE")
        path = None
        if cache:
            path = os.path.join(cache, f"cl_{self.n}_{self.m}_{self.beta}_{self.dmax}_{self.seed}.npz")
            if os.path.exists(path):
                with np.load(path) as z:
                    return CSR(z["row_ptr"], z["col"], name)
        g = chung_lu(self.n, self.m, self.beta, self.dmax, self.seed, name=name)
        if path:
            os.makedirs(cache, exist_ok=True)
            tmp = path + ".tmp.npz"
            np.savez(tmp, row_ptr=g.row_ptr, col=g.col)
            os.replace(tmp, path)
        return g

    def build_device(self, device="cuda"):
        """(row_ptr, col) int32 tensors generated on the device (see chung_lu_device)."""
        from .chung_lu_device import chung_lu_device
        return chung_lu_device(self.n, self.m, self.beta, self.dmax, self.seed, device)


CONFIGS = {
    "C1": dict(graph=GraphSpec(2_000, 10_000, 2.5, 200, 1), k=4, samples=100_000, seed=1),
    "C2": dict(graph=GraphSpec(100_000, 1_000_000, 2.2, 3_000, 2), k=4, samples=10_000_000, seed=1),
    "C3": dict(graph=GraphSpec(1_000_000, 10_000_000, 2.1, 20_000, 3), k=5, samples=100_000_000, seed=1),
}


def config_graph(name: str):
    return CONFIGS[name]["graph"].build()


def _family_spec(m: int, seed: int) -> GraphSpec:
    n = max(100, m // 10)
    m = min(m, n * (n - 1) // 4)
    return GraphSpec(n, m, 2.2, float(min(3000, n // 4)), seed)


def graph_family(count: int, m_lo: float, m_hi: float, seed: int, largest: GraphSpec | None = None):
    """Specs of `count` graphs with m log-uniform in [m_lo, m_hi] (PCG64(seed))."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ms = np.rint(10 ** rng.uniform(math.log10(m_lo), math.log10(m_hi), size=count)).astype(np.int64)
    specs = [_family_spec(int(m), 1000 * seed + i) for i, m in enumerate(ms)]
    if largest is not None:
        specs[-1] = largest
    return specs


@dataclasses.dataclass(frozen=True)
class Request:
    graph: int
    k: int
    samples: int
    seed: int
    arrival_s: float = 0.0


def batch_workload(n_requests: int = 256, n_graphs: int = 32, budget_lo: float = 1e4,
                   budget_hi: float = 1e7, seed: int = 4):
    """C4: graph specs plus the request list (graph uniform, k in {4,5}, log-uniform budget)."""
    specs = graph_family(n_graphs, 1e3, 5e6, seed)
    rng = np.random.Generator(np.random.PCG64(seed))
    g = rng.integers(0, n_graphs, size=n_requests)
    k = np.where(rng.random(n_requests) < 0.5, 4, 5)
    b = np.rint(10 ** rng.uniform(math.log10(budget_lo), math.log10(budget_hi), size=n_requests))
    reqs = [Request(int(g[i]), int(k[i]), int(b[i]), i + 1) for i in range(n_requests)]
    return specs, reqs


def serving_workload(n_requests: int = 5000, n_graphs: int = 64, rate: float = 500.0,
                     budget_lo: float = 1e4, budget_hi: float = 1e8, m_hi: float = 3.5e7,
                     largest: GraphSpec | None = GraphSpec(4_000_000, 35_000_000, 2.0, 20_000, 5063),
                     seed: int = 5):
    """C5: graph specs plus a Poisson request stream (exponential gaps at `rate`/s)."""
    specs = graph_family(n_graphs, 1e3, m_hi, seed, largest=largest)
    rng = np.random.Generator(np.random.PCG64(seed))
    gaps = rng.exponential(1.0 / rate, size=n_requests)
    t = np.cumsum(gaps)
    g = rng.integers(0, n_graphs, size=n_requests)
    k = np.where(rng.random(n_requests) < 0.5, 4, 5)
    b = np.rint(10 ** rng.uniform(math.log10(budget_lo), math.log10(budget_hi), size=n_requests))
    reqs = [Request(int(g[i]), int(k[i]), int(b[i]), i + 1, float(t[i])) for i in range(n_requests)]
    return specs, reqs
