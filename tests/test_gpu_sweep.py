"""A seeded sweep of GPU-vs-oracle parity over many small graphs of different shapes.

Each case draws a graph (G(n,p) at several densities, power-law Chung-Lu, stars,
wheels, complete and complete bipartite graphs, disjoint unions), a sampler, a seed and
a ragged sample range, and compares the GPU's hit counts and per-sample classes with the
oracle's bit for bit, and the finals of a whole estimate within 1e-12."""
import numpy as np
import pytest
import torch

import graphgen as gg
import oracle
from gpu_util import ORACLE_SAMPLER, assert_result_matches
from paper_1509_08089_amd import moss

pytestmark = pytest.mark.gpu

SAMPLERS = (moss.MOSS_SAMPLER_MOSS4, moss.MOSS_SAMPLER_MOSS4MIN, moss.MOSS_SAMPLER_T5, moss.MOSS_SAMPLER_PATH5)


def _union(a, b):
    ea = gg.edges_of(a)
    eb = gg.edges_of(b) + a.n
    return gg.from_edges(a.n + b.n, np.concatenate([ea, eb]), f"{a.name}+{b.name}")


def _graph(rng, i):
    kind = i % 7
    if kind == 0:
        n = int(rng.integers(6, 60))
        return gg.gnp(n, float(rng.uniform(0.05, 0.9)), int(rng.integers(1, 10**6)))
    if kind == 1:
        n = int(rng.integers(50, 3000))
        m = int(n * rng.uniform(1.5, 8))
        return gg.chung_lu(n, m, float(rng.uniform(2.05, 3.0)), max(8.0, n / rng.uniform(3, 30)),
                           int(rng.integers(1, 10**6)))
    if kind == 2:
        return gg.star(int(rng.integers(3, 400)))
    if kind == 3:
        return gg.wheel(int(rng.integers(4, 600)))
    if kind == 4:
        return gg.complete(int(rng.integers(4, 40)))
    if kind == 5:
        return gg.complete_bipartite(int(rng.integers(1, 12)), int(rng.integers(2, 500)))
    return _union(gg.gnp(int(rng.integers(5, 30)), 0.4, int(rng.integers(1, 999))), gg.star(int(rng.integers(3, 80))))


@pytest.mark.parametrize("case", range(40))
def test_sweep_sample_ranges(case):
    rng = np.random.Generator(np.random.PCG64(7000 + case))
    g = _graph(rng, case)
    G, og = moss.Graph(g), oracle.Graph(g)
    for sampler in SAMPLERS:
        osid = ORACLE_SAMPLER[sampler]
        total = og.totals()[{oracle.MOSS4: "gamma", oracle.MOSS4MIN: "gamma_min", oracle.T5: "gamma1",
                             oracle.PATH5: "gamma2"}[osid]]
        seed = int(rng.integers(0, 2**63))
        k0 = int(rng.integers(0, 2**40))
        n = int(rng.integers(1, 30_000))
        cls = torch.zeros(n, dtype=torch.uint8, device="cuda")
        hits = G.sample_range(sampler, seed, k0, k0 + n, cls)
        np.testing.assert_array_equal(hits, og.run(osid, seed, k0, k0 + n, 8), err_msg=f"{g.name} {sampler}")
        if total == 0:
            assert not hits.any() and not cls.any()
            continue
        idx = rng.integers(0, n, size=min(n, 200))
        c = cls.cpu().numpy()
        for j in idx:
            assert int(c[j]) == og.sample(osid, seed, k0 + int(j))[0], (g.name, sampler, int(j))


@pytest.mark.parametrize("case", range(20))
def test_sweep_estimates(case):
    rng = np.random.Generator(np.random.PCG64(9000 + case))
    g = _graph(rng, case + 3)
    G, og = moss.Graph(g), oracle.Graph(g)
    K = int(rng.integers(2, 200_000))
    seed = int(rng.integers(0, 2**63))
    mix = int(rng.integers(0, 2))
    t = og.totals()
    assert_result_matches(G.estimate(4, K, seed, mix), og.estimate(4, K, seed, mix, threads=8), float(t["lambda3"]))
    assert_result_matches(G.estimate(4, K, seed, mix | moss.MOSS_K4_MIN), og.estimate4min(K, seed, mix, threads=8),
                          float(t["lambda3"]))
    assert_result_matches(G.estimate(5, K, seed, mix), og.estimate(5, K, seed, mix, threads=8), float(t["lambda4"]))
