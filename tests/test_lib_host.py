"""The C-ABI library on the CPU: it loads, exports every declared symbol, and its
host-side logic (classification tables, estimator finals) agrees with the oracle.
No call here touches a GPU."""
import os
import re

import numpy as np
import pytest

import oracle
from paper_1509_08089_amd import moss

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "moss.h")).read()
    return sorted(set(re.findall(r"^(?:moss_status|const char \*)\s*(moss_\w+)\(", text, re.M)))


def test_library_exports_every_declared_symbol():
    L = moss.lib()
    decl = declared_symbols()
    assert len(decl) >= 20
    assert set(decl) == set(moss.EXPORTED)
    for name in decl:
        assert hasattr(L, name), name


def test_status_strings():
    for code in moss.STATUS:
        assert moss.moss_status_string(code)


# node order v, u, w, r, t; pairs fixed by each sampler, then the probed pairs in bit order
STRUCTURE = {
    moss.MOSS_SAMPLER_MOSS4: (4, [(0, 1), (0, 2), (1, 3)], [(1, 2), (0, 3), (2, 3)]),
    moss.MOSS_SAMPLER_MOSS4MIN: (4, [(0, 1), (0, 2), (1, 3)], [(1, 2), (0, 3), (2, 3)]),
    moss.MOSS_SAMPLER_T5: (5, [(0, 1), (0, 2), (0, 3), (1, 4)], [(1, 2), (1, 3), (2, 3), (0, 4), (2, 4), (3, 4)]),
    moss.MOSS_SAMPLER_PATH5: (5, [(0, 1), (0, 2), (1, 3), (2, 4)], [(0, 3), (0, 4), (1, 2), (1, 4), (2, 3), (3, 4)]),
}


@pytest.mark.parametrize("sampler", list(STRUCTURE))
def test_class_tables_match_oracle_classifier(sampler):
    k, known, probes = STRUCTURE[sampler]
    lut = moss.moss_class_lut(sampler)
    assert len(lut) == 1 << len(probes)
    for mask in range(1 << len(probes)):
        adj = np.zeros((k, k), np.uint8)
        for a, b in known:
            adj[a, b] = adj[b, a] = 1
        for i, (a, b) in enumerate(probes):
            if mask >> i & 1:
                adj[a, b] = adj[b, a] = 1
        assert int(lut[mask]) == oracle.classify(k, adj), (sampler, mask)


def _same(a, b):
    """The library's finals and the oracle's evaluate the same written formulas in the
    same order in double, so they must agree to the last bit (stricter than the 1e-12
    relative bound the estimates are held to)."""
    return a == b or (a != a and b != b)


@pytest.mark.parametrize("seed", range(100))
def test_finals4_match_oracle(seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    K = int(rng.integers(1, 10**9))
    hits = rng.multinomial(K, rng.dirichlet(np.ones(7))).astype(np.uint64)
    hits[2] = 0  # class 2 is never sampled by MOSS-4
    K = int(hits.sum()) or 1
    gamma = int(rng.integers(0, 2**62)) if seed % 4 else 0
    lam = int(rng.integers(0, 2**60))
    r = moss.moss_result()
    r.k, r.K[0], r.gamma[0], r.lambda_ = 4, K, gamma, lam
    for i in range(7):
        r.hits[0][i] = int(hits[i])
    moss.moss_finals(r)
    est, var = oracle.finals4(K, hits, gamma, lam)
    for i in range(6):
        assert _same(r.estimate[i], est[i]), (i, r.estimate[i], est[i])
        assert _same(r.variance[i], var[i]), (i, r.variance[i], var[i])


@pytest.mark.parametrize("seed", range(100))
@pytest.mark.parametrize("mix", [moss.MOSS_MIX_POOLED, moss.MOSS_MIX_PAPER])
def test_finals5_match_oracle(seed, mix):
    rng = np.random.Generator(np.random.PCG64(100 + seed))
    K1 = int(rng.integers(1, 10**8))
    K2 = K1 - int(rng.integers(0, 2)) or 1
    h1 = rng.multinomial(K1, rng.dirichlet(np.ones(22) * 0.5)).astype(np.uint64)
    h2 = rng.multinomial(K2, rng.dirichlet(np.ones(22) * 0.5)).astype(np.uint64)
    g1 = int(rng.integers(0, 2**60)) if seed % 5 else 0
    g2 = int(rng.integers(0, 2**60)) if seed % 7 else 0
    lam = int(rng.integers(0, 2**62))
    r = moss.moss_result()
    r.k, r.flags, r.K[0], r.K[1], r.lambda_ = 5, mix, K1, K2, lam
    r.gamma[0], r.gamma[1] = g1, g2
    for i in range(22):
        r.hits[0][i] = int(h1[i])
        r.hits[1][i] = int(h2[i])
    moss.moss_finals(r)
    est, var, _ = oracle.finals5(K1, K2, h1, h2, g1, g2, lam, mix)
    for i in range(21):
        assert _same(r.estimate[i], est[i]), (i, r.estimate[i], est[i])
        assert _same(r.variance[i], var[i]), (i, r.variance[i], var[i])


@pytest.mark.parametrize("seed", range(100))
@pytest.mark.parametrize("mix", [moss.MOSS_MIX_POOLED, moss.MOSS_MIX_PAPER])
def test_finals4_min_match_oracle(seed, mix):
    """MOSS-4 mixed with MOSS-4Min (reach-count bins in hits[1][7..9])."""
    rng = np.random.Generator(np.random.PCG64(300 + seed))
    K = int(rng.integers(1, 10**8))
    Kc = K - int(rng.integers(0, 2)) or 1
    h4 = rng.multinomial(K, rng.dirichlet(np.ones(7))).astype(np.uint64)
    hm = np.zeros(22, np.uint64)
    hm[:7] = rng.multinomial(Kc, rng.dirichlet(np.ones(7)))
    hm[7:10] = rng.multinomial(int(hm[5]), rng.dirichlet(np.ones(3)))
    gamma = int(rng.integers(1, 2**60)) if seed % 5 else 0
    gmin = int(rng.integers(0, gamma + 1)) if seed % 3 else 0
    lam = int(rng.integers(0, 2**60))
    r = moss.moss_result()
    r.k, r.flags, r.K[0], r.K[1], r.lambda_ = 4, mix | moss.MOSS_K4_MIN, K, Kc, lam
    r.gamma[0], r.gamma[1] = gamma, gmin
    for i in range(22):
        r.hits[0][i] = int(h4[i]) if i < 7 else 0
        r.hits[1][i] = int(hm[i])
    moss.moss_finals(r)
    est, var = oracle.finals4min(K, h4, gamma, lam, Kc, hm[:10], gmin, mix)
    for i in range(6):
        assert _same(r.estimate[i], est[i]), (i, r.estimate[i], est[i])
        assert _same(r.variance[i], var[i]), (i, r.variance[i], var[i])


def _pilot_pair(rng, n_motifs):
    """The same pilot result as the library's struct and the oracle's."""
    est = rng.lognormal(8, 3, n_motifs) * (rng.random(n_motifs) < 0.8)
    est[rng.random(n_motifs) < 0.1] *= -1
    var = rng.lognormal(10, 4, n_motifs) * (rng.random(n_motifs) < 0.9)
    K = [int(rng.integers(1, 10**9)), int(rng.integers(0, 10**9)) if n_motifs == 21 else 0]
    r = moss.moss_result()
    o = oracle._Result()
    for x in (r, o):
        x.k, x.n_motifs = (4, 6) if n_motifs == 6 else (5, 21)
        x.K[0], x.K[1] = K
        for i in range(n_motifs):
            x.estimate[i], x.variance[i] = float(est[i]), float(var[i])
    return r, oracle.Result(o)


@pytest.mark.parametrize("seed", range(20))
def test_plan_budget_matches_oracle(seed):
    rng = np.random.Generator(np.random.PCG64(500 + seed))
    r, o = _pilot_pair(rng, 6 if seed % 2 else 21)
    eps = float(10 ** rng.uniform(-3, -0.5))
    delta = float(10 ** rng.uniform(-8, -0.1))
    mask = int(rng.integers(0, 1 << 21)) if seed % 3 else 0
    b, mx = moss.moss_plan_budget(r, eps, delta, mask)
    ob, omx = oracle.plan_budget(o, eps, delta, mask)
    np.testing.assert_array_equal(b, ob)
    assert mx == omx
    np.testing.assert_allclose(moss.moss_concentrations(r), oracle.concentrations(o), rtol=1e-14, atol=0)


def test_plan_budget_rejects_bad_arguments():
    r, _ = _pilot_pair(np.random.Generator(np.random.PCG64(1)), 6)
    for eps, delta in ((0.0, 0.1), (-1.0, 0.1), (0.1, 0.0), (0.1, 1.0), (float("nan"), 0.1)):
        with pytest.raises(moss.MossError):
            moss.moss_plan_budget(r, eps, delta)


def test_finals_reject_bad_arguments():
    r = moss.moss_result()
    r.k = 3
    with pytest.raises(moss.MossError):
        moss.moss_finals(r)
    r.k, r.K[0] = 4, 0
    with pytest.raises(moss.MossError):
        moss.moss_finals(r)
    r.k, r.K[0], r.K[1], r.flags = 4, 10, 0, moss.MOSS_K4_MIN  # no MOSS-4Min samples
    with pytest.raises(moss.MossError):
        moss.moss_finals(r)
    r.k, r.K[0], r.K[1], r.flags = 5, 10, 10, moss.MOSS_K4_MIN  # the flag is for k = 4
    with pytest.raises(moss.MossError):
        moss.moss_finals(r)


def test_probe_library_exports_and_rejects_bad_arguments():
    """libmoss_probe.so (the benchmark's gather probe) exports what moss_probe.h declares
    and rejects bad arguments before any launch."""
    import ctypes
    from paper_1509_08089_amd import probe
    text = open(os.path.join(ROOT, "include", "moss_probe.h")).read()
    decl = sorted(set(re.findall(r"^int\s+(moss_probe_\w+)\(", text, re.M)))
    assert decl == sorted(probe.EXPORTED)
    L = probe.lib()
    P = ctypes.c_void_p
    fake = P(4096)  # never dereferenced: every call below fails its argument checks first
    assert L.moss_probe_fill(None, 10, 1, None) == -1
    assert L.moss_probe_fill(fake, 0, 1, None) == -1
    assert L.moss_probe_gather(None, 10, 1, 1, 1, fake, None) == -1
    assert L.moss_probe_gather(fake, 10, 1, 1, 1, None, None) == -1
    assert L.moss_probe_gather(fake, 0, 1, 1, 1, fake, None) == -1
    assert L.moss_probe_gather(fake, 10, 0, 1, 1, fake, None) == -1
    assert L.moss_probe_gather(fake, 10, (1 << 20) + 1, 1, 1, fake, None) == -1
    assert L.moss_probe_gather(fake, 10, 1, 0, 1, fake, None) == -1
    assert L.moss_probe_gather(fake, 10, 1, (1 << 20) + 1, 1, fake, None) == -1
    for chains in (0, 3, 5, 16):
        assert L.moss_probe_gather(fake, 10, 1, 1, chains, fake, None) == -1

def test_tuning_knobs_round_trip_and_bounds():
    """The launch knobs are host state: set, read back, and bad values refused."""
    try:
        moss.moss_set_tuning(4096, 6, 256, moss.MOSS_SCHEDULE_XCD, 19, 8, 256)
        t = moss.moss_get_tuning()
        assert (t.tile_samples, t.blocks_per_cu, t.threads_per_block, t.schedule, t.group_min_samples_log2,
                t.group_min_footprint_mb, t.sort_window) == (4096, 6, 256, moss.MOSS_SCHEDULE_XCD, 19, 8, 256)
        for bad in ((0, 0, 96, 0, 0, 0), (0, 65, 0, 0, 0, 0), (0, 0, 0, 3, 0, 0), (0, 0, 0, 0, 41, 0),
                    (0, 0, 0, 0, 0, (1 << 20) + 1), (0, 0, 0, 0, 0, 0, 100), (0, 0, 0, 0, 0, 0, 576)):
            with pytest.raises(moss.MossError):
                moss.moss_set_tuning(*bad)
    finally:
        moss.moss_set_tuning(0, 0, 0)
    assert moss.moss_get_tuning().group_min_samples_log2 == 0 and moss.moss_get_tuning().sort_window == 0
