"""Launch schedules: the XCD-grouped schedule (samples grouped by the top bits of their
first random word, one group per XCD) must draw every sample exactly once with the
outcome the plain grid-stride schedule and the oracle give it, for any range, block
size and occupancy, and across its internal chunks."""
import numpy as np
import pytest
import torch

import graphgen as gg
import oracle
from gpu_util import ORACLE_SAMPLER
from paper_1509_08089_amd import moss

pytestmark = pytest.mark.gpu

SAMPLERS = [moss.MOSS_SAMPLER_MOSS4, moss.MOSS_SAMPLER_T5, moss.MOSS_SAMPLER_PATH5]


@pytest.fixture
def schedule():
    def set_(sch, bpc=0, tpb=0):
        moss.moss_set_tuning(0, bpc, tpb, sch)
    yield set_
    moss.moss_set_tuning(0, 0, 0, 0)


@pytest.fixture(scope="module")
def small():
    return gg.chung_lu(2000, 10000, 2.5, 200, 1)


@pytest.fixture(scope="module")
def mid():
    return gg.chung_lu(20000, 150000, 2.1, 2000, 34)


@pytest.mark.parametrize("sampler", SAMPLERS)
@pytest.mark.parametrize("bpc,tpb", [(0, 0), (1, 64), (3, 128), (8, 256)])
def test_grouped_per_sample_classes(small, schedule, sampler, bpc, tpb):
    G, og = moss.Graph(small), oracle.Graph(small)
    k0, k1 = 1234, 1234 + 70_001  # not a multiple of the group window
    schedule(moss.MOSS_SCHEDULE_XCD, bpc, tpb)
    cls = torch.full((k1 - k0,), 255, dtype=torch.uint8, device="cuda")
    hits = G.sample_range(sampler, 7, k0, k1, cls)
    c = cls.cpu().numpy()
    osid = ORACLE_SAMPLER[sampler]
    want = np.array([og.sample(osid, 7, k)[0] for k in range(k0, k1)], dtype=np.uint8)
    np.testing.assert_array_equal(c, want)  # every sample drawn once, with its own outcome
    np.testing.assert_array_equal(hits, np.bincount(want, minlength=22)[:22])


@pytest.mark.parametrize("k", [4, 5])
def test_grouped_estimate_equals_plain(mid, schedule, k):
    G = moss.Graph(mid)
    schedule(moss.MOSS_SCHEDULE_PLAIN)
    a = G.estimate(k, 3_000_001, 9)
    schedule(moss.MOSS_SCHEDULE_XCD)
    b = G.estimate(k, 3_000_001, 9)
    np.testing.assert_array_equal(a.hits_np, b.hits_np)
    np.testing.assert_array_equal(a.estimate_np, b.estimate_np)


def test_grouped_across_chunks(mid, schedule):
    """More samples than one grouped launch takes (2^25): the chunks must join up."""
    G = moss.Graph(mid)
    n = (1 << 25) * 2 + 12_345
    schedule(moss.MOSS_SCHEDULE_PLAIN)
    a = G.sample_range(moss.MOSS_SAMPLER_MOSS4, 3, 5, 5 + n)
    schedule(moss.MOSS_SCHEDULE_XCD)
    b = G.sample_range(moss.MOSS_SAMPLER_MOSS4, 3, 5, 5 + n)
    np.testing.assert_array_equal(a, b)
    assert int(b.sum()) == n


@pytest.mark.parametrize("n", [64 * 8192, 65 * 8192 + 333])
def test_grouped_classes_over_many_count_rows(mid, schedule, n):
    """Past 64 blocks of 8192 samples the grouping passes sum several count rows per run
    before scanning across runs (64 rows: one per run; 66 rows: two per run in 33 runs);
    every sample must still be drawn exactly once, with the outcome the plain launch
    gives it."""
    G = moss.Graph(mid)
    k0 = 11
    out = []
    for sch in (moss.MOSS_SCHEDULE_PLAIN, moss.MOSS_SCHEDULE_XCD):
        schedule(sch)
        cls = torch.full((n,), 255, dtype=torch.uint8, device="cuda")
        hits = G.sample_range(moss.MOSS_SAMPLER_MOSS4, 4, k0, k0 + n, cls)
        out.append((hits, cls.cpu().numpy()))
    (ha, ca), (hb, cb) = out
    assert (ca != 255).all()
    np.testing.assert_array_equal(ca, cb)
    np.testing.assert_array_equal(ha, hb)


def test_tiny_and_empty_ranges(small, schedule):
    G, og = moss.Graph(small), oracle.Graph(small)
    schedule(moss.MOSS_SCHEDULE_XCD)
    for k0, k1 in [(0, 0), (5, 6), (100, 163), (0, 4096), (7, 4096 + 7 + 1)]:
        hits = G.sample_range(moss.MOSS_SAMPLER_T5, 2, k0, k1)
        np.testing.assert_array_equal(hits, og.run(oracle.T5, 2, k0, k1, 4))
