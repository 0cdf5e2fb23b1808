"""moss_sample_range_noalloc against moss_sample_range, through the C ABI.

The no-allocation call must give the same hits and per-sample classes as the call it is
a variant of, on two calls in a row where the second covers a smaller range (the fixed
scratch keeps the first call's contents), with the XCD-grouped schedule (which sorts
each chunk in the fixed scratch) and the plain one, for every sampler; and it must
refuse, without drawing anything, a range beyond its scratch and a graph whose tables
are not built."""
import numpy as np
import pytest
import torch

import graphgen as gg
from paper_1509_08089_amd import moss

pytestmark = pytest.mark.gpu

SAMPLERS = [moss.MOSS_SAMPLER_MOSS4, moss.MOSS_SAMPLER_MOSS4MIN, moss.MOSS_SAMPLER_T5, moss.MOSS_SAMPLER_PATH5]
ALL_TABLES = moss.MOSS_TABLES_K4 | moss.MOSS_TABLES_K5 | moss.MOSS_TABLES_K4MIN


@pytest.fixture(scope="module")
def big():
    """n = 1e5, m = 1e6: its sampled bytes pass 32 MB, so ranges of at least 1.5 * 2^20
    samples run XCD-grouped by default."""
    G = moss.Graph(gg.config_graph("C2"))
    G.build_tables(ALL_TABLES)
    assert G.info().sampling_bytes >= 32 << 20
    return G


def _same(G, sampler, seed, k0, k1):
    n = k1 - k0
    c_ref = torch.zeros(max(n, 1), dtype=torch.uint8, device="cuda")
    c_new = torch.full((max(n, 1),), 0xAB, dtype=torch.uint8, device="cuda")
    h_ref = moss.moss_sample_range(G.h, sampler, seed, k0, k1, c_ref if n else None)
    h_new = moss.moss_sample_range_noalloc(G.h, sampler, seed, k0, k1, c_new if n else None)
    np.testing.assert_array_equal(h_new, h_ref)
    if n:
        assert torch.equal(c_new[:n], c_ref[:n]), (sampler, k0, k1)
    return h_new


@pytest.mark.parametrize("sampler", SAMPLERS)
def test_grouped_two_calls_second_smaller(big, sampler):
    top = moss.MOSS_NOALLOC_MAX_SAMPLES
    h1 = _same(big, sampler, 7, 123, 123 + top)              # the largest range: one full chunk
    h2 = _same(big, sampler, 7, 2**40 + 5, 2**40 + 5 + 1_600_000)  # smaller, grouped as well
    drawn = lambda h: int(h[:7].sum()) if sampler == moss.MOSS_SAMPLER_MOSS4MIN else int(h.sum())  # noqa: E731
    assert drawn(h1) == top and drawn(h2) == 1_600_000


@pytest.mark.parametrize("schedule", [moss.MOSS_SCHEDULE_XCD, moss.MOSS_SCHEDULE_PLAIN])
@pytest.mark.parametrize("sampler", SAMPLERS)
def test_forced_schedules(big, sampler, schedule):
    moss.moss_set_tuning(0, 0, 0, schedule)
    try:
        _same(big, sampler, 11, 0, 300_001)
        _same(big, sampler, 11, 2**63 - 70_000, 2**63 - 3)  # smaller, ragged, far into the index space
        _same(big, sampler, 11, 5, 5)                       # empty
    finally:
        moss.moss_set_tuning(0, 0, 0, 0)


def test_splitting_a_range_adds_up(big):
    """A range beyond the scratch goes as several calls; their hits add up to the whole."""
    top = moss.MOSS_NOALLOC_MAX_SAMPLES
    whole = moss.moss_sample_range(big.h, moss.MOSS_SAMPLER_T5, 3, 0, 2 * top + 1000)
    parts = sum(moss.moss_sample_range_noalloc(big.h, moss.MOSS_SAMPLER_T5, 3, a, b)
                for a, b in ((0, top), (top, 2 * top), (2 * top, 2 * top + 1000)))
    np.testing.assert_array_equal(parts, whole)


def test_zero_weight_sampler_clears_classes():
    """A star has no 3-path (Gamma = 0): no sample is drawn and every class byte is 0."""
    G = moss.Graph(gg.star(40))
    G.build_tables(moss.MOSS_TABLES_K4)
    c = torch.full((5000,), 0xAB, dtype=torch.uint8, device="cuda")
    h = moss.moss_sample_range_noalloc(G.h, moss.MOSS_SAMPLER_MOSS4, 1, 10, 5010, c)
    assert int(h.sum()) == 0 and int(c.sum().item()) == 0


def test_refuses_without_drawing(big):
    with pytest.raises(moss.MossError) as e:
        moss.moss_sample_range_noalloc(big.h, moss.MOSS_SAMPLER_MOSS4, 1, 0, moss.MOSS_NOALLOC_MAX_SAMPLES + 1)
    assert e.value.status == moss.MOSS_E_TOO_LARGE
    G = moss.Graph(gg.gnp(60, 0.2, 5))  # no tables built: the call must not build them
    before = G.info().device_bytes
    with pytest.raises(moss.MossError) as e:
        moss.moss_sample_range_noalloc(G.h, moss.MOSS_SAMPLER_T5, 1, 0, 1000)
    assert e.value.status == moss.MOSS_E_NOT_BUILT
    assert G.info().built_mask == 0 and G.info().device_bytes == before
