"""Batched persistent launches and the serving loop: each request's result must be
identical to the same request run alone (moss_estimate), whatever else shares the
launch, the tile size, the occupancy, the chunking or the arrival order."""
import time

import numpy as np
import pytest

import graphgen as gg
import oracle
from gpu_util import assert_result_matches
from paper_1509_08089_amd import moss

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def graphs():
    gs = [gg.chung_lu(300, 1500, 2.4, 40, 31), gg.chung_lu(4000, 30000, 2.2, 500, 32),
          gg.gnp(25, 0.3, 33), gg.star(12), gg.cycle(12), gg.chung_lu(20000, 150000, 2.1, 2000, 34)]
    return gs, [moss.Graph(g) for g in gs]


def _requests(handles, n, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(n):
        k = 4 if rng.random() < 0.5 else 5
        budget = int(10 ** rng.uniform(1, 6))
        out.append((handles[int(rng.integers(0, len(handles)))].h, k, max(budget, 2), i + 1,
                    int(rng.integers(0, 2))))
    return out


def _alone(req):
    g, k, ns, seed, flags = req
    return moss.moss_estimate(g, k, ns, seed, flags)


def test_batch_equals_single_requests(graphs):
    gs, handles = graphs
    reqs = _requests(handles, 60, 1)
    alone = [_alone(q) for q in reqs]
    for rep in range(3):  # replays of the captured graph, with other work in between
        got = moss.moss_estimate_batch(reqs)
        for a, b in zip(alone, got):
            np.testing.assert_array_equal(a.hits_np, b.hits_np)
            np.testing.assert_array_equal(a.estimate_np, b.estimate_np)
        _alone(reqs[rep])


def test_batch_matches_oracle(graphs):
    gs, handles = graphs
    reqs = [(handles[1].h, 4, 123_457, 5, 0), (handles[1].h, 5, 98_765, 6, 0), (handles[0].h, 5, 4_001, 7, 1)]
    got = moss.moss_estimate_batch(reqs)
    for (h, k, ns, seed, flags), r, g in zip(reqs, got, [gs[1], gs[1], gs[0]]):
        og = oracle.Graph(g)
        lam = og.totals()["lambda3" if k == 4 else "lambda4"]
        assert_result_matches(r, og.estimate(k, ns, seed, flags, threads=8), float(lam))


@pytest.mark.parametrize("tile", [256, 4096])
def test_sorted_batch_equals_single_requests(graphs, tile):
    """With the XCD schedule forced, every batched item runs as grouped launches of its
    own after the persistent kernel (one item spans two 2^25-sample chunks): the hits
    must equal each request run alone."""
    gs, handles = graphs
    reqs = _requests(handles, 30, 3) + [(handles[1].h, 4, (1 << 25) + 4097, 77, 0),
                                        (handles[5].h, 5, 300_001, 78, 0), (handles[0].h, 4, 2, 79, 1)]
    alone = [_alone(q) for q in reqs]
    moss.moss_set_tuning(tile, 0, 0, moss.MOSS_SCHEDULE_XCD)
    try:
        for _ in range(2):
            got = moss.moss_estimate_batch(reqs)
            for a, b in zip(alone, got):
                np.testing.assert_array_equal(a.hits_np, b.hits_np)
                np.testing.assert_array_equal(a.estimate_np, b.estimate_np)
    finally:
        moss.moss_set_tuning(0, 0, 0, 0)


def test_large_items_sorted_by_default():
    """A graph past 32 MB of sampled bytes with items of 2^20 samples or more: drawn by
    grouped launches beside the persistent kernel by default; results equal the
    requests alone, mixed with small items."""
    G = moss.Graph(gg.config_graph("C2"))
    small = moss.Graph(gg.chung_lu(300, 1500, 2.4, 40, 31))
    reqs = [(G.h, 4, 1_500_000, 11, 0), (G.h, 5, 1_200_001, 12, 1), (G.h, 4, 2_000_000, 13, moss.MOSS_K4_MIN),
            (small.h, 4, 50_000, 14, 0), (G.h, 4, 1000, 15, 0)]
    assert moss.moss_graph_get_info(G.h).sampling_bytes >= 32 << 20
    alone = [_alone(q) for q in reqs]
    got = moss.moss_estimate_batch(reqs)
    for a, b in zip(alone, got):
        np.testing.assert_array_equal(a.hits_np, b.hits_np)
        np.testing.assert_array_equal(a.estimate_np, b.estimate_np)


@pytest.mark.parametrize("tile,bpc", [(256, 1), (4096, 2), (65536, 8), (1 << 20, 4)])
def test_tile_size_and_occupancy_do_not_change_results(graphs, tile, bpc):
    gs, handles = graphs
    reqs = _requests(handles, 24, 2)
    ref = [_alone(q) for q in reqs]
    moss.moss_set_tuning(tile, bpc, 0)
    try:
        got = moss.moss_estimate_batch(reqs)
    finally:
        moss.moss_set_tuning(0, 0, 0)
    for a, b in zip(ref, got):
        np.testing.assert_array_equal(a.hits_np, b.hits_np)


@pytest.mark.parametrize("lg,mb", [(10, 0), (12, 1), (17, 4), (40, 1 << 20)])
def test_grouping_thresholds_do_not_change_results(graphs, lg, mb):
    """Items of at least 2^lg samples on graphs of at least mb MB of sampled bytes leave the
    persistent kernel for grouped launches of their own (with 2^10 samples and 0 = the
    default 32 MB, then 1 MB, most items of the larger graphs do; with 2^40, none)."""
    gs, handles = graphs
    reqs = _requests(handles, 24, 5)
    ref = [_alone(q) for q in reqs]
    moss.moss_set_tuning(0, 0, 0, 0, lg, mb)
    try:
        t = moss.moss_get_tuning()
        assert (t.group_min_samples_log2, t.group_min_footprint_mb) == (lg, mb)
        got = moss.moss_estimate_batch(reqs)
    finally:
        moss.moss_set_tuning(0, 0, 0)
    for a, b in zip(ref, got):
        np.testing.assert_array_equal(a.hits_np, b.hits_np)
        np.testing.assert_array_equal(a.estimate_np, b.estimate_np)


@pytest.mark.parametrize("window", [64, 128, 512])
def test_sort_window_does_not_change_results(graphs, window):
    """The sorted kernel's window (samples a block takes at a time) only changes which
    lanes draw which samples: batched items sent to grouped launches (every item of
    2^10 samples or more on graphs of 1 MB or more) and a plain estimate on the largest
    graph, drawn grouped, give the results they give alone with the default window."""
    gs, handles = graphs
    reqs = _requests(handles, 24, 6)
    ref = [_alone(q) for q in reqs]
    plain_ref = moss.moss_estimate(handles[5].h, 4, 3_000_000, 9, 0)
    moss.moss_set_tuning(0, 0, 0, moss.MOSS_SCHEDULE_XCD, 10, 1, window)
    try:
        assert moss.moss_get_tuning().sort_window == window
        got = moss.moss_estimate_batch(reqs)
        plain = moss.moss_estimate(handles[5].h, 4, 3_000_000, 9, 0)
    finally:
        moss.moss_set_tuning(0, 0, 0)
    for a, b in zip(ref, got):
        np.testing.assert_array_equal(a.hits_np, b.hits_np)
        np.testing.assert_array_equal(a.estimate_np, b.estimate_np)
    np.testing.assert_array_equal(plain_ref.hits_np, plain.hits_np)


def test_autotune_keeps_results(graphs):
    gs, handles = graphs
    reqs = _requests(handles, 16, 3)
    best, ms = moss.moss_autotune(reqs)
    assert best.tile_samples > 0 and ms > 0 and best.group_min_samples_log2 in (0, *range(17, 23))
    got = moss.moss_estimate_batch(reqs)
    for q, b in zip(reqs, got):
        np.testing.assert_array_equal(_alone(q).hits_np, b.hits_np)
    moss.moss_set_tuning(0, 0, 0)


@pytest.mark.parametrize("express", [True, False])
def test_server_alone_and_in_mix(graphs, express):
    gs, handles = graphs
    reqs = _requests(handles, 80, 4)
    srv = moss.moss_server_create(0, 16, 50_000, express_samples=20_000, express=express)
    try:
        ids = [moss.moss_server_add_graph(srv, h.h) for h in handles]
        gid = {h.h.value: i for i, h in enumerate(handles)}
        tickets = []
        for j, (g, k, ns, seed, flags) in enumerate(reqs):
            tickets.append(moss.moss_server_submit(srv, ids[gid[g.value]], k, ns, seed, flags))
            if j % 10 == 0:
                time.sleep(0.002)  # arrivals while earlier requests run
        for q, t in zip(reqs, tickets):
            r = moss.moss_server_wait(srv, t, 60_000)
            a = _alone(q)
            np.testing.assert_array_equal(a.hits_np, r.hits_np)
            np.testing.assert_array_equal(a.estimate_np, r.estimate_np)
        st = moss.moss_server_stats_get(srv)
        assert st.completed == len(reqs) and st.p99_ms >= st.p50_ms > 0
        small = sum(1 for q in reqs if q[2] <= 20_000)
        assert 0 < small < len(reqs)
        if express:
            assert st.express_launches >= 1 and st.iterations >= 1
        else:
            assert st.express_launches == 0 and st.iterations >= 1
    finally:
        moss.moss_server_destroy(srv)


def test_server_concurrent_clients(graphs):
    """Four client threads submit and wait at once (the C calls release the interpreter
    lock), small requests and large ones on shared graphs: every result equals the same
    request alone (computed afterwards from this thread: a graph takes one direct call at
    a time, so the clients do not make their own)."""
    import threading
    gs, handles = graphs
    srv = moss.moss_server_create(0, 32, 1 << 18, iteration_samples=1 << 20, express_samples=50_000)
    errors, served = [], []
    try:
        ids = [moss.moss_server_add_graph(srv, h.h) for h in handles]

        def client(c):
            try:
                rng = np.random.Generator(np.random.PCG64(100 + c))
                mine = []
                for i in range(12):
                    gi = int(rng.integers(0, len(handles)))
                    k = 4 if rng.random() < 0.5 else 5
                    n = int(10 ** rng.uniform(3, 6.3))
                    seed = 1000 * c + i
                    mine.append((gi, k, n, seed, moss.moss_server_submit(srv, ids[gi], k, n, seed)))
                for gi, k, n, seed, t in mine:
                    served.append(((gi, k, n, seed), moss.moss_server_wait(srv, t, 120_000)))
            except Exception as e:  # reported below, from the test's own thread
                errors.append(e)

        threads = [threading.Thread(target=client, args=(c,)) for c in range(4)]
        for t in threads:
            t.start()
        for t in threads:
            t.join(300)
        assert not any(t.is_alive() for t in threads)
        assert not errors, errors[0]
        st = moss.moss_server_stats_get(srv)
        assert st.completed == 48 and st.queued == 0 and st.active == 0
    finally:
        moss.moss_server_destroy(srv)
    assert len(served) == 48
    for (gi, k, n, seed), r in served:
        a = moss.moss_estimate(handles[gi].h, k, n, seed, 0)
        np.testing.assert_array_equal(a.hits_np, r.hits_np)
        np.testing.assert_array_equal(a.estimate_np, r.estimate_np)


def test_server_express_beside_a_long_request(graphs):
    """Small requests submitted while a long request runs in the iterations take the
    express path: they finish while it is still running, with the results they have
    alone, and so does the long request.  Their graph is a fresh copy without tables,
    so its tables are built by the server's builder thread beside the long request
    before the express thread takes them."""
    gs, handles = graphs
    fresh = moss.Graph(gs[1])
    srv = moss.moss_server_create(0, 16, 1 << 20, iteration_samples=1 << 20)
    try:
        gid = moss.moss_server_add_graph(srv, handles[5].h)
        sid = moss.moss_server_add_graph(srv, fresh.h)
        t_long = moss.moss_server_submit(srv, gid, 5, 200_000_000, 7)
        small = [(sid, 4 + (i % 2), 50_000 + 1000 * i, 100 + i) for i in range(6)]
        ts = [moss.moss_server_submit(srv, *q) for q in small]
        for q, t in zip(small, ts):
            r = moss.moss_server_wait(srv, t, 60_000)
            a = moss.moss_estimate(handles[1].h, q[1], q[2], q[3], 0)
            np.testing.assert_array_equal(a.hits_np, r.hits_np)
            np.testing.assert_array_equal(a.estimate_np, r.estimate_np)
        st = moss.moss_server_stats_get(srv)
        assert st.express_launches >= 1
        assert st.active == 1  # the long request is still in its iterations
        r = moss.moss_server_wait(srv, t_long, 120_000)
        a = moss.moss_estimate(handles[5].h, 5, 200_000_000, 7, 0)
        np.testing.assert_array_equal(a.hits_np, r.hits_np)
    finally:
        moss.moss_server_destroy(srv)
        fresh.close()


def test_server_memory_budget_evicts_and_rejects():
    gs = [gg.chung_lu(3000, 20000, 2.2, 300, 40 + i) for i in range(4)]
    hs = [moss.Graph(g) for g in gs]
    probe = moss.Graph(gs[0])
    probe.build_tables(moss.MOSS_TABLES_K4)
    need = max(probe.info().device_bytes for _ in range(1))  # 4-node tables of one such graph
    probe.close()
    srv = moss.moss_server_create(int(need * 1.5), 4, 10_000)
    try:
        ids = [moss.moss_server_add_graph(srv, h.h) for h in hs]
        ts = [moss.moss_server_submit(srv, ids[i % 4], 4, 30_000, i + 1) for i in range(8)]
        for i, t in enumerate(ts):
            r = moss.moss_server_wait(srv, t, 60_000)
            np.testing.assert_array_equal(r.hits_np, hs[i % 4].estimate(4, 30_000, i + 1).hits_np)
            hs[i % 4].h  # keep alive
        st = moss.moss_server_stats_get(srv)
        assert st.evictions >= 1
        # a request whose tables can never fit the budget is refused, not queued forever
        big = moss.Graph(gg.chung_lu(50000, 400000, 2.2, 2000, 49))
        bid = moss.moss_server_add_graph(srv, big.h)
        t = moss.moss_server_submit(srv, bid, 5, 1000, 1)
        with pytest.raises(moss.MossError) as e:
            moss.moss_server_wait(srv, t, 60_000)
        assert e.value.status == moss.MOSS_E_ADMISSION
    finally:
        moss.moss_server_destroy(srv)


def _table_bytes(g, mask):
    """Device bytes that building `mask` on a fresh copy of graph g adds."""
    h = moss.Graph(g)
    try:
        before = h.info().device_bytes
        h.build_tables(mask)
        return h.info().device_bytes - before
    finally:
        h.close()


def test_server_evicts_own_idle_tables():
    """A budget that holds the 5-node tables alone but not beside the 4-node ones: after a
    k=4 request, a k=5 request on the same graph must evict the graph's own idle 4-node
    tables (not wait forever for memory no one will release), and the k=4 request after
    it must evict the 5-node ones."""
    g = gg.chung_lu(3000, 20000, 2.2, 300, 47)
    b4, b5, b45 = (_table_bytes(g, m) for m in
                   (moss.MOSS_TABLES_K4, moss.MOSS_TABLES_K5, moss.MOSS_TABLES_K4 | moss.MOSS_TABLES_K5))
    budget = b5 + (b45 - b5) // 2
    assert b4 <= budget and b5 <= budget < b45
    h = moss.Graph(g)
    srv = moss.moss_server_create(budget, 4, 10_000)
    try:
        gid = moss.moss_server_add_graph(srv, h.h)
        for i, k in enumerate((4, 5, 4, 5)):
            t = moss.moss_server_submit(srv, gid, k, 30_000, i + 1)
            r = moss.moss_server_wait(srv, t, 60_000)
            a = moss.Graph(g).estimate(k, 30_000, i + 1)
            np.testing.assert_array_equal(r.hits_np, a.hits_np)
            np.testing.assert_array_equal(r.estimate_np, a.estimate_np)
        st = moss.moss_server_stats_get(srv)
        assert st.evictions >= 3 and st.completed == 4 and st.table_bytes <= budget
    finally:
        moss.moss_server_destroy(srv)


def test_server_evicts_largest_idle_tables_first():
    """Two small graphs and a large one, used small, large, then the other small one,
    under a budget that holds the large tables and one small set but not a second small
    set beside them: the third request must evict the large graph's tables (the largest
    idle ones) and keep the first small graph's, though that one was used longer ago."""
    small = [gg.chung_lu(2000, 12000, 2.2, 200, 60 + i) for i in range(2)]
    large = gg.chung_lu(12000, 90000, 2.2, 800, 62)
    bs = max(_table_bytes(g, moss.MOSS_TABLES_K4) for g in small)
    bl = _table_bytes(large, moss.MOSS_TABLES_K4)
    budget = bl + bs + bs // 2
    assert bl > bs and bl + 2 * bs > budget
    hs = [moss.Graph(g) for g in small]
    hl = moss.Graph(large)
    base = [h.info().device_bytes for h in hs], hl.info().device_bytes
    srv = moss.moss_server_create(budget, 4, 10_000)
    try:
        ids = [moss.moss_server_add_graph(srv, h.h) for h in (hs[0], hl, hs[1])]
        for i, (gid, g) in enumerate(zip(ids, (small[0], large, small[1]))):
            r = moss.moss_server_wait(srv, moss.moss_server_submit(srv, gid, 4, 30_000, i + 1),
                                      60_000)
            np.testing.assert_array_equal(r.hits_np, moss.Graph(g).estimate(4, 30_000, i + 1).hits_np)
        st = moss.moss_server_stats_get(srv)
        assert st.evictions == 1 and st.table_bytes <= budget
        assert hl.info().device_bytes == base[1]            # large tables evicted
        assert hs[0].info().device_bytes > base[0][0]       # first small graph's kept
        assert hs[1].info().device_bytes > base[0][1]
    finally:
        moss.moss_server_destroy(srv)


def test_server_refuses_sets_that_never_fit_together():
    """MOSS-4 + MOSS-4Min needs the 4-node and the MOSS-4Min tables at once; with a budget
    below their sum and the 4-node tables already resident, the request is refused with
    MOSS_E_ADMISSION (no other graph or set can be evicted), and the server stays usable."""
    g = gg.chung_lu(3000, 20000, 2.2, 300, 48)
    both = _table_bytes(g, moss.MOSS_TABLES_K4 | moss.MOSS_TABLES_K4MIN)
    h = moss.Graph(g)
    srv = moss.moss_server_create(both - 1, 4, 10_000)
    try:
        gid = moss.moss_server_add_graph(srv, h.h)
        r = moss.moss_server_wait(srv, moss.moss_server_submit(srv, gid, 4, 20_000, 1), 60_000)
        np.testing.assert_array_equal(r.hits_np, moss.Graph(g).estimate(4, 20_000, 1).hits_np)
        t = moss.moss_server_submit(srv, gid, 4, 20_000, 2, moss.MOSS_K4_MIN)
        with pytest.raises(moss.MossError) as e:
            moss.moss_server_wait(srv, t, 60_000)
        assert e.value.status == moss.MOSS_E_ADMISSION
        r = moss.moss_server_wait(srv, moss.moss_server_submit(srv, gid, 4, 20_000, 3), 60_000)
        np.testing.assert_array_equal(r.hits_np, moss.Graph(g).estimate(4, 20_000, 3).hits_np)
    finally:
        moss.moss_server_destroy(srv)


def test_server_cancel_and_timeout(graphs):
    gs, handles = graphs
    srv = moss.moss_server_create(0, 2, 1 << 16)
    try:
        gid = moss.moss_server_add_graph(srv, handles[5].h)
        t_long = moss.moss_server_submit(srv, gid, 5, 2_000_000_000, 1)
        with pytest.raises(moss.MossError) as e:
            moss.moss_server_wait(srv, t_long, 1)
        assert e.value.status == moss.MOSS_E_TIMEOUT
        moss.moss_server_cancel(srv, t_long)
        with pytest.raises(moss.MossError) as e:
            moss.moss_server_wait(srv, t_long, 60_000)
        assert e.value.status == moss.MOSS_E_CANCELLED
        t = moss.moss_server_submit(srv, gid, 4, 1000, 2)
        r = moss.moss_server_wait(srv, t, 60_000)
        np.testing.assert_array_equal(r.hits_np, handles[5].estimate(4, 1000, 2).hits_np)
    finally:
        moss.moss_server_destroy(srv)
