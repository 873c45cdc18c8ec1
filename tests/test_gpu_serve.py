"""Served form: continuous batching returns, for every request, exactly the
rows the query has alone (and the oracle's), whatever else is in flight."""
import time

import numpy as np
import pytest

import oracle
import workload
from helpers import engine_rows, sort_rows

gs = pytest.importorskip("paper_2106_14038_amd")
pytestmark = pytest.mark.gpu


def ocount(G, q, cap):
    try:
        return G.eval(q, rows=False, work_cap=cap)[0]
    except oracle.OracleError:
        return -1


@pytest.fixture(scope="module")
def c0_mix():
    trip = workload.c0_graph()
    n, P = workload.C0["n"], workload.C0["n_labels"]
    G = oracle.Graph(trip, n, P)
    qs = workload.walk_queries(trip, n, 21, "mixed", 150, max_consts=2)
    for shape in ("chain4", "star5", "snowflake8", "triangle"):
        qs += workload.walk_queries(trip, n, 22, shape, 10)
    qs = [q for q in qs if 0 <= ocount(G, q, 20_000_000) <= 300_000]
    return trip, n, P, G, qs


def serve(eng, qs, rate, opts=None, flags=0, timeout=120):
    srv = gs.gs_server_start(eng, opts)
    arr = workload.poisson_arrivals(5, rate, 10.0)[:len(qs)]
    t0 = time.perf_counter()
    tickets = []
    for q, ta in zip(qs, arr):
        while time.perf_counter() - t0 < ta:
            pass
        tickets.append(gs.gs_submit(srv, q, flags))
    out = {}
    deadline = time.time() + timeout
    while len(out) < len(tickets) and time.time() < deadline:
        for t in tickets:
            if t in out:
                continue
            try:
                r = gs.gs_poll(srv, t)
            except gs.GsError as e:
                out[t] = e
                continue
            if r is not None:
                out[t] = r
        time.sleep(0.001)
    stats = gs.gs_server_stop(srv)
    assert len(out) == len(tickets), "requests still pending at the deadline"
    return [out[t] for t in tickets], stats


def test_served_mix_equals_alone_and_oracle(c0_mix):
    trip, n, P, G, qs = c0_mix
    eng = gs.gs_engine_create(gs.options(tree_bytes=2 << 30, scratch_bytes=1 << 30))
    try:
        gs.gs_load_triples(eng, n, P, trip)
        alone = [engine_rows(gs, eng, q) for q in qs]
        res, stats = serve(eng, qs, rate=5000.0)
        assert stats.completed == len(qs) and stats.rejected == 0
        assert stats.max_active_seen > 1                      # work overlapped on the device
        lat = []
        for q, (cnt, rows), r in zip(qs, alone, res):
            assert not isinstance(r, Exception), r
            assert gs.gs_result_count(r) == cnt
            assert np.array_equal(sort_rows(gs.gs_result_rows(r)), rows), q
            lat.append(gs.gs_result_stats(r).latency_ms)
            gs.gs_result_free(r)
        assert min(lat) > 0
        for q, (cnt, _) in zip(qs[:60], alone[:60]):
            assert ocount(G, q, 0) == cnt
    finally:
        gs.gs_engine_destroy(eng)


def test_served_small_budget_queues_and_count_only(c0_mix):
    trip, n, P, G, qs = c0_mix
    eng = gs.gs_engine_create(gs.options(tree_bytes=2 << 30, scratch_bytes=1 << 30))
    try:
        gs.gs_load_triples(eng, n, P, trip)
        alone = [engine_rows(gs, eng, q, gs.GS_COUNT_ONLY)[0] for q in qs[:80]]
        opts = gs.gs_server_options(max_active=4, tree_budget_bytes=1 << 16, flags=0)
        res, stats = serve(eng, qs[:80], rate=20000.0, opts=opts, flags=gs.GS_COUNT_ONLY)
        assert stats.max_active_seen <= 4
        for cnt, r in zip(alone, res):
            assert gs.gs_result_count(r) == cnt
            gs.gs_result_free(r)
    finally:
        gs.gs_engine_destroy(eng)


def test_served_tiny_arena_requeues_or_fails_cleanly(c0_mix):
    trip, n, P, G, qs = c0_mix
    big = sorted(qs, key=lambda q: -ocount(G, q, 20_000_000))[:6]
    small = [q for q in qs if ocount(G, q, 20_000_000) <= 50][:20]
    eng = gs.gs_engine_create(gs.options(tree_bytes=1 << 20, scratch_bytes=1 << 28))
    try:
        gs.gs_load_triples(eng, n, P, trip)
        res, stats = serve(eng, big + small, rate=50000.0)
        for q, r in zip(big + small, res):
            if isinstance(r, gs.GsError):
                assert r.status == gs.GS_ENOMEM
            else:
                assert gs.gs_result_count(r) == ocount(G, q, 0)
                gs.gs_result_free(r)
        for r in res[len(big):]:
            assert not isinstance(r, gs.GsError)           # small requests all complete
    finally:
        gs.gs_engine_destroy(eng)


def test_served_errors_and_constant_queries(c0_mix):
    trip, n, P, G, qs = c0_mix
    eng = gs.gs_engine_create(gs.options(tree_bytes=1 << 30, scratch_bytes=1 << 28))
    try:
        gs.gs_load_triples(eng, n, P, trip)
        s, p, o = (int(x) for x in trip[0])
        reqs = [{"n_qv": 2, "qv_const": [-1, -1], "edges": [(0, P + 1, 1)]},       # label out of range
                {"n_qv": 2, "qv_const": [s, o], "edges": [(0, p, 1)]},             # constants only, holds
                {"n_qv": 2, "qv_const": [o, s], "edges": [(0, p, 1)]}] + qs[:5]
        res, stats = serve(eng, reqs, rate=1000.0)
        assert isinstance(res[0], gs.GsError) and res[0].status == gs.GS_ERANGE
        exp2 = int(bool(((trip[:, 0] == o) & (trip[:, 1] == p) & (trip[:, 2] == s)).any()))
        assert gs.gs_result_count(res[1]) == 1 and gs.gs_result_count(res[2]) == exp2
        for q, r in zip(qs[:5], res[3:]):
            assert gs.gs_result_count(r) == ocount(G, q, 0)
        for r in res[1:]:
            gs.gs_result_free(r)
    finally:
        gs.gs_engine_destroy(eng)


def test_poll_ready_drains_every_request_once(c0_mix):
    trip, n, P, G, qs = c0_mix
    eng = gs.gs_engine_create(gs.options(tree_bytes=1 << 30, scratch_bytes=1 << 28))
    try:
        gs.gs_load_triples(eng, n, P, trip)
        srv = gs.gs_server_start(eng, None)
        tickets = {gs.gs_submit(srv, q, gs.GS_COUNT_ONLY): i for i, q in enumerate(qs[:60])}
        seen = {}
        deadline = time.time() + 60
        while len(seen) < len(tickets) and time.time() < deadline:
            for tk, status, r in gs.gs_poll_ready(srv, cap=7):
                assert tk in tickets and tk not in seen and status == gs.GS_OK
                seen[tk] = gs.gs_result_count(r)
                gs.gs_result_free(r)
            time.sleep(0.001)
        gs.gs_server_stop(srv)
        assert len(seen) == len(tickets)
        for tk, i in tickets.items():
            assert seen[tk] == ocount(G, qs[i], 0)
    finally:
        gs.gs_engine_destroy(eng)


def test_server_and_direct_use_are_exclusive():
    """The server uses the whole tree arena: it does not start while a direct
    result is live, and direct evaluation is refused while it runs."""
    n, P = 2000, 4
    trip = workload.uniform_graph(4, n, P, 20_000)
    q = {"n_qv": 2, "qv_const": [-1, -1], "edges": [(0, 1, 1)]}
    e = gs.gs_engine_create(gs.options(tree_bytes=1 << 28, scratch_bytes=1 << 27))
    try:
        gs.gs_load_triples(e, n, P, trip)
        r = gs.gs_query_run(e, q)
        with pytest.raises(gs.GsError) as ei:
            gs.gs_server_start(e)
        assert ei.value.status == gs.GS_ESTATE
        expect = gs.gs_result_count(r)
        gs.gs_result_free(r)
        srv = gs.gs_server_start(e)
        with pytest.raises(gs.GsError) as ei:
            gs.gs_query_run(e, q)
        assert ei.value.status == gs.GS_ESTATE
        with pytest.raises(gs.GsError) as ei:
            gs.gs_server_start(e)
        assert ei.value.status == gs.GS_ESTATE
        t = gs.gs_submit(srv, q, gs.GS_COUNT_ONLY)
        deadline = time.time() + 30
        got = None
        while got is None and time.time() < deadline:
            got = gs.gs_poll(srv, t)
        assert got is not None and gs.gs_result_count(got) == expect
        gs.gs_result_free(got)
        gs.gs_server_stop(srv)
        r = gs.gs_query_run(e, q, gs.GS_COUNT_ONLY)   # direct use again after the stop
        assert gs.gs_result_count(r) == expect
        gs.gs_result_free(r)
    finally:
        gs.gs_engine_destroy(e)
