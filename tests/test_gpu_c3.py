"""The served form on the power-law graph (N = 10M, M = 100M, 256 labels, held
resident): the served query set (400 walk queries of mixed shape, 1-12 edges,
0-2 constants, counts up to 1e7) arrives as a Poisson stream and is served with
continuous batching, rows kept. Every request's rows have the oracle's count and
order-independent row digest stored with the set, and equal the rows the same
query has alone (plain form), whatever else was in flight."""
import json
import os
import time

import pytest

import workload

gs = pytest.importorskip("paper_2106_14038_amd")
pytestmark = [pytest.mark.gpu, pytest.mark.slow]

DATA = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "workload", "data", "c3_queries.json")


@pytest.mark.timeout(1200)
def test_c3_served_rows_match_oracle_and_alone():
    if not os.path.exists(DATA):
        pytest.skip("query set not generated")
    qs = json.load(open(DATA))
    if "digest_sum" not in qs["queries"][0]:
        pytest.skip("query set has no stored digests")
    for q in qs["queries"]:
        q["query"]["edges"] = [tuple(e) for e in q["query"]["edges"]]
    queries = [q["query"] for q in qs["queries"]]
    want = [(q["count"], int(q["digest_sum"]), int(q["digest_xor"])) for q in qs["queries"]]
    print("[c3] generating graph", flush=True)
    trip = workload.c1_graph(qs["scale"])
    eng = gs.gs_engine_create(gs.options())
    try:
        gs.gs_load_triples(eng, qs["n"], qs["n_labels"], trip)
        print("[c3] plain form, one query at a time", flush=True)
        alone = []
        for q in queries:
            r = gs.gs_query_run(eng, q)
            alone.append(gs.gs_result_digest(r))
            gs.gs_result_free(r)
        bad = [i for i, (a, w) in enumerate(zip(alone, want)) if a != w]
        assert not bad, bad[:10]
        print("[c3] served, Poisson arrivals at 5000/s", flush=True)
        srv = gs.gs_server_start(eng, gs.gs_server_options(max_active=1024, tree_budget_bytes=0, flags=0))
        arr = workload.poisson_arrivals(9, 5000.0, 10.0)[:len(queries)]
        t0 = time.perf_counter()
        tickets = {}
        got = {}
        i = 0
        deadline = time.time() + 600
        while (i < len(queries) or len(got) < len(queries)) and time.time() < deadline:
            now = time.perf_counter() - t0
            while i < len(queries) and arr[i] <= now:
                tickets[gs.gs_submit(srv, queries[i], 0)] = i
                i += 1
            for tk, status, r in gs.gs_poll_ready(srv):
                assert status == gs.GS_OK, (tickets[tk], status)
                got[tickets[tk]] = gs.gs_result_digest(r)   # host-owned rows: digest on the host
                gs.gs_result_free(r)
        st = gs.gs_server_stop(srv)
        assert len(got) == len(queries), "requests still pending at the deadline"
        assert st.rejected == 0 and st.max_active_seen > 1
        bad = [k for k in range(len(queries)) if got[k] != want[k]]
        assert not bad, bad[:10]
    finally:
        gs.gs_engine_destroy(eng)
