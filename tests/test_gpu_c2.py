"""The batched query set at full size (power-law graph, N = 10M, M = 100M,
256 labels; 1024 queries of the four shapes with random constants, counts
spread over decades 1 .. 1e7): every query's rows from the batched form (in
waves of 128) have the oracle's count and order-independent row digest stored
with the set; the whole set as one count-only batch (the configuration the
benchmark times) gives every stored count; the plain form gives the same
digests on a seeded sample."""
import json
import os

import numpy as np
import pytest

import workload

gs = pytest.importorskip("paper_2106_14038_amd")
pytestmark = [pytest.mark.gpu, pytest.mark.slow]

DATA = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "workload", "data", "c2_queries.json")


@pytest.mark.timeout(1200)
def test_c2_batched_counts_match_oracle():
    if not os.path.exists(DATA):
        pytest.skip("query set not generated")
    qs = json.load(open(DATA))
    for q in qs["queries"]:
        q["query"]["edges"] = [tuple(e) for e in q["query"]["edges"]]
    queries = [q["query"] for q in qs["queries"]]
    expect = [q["count"] for q in qs["queries"]]
    print("[c2] generating graph", flush=True)
    trip = workload.c1_graph(qs["scale"])
    eng = gs.gs_engine_create(gs.options())
    try:
        gs.gs_load_triples(eng, qs["n"], qs["n_labels"], trip)
        digests = [(q["count"], int(q["digest_sum"]), int(q["digest_xor"])) for q in qs["queries"]] \
            if "digest_sum" in qs["queries"][0] else None
        got = []
        for i in range(0, len(queries), 128):
            print(f"[c2] wave {i // 128}", flush=True)
            rs = gs.gs_batch_run(eng, queries[i:i + 128])
            got += [gs.gs_result_digest(r) for r in rs]
            for r in rs:
                gs.gs_result_free(r)
        assert [g[0] for g in got] == expect
        if digests:
            bad = [i for i, (g, d) in enumerate(zip(got, digests)) if g != d]
            assert not bad, bad[:10]
        print("[c2] the whole set as one batch", flush=True)   # the configuration the benchmark times
        rs = gs.gs_batch_run(eng, queries, gs.GS_COUNT_ONLY)
        whole = [gs.gs_result_count(r) for r in rs]
        for r in rs:
            gs.gs_result_free(r)
        assert whole == expect
        rng = np.random.default_rng(2)
        for i in rng.choice(len(queries), size=64, replace=False):
            r = gs.gs_query_run(eng, queries[i])
            assert gs.gs_result_digest(r) == got[i], i
            gs.gs_result_free(r)
    finally:
        gs.gs_engine_destroy(eng)
