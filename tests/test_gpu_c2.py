"""The batched query set at full size (power-law graph, N = 10M, M = 100M,
256 labels; walk queries of the four shapes with 0-2 constants, stratified by
shape and count decade over 1 .. 1e8): every query's rows from the batched
form (in waves of up to 128) have the oracle's count and, where the set holds
one, its order-independent row digest; the whole set as one count-only batch
(the configuration the benchmark times) gives every stored count; the plain
form gives the same digests on a seeded sample."""
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
        # the oracle's digest where it has one (its backtracking has a time limit per query:
        # the set lists the queries left with their count only)
        digests = [(q["count"], int(q["digest_sum"]), int(q["digest_xor"])) if "digest_sum" in q else None
                   for q in qs["queries"]]
        assert sum(d is not None for d in digests) >= len(digests) - len(qs.get("no_digest", []))
        got, i, wave = [], 0, 128
        while i < len(queries):
            print(f"[c2] queries {i}.. in a wave of {wave}", flush=True)
            try:
                rs = gs.gs_batch_run(eng, queries[i:i + wave])
            except gs.GsError as err:   # the wave's trees exceed the tree arena: smaller waves
                assert err.status == gs.GS_ENOMEM and wave > 1
                wave //= 2
                continue
            got += [gs.gs_result_digest(r) for r in rs]
            for r in rs:
                gs.gs_result_free(r)
            i += wave
        assert [g[0] for g in got] == expect
        bad = [i for i, (g, d) in enumerate(zip(got, digests)) if d is not None and g != d]
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
