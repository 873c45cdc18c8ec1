"""Parity on the 2B-triple graph (N = 2e8; the distinct triples among 2e9
Chung-Lu draws, beta 2.0, 1024 Zipf labels, typed domains; 64-bit row offsets),
against the oracle's counts and order-independent row digests stored with its
query set (workload/data/c4_queries.json), and on the same recipe at 1% scale
(N = 2e6, 2e7 draws; workload/data/c4s0.01_queries.json):

- the selective set (256 walk queries with constants: snowflake-8, star-5,
  chain-4), batched in one launch sequence with rows kept: every query's count
  and row digest (computed on the device) equal the oracle's;
- the large set (chain-4 and star-5 with one constant, 1e7 to 1e9 rows):
  counts batched count-only; every query's rows alone (plain form, rows kept)
  have the oracle's digest; the rows of the smallest one streamed to the host
  in chunks have it too.
"""
import json
import os

import numpy as np
import pytest

import workload
from helpers import row_digest_np

gs = pytest.importorskip("paper_2106_14038_amd")
pytestmark = pytest.mark.gpu

DATA = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "workload", "data")


def stored(rec):
    return rec["count"], int(rec["digest_sum"]), int(rec["digest_xor"])


@pytest.fixture(scope="module", params=["c4s0.01", pytest.param("c4", marks=pytest.mark.slow)])
def c4(request):
    path = os.path.join(DATA, f"{request.param}_queries.json")
    if not os.path.exists(path):
        pytest.skip("query set not generated")
    torch = pytest.importorskip("torch")
    qs = json.load(open(path))
    for q in qs["queries"]:
        q["query"]["edges"] = [tuple(e) for e in q["query"]["edges"]]
    print(f"[{request.param}] drawing the graph on the device", flush=True)
    st = workload.c4_stream(qs["scale"])
    trip = st.device_graph(qs["draws"])
    torch.cuda.synchronize()
    eng = gs.gs_engine_create(gs.options(tree_bytes=64 << 30, scratch_bytes=16 << 30, offset_bytes=8,
                                         hip_stream=torch.cuda.current_stream().cuda_stream))
    print("[c4] engine load", flush=True)
    gs.gs_load_triples(eng, qs["n"], qs["n_labels"], trip)
    torch.cuda.synchronize()
    del trip, st
    torch.cuda.empty_cache()
    yield qs, eng
    gs.gs_engine_destroy(eng)


@pytest.mark.timeout(1200)
def test_c4_distinct_count(c4):
    qs, eng = c4
    n, P, m, _ = gs.gs_graph_info(eng)
    assert (n, P, m) == (qs["n"], qs["n_labels"], qs["m"])


@pytest.mark.timeout(1200)
def test_c4_selective_batched_digests(c4):
    qs, eng = c4
    recs = [q for q in qs["queries"] if q["group"] == "selective"]
    print(f"[c4] {len(recs)} selective queries batched", flush=True)
    rs = gs.gs_batch_run(eng, [q["query"] for q in recs])
    try:
        got = [gs.gs_result_digest(r) for r in rs]
    finally:
        for r in rs:
            gs.gs_result_free(r)
    bad = [i for i, (g, q) in enumerate(zip(got, recs)) if g != stored(q)]
    assert not bad, bad[:10]
    rng = np.random.default_rng(4)
    for i in rng.choice(len(recs), size=min(32, len(recs)), replace=False):   # the plain form
        r = gs.gs_query_run(eng, recs[i]["query"])
        assert gs.gs_result_digest(r) == stored(recs[i]), i
        gs.gs_result_free(r)


@pytest.mark.timeout(1200)
def test_c4_large_counts_and_digests(c4):
    qs, eng = c4
    recs = [q for q in qs["queries"] if q["group"] == "large"]
    print(f"[c4] {len(recs)} large queries count-only, batched in waves of 4", flush=True)
    for i in range(0, len(recs), 4):
        rs = gs.gs_batch_run(eng, [q["query"] for q in recs[i:i + 4]], gs.GS_COUNT_ONLY)
        got = [gs.gs_result_count(r) for r in rs]
        for r in rs:
            gs.gs_result_free(r)
        assert got == [q["count"] for q in recs[i:i + 4]], i
    for i, rec in enumerate(recs):
        print(f"[c4] large query {i} {rec['shape']} count={rec['count']} rows kept", flush=True)
        r = gs.gs_query_run(eng, rec["query"])
        try:
            assert gs.gs_result_digest(r) == stored(rec), i
        finally:
            gs.gs_result_free(r)


@pytest.mark.timeout(1200)
def test_c4_streamed_rows_digest(c4):
    qs, eng = c4
    rec = min((q for q in qs["queries"] if q["group"] == "large"), key=lambda q: q["count"])
    print(f"[c4] streaming {rec['count']} rows to the host", flush=True)
    r = gs.gs_query_run(eng, rec["query"])
    try:
        k = gs.gs_result_width(r)
        n, s, x = 0, 0, 0
        chunk = 1 << 24
        for first in range(0, rec["count"], chunk):
            rows = gs.gs_result_rows(r, first, chunk)
            c, cs, cx = row_digest_np(rows.reshape(-1, k))
            n, s, x = n + c, (s + cs) % (1 << 64), x ^ cx
        assert (n, s, x) == stored(rec)
    finally:
        gs.gs_result_free(r)
