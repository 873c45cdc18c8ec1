"""Batched form with the launch sequence captured in a hipGraph: every replay,
interleaved with other device work and synchronisations, gives the eager
engine's results."""
import numpy as np
import pytest

import oracle
import workload
from helpers import sort_rows

gs = pytest.importorskip("paper_2106_14038_amd")
pytestmark = pytest.mark.gpu


def batch_results(eng, qs, flags=0):
    rs = gs.gs_batch_run(eng, qs, flags)
    try:
        out = []
        for r in rs:
            cnt = gs.gs_result_count(r)
            rows = sort_rows(gs.gs_result_rows(r)) if not flags & gs.GS_COUNT_ONLY else None
            out.append((cnt, rows))
        return out
    finally:
        for r in rs:
            gs.gs_result_free(r)


def test_graph_replays_match_eager():
    import torch
    trip = workload.c0_graph()
    n, P = workload.C0["n"], workload.C0["n_labels"]
    G = oracle.Graph(trip, n, P)
    qs = []
    for shape in ("chain4", "star5", "snowflake8", "triangle", "mixed"):
        qs += workload.walk_queries(trip, n, 31, shape, 8)
    keep = []
    for q in qs:
        try:
            if G.eval(q, rows=False, work_cap=5_000_000)[0] <= 200_000:
                keep.append(q)
        except oracle.OracleError:
            pass
    eager = gs.gs_engine_create(gs.options(tree_bytes=1 << 30, scratch_bytes=1 << 28))
    graph = gs.gs_engine_create(gs.options(tree_bytes=1 << 30, scratch_bytes=1 << 28, use_graphs=1))
    try:
        gs.gs_load_triples(eager, n, P, trip)
        gs.gs_load_triples(graph, n, P, trip)
        ref = batch_results(eager, keep)
        x = torch.arange(1 << 20, device="cuda")
        for rep in range(4):
            got = batch_results(graph, keep)
            for (c0, r0), (c1, r1), q in zip(ref, got, keep):
                assert c0 == c1 and np.array_equal(r0, r1), (rep, q)
            # the program's own eager work between replays
            y = (x * rep).sum().item()
            r = gs.gs_query_run(graph, keep[rep])
            assert gs.gs_result_count(r) == ref[rep][0]
            gs.gs_result_free(r)
            torch.cuda.synchronize()
        for rep in range(2):
            got = batch_results(graph, keep, gs.GS_COUNT_ONLY)
            assert [c for c, _ in got] == [c for c, _ in ref]
    finally:
        gs.gs_engine_destroy(eager)
        gs.gs_engine_destroy(graph)


def test_autotune_keeps_results_and_is_recorded(tmp_path):
    """The tuned pair changes no result; it is recorded in the autotune cache for the
    graph's sizes, and an engine loading a graph of those sizes starts from it."""
    trip = workload.c0_graph()
    n, P = workload.C0["n"], workload.C0["n_labels"]
    qs = workload.walk_queries(trip, n, 41, "triangle", 6) + workload.walk_queries(trip, n, 41, "star5", 6)
    cache = str(tmp_path / "tune.txt")
    eng = gs.gs_engine_create(gs.options(tree_bytes=1 << 30, scratch_bytes=1 << 28, autotune_cache=cache.encode()))
    try:
        gs.gs_load_triples(eng, n, P, trip)
        before = batch_results(eng, qs)
        tr = gs.gs_autotune(eng, qs)
        assert tr.n_tried == 17 and tr.best_ms <= tr.default_ms and tr.grid_blocks > 0
        assert tr.write_block in (128, 256, 512)
        after = batch_results(eng, qs)
        for (c0, r0), (c1, r1) in zip(before, after):
            assert c0 == c1 and np.array_equal(r0, r1)
        line = open(cache).read().split()
        assert [int(x) for x in line[:4]] == [n, gs.gs_graph_info(eng)[2], P, tr.grid_blocks]
        assert abs(float(line[4]) - tr.push_pull_theta) < 1e-6 and int(line[5]) == tr.write_block
    finally:
        gs.gs_engine_destroy(eng)
    eng = gs.gs_engine_create(gs.options(tree_bytes=1 << 30, scratch_bytes=1 << 28, autotune_cache=cache.encode()))
    try:
        gs.gs_load_triples(eng, n, P, trip)
        again = batch_results(eng, qs)
        for (c0, r0), (c1, r1) in zip(before, again):
            assert c0 == c1 and np.array_equal(r0, r1)
    finally:
        gs.gs_engine_destroy(eng)
    # every write-pass workgroup size, applied from a recorded setting, gives the same rows
    for wb in (128, 256, 512):
        with open(cache, "w") as f:
            f.write(f"{line[0]} {line[1]} {line[2]} {line[3]} {line[4]} {wb}\n")
        eng = gs.gs_engine_create(gs.options(tree_bytes=1 << 30, scratch_bytes=1 << 28, autotune_cache=cache.encode()))
        try:
            gs.gs_load_triples(eng, n, P, trip)
            got = batch_results(eng, qs)
            for (c0, r0), (c1, r1) in zip(before, got):
                assert c0 == c1 and np.array_equal(r0, r1), wb
        finally:
            gs.gs_engine_destroy(eng)
        eng = gs.gs_engine_create(gs.options(tree_bytes=1 << 30, scratch_bytes=1 << 28, write_block=wb))
        try:
            gs.gs_load_triples(eng, n, P, trip)
            got = batch_results(eng, qs)
            for (c0, r0), (c1, r1) in zip(before, got):
                assert c0 == c1 and np.array_equal(r0, r1), wb
        finally:
            gs.gs_engine_destroy(eng)
    with pytest.raises(gs.GsError):
        gs.gs_engine_create(gs.options(write_block=100))
