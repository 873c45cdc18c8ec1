"""The per-query reduced matrix built on the device (Section 6.2.1, 6.2.2;
Ex. 6.3, 6.4) against the oracle's reduction, and the one-shot load that keeps
only a query's predicates (step 1 of both sections) against the full load and
the oracle."""
import os
import random

import numpy as np
import pytest

import oracle
import workload
from helpers import engine_rows, random_query
from oracle import reduce as ored
from test_reduce_cpu import example_query, example_triples

gs = pytest.importorskip("paper_2106_14038_amd")
pytestmark = pytest.mark.gpu

SMALL = dict(tree_bytes=1 << 30, scratch_bytes=1 << 28)


def make_engine(trip, n, P, **kw):
    e = gs.gs_engine_create(gs.options(**{**SMALL, **kw}))
    gs.gs_load_triples(e, n, P, trip)
    return e


def check_reduction(e, trip, n, q, traversal):
    """Engine's reduced parts equal the oracle's for the labels the plan's groups give."""
    info = gs.gs_plan_query(q, engine=e, traversal=traversal)
    direction = traversal == gs.GS_TRAVERSAL_DIRECTION
    rows, cols = ored.orientation_labels(q, list(info.edge_group), list(info.group_vertex), direction)
    red = gs.gs_lspm_reduce(e, q, traversal)
    assert red["n"] == n
    for o, labels in ((0, rows), (1, cols)):
        part = red["parts"][o]
        assert part["labels"] == labels, (o, q)
        M, P, val, idx = ored.reduce_part(trip, n, labels, o)
        assert np.array_equal(part["M"], M), (o, q)
        assert np.array_equal(part["P"], P), (o, q)
        assert np.array_equal(part["val"], val) and np.array_equal(part["idx"], idx), (o, q)


def test_examples_6_3_and_6_4_on_the_device():
    g, trip = example_triples()
    q = example_query()
    e = make_engine(trip, g["n"], g["n_labels"])
    try:
        red = gs.gs_lspm_reduce(e, q, gs.GS_TRAVERSAL_DIRECTION)
        p0 = red["parts"][0]
        assert p0["M"].tolist() == g["Mr"] and p0["P"].tolist() == g["Pr"] and red["parts"][1]["nnz"] == 0
        for r in range(len(g["Pr"]) - 1):
            a, b = g["Pr"][r], g["Pr"][r + 1]
            assert sorted(zip(p0["val"][a:b].tolist(), p0["idx"][a:b].tolist())) == \
                sorted(zip(g["Val"][a:b], g["Col"][a:b]))
        red = gs.gs_lspm_reduce(e, q, gs.GS_TRAVERSAL_DEGREE)
        ex = g["example_6_4_csr_without_label_3"]
        assert red["parts"][0]["rows"] == ex["nonempty_rows"] and red["parts"][0]["nnz"] == ex["nonzeros"]
        assert red["parts"][1]["nnz"] == g["example_6_4_csc_without_label_2"]["nonzeros"]
        for trav in (gs.GS_TRAVERSAL_DIRECTION, gs.GS_TRAVERSAL_DEGREE):
            check_reduction(e, trip, g["n"], q, trav)
    finally:
        gs.gs_engine_destroy(e)


@pytest.mark.parametrize("seed", range(2))
def test_random_graphs_and_queries(seed):
    rng = random.Random(1300 + seed)
    for case in range(20):
        n, P = rng.randint(2, 40), rng.randint(1, 6)
        trip = workload.uniform_graph(rng.randrange(1 << 30), n, P, rng.randint(1, min(n * n * P, 3000)))
        e = make_engine(trip, n, P)
        try:
            for _ in range(4):
                nv = rng.randint(2, 5)
                q = random_query(rng, n, P, nv, rng.randint(0, 1), n_edges=rng.randint(nv - 1, nv + 2))
                deg = [0] * q["n_qv"]
                for a, _, b in q["edges"]:
                    deg[a] += 1
                    deg[b] += 1
                if any(d == 0 and q["qv_const"][i] < 0 for i, d in enumerate(deg)):
                    continue
                print(f"[reduce] seed={seed} case={case} q={q}", flush=True)
                for trav in (gs.GS_TRAVERSAL_DEGREE, gs.GS_TRAVERSAL_DIRECTION):
                    check_reduction(e, trip, n, q, trav)
        finally:
            gs.gs_engine_destroy(e)


def test_power_law_rows_and_wide_labels():
    """Hub rows (binary-searched label sub-segments) and 2-byte labels (600 labels)."""
    for P, zipf in ((4, 1.1), (600, 1.1)):
        n = 20000
        trip = workload.chunglu_graph(9, n, P, 200_000, beta=2.0, zipf_s=zipf)
        e = make_engine(trip, n, P)
        try:
            qs = workload.walk_queries(trip, n, 3, "star5", 6, const_prob=0.3) + \
                workload.walk_queries(trip, n, 4, "triangle", 4, const_prob=0.0)
            for q in qs:
                for trav in (gs.GS_TRAVERSAL_DEGREE, gs.GS_TRAVERSAL_DIRECTION):
                    check_reduction(e, trip, n, q, trav)
        finally:
            gs.gs_engine_destroy(e)


def test_one_shot_load_keeps_only_the_query_predicates():
    torch = pytest.importorskip("torch")
    trip = workload.c0_graph()
    n, P = workload.C0["n"], workload.C0["n_labels"]
    G = oracle.Graph(trip, n, P)
    full = make_engine(trip, n, P)
    try:
        qs = []
        for shape in ("chain4", "star5", "triangle", "snowflake8"):
            qs += workload.walk_queries(trip, n, 21, shape, 3)
        for i, q in enumerate(qs):
            labels = gs.query_labels(q)
            e = gs.gs_engine_create(gs.options(**SMALL))
            try:
                src = torch.from_numpy(trip).cuda() if i % 2 else trip   # device and host input
                gs.gs_load_triples_labels(e, n, P, src, labels)
                _, _, m, _ = gs.gs_graph_info(e)
                t = np.unique(trip, axis=0)
                assert m == int(np.isin(t[:, 1], labels).sum())
                cnt, rows = engine_rows(gs, e, q)
                cf, rf = engine_rows(gs, full, q)
                assert cnt == cf and np.array_equal(rows, rf), (i, q)
                if cnt < 200_000:
                    oc, orows = G.eval(q, rows_cap=cnt + 1)
                    assert oc == cnt and np.array_equal(rows, orows)
            finally:
                gs.gs_engine_destroy(e)
        e = gs.gs_engine_create(gs.options(**SMALL))
        try:
            with pytest.raises(gs.GsError) as err:
                gs.gs_load_triples_labels(e, n, P, trip, [P + 1])
            assert err.value.status == gs.GS_ERANGE
        finally:
            gs.gs_engine_destroy(e)
    finally:
        gs.gs_engine_destroy(full)
