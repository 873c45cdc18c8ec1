"""Host-side checks of the C-ABI library (no device needed): every declared
symbol is exported, the planner follows the degree-driven traversal of
Section 6.1.2, and argument errors come back as status codes."""
import json
import os
import random
import re

import pytest

import paper_2106_14038_amd as gs
from helpers import random_query

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLD = os.path.join(ROOT, "tests", "golden")


def header_functions():
    with open(os.path.join(ROOT, "include", "gsmart.h")) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gs_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    names = header_functions()
    assert len(names) >= 20
    L = gs.lib()
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(gs.SIGNATURES), set(names) ^ set(gs.SIGNATURES)


def test_planner_example_6_2():
    ex = json.load(open(os.path.join(GOLD, "query_example_7_2.json")))
    q = ex["query"]
    q = {"n_qv": q["n_qv"], "qv_const": q["qv_const"], "edges": [tuple(e) for e in q["edges"]]}
    info = gs.gs_plan_query(q)
    plan = ex["example_6_2_degree_plan"]
    assert list(info.roots[:info.n_roots]) == [plan["root"]]
    groups = {}
    for k, (a, _, b) in enumerate(q["edges"]):
        groups.setdefault(info.edge_group[k], []).append([a, b])
    assert [groups[g] for g in sorted(groups)] == plan["groups"]
    assert list(info.group_vertex[:info.n_groups]) == [2, 0]
    # binding order follows the pops: v2, then v0 (it pops first), then v1 and v3
    assert list(info.order[:4]) == [2, 0, 1, 3]
    assert info.parent_edge[0] == -1


def test_planner_example_6_1_direction():
    # Section 6.1.1, Example 6.1: roots v0 and v3, groups {v0v1, v0v2}, {v2v1}, {v3v2}
    ex = json.load(open(os.path.join(GOLD, "query_example_7_2.json")))
    q = ex["query"]
    q = {"n_qv": q["n_qv"], "qv_const": q["qv_const"], "edges": [tuple(e) for e in q["edges"]]}
    info = gs.gs_plan_query(q, traversal=gs.GS_TRAVERSAL_DIRECTION)
    plan = ex["example_6_1_direction_roots"]
    assert list(info.roots[:info.n_roots]) == plan["roots"]
    groups = {}
    for k, (a, _, b) in enumerate(q["edges"]):
        groups.setdefault(info.edge_group[k], []).append([a, b])
    assert [sorted(groups[g]) for g in sorted(groups)] == plan["groups"]
    assert list(info.group_vertex[:info.n_groups]) == [0, 2, 3]
    # a level reached by the traversal reads its edge along its direction (from the bound
    # source); the further root v3 has an edge to v2, placed before it, and the single binding
    # tree binds it through that edge, read against its direction
    level = {v: j for j, v in enumerate(info.order[:info.n_vars])}
    for j in range(info.n_vars):
        pe = info.parent_edge[j]
        v = info.order[j]
        if v == plan["roots"][0]:
            assert pe == -1
            continue
        a, _, b = q["edges"][pe]
        if v in plan["roots"]:
            assert a == v and level[b] < j
        else:
            assert b == v and level[a] < j


def test_planner_direction_cycle_and_constants():
    # a directed cycle has no vertex without incoming edges: the root is the one with the most
    # outgoing edges (lowest index on ties); with a constant the degree-driven plan applies
    cyc = {"n_qv": 3, "qv_const": [-1, -1, -1], "edges": [(0, 1, 1), (1, 1, 2), (2, 1, 0)]}
    info = gs.gs_plan_query(cyc, traversal=gs.GS_TRAVERSAL_DIRECTION)
    assert list(info.roots[:info.n_roots]) == [0] and list(info.group_vertex[:info.n_groups]) == [0, 1, 2]
    cq = {"n_qv": 4, "qv_const": [-1, 5, -1, -1], "edges": [(0, 1, 1), (0, 2, 2), (2, 3, 3)]}
    a = gs.gs_plan_query(cq, traversal=gs.GS_TRAVERSAL_DIRECTION)
    b = gs.gs_plan_query(cq, traversal=gs.GS_TRAVERSAL_DEGREE)
    assert list(a.order[:a.n_vars]) == list(b.order[:b.n_vars]) and list(a.roots[:1]) == list(b.roots[:1])


def test_planner_direction_valid_on_random_queries():
    rng = random.Random(5)
    for _ in range(500):
        nv = rng.randint(1, 8)
        q = random_query(rng, 50, 5, nv, rng.randint(0, 1), connected=rng.random() < 0.7)
        deg = [0] * q["n_qv"]
        for a, _, b in q["edges"]:
            deg[a] += 1
            deg[b] += 1
        if any(d == 0 and q["qv_const"][i] < 0 for i, d in enumerate(deg)):
            continue
        info = gs.gs_plan_query(q, traversal=gs.GS_TRAVERSAL_DIRECTION)
        _check_plan_valid(q, info)
        roots = list(info.roots[:info.n_roots])
        level = {v: j for j, v in enumerate(info.order[:info.n_vars])}
        for j in range(info.n_vars):
            v, pe = info.order[j], info.parent_edge[j]
            if pe < 0:   # bound by nothing earlier: no edge to an earlier level
                assert all(not ((a == v and b in level and level[b] < j) or (b == v and a in level and level[a] < j))
                           for a, _, b in q["edges"]), (q, j)
            elif all(c < 0 for c in q["qv_const"]) and v not in roots:
                assert q["edges"][pe][2] == v   # generating edges are read along their direction


def test_planner_constants_first():
    # (?x p c) and (?x q ?y), (?y r ?z): the constant's edge is evaluated first and ?x is the root
    q = {"n_qv": 4, "qv_const": [-1, 5, -1, -1], "edges": [(0, 1, 1), (0, 2, 2), (2, 3, 3)]}
    info = gs.gs_plan_query(q)
    assert info.group_vertex[0] == -1 and info.edge_group[0] == 0
    assert info.roots[0] == 0 and list(info.order[:3]) == [0, 2, 3]


def _check_plan_valid(q, info):
    var = [i for i, c in enumerate(q["qv_const"]) if c < 0]
    order = list(info.order[:info.n_vars])
    assert sorted(order) == var
    level = {v: j for j, v in enumerate(order)}
    for j, v in enumerate(order):
        pe = info.parent_edge[j]
        if pe >= 0:
            a, _, b = q["edges"][pe]
            u = b if a == v else a
            assert v in (a, b) and u in level and level[u] < j
    seen = {}
    for k, e in enumerate(q["edges"]):
        g = info.edge_group[k]
        if e in seen:
            assert g == -1
        else:
            seen[e] = g
            assert 0 <= g < info.n_groups
            gv = info.group_vertex[g]
            if gv >= 0:
                assert gv in (e[0], e[2])
            else:
                assert q["qv_const"][e[0]] >= 0 or q["qv_const"][e[2]] >= 0


def test_planner_valid_on_random_queries():
    rng = random.Random(4)
    for _ in range(500):
        nv = rng.randint(1, 8)
        q = random_query(rng, 50, 5, nv, rng.randint(0, 2), connected=rng.random() < 0.7)
        deg = [0] * q["n_qv"]
        for a, _, b in q["edges"]:
            deg[a] += 1
            deg[b] += 1
        if any(d == 0 and q["qv_const"][i] < 0 for i, d in enumerate(deg)):
            continue
        _check_plan_valid(q, gs.gs_plan_query(q))


def test_argument_errors_without_device():
    with pytest.raises(gs.GsError) as e:
        gs.gs_plan_query({"n_qv": 2, "qv_const": [-1, -1], "edges": []})
    assert e.value.status == gs.GS_EINVAL
    with pytest.raises(gs.GsError) as e:
        gs.gs_plan_query({"n_qv": 2, "qv_const": [-1, -1], "edges": [(0, 1, 5)]})
    assert e.value.status == gs.GS_EINVAL
    with pytest.raises(gs.GsError) as e:
        gs.gs_plan_query({"n_qv": 3, "qv_const": [-1, -1, -1], "edges": [(0, 1, 1)]})   # ?2 has no edge
    assert e.value.status == gs.GS_EINVAL
    many = {"n_qv": 66, "qv_const": [-1] * 66, "edges": [(i, 1, i + 1) for i in range(65)]}
    with pytest.raises(gs.GsError) as e:
        gs.gs_plan_query(many)
    assert e.value.status == gs.GS_EUNSUPPORTED


def test_engine_create_reports_missing_device():
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a device is present")
    except ImportError:
        pass
    with pytest.raises(gs.GsError) as e:
        gs.gs_engine_create()
    assert e.value.status in (gs.GS_EDEVICE, gs.GS_EINVAL)
