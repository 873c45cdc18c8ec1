"""The per-query reduced matrix and the N-Triples encoder on the host: the
oracle's reduction against the arrays Examples 6.3 and 6.4 print and against a
loop-by-loop restatement on tiny graphs; the engine's encoder (host code in
the library, no device needed) against the oracle's on seeded text."""
import json
import os
import random

import numpy as np
import pytest

import paper_2106_14038_amd as gs
import workload
from oracle import ntriples, reduce as ored

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def example_triples():
    g = load("lspm_example_6_3.json")
    trip = []
    for i in range(g["n"]):
        if g["Mr"][i + 1] - g["Mr"][i] == 1:
            r = g["Mr"][i]
            for k in range(g["Pr"][r], g["Pr"][r + 1]):
                trip.append((i, g["Val"][k], g["Col"][k]))
    return g, np.array(trip, np.int32)


def example_query():
    q = load("query_example_7_2.json")["query"]
    return {"n_qv": q["n_qv"], "qv_const": q["qv_const"], "edges": [tuple(e) for e in q["edges"]]}


def test_example_6_3_direction_driven_reduction():
    """Section 6.2.1, Ex. 6.3: the direction-driven plan keeps every predicate of the query
    in one row-wise part; its Mr and Pr are the printed arrays, each row's (Val, Col) the
    printed multiset."""
    g, trip = example_triples()
    q = example_query()
    info = gs.gs_plan_query(q, traversal=gs.GS_TRAVERSAL_DIRECTION)
    rows, cols = ored.orientation_labels(q, list(info.edge_group), list(info.group_vertex), True)
    assert rows == [1, 2, 3] and cols == []
    M, P, val, idx = ored.reduce_part(trip, g["n"], rows, 0)
    assert M.tolist() == g["Mr"] and P.tolist() == g["Pr"]
    for r in range(len(P) - 1):
        ours = sorted(zip(val[P[r]:P[r + 1]].tolist(), idx[P[r]:P[r + 1]].tolist()))
        theirs = sorted(zip(g["Val"][g["Pr"][r]:g["Pr"][r + 1]], g["Col"][g["Pr"][r]:g["Pr"][r + 1]]))
        assert ours == theirs
    # the row-wise order the engine stores: by (label, column) within a row
    for r in range(len(P) - 1):
        seg = list(zip(val[P[r]:P[r + 1]].tolist(), idx[P[r]:P[r + 1]].tolist()))
        assert seg == sorted(seg)


def test_example_6_4_degree_driven_reduction():
    """Section 6.2.2, Ex. 6.4: with the degree-driven plan (Ex. 6.2) the row-wise part drops
    director (label 3) and holds 5 rows and 7 nonzeros; the column-wise part drops actor
    (label 2) and holds 8 rows and 9 nonzeros (the printed column count disagrees with
    Ex. 6.3's arrays and is not pinned)."""
    g, trip = example_triples()
    q = example_query()
    info = gs.gs_plan_query(q, traversal=gs.GS_TRAVERSAL_DEGREE)
    rows, cols = ored.orientation_labels(q, list(info.edge_group), list(info.group_vertex), False)
    assert rows == [1, 2] and cols == [1, 3]
    M, P, val, _ = ored.reduce_part(trip, g["n"], rows, 0)
    ex = g["example_6_4_csr_without_label_3"]
    assert len(P) - 1 == ex["nonempty_rows"] and len(val) == ex["nonzeros"] and 3 not in val.tolist()
    M, P, val, _ = ored.reduce_part(trip, g["n"], cols, 1)
    ex = g["example_6_4_csc_without_label_2"]
    assert len(M) - 1 == ex["rows"] and len(val) == ex["nonzeros"]
    assert 2 not in val.tolist()


def test_reduction_against_loops_on_tiny_graphs():
    """The numpy reduction against the definition restated with loops (dict of rows)."""
    rng = random.Random(11)
    for _ in range(200):
        n, P = rng.randint(1, 12), rng.randint(1, 5)
        trip = workload.uniform_graph(rng.randrange(1 << 30), n, P, rng.randint(0, n * n * P)) \
            if rng.random() < 0.9 else np.zeros((0, 3), np.int32)
        if len(trip) and rng.random() < 0.5:   # repeats: the reduction takes the triples as a set
            trip = np.concatenate([trip, trip[rng.randrange(len(trip)):]])
        labels = sorted(rng.sample(range(1, P + 1), rng.randint(0, P)))
        for o in (0, 1):
            M, Pp, val, idx = ored.reduce_part(trip, n, labels, o)
            rowmap = {}
            for s, p, t in set(map(tuple, trip.tolist())):
                if p in labels:
                    a, b = (s, t) if o == 0 else (t, s)
                    rowmap.setdefault(a, []).append((p, b))
            kept = sorted(rowmap)
            assert M[0] == 0 and len(M) == n + 1
            for i in range(n):
                assert M[i + 1] - M[i] == (1 if i in rowmap else 0)
            assert len(Pp) == len(kept) + 1 and Pp[0] == 0
            for r, i in enumerate(kept):
                assert M[i] == r
                got = list(zip(val[Pp[r]:Pp[r + 1]].tolist(), idx[Pp[r]:Pp[r + 1]].tolist()))
                assert got == sorted(rowmap[i])
            ptr = ored.expand_rows(M, Pp, n)
            assert all(ptr[i + 1] - ptr[i] == len(rowmap.get(i, [])) for i in range(n))


def test_orientation_labels_constants_and_repeats():
    # an edge out of a constant is row-wise, into a constant column-wise, a repeated edge with its first copy
    q = {"n_qv": 3, "qv_const": [-1, 7, -1], "edges": [(1, 4, 0), (0, 5, 1), (0, 6, 2), (0, 6, 2)]}
    info = gs.gs_plan_query(q)
    rows, cols = ored.orientation_labels(q, list(info.edge_group), list(info.group_vertex), False)
    assert 4 in rows and 5 in cols
    g = info.edge_group[2]
    assert (6 in rows) == (info.group_vertex[g] == 0) and (6 in cols) == (info.group_vertex[g] == 2)
    assert info.edge_group[3] == -1


# ---- N-Triples

SMALL = (
    "# a hand-worked example\n"
    "<http://x/a> <http://x/knows> <http://x/b> .\n"
    "\n"
    "<http://x/b> <http://x/name> \"Bee \\\"B\\\"\"@en-GB .\r\n"
    "_:n1 <http://x/knows> <http://x/a>.   # trailing comment\n"
    "<http://x/a> <http://x/age> \"42\"^^<http://www.w3.org/2001/XMLSchema#integer> .\n"
    "<http://x/a> <http://x/knows> <http://x/b> .\n"
)


def test_ntriples_hand_worked():
    """Ids by first appearance, worked by hand: vertices a=0, b=1, "Bee..."=2, _:n1=3, "42"=4;
    predicates knows=1, name=2, age=3; the repeated line stays."""
    t, v, p = ntriples.encode(SMALL)
    assert t == [(0, 1, 1), (1, 2, 2), (3, 1, 0), (0, 3, 4), (0, 1, 1)]
    assert v == ["<http://x/a>", "<http://x/b>", '"Bee \\"B\\""@en-GB', "_:n1",
                 '"42"^^<http://www.w3.org/2001/XMLSchema#integer>']
    assert p == ["<http://x/knows>", "<http://x/name>", "<http://x/age>"]


@pytest.mark.parametrize("bad", ["<a> <p> .", "<a> <p> <b>", "\"lit\" <p> <b> .", "<a> _:p <b> .",
                                 "<a> <p> \"open .", "<a> <p> <b> . junk", "<a <p> <b> .", "x <p> <b> ."])
def test_ntriples_errors(bad):
    with pytest.raises(ntriples.NTriplesError):
        ntriples.encode("<ok> <ok> <ok> .\n" + bad + "\n")
    with pytest.raises(gs.GsError) as err:
        gs.gs_encode_ntriples("<ok> <ok> <ok> .\n" + bad + "\n")
    assert err.value.status == gs.GS_EINVAL and "line 2" in str(err.value)


def random_ntriples(rng, lines):
    iri = lambda k: f"<http://example.org/r/{k}>"
    out = []
    for _ in range(lines):
        r = rng.random()
        if r < 0.05:
            out.append("# c " + str(rng.random()))
            continue
        if r < 0.08:
            out.append("   ")
            continue
        s = iri(rng.randrange(60)) if rng.random() < 0.8 else f"_:b{rng.randrange(20)}"
        p = f"<http://example.org/p/{rng.randrange(12)}>"
        k = rng.random()
        if k < 0.6:
            o = iri(rng.randrange(60))
        elif k < 0.7:
            o = f"_:b{rng.randrange(20)}"
        else:
            body = "".join(rng.choice(["a", "b", " ", "\\\"", "\\\\", "\\n", "é", "x"]) for _ in range(rng.randint(0, 6)))
            tail = rng.choice(["", "@en", "@de-AT", "^^<http://www.w3.org/2001/XMLSchema#string>"])
            o = f"\"{body}\"{tail}"
        sep = rng.choice([" ", "\t", "  "])
        end = rng.choice([" .", ".", " . # t"])
        out.append(f"{s}{sep}{p}{sep}{o}{end}")
    return rng.choice(["\n", "\r\n"]).join(out) + rng.choice(["", "\n"])


@pytest.mark.parametrize("seed", range(4))
def test_ntriples_engine_matches_oracle(seed):
    rng = random.Random(seed)
    text = random_ntriples(rng, rng.randint(0, 400))
    t, v, p = ntriples.encode(text)
    d = gs.gs_encode_ntriples(text)
    assert (d.n_triples, d.n_vertices, d.n_labels) == (len(t), len(v), len(p))
    assert d.triples().tolist() == [list(x) for x in t]
    assert [d.vertex(i) for i in range(len(v))] == v
    assert [d.label(k + 1) for k in range(len(p))] == p
    for i, term in enumerate(v[:20]):
        assert d.find_vertex(term) == i
    assert d.find_vertex("<http://example.org/absent>") == -1 and d.find_label("<nope>") == 0
