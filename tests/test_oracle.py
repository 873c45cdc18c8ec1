"""Pins for the oracle: the paper's worked examples, brute force, closed forms
and invariants. Each check is independent of the oracle's own code (numpy
definitions or printed values), so a dropped term, a wrong direction or a
swapped operand in the oracle fails at least one of them."""
import itertools
import json
import math
import os
import random

import numpy as np
import pytest

import oracle
import workload
from helpers import _mix64, brute_force, dense_tensor, random_query, row_digest, sort_rows

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def load(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


# ------------------------------------------------------------------ paper values
def test_algebra_examples_section_2_1():
    g = load("algebra_3x3.json")
    G = oracle.Graph(np.array(g["triples"], np.int32), g["n"], g["n_labels"])
    # Eq. (6): rows holding b; Eq. (7): columns holding b
    assert G.label_exists(g["eq6_rows_holding_b"]["label"], 0).tolist() == g["eq6_rows_holding_b"]["expect"]
    assert G.label_exists(g["eq7_columns_holding_b"]["label"], 1).tolist() == g["eq7_columns_holding_b"]["expect"]
    # Eq. (9) / (12)-(13): S_c (x) A marks the positions of c, i.e. the single-edge query ?x c ?y
    cnt, rows = G.eval({"n_qv": 2, "qv_const": [-1, -1], "edges": [(0, g["eq9_positions_of_c"]["label"], 1)]})
    assert rows.tolist() == g["eq9_positions_of_c"]["expect_pairs"]
    # Eq. (2)/(3) with Eq. (10)/(11): the frontier restricted product keeps exactly the selected rows / columns
    x = np.array(g["eq10_vector_and"]["x"], np.uint8)
    y = np.array(g["eq10_vector_and"]["y"], np.uint8)
    assert (x & y).tolist() == g["eq10_vector_and"]["expect"]
    assert (x | y).tolist() == g["eq11_vector_or"]["expect"]
    sel = np.zeros(3, np.uint8)
    sel[g["eq2_row_selection"]["rows"]] = 1
    kept = [p for p in range(1, 10) if G.frontier_domain(sel, p, 0).any()]
    assert kept == g["eq2_row_selection"]["expect_labels_kept"]
    sel = np.zeros(3, np.uint8)
    sel[g["eq3_column_selection"]["cols"]] = 1
    kept = [p for p in range(1, 10) if G.frontier_domain(sel, p, 1).any()]
    assert kept == g["eq3_column_selection"]["expect_labels_kept"]
    # row 2 = [g h i] = labels 7 8 9: along h (8) from row 2 the only column reached is 1
    f = np.array([0, 0, 1], np.uint8)
    assert G.frontier_domain(f, 8, 0).tolist() == [0, 1, 0]
    # along c (3) into column 2 the only row reached is 0
    assert G.frontier_domain(np.array([0, 0, 1], np.uint8), 3, 1).tolist() == [1, 0, 0]


def decode_example_6_3():
    g = load("lspm_example_6_3.json")
    Mr, Pr, Val, Col = g["Mr"], g["Pr"], g["Val"], g["Col"]
    trip = []
    for i in range(g["n"]):
        if Mr[i + 1] - Mr[i] == 1:
            r = Mr[i]
            for k in range(Pr[r], Pr[r + 1]):
                trip.append((i, Val[k], Col[k]))
    return g, np.array(trip, np.int32)


def test_lspm_example_6_3():
    g, trip = decode_example_6_3()
    assert len(trip) == 11
    G = oracle.Graph(trip, g["n"], g["n_labels"])
    rp, col, lab = G.csr()
    # non-empty rows and the reduced pointer array match Mr / Pr
    nonempty = [i for i in range(g["n"]) if rp[i + 1] > rp[i]]
    Mr = [0]
    for i in range(g["n"]):
        Mr.append(Mr[-1] + (1 if i in nonempty else 0))
    assert Mr == g["Mr"]
    assert [int(rp[i]) for i in nonempty] + [int(rp[-1])] == g["Pr"]
    # each row holds the paper's (label, column) multiset, sorted by (label, column)
    for r_red, i in enumerate(nonempty):
        ours = list(zip(lab[rp[i]:rp[i + 1]].tolist(), col[rp[i]:rp[i + 1]].tolist()))
        theirs = sorted(zip(g["Val"][g["Pr"][r_red]:g["Pr"][r_red + 1]], g["Col"][g["Pr"][r_red]:g["Pr"][r_red + 1]]))
        assert ours == theirs
    # Example 6.4: without label 3 the row-wise part has 5 non-empty rows and 7 nonzeros
    keep = trip[trip[:, 1] != 3]
    G2 = oracle.Graph(keep, g["n"], g["n_labels"])
    rp2, _, _ = G2.csr()
    ex = g["example_6_4_csr_without_label_3"]
    assert int((np.diff(rp2) > 0).sum()) == ex["nonempty_rows"] and G2.m == ex["nonzeros"]
    # the column-wise arrays hold the same nonzeros, grouped by column
    cp, row, labc = G.csc()
    got = sorted((int(row[k]), int(labc[k]), c) for c in range(g["n"]) for k in range(cp[c], cp[c + 1]))
    assert got == sorted(map(tuple, trip.tolist()))


def test_reconstructed_query_example_7_2():
    g, trip = decode_example_6_3()
    ex = load("query_example_7_2.json")
    q = ex["query"]
    q = {"n_qv": q["n_qv"], "qv_const": q["qv_const"], "edges": [tuple(e) for e in q["edges"]]}
    bf = brute_force(trip, ex["n"], ex["n_labels"], q)
    assert bf.tolist() == ex["expect_rows"]
    G = oracle.Graph(trip, ex["n"], ex["n_labels"])
    cnt, rows = G.eval(q)
    assert cnt == 2 and rows.tolist() == ex["expect_rows"]
    # Example 7.2's per-root outcomes: restricting v2 to 0, 4 or 5 leaves nothing, v2 = 1 leaves both rows
    for v2, expect in [(0, 0), (4, 0), (5, 0), (1, 2)]:
        mask = np.zeros(ex["n"], np.uint8)
        mask[v2] = 1
        assert G.eval(q, restrict=(2, mask))[0] == expect
    # Example 8.1: v1 = 5 is reachable from v0 = 2 along label 2 but not from v2 = 1 along label 1
    assert (2, 2, 5) in set(map(tuple, trip.tolist())) and (1, 1, 5) not in set(map(tuple, trip.tolist()))
    assert 5 not in rows[:, 1]
    # adding triples of an unused label (FriendOf) changes nothing
    extra = np.array([[0, 4, 3], [3, 4, 6], [5, 4, 1]], np.int32)
    G4 = oracle.Graph(np.concatenate([trip, extra]), ex["n"], 4)
    assert G4.eval(q)[1].tolist() == ex["expect_rows"]


# ------------------------------------------------------------------ brute force
@pytest.mark.parametrize("seed", range(6))
def test_eval_matches_brute_force(seed):
    rng = random.Random(1000 + seed)
    for case in range(60):
        n = rng.randint(1, 9)
        P = rng.randint(1, 4)
        dens = rng.choice([0.05, 0.2, 0.5])
        m = max(0, min(int(dens * n * n * P), n * n * P))
        trip = workload.uniform_graph(rng.randrange(1 << 30), n, P, m) if m else np.zeros((0, 3), np.int32)
        nv = rng.randint(0, 4)
        nc = rng.randint(0 if nv else 1, 2)
        q = random_query(rng, n, P, nv, nc, connected=rng.random() < 0.8)
        G = oracle.Graph(trip, n, P)
        cnt, rows = G.eval(q)
        bf = brute_force(trip, n, P, q)
        assert cnt == len(bf), (case, q)
        if nv:
            assert np.array_equal(rows, bf), (case, q)


def test_eval_multilabel_pairs_and_self_loops():
    # several labels on one (s, o) pair, self loops, parallel and antiparallel query edges
    trip = np.array([[0, 1, 1], [0, 2, 1], [1, 1, 0], [1, 1, 1], [2, 2, 2], [2, 1, 0], [0, 1, 0]], np.int32)
    qs = [
        {"n_qv": 2, "qv_const": [-1, -1], "edges": [(0, 1, 1), (0, 2, 1)]},
        {"n_qv": 2, "qv_const": [-1, -1], "edges": [(0, 1, 1), (1, 1, 0)]},
        {"n_qv": 1, "qv_const": [-1], "edges": [(0, 1, 0)]},
        {"n_qv": 2, "qv_const": [-1, 2], "edges": [(1, 2, 1), (1, 1, 0), (0, 1, 0)]},
        {"n_qv": 2, "qv_const": [-1, -1], "edges": [(0, 1, 1), (0, 1, 1)]},
    ]
    G = oracle.Graph(trip, 3, 2)
    for q in qs:
        cnt, rows = G.eval(q)
        assert np.array_equal(rows, brute_force(trip, 3, 2, q)), q


# ------------------------------------------------------------------ closed forms
def _small_graph(seed, n=12, P=3, m=90):
    return workload.uniform_graph(seed, n, P, m), n, P


def test_single_edge_count_is_label_nnz():
    trip, n, P = _small_graph(7, n=30, P=5, m=900)
    G = oracle.Graph(trip, n, P)
    for p in range(1, P + 1):
        q = {"n_qv": 2, "qv_const": [-1, -1], "edges": [(0, p, 1)]}
        assert G.eval(q, rows=False)[0] == int((trip[:, 1] == p).sum())
        assert G.count_acyclic(q) == int((trip[:, 1] == p).sum())


def test_chain_count_is_walk_count():
    trip, n, P = _small_graph(11, n=15, P=3, m=200)
    A = dense_tensor(trip, n, P).astype(np.int64)
    G = oracle.Graph(trip, n, P)
    rng = random.Random(5)
    for _ in range(40):
        k = rng.randint(1, 4)
        labels = [rng.randint(1, P) for _ in range(k)]
        dirs = [rng.randint(0, 1) for _ in range(k)]
        edges = []
        M = np.eye(n, dtype=np.int64)
        for i, (p, d) in enumerate(zip(labels, dirs)):
            edges.append((i, p, i + 1) if d == 0 else (i + 1, p, i))
            M = M @ (A[p] if d == 0 else A[p].T)
        q = {"n_qv": k + 1, "qv_const": [-1] * (k + 1), "edges": edges}
        expect = int(M.sum())
        assert G.eval(q, rows=False)[0] == expect
        assert G.count_acyclic(q) == expect


def test_star_count_is_degree_product():
    trip, n, P = _small_graph(13, n=20, P=3, m=300)
    A = dense_tensor(trip, n, P).astype(np.int64)
    G = oracle.Graph(trip, n, P)
    rng = random.Random(9)
    for _ in range(30):
        k = rng.randint(1, 5)
        edges, per = [], []
        for i in range(k):
            p, d = rng.randint(1, P), rng.randint(0, 1)
            edges.append((0, p, i + 1) if d == 0 else (i + 1, p, 0))
            per.append(A[p].sum(axis=1) if d == 0 else A[p].sum(axis=0))
        expect = int(np.prod(np.stack(per), axis=0).sum())
        q = {"n_qv": k + 1, "qv_const": [-1] * (k + 1), "edges": edges}
        assert G.eval(q, rows=False)[0] == expect
        assert G.count_acyclic(q) == expect


def test_triangle_count_is_trace():
    trip, n, P = _small_graph(17, n=14, P=2, m=150)
    A = dense_tensor(trip, n, P).astype(np.int64)
    G = oracle.Graph(trip, n, P)
    for p1, p2, p3 in itertools.product(range(1, P + 1), repeat=3):
        for d in itertools.product([0, 1], repeat=3):
            mats, edges = [], []
            for i, (p, di) in enumerate(zip((p1, p2, p3), d)):
                a, b = i, (i + 1) % 3
                edges.append((a, p, b) if di == 0 else (b, p, a))
                mats.append(A[p] if di == 0 else A[p].T)
            expect = int(np.trace(mats[0] @ mats[1] @ mats[2]))
            q = {"n_qv": 3, "qv_const": [-1] * 3, "edges": edges}
            assert G.eval(q, rows=False)[0] == expect
            with pytest.raises(oracle.OracleError):
                G.count_acyclic(q)


@pytest.mark.parametrize("seed", range(3))
def test_count_dp_matches_eval_on_acyclic(seed):
    rng = random.Random(300 + seed)
    for _ in range(40):
        n, P = rng.randint(2, 25), rng.randint(1, 4)
        m = rng.randint(1, min(3 * n * n, n * n * P))
        trip = workload.uniform_graph(rng.randrange(1 << 30), n, P, m)
        nv = rng.randint(1, 6)
        q = random_query(rng, n, P, nv, rng.randint(0, 2), n_edges=0, connected=True)
        # a tree over variables and constants, plus optional parallel edges and self loops
        e = list(q["edges"])
        for _ in range(rng.randint(0, 2) if e else 0):
            a, p, b = rng.choice(e)
            e.append((b, rng.randint(1, P), a) if rng.random() < 0.5 else (a, rng.randint(1, P), b))
        if rng.random() < 0.3 or not e:
            v = rng.randrange(q["n_qv"])
            e.append((v, rng.randint(1, P), v))
        q["edges"] = e
        G = oracle.Graph(trip, n, P)
        expect = G.eval(q, rows=False)[0]
        assert G.count_acyclic(q) == expect, q
        assert G.count_acyclic(q, threads=3) == expect, q   # vertex loops split over threads


# ------------------------------------------------------------------ invariants
def test_result_independent_of_order():
    rng = random.Random(77)
    for _ in range(25):
        n, P = rng.randint(3, 10), rng.randint(1, 3)
        trip = workload.uniform_graph(rng.randrange(1 << 30), n, P, rng.randint(5, n * n))
        q = random_query(rng, n, P, rng.randint(2, 4), rng.randint(0, 1))
        G = oracle.Graph(trip, n, P)
        base = G.eval(q)[1]
        var_qv = [i for i, c in enumerate(q["qv_const"]) if c < 0]
        for perm in itertools.permutations(var_qv):
            assert np.array_equal(G.eval(q, order=list(perm))[1], base)


def test_adding_triples_never_removes_rows():
    rng = random.Random(78)
    for _ in range(20):
        n, P = rng.randint(3, 12), rng.randint(1, 3)
        full = workload.uniform_graph(rng.randrange(1 << 30), n, P, rng.randint(min(10, n * n), n * n))
        part = full[: len(full) // 2]
        q = random_query(rng, n, P, rng.randint(1, 4), rng.randint(0, 1))
        r_small = oracle.Graph(part, n, P).eval(q)[1]
        r_big = oracle.Graph(full, n, P).eval(q)[1]
        assert len(r_big) >= len(r_small)
        big = set(map(tuple, r_big.tolist()))
        assert all(tuple(r) in big for r in r_small.tolist())


def test_constant_substitution():
    rng = random.Random(79)
    for _ in range(20):
        n, P = rng.randint(3, 10), rng.randint(1, 3)
        trip = workload.uniform_graph(rng.randrange(1 << 30), n, P, rng.randint(min(10, n * n), n * n))
        q = random_query(rng, n, P, rng.randint(2, 4), 0)
        G = oracle.Graph(trip, n, P)
        rows = G.eval(q)[1]
        x = rng.randrange(q["n_qv"])
        c = rng.randrange(n)
        q2 = dict(q, qv_const=[c if i == x else v for i, v in enumerate(q["qv_const"])])
        expect = sort_rows(np.delete(rows[rows[:, x] == c], x, axis=1)) if len(rows) else np.zeros((0, q["n_qv"] - 1), np.int32)
        got = G.eval(q2)[1]
        assert np.array_equal(got.reshape(-1, q["n_qv"] - 1), expect.reshape(-1, q["n_qv"] - 1))


def test_disjoint_union_is_product():
    rng = random.Random(80)
    for _ in range(20):
        n, P = rng.randint(3, 10), rng.randint(1, 3)
        trip = workload.uniform_graph(rng.randrange(1 << 30), n, P, rng.randint(min(10, n * n), n * n))
        G = oracle.Graph(trip, n, P)
        q1 = random_query(rng, n, P, rng.randint(1, 2), 0)
        q2 = random_query(rng, n, P, rng.randint(1, 2), 0)
        k1 = q1["n_qv"]
        qu = {"n_qv": k1 + q2["n_qv"], "qv_const": q1["qv_const"] + q2["qv_const"],
              "edges": q1["edges"] + [(a + k1, p, b + k1) for a, p, b in q2["edges"]]}
        assert G.eval(qu, rows=False)[0] == G.eval(q1, rows=False)[0] * G.eval(q2, rows=False)[0]


def test_zero_variable_and_constant_only_queries():
    trip = np.array([[0, 1, 1], [1, 2, 2]], np.int32)
    G = oracle.Graph(trip, 3, 2)
    assert G.eval({"n_qv": 2, "qv_const": [0, 1], "edges": [(0, 1, 1)]}, rows=False)[0] == 1
    assert G.eval({"n_qv": 2, "qv_const": [0, 1], "edges": [(1, 1, 0)]}, rows=False)[0] == 0
    # a constant with no matching edge gives nothing
    assert G.eval({"n_qv": 2, "qv_const": [-1, 2], "edges": [(1, 1, 0)]}, rows=False)[0] == 0


def test_out_of_range_rejected():
    trip = np.array([[0, 1, 1]], np.int32)
    G = oracle.Graph(trip, 2, 1)
    with pytest.raises(oracle.OracleError):
        G.eval({"n_qv": 2, "qv_const": [-1, -1], "edges": [(0, 2, 1)]})
    with pytest.raises(oracle.OracleError):
        G.eval({"n_qv": 2, "qv_const": [-1, 5], "edges": [(0, 1, 1)]})
    with pytest.raises(oracle.OracleError):
        oracle.Graph(np.array([[0, 1, 3]], np.int32), 2, 1)


def test_c0_workload_star_nonempty():
    trip = workload.c0_graph()
    q = workload.c0_star_query(trip, workload.C0["n"])
    G = oracle.Graph(trip, workload.C0["n"], workload.C0["n_labels"])
    assert G.m == workload.C0["m"]
    cnt, rows = G.eval(q)
    assert cnt >= 1 and cnt == G.count_acyclic(q)
    # every row satisfies every pattern
    S = set(map(tuple, trip.tolist()))
    var_qv = [i for i, c in enumerate(q["qv_const"]) if c < 0]
    for r in rows.tolist():
        val = {v: r[i] for i, v in enumerate(var_qv)}
        val.update({i: c for i, c in enumerate(q["qv_const"]) if c >= 0})
        assert all((val[s], p, val[o]) in S for s, p, o in q["edges"])


# ------------------------------------------------------------------ set semantics of the load
def test_duplicate_and_permuted_triples_form_a_set():
    # Section 2.2.1: a dataset is a set of triples. Repeated and reordered input triples must
    # give the same index, the same distinct count and the same results as the distinct set.
    rng = np.random.default_rng(21)
    for case in range(20):
        n, P = int(rng.integers(2, 12)), int(rng.integers(1, 4))
        base = np.stack([rng.integers(0, n, 60), rng.integers(1, P + 1, 60), rng.integers(0, n, 60)], 1)
        dup = np.concatenate([base, base[rng.integers(0, len(base), 80)]])
        dup = dup[rng.permutation(len(dup))].astype(np.int32)
        uniq = np.unique(base, axis=0)
        G = oracle.Graph(dup, n, P)
        assert G.m == len(uniq)
        # row-wise arrays straight from the distinct set: rows by s, each row by (p, o)
        order = np.lexsort((uniq[:, 2], uniq[:, 1], uniq[:, 0]))
        u = uniq[order]
        rp, col, lab = G.csr()
        assert np.array_equal(rp, np.searchsorted(u[:, 0], np.arange(n + 1), side="left"))
        assert np.array_equal(col, u[:, 2]) and np.array_equal(lab, u[:, 1])
        order = np.lexsort((uniq[:, 0], uniq[:, 1], uniq[:, 2]))
        u = uniq[order]
        cp, row, labc = G.csc()
        assert np.array_equal(cp, np.searchsorted(u[:, 2], np.arange(n + 1), side="left"))
        assert np.array_equal(row, u[:, 0]) and np.array_equal(labc, u[:, 1])
        r = random.Random(case)
        for _ in range(5):
            q = random_query(r, n, P, r.randint(1, 3), r.randint(0, 1))
            cnt, rows = G.eval(q)
            bf = brute_force(uniq, n, P, q)
            assert cnt == len(bf) and (rows.shape[1] == 0 or np.array_equal(rows, bf)), q


def test_streamed_build_equals_one_array():
    # the set built from chunks (repeats across chunks, rows sorted on several threads) is the
    # set built from one array: same distinct count, same row-wise and column-wise arrays
    rng = np.random.default_rng(22)
    n, P = 300, 5
    base = np.stack([rng.integers(0, n, 4000), rng.integers(1, P + 1, 4000), rng.integers(0, n, 4000)], 1)
    dup = np.concatenate([base, base[rng.integers(0, len(base), 3000)]]).astype(np.int32)
    dup = dup[rng.permutation(len(dup))]
    chunks = np.array_split(dup, 7)
    one = oracle.Graph(dup, n, P)
    for threads in (1, 3):
        st = oracle.Graph.from_chunks(lambda: iter(chunks), n, P, threads=threads)
        assert st.m == one.m == len(np.unique(base, axis=0))
        for a, b in zip(st.csr() + st.csc(), one.csr() + one.csc()):
            assert np.array_equal(a, b)
    with pytest.raises(oracle.OracleError):
        bad = dup.copy()
        bad[5, 1] = P + 1
        oracle.Graph.from_chunks(lambda: iter([bad]), n, P)


# ------------------------------------------------------------------ row digest and the timing mode
def test_splitmix64_output_function_reference_values():
    # the first outputs of splitmix64 started from state 0 (Steele, Lea and Flood 2014): its
    # output function applied to 1, 2 and 3 times the golden-ratio increment
    g = 0x9E3779B97F4A7C15
    got = [_mix64((i * g) % (1 << 64)) for i in (1, 2, 3)]
    assert got == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


@pytest.mark.parametrize("seed", range(3))
def test_digest_matches_brute_force_rows(seed):
    rng = random.Random(500 + seed)
    for case in range(40):
        n, P = rng.randint(1, 8), rng.randint(1, 3)
        m = rng.randint(0, n * n * P)
        trip = workload.uniform_graph(rng.randrange(1 << 30), n, P, m) if m else np.zeros((0, 3), np.int32)
        nv = rng.randint(0, 4)
        q = random_query(rng, n, P, nv, rng.randint(0 if nv else 1, 2), connected=rng.random() < 0.8)
        G = oracle.Graph(trip, n, P)
        bf = brute_force(trip, n, P, q)
        expect = row_digest(bf, nv)
        assert G.digest(q) == expect, (case, q)
        assert G.digest(q, threads=3) == expect, (case, q)
        assert G.digest(q, support_filter=True) == expect, (case, q)
        assert G.digest(q, threads=3, support_filter=True) == expect, (case, q)


@pytest.mark.parametrize("seed", range(2))
def test_support_filter_keeps_every_row(seed):
    # denser graphs, longer and cyclic patterns, parallel and antiparallel edges, self loops,
    # constants: the arc-consistency domains never drop a value of a row (brute force)
    rng = random.Random(900 + seed)
    for case in range(30):
        n, P = rng.randint(2, 7), rng.randint(1, 2)
        trip = workload.uniform_graph(rng.randrange(1 << 30), n, P, rng.randint(n, n * n * P))
        nv = rng.randint(2, 4)
        q = random_query(rng, n, P, nv, rng.randint(0, 1), n_edges=rng.randint(nv, nv + 3),
                         connected=rng.random() < 0.9)
        G = oracle.Graph(trip, n, P)
        expect = row_digest(brute_force(trip, n, P, q), nv)
        assert G.digest(q, support_filter=True) == expect, (case, q)


def test_support_filter_cuts_the_search():
    # a branch that can never be completed (no vertex has an out-edge of label 2 and an
    # in-edge of label 1 at once): without the filter the search walks every partial row of
    # the first branch before finding that out; with it the domains are empty at once
    n = 200
    a = np.arange(n, dtype=np.int32)
    trip = np.concatenate([np.stack([a, np.ones(n, np.int32), (a + 1) % n], 1),
                           np.stack([a[: n // 2], np.full(n // 2, 2, np.int32), a[n // 2:]], 1),
                           np.stack([np.zeros(n, np.int32), np.full(n, 3, np.int32), a], 1)]).astype(np.int32)
    keep = ~((trip[:, 1] == 1) & (trip[:, 2] < n // 2))   # label-1 edges only into the upper half
    trip = trip[keep]
    G = oracle.Graph(trip, n, 3)
    q = {"n_qv": 4, "qv_const": [-1] * 4, "edges": [(0, 3, 1), (0, 3, 2), (2, 1, 3), (3, 2, 1)]}
    assert G.eval(q, rows=False)[0] == 0
    with pytest.raises(oracle.OracleError):
        G.digest(q, work_cap=2000)
    assert G.digest(q, support_filter=True, work_cap=2000) == (0, 0, 0)


def test_digest_detects_a_changed_row():
    # a row with one value changed, dropped or repeated changes the digest
    rows = np.array([[1, 2, 3], [4, 5, 6], [1, 2, 4]], np.int32)
    d = row_digest(rows, 3)
    assert row_digest(rows[[0, 1]], 3) != d
    assert row_digest(np.array([[1, 2, 3], [4, 5, 6], [1, 2, 5]]), 3) != d
    assert row_digest(np.array([[1, 2, 3], [4, 5, 6], [1, 2, 3]]), 3)[1:] != d[1:]
    assert row_digest(rows[[2, 0, 1]], 3) == d


def test_digest_on_all_cores_equals_one_thread():
    # the timing mode: the first variable's candidates split over threads gives the same
    # count and digest as the plain evaluation, with and without a constant anchoring them
    n, P = 3000, 4
    trip = workload.uniform_graph(3, n, P, 30000)
    G = oracle.Graph(trip, n, P)
    shapes = ["chain4", "star5", "snowflake8", "triangle"]
    qs = []
    for i, sh in enumerate(shapes):
        qs += workload.walk_queries(trip, n, 40 + i, sh, 2)
    qs.append({"n_qv": 3, "qv_const": [-1, -1, int(trip[0, 0])], "edges": [(2, int(trip[0, 1]), 0), (0, 1, 1)]})
    for q in qs:
        one = G.digest(q)
        assert one[0] == G.eval(q, rows=False)[0]
        for t in (2, 8):
            assert G.digest(q, threads=t) == one, (q, t)
            assert G.digest(q, threads=t, support_filter=True) == one, (q, t)


def test_digest_work_cap_aborts():
    n, P = 400, 2
    trip = workload.uniform_graph(4, n, P, 20000)
    G = oracle.Graph(trip, n, P)
    q = {"n_qv": 4, "qv_const": [-1] * 4, "edges": [(0, 1, 1), (1, 1, 2), (2, 2, 3)]}
    for t in (1, 4):
        with pytest.raises(oracle.OracleError):
            G.digest(q, threads=t, work_cap=100_000)
