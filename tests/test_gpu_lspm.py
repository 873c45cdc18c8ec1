"""Device LSpM builder (Section 6.2) and the matrix-algebra primitives of
Section 2.1 against the oracle, bit for bit."""
import numpy as np
import pytest

import oracle
import workload
from helpers import pack_bits, unpack_bits

gs = pytest.importorskip("paper_2106_14038_amd")
pytestmark = pytest.mark.gpu

SMALL = dict(tree_bytes=1 << 30, scratch_bytes=1 << 29)


def make_engine(trip, n, P, **kw):
    opts = gs.options(**{**SMALL, **kw})
    e = gs.gs_engine_create(opts)
    gs.gs_load_triples(e, n, P, trip)
    return e


CASES = [  # (name, n, P, m, duplicates)
    ("tiny", 3, 2, 7, 3),
    ("one_vertex", 1, 1, 1, 2),
    ("single_label", 2000, 1, 30000, 500),
    ("ragged", 7777, 13, 123457, 1000),
    ("wide_labels", 5000, 300, 80000, 100),
    ("power_law", 50000, 64, 400000, 0),
]


def graph(name, n, P, m, dups, seed=3):
    if name == "power_law":
        t = workload.chunglu_graph(seed, n, P, m)
    else:
        t = workload.uniform_graph(seed, n, P, m)
    if dups:
        rng = np.random.default_rng(seed)
        t = np.concatenate([t, t[rng.integers(0, len(t), dups)]])
        t = t[rng.permutation(len(t))]
    return t


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_lspm_arrays_match_oracle(case):
    name, n, P, m, dups = case
    t = graph(*case)
    print(f"[lspm] case={name} n={n} P={P} m={len(t)}", flush=True)
    G = oracle.Graph(t, n, P)
    e = make_engine(t, n, P)
    try:
        nn, pp, mm, _ = gs.gs_graph_info(e)
        assert (nn, pp, mm) == (n, P, G.m)
        rp, col, lab = gs.gs_lspm_export(e, 0)
        orp, ocol, olab = G.csr()
        assert np.array_equal(rp, orp) and np.array_equal(col, ocol) and np.array_equal(lab, olab)
        cp, row, labc = gs.gs_lspm_export(e, 1)
        ocp, orow, olabc = G.csc()
        assert np.array_equal(cp, ocp) and np.array_equal(row, orow) and np.array_equal(labc, olabc)
        nnz, rows, cols = gs.gs_label_stats(e)
        for p in range(1, P + 1):
            out = G.label_exists(p, 0)
            inn = G.label_exists(p, 1)
            assert np.array_equal(gs.gs_label_exists(e, p, 0), pack_bits(out)), p
            assert np.array_equal(gs.gs_label_exists(e, p, 1), pack_bits(inn)), p
            assert nnz[p - 1] == int((olab == p).sum()) and rows[p - 1] == out.sum() and cols[p - 1] == inn.sum()
    finally:
        gs.gs_engine_destroy(e)


def test_empty_graph_and_bad_ids():
    e = make_engine(np.zeros((0, 3), np.int32), 10, 3)
    try:
        rp, col, lab = gs.gs_lspm_export(e, 0)
        assert rp.tolist() == [0] * 11 and len(col) == 0
    finally:
        gs.gs_engine_destroy(e)
    for bad in ([[0, 1, 10]], [[0, 0, 1]], [[0, 4, 1]], [[-1, 1, 1]]):
        e = gs.gs_engine_create(gs.options(**SMALL))
        try:
            with pytest.raises(gs.GsError) as err:
                gs.gs_load_triples(e, 10, 3, np.array(bad, np.int32))
            assert err.value.status == gs.GS_ERANGE
        finally:
            gs.gs_engine_destroy(e)
    e = make_engine(np.array([[0, 1, 1]], np.int32), 2, 1)
    try:
        with pytest.raises(gs.GsError) as err:
            gs.gs_load_triples(e, 2, 1, np.array([[0, 1, 1]], np.int32))
        assert err.value.status == gs.GS_ESTATE
    finally:
        gs.gs_engine_destroy(e)


@pytest.mark.parametrize("seed", [1, 2])
def test_frontier_domain_push_pull_match_oracle(seed):
    n, P = 6000, 5
    t = workload.chunglu_graph(seed, n, P, 90000, domain_mod=1)
    G = oracle.Graph(t, n, P)
    e = make_engine(t, n, P)
    rng = np.random.default_rng(seed)
    try:
        for dens in (0.001, 0.05, 0.6):
            F = (rng.random(n) < dens).astype(np.uint8)
            mask = (rng.random(n) < 0.5).astype(np.uint8)
            for p in range(1, P + 1):
                for d in (0, 1):
                    ref = G.frontier_domain(F, p, d)
                    push = gs.gs_frontier_domain(e, pack_bits(F), p, d, gs.GS_DOMAIN_PUSH)
                    pull = gs.gs_frontier_domain(e, pack_bits(F), p, d, gs.GS_DOMAIN_PULL)
                    pullm = gs.gs_frontier_domain(e, pack_bits(F), p, d, gs.GS_DOMAIN_PULL, pack_bits(mask))
                    assert np.array_equal(unpack_bits(push, n), ref)
                    assert np.array_equal(unpack_bits(pull, n), ref)
                    assert np.array_equal(unpack_bits(pullm, n), ref & mask)
    finally:
        gs.gs_engine_destroy(e)


def test_bitmap_and_compact():
    for n in (1, 63, 64, 65, 70001):
        t = workload.uniform_graph(5, n, 2, min(10, n * n * 2))
        e = make_engine(t, n, 2)
        rng = np.random.default_rng(n)
        try:
            for k in (0, 1, 3):
                vs = [(rng.random(n) < 0.7).astype(np.uint8) for _ in range(k)]
                ref = np.ones(n, np.uint8)
                for v in vs:
                    ref &= v
                got = gs.gs_bitmap_and_compact(e, [pack_bits(v) for v in vs])
                assert np.array_equal(got, np.nonzero(ref)[0].astype(np.int32))
        finally:
            gs.gs_engine_destroy(e)
