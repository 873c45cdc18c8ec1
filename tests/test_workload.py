"""The seeded input generators: Philox4x32-10 known-answer vectors, determinism,
set semantics and the shape rules of the synthetic workloads."""
import numpy as np

import workload


def test_philox_known_answers():
    # Random123 known-answer vectors for Philox4x32-10 (Salmon et al., SC'11)
    assert workload.philox4x32_10([0, 0, 0, 0], [0, 0]).tolist() == [0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8]
    assert workload.philox4x32_10([0xFFFFFFFF] * 4, [0xFFFFFFFF] * 2).tolist() == [0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD]
    assert workload.philox4x32_10([0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344],
                                  [0xA4093822, 0x299F31D0]).tolist() == [0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1]


def _key(t):
    return (t[:, 0].astype(np.int64) << 40) | (t[:, 1].astype(np.int64) << 28) | t[:, 2].astype(np.int64)


def test_uniform_graph_set_and_determinism():
    a = workload.uniform_graph(3, 500, 7, 20000)
    b = workload.uniform_graph(3, 500, 7, 20000)
    assert np.array_equal(a, b)
    assert len(np.unique(_key(a))) == len(a)
    assert a[:, [0, 2]].min() >= 0 and a[:, [0, 2]].max() < 500 and a[:, 1].min() >= 1 and a[:, 1].max() <= 7
    # a prefix of a longer draw sequence: the first m distinct triples in draw order
    c = workload.uniform_graph(3, 500, 7, 25000)
    assert np.array_equal(c[:20000], a)


def test_chunglu_graph_shape():
    n, m = 100_000, 1_000_000
    t = workload.chunglu_graph(1, n, 256, m)
    assert t.shape == (m, 3) and len(np.unique(_key(t))) == m
    assert t[:, [0, 2]].max() < n and t[:, 1].min() >= 1 and t[:, 1].max() <= 256
    deg = np.bincount(t[:, 0], minlength=n) + np.bincount(t[:, 2], minlength=n)
    # heavy tail: the top vertex holds far more than the mean
    assert deg.max() > 100 * deg.mean()
    # Zipf labels: label 1 is the most frequent and label frequencies fall off
    cnt = np.bincount(t[:, 1], minlength=257)[1:]
    assert cnt[0] == cnt.max() and cnt[0] > 5 * cnt[99]
    # typed domains: each label's objects come from a fifth of the vertices
    for p in (1, 2, 3):
        objs = np.unique(t[t[:, 1] == p, 2])
        assert len(objs) < 0.2 * n + 1
    assert np.array_equal(t, workload.chunglu_graph(1, n, 256, m))


def test_walk_queries_have_witness_and_shape():
    n, m = 20_000, 200_000
    t = workload.chunglu_graph(5, n, 32, m)
    S = set(map(tuple, t.tolist()))
    sizes = {"chain4": (5, 4), "star5": (6, 5), "snowflake8": (9, 8), "triangle": (3, 3)}
    for shape, (nqv, ne) in sizes.items():
        qs = workload.walk_queries(t, n, 11, shape, 8)
        assert len(qs) == 8
        for q in qs:
            assert q["n_qv"] == nqv and len(q["edges"]) == ne
            assert sum(c >= 0 for c in q["qv_const"]) <= 1
            for s, p, o in q["edges"]:
                assert 0 <= s < nqv and 0 <= o < nqv and 1 <= p <= 32
    assert workload.walk_queries(t, n, 11, "star5", 4) == workload.walk_queries(t, n, 11, "star5", 4)
    # mixed shapes: 1..12 edges, at most 2 constants
    for q in workload.walk_queries(t, n, 2, "mixed", 50):
        assert 1 <= len(q["edges"]) <= 12 and sum(c >= 0 for c in q["qv_const"]) <= 2


def test_poisson_arrivals():
    a = workload.poisson_arrivals(1, 5000.0, 2.0)
    assert np.all(np.diff(a) > 0) and a[-1] < 2.0
    assert abs(len(a) - 10000) < 400
