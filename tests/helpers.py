"""Test-side helpers: a brute-force evaluator written directly from the
definition of a basic graph pattern's result (every assignment of vertices to
variables under which every triple pattern is in the dataset), and seeded
random query graphs. Independent of both the oracle and the engine."""
from __future__ import annotations

import itertools
import random

import numpy as np


def dense_tensor(triples, n, n_labels):
    """A[p][s][o] = True iff (s, p, o) is a triple (p 1-based; index 0 unused)."""
    A = np.zeros((n_labels + 1, n, n), dtype=bool)
    t = np.asarray(triples, dtype=np.int64).reshape(-1, 3)
    if len(t):
        A[t[:, 1], t[:, 0], t[:, 2]] = True
    return A


def brute_force(triples, n, n_labels, q):
    """All rows (variables in ascending query-vertex index), sorted; every assignment in [0,n)^k."""
    A = dense_tensor(triples, n, n_labels)
    consts = q["qv_const"]
    var_qv = [i for i, c in enumerate(consts) if c < 0]
    k = len(var_qv)
    if k == 0:
        grid = np.zeros((1, 0), dtype=np.int64)
    else:
        grid = np.array(list(itertools.product(range(n), repeat=k)), dtype=np.int64).reshape(-1, k)
    ok = np.ones(len(grid), dtype=bool)

    def col(v):
        if consts[v] >= 0:
            return np.full(len(grid), consts[v], dtype=np.int64)
        return grid[:, var_qv.index(v)]

    for (s, p, o) in q["edges"]:
        ok &= A[p, col(s), col(o)]
    rows = grid[ok]
    if k == 0:
        return np.zeros((int(ok.sum()), 0), np.int32)
    order = np.lexsort(rows.T[::-1])
    return rows[order].astype(np.int32)


def random_query(rng: random.Random, n, n_labels, n_vars, n_consts=0, n_edges=None, connected=True,
                 allow_self=True):
    nqv = n_vars + n_consts
    qv_const = [-1] * nqv
    cpos = rng.sample(range(nqv), n_consts) if n_consts else []
    for c in cpos:
        qv_const[c] = rng.randrange(n)
    if n_edges is None:
        n_edges = rng.randint(max(1, nqv - 1), nqv + 2)
    edges = []
    verts = list(range(nqv))
    rng.shuffle(verts)
    if connected and nqv > 1:
        for i in range(1, nqv):
            a, b = verts[i], verts[rng.randrange(i)]
            if rng.random() < 0.5:
                a, b = b, a
            edges.append((a, rng.randint(1, n_labels), b))
    while len(edges) < n_edges:
        a = rng.randrange(nqv)
        b = rng.randrange(nqv) if allow_self or nqv == 1 else rng.choice([v for v in range(nqv) if v != a])
        edges.append((a, rng.randint(1, n_labels), b))
    return {"n_qv": nqv, "qv_const": qv_const, "edges": edges}


def sort_rows(rows):
    rows = np.asarray(rows, dtype=np.int64)
    if rows.ndim == 1 or rows.shape[1] == 0 or len(rows) == 0:
        return rows.astype(np.int32)
    return rows[np.lexsort(rows.T[::-1])].astype(np.int32)


def pack_bits(v):
    """uint8 0/1 vector -> uint64 words, bit i = word i//64, bit i%64."""
    v = np.asarray(v, dtype=np.uint8)
    n = len(v)
    w = (n + 63) // 64
    pad = np.zeros(w * 64, np.uint8)
    pad[:n] = v
    bits = pad.reshape(w, 64).astype(np.uint64)
    return (bits << np.arange(64, dtype=np.uint64)).sum(axis=1).astype(np.uint64)


def unpack_bits(words, n):
    words = np.asarray(words, dtype=np.uint64)
    bits = ((words[:, None] >> np.arange(64, dtype=np.uint64)) & np.uint64(1)).astype(np.uint8)
    return bits.reshape(-1)[:n]


def engine_rows(gs, engine, q, flags=0):
    """Run one query through the C-ABI; (count, rows sorted lexicographically)."""
    r = gs.gs_query_run(engine, q, flags)
    try:
        cnt = gs.gs_result_count(r)
        rows = gs.gs_result_rows(r) if not (flags & gs.GS_COUNT_ONLY) else None
    finally:
        gs.gs_result_free(r)
    return cnt, (sort_rows(rows) if rows is not None else None)


_M64 = (1 << 64) - 1


def _mix64(z):
    # output function of splitmix64 (Steele, Lea and Flood, OOPSLA 2014), on Python ints
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def row_digest(rows, width):
    """(count, sum of row hashes mod 2^64, XOR of row hashes) of a bag of rows; a row
    (v_0..v_{k-1}) hashes to h_k with h_0 = k, h_{i+1} = mix64(h_i + 0x9E3779B97F4A7C15 + v_i)."""
    s = x = 0
    n = 0
    for r in np.asarray(rows, dtype=np.int64).reshape(-1, width).tolist() if width else [[]] * len(rows):
        h = width
        for v in r:
            h = _mix64((h + 0x9E3779B97F4A7C15 + (v & 0xFFFFFFFF)) & _M64)
        s = (s + h) & _M64
        x ^= h
        n += 1
    return n, s, x


def row_digest_np(rows):
    """row_digest for an (n, k) int32 array, vectorised (same hash, uint64 arithmetic)."""
    rows = np.asarray(rows)
    n, k = rows.shape
    with np.errstate(over="ignore"):
        h = np.full(n, k, dtype=np.uint64)
        for i in range(k):
            z = h + np.uint64(0x9E3779B97F4A7C15) + rows[:, i].astype(np.uint32).astype(np.uint64)
            z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
            z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
            h = z ^ (z >> np.uint64(31))
        return n, int(h.sum(dtype=np.uint64)), int(np.bitwise_xor.reduce(h)) if n else 0
