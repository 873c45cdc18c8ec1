"""ORACLE — test infrastructure only (only the test suite may import it).

Per-query reduction of the RDF matrix, written from its definition in
Section 6.2.1 (direction-driven LSpM: one row-wise part) and Section 6.2.2
(degree-driven LSpM: a row-wise part for the direction-consistent edges, a
column-wise part for the direction-opposite ones; Examples 6.3 and 6.4):
keep the nonzeros whose predicate the query reads in that orientation, drop
the rows (columns) that are left empty, number the kept ones in order, and
store them compressed. Plain numpy; shares nothing with the engine.
"""
from __future__ import annotations

import numpy as np


def orientation_labels(query: dict, edge_group, group_vertex, direction_driven: bool):
    """The predicates (1-based) of the row-wise and of the column-wise part.

    Direction-driven plan without constants (Section 6.2.1): every edge is read along its
    direction, so there is one row-wise part holding every predicate of the query.
    Otherwise (Section 6.2.2; a query with constants takes the degree-driven plan, Section
    6.1.1): an edge evaluated in the group of its subject is direction-consistent (row-wise),
    one evaluated in the group of its object direction-opposite (column-wise); an edge out of a
    constant is row-wise and an edge into a constant column-wise. A repeated edge (group -1)
    goes where its first copy goes."""
    consts = query["qv_const"]
    has_const = any(c >= 0 for c in consts)
    rows, cols = set(), set()
    for k, (s, p, o) in enumerate(query["edges"]):
        if direction_driven and not has_const:
            rows.add(p)
            continue
        if consts[s] >= 0 or consts[o] >= 0:
            if consts[s] >= 0:
                rows.add(p)
            if consts[o] >= 0:
                cols.add(p)
            continue
        g = edge_group[k]
        if g < 0:
            continue
        (rows if group_vertex[g] == s else cols).add(p)
    return sorted(rows), sorted(cols)


def reduce_part(triples: np.ndarray, n: int, labels, orientation: int):
    """One part of the reduced matrix. orientation 0: rows are subjects (LSpM_CSR), 1: rows
    are objects (LSpM_CSC). The triples are taken as a set. Returns (M, P, Val, Idx):
    M has n + 1 entries, M[i + 1] - M[i] == 1 exactly when row i keeps a nonzero and then
    M[i] is its index among the kept rows; P points into Val / Idx per kept row (kept rows + 1
    entries); Val holds the 1-based predicates, Idx the other endpoint, a row's entries in
    ascending (predicate, endpoint) order."""
    t = np.unique(np.asarray(triples, np.int64).reshape(-1, 3), axis=0)
    t = t[np.isin(t[:, 1], np.asarray(sorted(labels), np.int64))]
    a = t[:, 0] if orientation == 0 else t[:, 2]
    b = t[:, 2] if orientation == 0 else t[:, 0]
    order = np.lexsort((b, t[:, 1], a))
    a, p, b = a[order], t[order, 1], b[order]
    cnt = np.bincount(a, minlength=n)[:n]
    M = np.concatenate([[0], np.cumsum(cnt > 0)]).astype(np.int64)
    P = np.concatenate([[0], np.cumsum(cnt[cnt > 0])]).astype(np.int64)
    return M, P, p.astype(np.int32), b.astype(np.int32)


def expand_rows(M, P, n):
    """Row pointers of the unreduced layout from a reduced part: row i spans
    [P[M[i]], P[M[i + 1]]) (empty when the row was dropped)."""
    M = np.asarray(M)
    return np.asarray(P)[M[: n + 1]]
