"""ORACLE — test infrastructure only.

Plain CPU reference for SPARQL basic-graph-pattern evaluation over an RDF
triple set and for the matrix-algebra primitives of gSmart (arXiv 2106.14038,
Sections 2.1, 2.2 and 6.2). Only the test suite, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py`` may import it; the engine never does.

The C source (``oracle.c``) shares no code with the HIP engine. This module
only marshals numpy arrays into it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None

RC = {0: "ok", -1: "malformed query", -2: "id or label out of range", -3: "bad order",
      -4: "work cap reached", -5: "query graph is cyclic"}


class OracleError(RuntimeError):
    def __init__(self, rc):
        super().__init__(f"oracle: {RC.get(rc, rc)}")
        self.rc = rc


def build() -> str:
    src = os.path.join(_HERE, "oracle.c")
    subprocess.run(["gcc", "-O2", "-std=c11", "-Wall", "-shared", "-fPIC", "-pthread", "-o", _SO + ".tmp", src],
                   check=True)
    os.replace(_SO + ".tmp", _SO)
    return _SO


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_SO):
        build()
    lib = ctypes.CDLL(_SO)
    vp = ctypes.c_void_p
    i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
    i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
    u8p = np.ctypeslib.ndpointer(np.uint8, flags="C_CONTIGUOUS")
    lib.or_graph_new.argtypes = [i32p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32]
    lib.or_graph_new.restype = vp
    lib.or_graph_begin.argtypes = [ctypes.c_int64, ctypes.c_int32]
    lib.or_graph_begin.restype = vp
    lib.or_graph_count.argtypes = [vp, i32p, ctypes.c_int64]
    lib.or_graph_count.restype = ctypes.c_int
    lib.or_graph_alloc.argtypes = [vp]
    lib.or_graph_alloc.restype = ctypes.c_int
    lib.or_graph_fill.argtypes = [vp, i32p, ctypes.c_int64]
    lib.or_graph_finish.argtypes = [vp, ctypes.c_int32]
    lib.or_graph_finish.restype = ctypes.c_int
    lib.or_graph_free.argtypes = [vp]
    lib.or_graph_m.argtypes = [vp]
    lib.or_graph_m.restype = ctypes.c_int64
    lib.or_csr.argtypes = [vp, i64p, i32p, i32p]
    lib.or_csc.argtypes = [vp, i64p, i32p, i32p]
    lib.or_label_exists.argtypes = [vp, ctypes.c_int32, ctypes.c_int, u8p]
    lib.or_frontier_domain.argtypes = [vp, u8p, ctypes.c_int32, ctypes.c_int, u8p]
    lib.or_eval.argtypes = [vp, ctypes.c_int32, i32p, ctypes.c_int32, i32p, vp, ctypes.c_int32, vp,
                            ctypes.POINTER(ctypes.c_int64), vp, ctypes.c_int64, ctypes.c_int64,
                            ctypes.POINTER(ctypes.c_int32)]
    lib.or_eval.restype = ctypes.c_int
    lib.or_eval_digest.argtypes = [vp, ctypes.c_int32, i32p, ctypes.c_int32, i32p, vp, ctypes.c_int32,
                                   ctypes.c_int32, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_uint64),
                                   ctypes.POINTER(ctypes.c_uint64)]
    lib.or_eval_digest.restype = ctypes.c_int
    lib.or_count_acyclic.argtypes = [vp, ctypes.c_int32, i32p, ctypes.c_int32, i32p, ctypes.c_int32,
                                     ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32)]
    lib.or_count_acyclic.restype = ctypes.c_int
    _lib = lib
    return lib


def _qarrays(q: dict):
    consts = np.ascontiguousarray(q["qv_const"], dtype=np.int32)
    edges = np.ascontiguousarray(np.asarray(q["edges"], dtype=np.int32).reshape(-1))
    if len(consts) == 0:
        consts = np.zeros(1, np.int32)
    return consts, edges


class Graph:
    """The triple set of Section 2.2.1, indexed by (s,p,o) and (o,p,s)."""

    def __init__(self, triples: np.ndarray, n: int, n_labels: int):
        lib = _load()
        t = np.ascontiguousarray(triples, dtype=np.int32).reshape(-1)
        self.n, self.n_labels = int(n), int(n_labels)
        self._h = lib.or_graph_new(t if len(t) else np.zeros(3, np.int32), len(t) // 3, n, n_labels)
        if not self._h:
            raise OracleError(-2)
        self.m = lib.or_graph_m(self._h)

    @classmethod
    def from_chunks(cls, chunks, n: int, n_labels: int, threads: int = 1):
        """The triple set of a stream too large to hold at once: chunks() yields int32 arrays
        of triples; it is called twice (count, then fill) and must yield the same triples."""
        lib = _load()
        self = cls.__new__(cls)
        self.n, self.n_labels = int(n), int(n_labels)
        self._h = lib.or_graph_begin(n, n_labels)
        if not self._h:
            raise MemoryError("oracle graph")
        for c in chunks():
            c = np.ascontiguousarray(c, dtype=np.int32).reshape(-1)
            if len(c) and lib.or_graph_count(self._h, c, len(c) // 3) != 0:
                raise OracleError(-2)
        if lib.or_graph_alloc(self._h) != 0:
            raise MemoryError("oracle graph")
        for c in chunks():
            c = np.ascontiguousarray(c, dtype=np.int32).reshape(-1)
            if len(c):
                lib.or_graph_fill(self._h, c, len(c) // 3)
        if lib.or_graph_finish(self._h, int(threads)) != 0:
            raise RuntimeError("oracle graph: the two orientations disagree")
        self.m = lib.or_graph_m(self._h)
        return self

    def __del__(self):
        if getattr(self, "_h", None):
            _load().or_graph_free(self._h)
            self._h = None

    # -- LSpM (Section 6.2) --------------------------------------------------
    def csr(self):
        rp = np.zeros(self.n + 1, np.int64)
        col = np.zeros(max(self.m, 1), np.int32)
        lab = np.zeros(max(self.m, 1), np.int32)
        _load().or_csr(self._h, rp, col, lab)
        return rp, col[:self.m], lab[:self.m]

    def csc(self):
        cp = np.zeros(self.n + 1, np.int64)
        row = np.zeros(max(self.m, 1), np.int32)
        lab = np.zeros(max(self.m, 1), np.int32)
        _load().or_csc(self._h, cp, row, lab)
        return cp, row[:self.m], lab[:self.m]

    # -- algebra (Section 2.1) -----------------------------------------------
    def label_exists(self, p: int, direction: int) -> np.ndarray:
        """Eq. (4) (direction 0, rows holding p) or Eq. (5) (direction 1, columns)."""
        y = np.zeros(max(self.n, 1), np.uint8)
        _load().or_label_exists(self._h, p, direction, y)
        return y[:self.n]

    def frontier_domain(self, frontier: np.ndarray, p: int, direction: int) -> np.ndarray:
        """Eq. (14)-(16): vertices reached from the selected rows (0) / columns (1) along p."""
        f = np.ascontiguousarray(frontier, dtype=np.uint8)
        y = np.zeros(max(self.n, 1), np.uint8)
        _load().or_frontier_domain(self._h, f, p, direction, y)
        return y[:self.n]

    # -- queries ---------------------------------------------------------------
    def eval(self, q: dict, order=None, rows: bool = True, rows_cap: int = 10_000_000,
             restrict=None, work_cap: int = 0):
        """Backtracking evaluation. Returns (count, rows sorted lexicographically or None).

        restrict = (query_vertex, mask uint8[n]) keeps rows whose query_vertex value is in mask.
        """
        lib = _load()
        consts, edges = _qarrays(q)
        cnt = ctypes.c_int64(0)
        nv = ctypes.c_int32(0)
        o = np.ascontiguousarray(order, dtype=np.int32) if order is not None else None
        nvars = sum(1 for c in q["qv_const"] if c < 0)
        if restrict is not None:
            rq, mask = restrict
            mask = np.ascontiguousarray(mask, dtype=np.uint8)
        else:
            rq, mask = -1, None
        buf = None
        cap = 0
        if rows:
            cap = rows_cap
            buf = np.zeros(max(1, cap * max(nvars, 1)), np.int32)
        rc = lib.or_eval(self._h, q["n_qv"], consts, len(q["edges"]), edges,
                         o.ctypes.data if o is not None else None, rq,
                         mask.ctypes.data if mask is not None else None,
                         ctypes.byref(cnt), buf.ctypes.data if buf is not None else None, cap, work_cap,
                         ctypes.byref(nv))
        if rc != 0:
            raise OracleError(rc)
        if not rows:
            return cnt.value, None
        if cnt.value > cap:
            raise OracleError(-4)
        return cnt.value, buf[:cnt.value * nvars].reshape(cnt.value, nvars).copy()

    def digest(self, q: dict, order=None, threads: int = 1, work_cap: int = 0, support_filter: bool = False):
        """Backtracking evaluation keeping only (count, sum of row hashes mod 2^64, XOR of row
        hashes): the order-independent digest of the result rows (the row hash is defined in
        oracle.c). threads > 1 splits the first variable's candidates over that many threads;
        support_filter narrows candidates by arc consistency first (same rows, less search)."""
        consts, edges = _qarrays(q)
        cnt, hs, hx = ctypes.c_int64(0), ctypes.c_uint64(0), ctypes.c_uint64(0)
        o = np.ascontiguousarray(order, dtype=np.int32) if order is not None else None
        rc = _load().or_eval_digest(self._h, q["n_qv"], consts, len(q["edges"]), edges,
                                    o.ctypes.data if o is not None else None, int(threads),
                                    int(bool(support_filter)), int(work_cap),
                                    ctypes.byref(cnt), ctypes.byref(hs), ctypes.byref(hx))
        if rc != 0:
            raise OracleError(rc)
        return cnt.value, hs.value, hx.value

    def count_acyclic(self, q: dict, threads: int = 1) -> int:
        """Exact count by message passing over the query forest (acyclic queries only); the
        per-vertex loops split over `threads` threads."""
        consts, edges = _qarrays(q)
        cnt = ctypes.c_int64(0)
        sat = ctypes.c_int32(0)
        rc = _load().or_count_acyclic(self._h, q["n_qv"], consts, len(q["edges"]), edges, int(threads),
                                      ctypes.byref(cnt), ctypes.byref(sat))
        if rc != 0:
            raise OracleError(rc)
        if sat.value:
            raise OverflowError("count exceeds int64")
        return cnt.value
