"""MI355X engine for SPARQL basic graph patterns by grouped incident-edge
evaluation over a label-carrying sparse RDF matrix (after gSmart, arXiv
2106.14038).

This module is a thin ctypes binding of ``include/gsmart.h``: the functions
keep the C names and only marshal arguments. Every step of the evaluation runs
in the HIP library ``libgsmart.so`` built from ``csrc/``; importing this module
fails if that library is missing. PyTorch, when present, only supplies device
memory (its caching allocator) and streams.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgsmart.so")

GS_OK, GS_EINVAL, GS_ERANGE, GS_ENOMEM, GS_EDEVICE, GS_ESTATE, GS_EUNSUPPORTED, GS_EAGAIN = range(8)
GS_MEM_HOST, GS_MEM_DEVICE = 0, 1
GS_COUNT_ONLY, GS_PRUNE = 1, 2
GS_DOMAIN_AUTO, GS_DOMAIN_PUSH, GS_DOMAIN_PULL, GS_DOMAIN_OFF = 0, 1, 2, 3
GS_TRAVERSAL_DEGREE, GS_TRAVERSAL_DIRECTION, GS_TRAVERSAL_ENGINE = 0, 1, -1
STATUS_NAMES = ["GS_OK", "GS_EINVAL", "GS_ERANGE", "GS_ENOMEM", "GS_EDEVICE", "GS_ESTATE", "GS_EUNSUPPORTED",
                "GS_EAGAIN"]


class GsError(RuntimeError):
    def __init__(self, status, msg):
        name = STATUS_NAMES[status] if 0 <= status < len(STATUS_NAMES) else str(status)
        super().__init__(f"{name}: {msg}")
        self.status = status


class gs_triple(ctypes.Structure):
    _fields_ = [("s", ctypes.c_int32), ("p", ctypes.c_int32), ("o", ctypes.c_int32)]


class gs_edge(ctypes.Structure):
    _fields_ = [("src", ctypes.c_int32), ("label", ctypes.c_int32), ("dst", ctypes.c_int32)]


class gs_query(ctypes.Structure):
    _fields_ = [("n_qv", ctypes.c_int32), ("qv_const", ctypes.POINTER(ctypes.c_int32)),
                ("n_edges", ctypes.c_int32), ("edges", ctypes.POINTER(gs_edge))]


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class gs_options(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int), ("hip_stream", ctypes.c_void_p), ("tree_bytes", ctypes.c_uint64),
                ("scratch_bytes", ctypes.c_uint64), ("alloc", ALLOC_FN), ("free", FREE_FN),
                ("alloc_ctx", ctypes.c_void_p), ("domain_mode", ctypes.c_int32),
                ("push_pull_theta", ctypes.c_float), ("grid_blocks", ctypes.c_int32),
                ("use_graphs", ctypes.c_int32), ("profile_kernels", ctypes.c_int32),
                ("offset_bytes", ctypes.c_int32), ("autotune_cache", ctypes.c_char_p),
                ("traversal", ctypes.c_int32), ("write_block", ctypes.c_int32)]


class gs_query_stats(ctypes.Structure):
    _fields_ = [("count", ctypes.c_int64), ("n_levels", ctypes.c_int32), ("n_domains", ctypes.c_int32),
                ("level_nodes", ctypes.c_int64 * 64), ("t_expand", ctypes.c_int64), ("t_seed", ctypes.c_int64),
                ("t_push", ctypes.c_int64), ("t_pull", ctypes.c_int64), ("t_probe", ctypes.c_int64),
                ("t_total", ctypes.c_int64), ("bytes_alg", ctypes.c_int64), ("domain_push", ctypes.c_int32),
                ("domain_pull", ctypes.c_int32), ("gpu_ms", ctypes.c_double), ("latency_ms", ctypes.c_double),
                ("t_label", ctypes.c_int64), ("seg_lookups", ctypes.c_int64), ("bitmap_words", ctypes.c_int64),
                ("nodes_written", ctypes.c_int64), ("nodes_read", ctypes.c_int64)]


class gs_plan_info(ctypes.Structure):
    _fields_ = [("n_vars", ctypes.c_int32), ("order", ctypes.c_int32 * 64), ("parent_edge", ctypes.c_int32 * 64),
                ("n_groups", ctypes.c_int32), ("group_vertex", ctypes.c_int32 * 64),
                ("edge_group", ctypes.c_int32 * 64), ("n_roots", ctypes.c_int32), ("roots", ctypes.c_int32 * 64)]


class gs_reduced_info(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("rows", ctypes.c_int64 * 2), ("nnz", ctypes.c_int64 * 2),
                ("n_labels", ctypes.c_int32 * 2), ("labels", (ctypes.c_int32 * 64) * 2)]


class gs_kernel_stat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char_p), ("launches", ctypes.c_int64), ("ms", ctypes.c_double),
                ("bytes_alg", ctypes.c_double), ("bytes_impl", ctypes.c_double)]


class gs_tune_result(ctypes.Structure):
    _fields_ = [("grid_blocks", ctypes.c_int32), ("push_pull_theta", ctypes.c_float), ("best_ms", ctypes.c_double),
                ("default_ms", ctypes.c_double), ("n_tried", ctypes.c_int32), ("write_block", ctypes.c_int32)]


class gs_server_options(ctypes.Structure):
    _fields_ = [("max_active", ctypes.c_int32), ("tree_budget_bytes", ctypes.c_uint64), ("flags", ctypes.c_uint32)]


class gs_server_stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64), ("iterations", ctypes.c_int64),
                ("max_active_seen", ctypes.c_int64), ("rejected", ctypes.c_int64), ("requeued", ctypes.c_int64)]


# Every symbol the header declares, with its ctypes signature.
_vp, _i32, _i64, _u32, _u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64
_P = ctypes.POINTER
SIGNATURES = {
    "gs_engine_create": ([_P(gs_options), _P(_vp)], ctypes.c_int),
    "gs_engine_destroy": ([_vp], None),
    "gs_load_triples": ([_vp, _i64, _i32, _vp, _i64, ctypes.c_int], ctypes.c_int),
    "gs_load_triples_labels": ([_vp, _i64, _i32, _vp, _i64, ctypes.c_int, _vp, _i32], ctypes.c_int),
    "gs_lspm_reduce": ([_vp, _P(gs_query), _i32, _P(_vp)], ctypes.c_int),
    "gs_reduced_get_info": ([_vp, _P(gs_reduced_info)], ctypes.c_int),
    "gs_reduced_export": ([_vp, _i32, _vp, _vp, _vp, _vp], ctypes.c_int),
    "gs_reduced_free": ([_vp], ctypes.c_int),
    "gs_encode_ntriples": ([ctypes.c_char_p, _i64, _P(_vp)], ctypes.c_int),
    "gs_dict_info": ([_vp, _P(_i64), _P(_i64), _P(_i32)], ctypes.c_int),
    "gs_dict_triples": ([_vp, _vp], ctypes.c_int),
    "gs_dict_vertex": ([_vp, _i64, ctypes.c_char_p, _i64, _P(_i64)], ctypes.c_int),
    "gs_dict_label": ([_vp, _i32, ctypes.c_char_p, _i64, _P(_i64)], ctypes.c_int),
    "gs_dict_find_vertex": ([_vp, ctypes.c_char_p, _i64, _P(_i64)], ctypes.c_int),
    "gs_dict_find_label": ([_vp, ctypes.c_char_p, _i64, _P(_i32)], ctypes.c_int),
    "gs_dict_free": ([_vp], ctypes.c_int),
    "gs_graph_info": ([_vp, _P(_i64), _P(_i32), _P(_i64), _P(_u64)], ctypes.c_int),
    "gs_lspm_export": ([_vp, ctypes.c_int, _vp, _vp, _vp], ctypes.c_int),
    "gs_label_stats": ([_vp, _vp, _vp, _vp], ctypes.c_int),
    "gs_label_exists": ([_vp, _i32, ctypes.c_int, _vp], ctypes.c_int),
    "gs_frontier_domain": ([_vp, _vp, _i32, ctypes.c_int, ctypes.c_int, _vp, _vp], ctypes.c_int),
    "gs_bitmap_and_compact": ([_vp, _vp, _i32, _vp, _P(_i64)], ctypes.c_int),
    "gs_bitmap_and_compact_noalloc": ([_vp, _vp, _i32, _vp, _vp], ctypes.c_int),
    "gs_plan_query": ([_vp, _P(gs_query), _P(gs_plan_info)], ctypes.c_int),
    "gs_plan_query_ex": ([_vp, _P(gs_query), _i32, _P(gs_plan_info)], ctypes.c_int),
    "gs_query_run": ([_vp, _P(gs_query), _u32, _P(_vp)], ctypes.c_int),
    "gs_batch_run": ([_vp, _P(gs_query), _i32, _u32, _P(_vp)], ctypes.c_int),
    "gs_result_count": ([_vp, _P(_i64)], ctypes.c_int),
    "gs_result_width": ([_vp, _P(_i32)], ctypes.c_int),
    "gs_result_rows": ([_vp, _i64, _i64, _vp, ctypes.c_int, _P(_i64)], ctypes.c_int),
    "gs_result_stats": ([_vp, _P(gs_query_stats)], ctypes.c_int),
    "gs_result_digest": ([_vp, _P(_i64), _P(_u64), _P(_u64)], ctypes.c_int),
    "gs_result_level": ([_vp, _i32, _vp, _vp, _P(_i64)], ctypes.c_int),
    "gs_result_free": ([_vp], None),
    "gs_server_start": ([_vp, _P(gs_server_options), _P(_vp)], ctypes.c_int),
    "gs_submit": ([_vp, _P(gs_query), _u32, _P(_u64)], ctypes.c_int),
    "gs_poll": ([_vp, _u64, _P(_vp)], ctypes.c_int),
    "gs_server_stop": ([_vp, _P(gs_server_stats)], ctypes.c_int),
    "gs_poll_ready": ([_vp, _vp, _vp, _vp, _i32, _P(_i32)], ctypes.c_int),
    "gs_kernel_stats": ([_vp, _P(gs_kernel_stat), _i32, _P(_i32), ctypes.c_int], ctypes.c_int),
    "gs_autotune": ([_vp, _P(gs_query), _i32, _P(gs_tune_result)], ctypes.c_int),
    "gs_last_error": ([], ctypes.c_char_p),
}

_lib = None


def build() -> str:
    """Compile libgsmart.so for gfx950 (hipcc)."""
    from .csrc import build as _b
    return _b.build()


def lib():
    """The loaded HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run paper_2106_14038_amd.build() (hipcc, gfx950) first")
        # PyTorch ships its own HIP runtime under the same soname as the system one; whichever
        # is loaded first serves the whole process. Load PyTorch's first, so that the library
        # and any later torch.cuda use share one runtime (loaded the other way round, torch
        # finds no device).
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in SIGNATURES.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def last_error() -> str:
    return lib().gs_last_error().decode()


def _check(status):
    if status != GS_OK:
        raise GsError(status, last_error())


def make_query(q: dict):
    """Marshal a query dict into a gs_query (the arrays stay alive on the returned object)."""
    n = int(q["n_qv"])
    consts = (ctypes.c_int32 * max(n, 1))(*[int(c) for c in q["qv_const"]])
    edges = (gs_edge * max(len(q["edges"]), 1))(*[gs_edge(int(a), int(p), int(b)) for a, p, b in q["edges"]])
    g = gs_query(n, consts, len(q["edges"]), edges)
    g._keep = (consts, edges)
    return g


# ---- same-named wrappers ------------------------------------------------------------------
def gs_engine_create(options: gs_options | None = None):
    h = ctypes.c_void_p()
    _check(lib().gs_engine_create(ctypes.byref(options) if options is not None else None, ctypes.byref(h)))
    return h


def gs_engine_destroy(engine):
    lib().gs_engine_destroy(engine)


def gs_load_triples(engine, n_vertices: int, n_labels: int, triples, m: int | None = None):
    """triples: numpy (m,3) int32 on the host, or a torch int32 tensor on the device."""
    if hasattr(triples, "data_ptr") and getattr(triples, "is_cuda", False):
        t = triples.contiguous()
        _check(lib().gs_load_triples(engine, n_vertices, n_labels, ctypes.c_void_p(t.data_ptr()),
                                     t.numel() // 3, GS_MEM_DEVICE))
        return
    a = np.ascontiguousarray(triples, dtype=np.int32).reshape(-1, 3)
    _check(lib().gs_load_triples(engine, n_vertices, n_labels, a.ctypes.data_as(ctypes.c_void_p),
                                 len(a) if m is None else m, GS_MEM_HOST))


def gs_graph_info(engine):
    n, p, m, b = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int64(), ctypes.c_uint64()
    _check(lib().gs_graph_info(engine, ctypes.byref(n), ctypes.byref(p), ctypes.byref(m), ctypes.byref(b)))
    return n.value, p.value, m.value, b.value


def gs_lspm_export(engine, orientation: int):
    n, _, m, _ = gs_graph_info(engine)
    ptr = np.zeros(n + 1, np.int64)
    idx = np.zeros(max(m, 1), np.int32)
    lab = np.zeros(max(m, 1), np.int32)
    _check(lib().gs_lspm_export(engine, orientation, ptr.ctypes.data, idx.ctypes.data, lab.ctypes.data))
    return ptr, idx[:m], lab[:m]


def query_labels(q: dict) -> list:
    """The predicates (1-based) a query names: what gs_load_triples_labels keeps for it."""
    return sorted({int(p) for _, p, _ in q["edges"]})


def gs_load_triples_labels(engine, n_vertices: int, n_labels: int, triples, labels):
    """gs_load_triples keeping only the triples whose predicate is in `labels` (1-based)."""
    keep = np.ascontiguousarray(labels, dtype=np.int32)
    if hasattr(triples, "data_ptr") and getattr(triples, "is_cuda", False):
        t = triples.contiguous()
        _check(lib().gs_load_triples_labels(engine, n_vertices, n_labels, ctypes.c_void_p(t.data_ptr()),
                                            t.numel() // 3, GS_MEM_DEVICE, keep.ctypes.data, len(keep)))
        return
    a = np.ascontiguousarray(triples, dtype=np.int32).reshape(-1, 3)
    _check(lib().gs_load_triples_labels(engine, n_vertices, n_labels, a.ctypes.data_as(ctypes.c_void_p), len(a),
                                        GS_MEM_HOST, keep.ctypes.data, len(keep)))


def gs_lspm_reduce(engine, q: dict, traversal: int = GS_TRAVERSAL_ENGINE):
    """The query's reduced matrix: a dict with its info and, per part (0 row-wise, 1
    column-wise), the arrays M, P, val, idx (host copies)."""
    h = ctypes.c_void_p()
    _check(lib().gs_lspm_reduce(engine, ctypes.byref(make_query(q)), traversal, ctypes.byref(h)))
    try:
        info = gs_reduced_info()
        _check(lib().gs_reduced_get_info(h, ctypes.byref(info)))
        out = {"n": info.n, "parts": []}
        for o in range(2):
            rows, nnz = info.rows[o], info.nnz[o]
            M = np.zeros(info.n + 1, np.int64)
            P = np.zeros(rows + 1, np.int64)
            val = np.zeros(max(nnz, 1), np.int32)
            idx = np.zeros(max(nnz, 1), np.int32)
            _check(lib().gs_reduced_export(h, o, M.ctypes.data, P.ctypes.data, val.ctypes.data, idx.ctypes.data))
            out["parts"].append({"labels": list(info.labels[o][:info.n_labels[o]]), "rows": rows, "nnz": nnz,
                                 "M": M, "P": P, "val": val[:nnz], "idx": idx[:nnz]})
        return out
    finally:
        lib().gs_reduced_free(h)


class NTriplesDict:
    """Integer triples and dictionaries of N-Triples text (gs_encode_ntriples)."""

    def __init__(self, text):
        data = text.encode("utf-8") if isinstance(text, str) else bytes(text)
        self._h = ctypes.c_void_p()
        self._lib = lib()
        _check(self._lib.gs_encode_ntriples(data, len(data), ctypes.byref(self._h)))
        nt, nv, nl = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32()
        _check(self._lib.gs_dict_info(self._h, ctypes.byref(nt), ctypes.byref(nv), ctypes.byref(nl)))
        self.n_triples, self.n_vertices, self.n_labels = nt.value, nv.value, nl.value

    def triples(self) -> np.ndarray:
        out = np.zeros((self.n_triples, 3), np.int32)
        _check(self._lib.gs_dict_triples(self._h, out.ctypes.data))
        return out

    def _term(self, f, key) -> str:
        n = ctypes.c_int64()
        _check(f(self._h, key, None, 0, ctypes.byref(n)))
        buf = ctypes.create_string_buffer(n.value + 1)
        _check(f(self._h, key, buf, n.value + 1, ctypes.byref(n)))
        return buf.raw[:n.value].decode("utf-8")

    def vertex(self, i: int) -> str:
        return self._term(self._lib.gs_dict_vertex, i)

    def label(self, p: int) -> str:
        return self._term(self._lib.gs_dict_label, p)

    def find_vertex(self, term: str) -> int:
        b = term.encode("utf-8")
        out = ctypes.c_int64()
        _check(self._lib.gs_dict_find_vertex(self._h, b, len(b), ctypes.byref(out)))
        return out.value

    def find_label(self, term: str) -> int:
        b = term.encode("utf-8")
        out = ctypes.c_int32()
        _check(self._lib.gs_dict_find_label(self._h, b, len(b), ctypes.byref(out)))
        return out.value

    def __del__(self):
        if getattr(self, "_h", None) and self._h.value:
            self._lib.gs_dict_free(self._h)
            self._h = ctypes.c_void_p()


def gs_encode_ntriples(text) -> NTriplesDict:
    return NTriplesDict(text)


def gs_label_stats(engine):
    _, p, _, _ = gs_graph_info(engine)
    a, b, c = (np.zeros(p, np.int64) for _ in range(3))
    _check(lib().gs_label_stats(engine, a.ctypes.data, b.ctypes.data, c.ctypes.data))
    return a, b, c


def _words(engine):
    return (gs_graph_info(engine)[0] + 63) // 64


def gs_label_exists(engine, label: int, direction: int) -> np.ndarray:
    out = np.zeros(_words(engine), np.uint64)
    _check(lib().gs_label_exists(engine, label, direction, out.ctypes.data))
    return out


def gs_frontier_domain(engine, frontier_words, label: int, direction: int, mode: int, mask_words=None):
    f = np.ascontiguousarray(frontier_words, dtype=np.uint64)
    m = np.ascontiguousarray(mask_words, dtype=np.uint64) if mask_words is not None else None
    out = np.zeros(_words(engine), np.uint64)
    _check(lib().gs_frontier_domain(engine, f.ctypes.data, label, direction, mode,
                                    m.ctypes.data if m is not None else None, out.ctypes.data))
    return out


def gs_bitmap_and_compact(engine, bitmaps) -> np.ndarray:
    bms = [np.ascontiguousarray(b, dtype=np.uint64) for b in bitmaps]
    ptrs = (ctypes.c_void_p * max(len(bms), 1))(*[b.ctypes.data for b in bms])
    n = gs_graph_info(engine)[0]
    out = np.zeros(max(n, 1), np.int32)
    cnt = ctypes.c_int64()
    _check(lib().gs_bitmap_and_compact(engine, ptrs, len(bms), out.ctypes.data, ctypes.byref(cnt)))
    return out[:cnt.value].copy()


def gs_bitmap_and_compact_noalloc(engine, dev_bitmaps, dev_out, dev_count) -> None:
    """dev_bitmaps: device addresses (ints) of k bitmaps; dev_out, dev_count: device
    addresses of the id buffer (n int32) and of one int64. Stream-ordered, no sync."""
    ptrs = (ctypes.c_void_p * max(len(dev_bitmaps), 1))(*[int(p) for p in dev_bitmaps])
    _check(lib().gs_bitmap_and_compact_noalloc(engine, ptrs, len(dev_bitmaps), ctypes.c_void_p(int(dev_out)),
                                               ctypes.c_void_p(int(dev_count))))


def gs_plan_query(q: dict, engine=None, traversal: int | None = None) -> gs_plan_info:
    """The plan of query q: the engine's (label statistics) when an engine is given; traversal
    GS_TRAVERSAL_DEGREE / GS_TRAVERSAL_DIRECTION overrides the engine's choice."""
    info = gs_plan_info()
    if traversal is None:
        _check(lib().gs_plan_query(engine, ctypes.byref(make_query(q)), ctypes.byref(info)))
    else:
        _check(lib().gs_plan_query_ex(engine, ctypes.byref(make_query(q)), traversal, ctypes.byref(info)))
    return info


def gs_query_run(engine, q: dict, flags: int = 0):
    r = ctypes.c_void_p()
    _check(lib().gs_query_run(engine, ctypes.byref(make_query(q)), flags, ctypes.byref(r)))
    return r


def gs_batch_run(engine, qs: list, flags: int = 0):
    arr = (gs_query * len(qs))(*[make_query(q) for q in qs])
    outs = (ctypes.c_void_p * len(qs))()
    _check(lib().gs_batch_run(engine, arr, len(qs), flags, outs))
    return [ctypes.c_void_p(o) for o in outs]


def gs_result_count(result) -> int:
    c = ctypes.c_int64()
    _check(lib().gs_result_count(result, ctypes.byref(c)))
    return c.value


def gs_result_width(result) -> int:
    c = ctypes.c_int32()
    _check(lib().gs_result_width(result, ctypes.byref(c)))
    return c.value


def gs_result_rows(result, first: int = 0, n: int | None = None, dst=None) -> np.ndarray:
    """Rows as an (n, n_vars) int32 array (host), or into a device tensor dst."""
    k = gs_result_width(result)
    total = gs_result_count(result)
    if n is None:
        n = total - first
    written = ctypes.c_int64()
    if dst is not None:
        _check(lib().gs_result_rows(result, first, n, ctypes.c_void_p(dst.data_ptr()), GS_MEM_DEVICE,
                                    ctypes.byref(written)))
        return dst
    out = np.zeros((max(n, 0), k), np.int32)
    _check(lib().gs_result_rows(result, first, n, out.ctypes.data if out.size else None, GS_MEM_HOST,
                                ctypes.byref(written)))
    return out[:written.value]


def gs_result_stats(result) -> gs_query_stats:
    s = gs_query_stats()
    _check(lib().gs_result_stats(result, ctypes.byref(s)))
    return s


def gs_result_digest(result):
    """(count, sum of row hashes mod 2^64, XOR of row hashes), computed on the device."""
    c, hs, hx = ctypes.c_int64(), ctypes.c_uint64(), ctypes.c_uint64()
    _check(lib().gs_result_digest(result, ctypes.byref(c), ctypes.byref(hs), ctypes.byref(hx)))
    return c.value, hs.value, hx.value


def gs_result_level(result, level: int):
    n = ctypes.c_int64()
    _check(lib().gs_result_level(result, level, None, None, ctypes.byref(n)))
    par = np.zeros(max(n.value, 1), np.int32)
    vid = np.zeros(max(n.value, 1), np.int32)
    _check(lib().gs_result_level(result, level, par.ctypes.data, vid.ctypes.data, ctypes.byref(n)))
    return par[:n.value], vid[:n.value]


def gs_kernel_stats(engine, reset: bool = False) -> dict:
    arr = (gs_kernel_stat * 32)()
    n = ctypes.c_int32()
    _check(lib().gs_kernel_stats(engine, arr, 32, ctypes.byref(n), int(reset)))
    return {arr[i].name.decode(): {"launches": arr[i].launches, "ms": arr[i].ms, "bytes_alg": arr[i].bytes_alg,
                                   "bytes_impl": arr[i].bytes_impl}
            for i in range(min(n.value, 32))}


def gs_autotune(engine, qs: list) -> gs_tune_result:
    arr = (gs_query * len(qs))(*[make_query(q) for q in qs])
    out = gs_tune_result()
    _check(lib().gs_autotune(engine, arr, len(qs), ctypes.byref(out)))
    return out


def gs_result_free(result):
    lib().gs_result_free(result)


def gs_server_start(engine, options: gs_server_options | None = None):
    h = ctypes.c_void_p()
    _check(lib().gs_server_start(engine, ctypes.byref(options) if options is not None else None, ctypes.byref(h)))
    return h


def gs_submit(server, q: dict, flags: int = 0) -> int:
    t = ctypes.c_uint64()
    _check(lib().gs_submit(server, ctypes.byref(make_query(q)), flags, ctypes.byref(t)))
    return t.value


def gs_poll(server, ticket: int):
    """None while pending, else the result handle."""
    r = ctypes.c_void_p()
    st = lib().gs_poll(server, ticket, ctypes.byref(r))
    if st == GS_EAGAIN:
        return None
    _check(st)
    return r


def gs_poll_ready(server, cap: int = 4096):
    """Finished requests: list of (ticket, status, result handle or None)."""
    t = (ctypes.c_uint64 * cap)()
    st = (ctypes.c_int32 * cap)()
    rs = (ctypes.c_void_p * cap)()
    n = ctypes.c_int32()
    _check(lib().gs_poll_ready(server, t, st, rs, cap, ctypes.byref(n)))
    return [(t[i], st[i], ctypes.c_void_p(rs[i]) if rs[i] else None) for i in range(n.value)]


def gs_server_stop(server) -> gs_server_stats:
    s = gs_server_stats()
    _check(lib().gs_server_stop(server, ctypes.byref(s)))
    return s


# ---- PyTorch plumbing (device memory and streams) -------------------------------------------
_torch_cb = None


def torch_options(device: int = 0, **kw) -> gs_options:
    """Options that route device allocations through PyTorch's caching allocator
    and run on PyTorch's current stream of `device`."""
    import torch
    global _torch_cb
    if _torch_cb is None:
        def _alloc(ctx, size):
            try:
                return torch.cuda.caching_allocator_alloc(int(size), device=int(ctx or 0))
            except Exception:
                return None

        def _free(ctx, ptr):
            torch.cuda.caching_allocator_delete(ptr)
        _torch_cb = (ALLOC_FN(_alloc), FREE_FN(_free))
    o = gs_options()
    o.device = device
    o.hip_stream = torch.cuda.current_stream(device).cuda_stream
    o.alloc, o.free = _torch_cb
    o.alloc_ctx = device
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def options(**kw) -> gs_options:
    o = gs_options()
    for k, v in kw.items():
        setattr(o, k, v)
    return o
