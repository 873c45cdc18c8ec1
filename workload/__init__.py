"""Seeded synthetic inputs: RDF graphs, query graphs and arrival traces.

Shared by the engine's tests and benchmark and by the oracle's tests. The
module only draws inputs (Philox4x32-10 counter streams, see ``gen.c``); it
evaluates no query.

Queries are plain dicts, the Python form of ``gs_query``::

    {"n_qv": 4, "qv_const": [-1, -1, 7, -1], "edges": [(0, 3, 1), (1, 2, 2), ...]}

``qv_const[i] == -1`` marks a variable, any other value is a constant vertex
id. Edges are (src, label, dst) over query-vertex indices, labels 1-based.
"""
from __future__ import annotations

import ctypes
import os
import shutil
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libgswork.so")
_lib = None

SHAPES = {"chain4": 0, "star5": 1, "snowflake8": 2, "triangle": 3, "c0star": 4, "mixed": 5}


_DEV_SO = os.path.join(_HERE, "libgswork_dev.so")
_dev_lib = None


def build() -> str:
    """Compile gen.c into libgswork.so (gcc, OpenMP) and its device twin gen_dev.hip into
    libgswork_dev.so (hipcc, gfx950)."""
    src = os.path.join(_HERE, "gen.c")
    cmd = ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c11", "-Wall", "-Wno-unused-function",
           "-o", _SO + ".tmp", src, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_SO + ".tmp", _SO)
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    arch = os.environ.get("GS_OFFLOAD_ARCH", "gfx950")
    cmd = [hipcc, "-O3", "-std=c++17", "-fPIC", "-shared", f"--offload-arch={arch}", "-Xclang", "-target-feature",
           "-Xclang", "-packed-fp32-ops", "-o", _DEV_SO + ".tmp", os.path.join(_HERE, "gen_dev.hip")]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("gen_dev.hip: " + r.stderr)
    os.replace(_DEV_SO + ".tmp", _DEV_SO)
    return _SO


def _load_dev():
    """The device twin of the draw function (needs PyTorch's HIP runtime loaded first)."""
    global _dev_lib
    if _dev_lib is None:
        import torch  # noqa: F401  (one HIP runtime for both)
        lib = ctypes.CDLL(_DEV_SO)
        vp = ctypes.c_void_p
        lib.gsw_dev_cl_draws.argtypes = [vp, vp, ctypes.c_int64, vp, vp, ctypes.c_int32, vp, ctypes.c_uint64,
                                         ctypes.c_int32, ctypes.c_uint64, ctypes.c_int64, vp, vp]
        lib.gsw_dev_cl_draws.restype = ctypes.c_int
        _dev_lib = lib
    return _dev_lib


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_SO):
        build()
    lib = ctypes.CDLL(_SO)
    i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
    u32p = np.ctypeslib.ndpointer(np.uint32, flags="C_CONTIGUOUS")
    f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
    lib.gsw_philox4x32_10.argtypes = [u32p, u32p, u32p]
    lib.gsw_uniform_graph.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int32, ctypes.c_int64, i32p]
    lib.gsw_uniform_graph.restype = ctypes.c_int
    lib.gsw_chunglu_graph.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int32, ctypes.c_int64,
                                      ctypes.c_double, ctypes.c_double, ctypes.c_int32, i32p]
    lib.gsw_chunglu_graph.restype = ctypes.c_int
    lib.gsw_cl_new.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                               ctypes.c_int32]
    lib.gsw_cl_new.restype = ctypes.c_void_p
    lib.gsw_cl_free.argtypes = [ctypes.c_void_p]
    lib.gsw_cl_draws.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int64, i32p]
    lib.gsw_cl_draws.restype = ctypes.c_int64
    vpp = ctypes.POINTER(ctypes.c_void_p)
    lib.gsw_cl_tables.argtypes = [ctypes.c_void_p, vpp, vpp, vpp, vpp, vpp]
    lib.gsw_query_record_words.restype = ctypes.c_int
    lib.gsw_walk_queries.argtypes = [i32p, ctypes.c_int64, ctypes.c_int64, ctypes.c_uint64, ctypes.c_int32,
                                     ctypes.c_int64, ctypes.c_int32, ctypes.c_double, ctypes.c_int32, i32p]
    lib.gsw_walk_queries.restype = ctypes.c_int
    lib.gsw_walk_queries_ex.argtypes = [i32p, ctypes.c_int64, ctypes.c_int64, ctypes.c_uint64, ctypes.c_int32,
                                        ctypes.c_int64, ctypes.c_int32, ctypes.c_double, ctypes.c_int32,
                                        ctypes.c_int32, ctypes.c_int64, i32p]
    lib.gsw_walk_queries_ex.restype = ctypes.c_int
    lib.gsw_poisson_arrivals.argtypes = [ctypes.c_uint64, ctypes.c_double, ctypes.c_double, ctypes.c_int64, f64p]
    lib.gsw_poisson_arrivals.restype = ctypes.c_int64
    _lib = lib
    return lib


def philox4x32_10(counter, key) -> np.ndarray:
    out = np.zeros(4, np.uint32)
    _load().gsw_philox4x32_10(np.asarray(counter, np.uint32), np.asarray(key, np.uint32), out)
    return out


def uniform_graph(seed: int, n: int, n_labels: int, m: int) -> np.ndarray:
    """m distinct triples, s/o uniform over [0,n), p uniform over [1,n_labels]; (m,3) int32."""
    out = np.empty((m, 3), np.int32)
    rc = _load().gsw_uniform_graph(seed, n, n_labels, m, out)
    if rc != 0:
        raise ValueError(f"gsw_uniform_graph failed ({rc})")
    return out


def chunglu_graph(seed: int, n: int, n_labels: int, m: int, beta: float = 2.1, zipf_s: float = 1.1,
                  domain_mod: int = 5) -> np.ndarray:
    """m distinct Chung-Lu triples with Zipf labels and typed object domains; (m,3) int32."""
    out = np.empty((m, 3), np.int32)
    rc = _load().gsw_chunglu_graph(seed, n, n_labels, m, beta, zipf_s, domain_mod, out)
    if rc != 0:
        raise ValueError(f"gsw_chunglu_graph failed ({rc})")
    return out


class ChungLuStream:
    """The Chung-Lu draws of chunglu_graph as a stream (draw i is a pure function of
    (seed, i)), for graphs defined as the distinct triples among the first `draws` draws."""

    def __init__(self, seed: int, n: int, n_labels: int, beta: float, zipf_s: float, domain_mod: int):
        self.n, self.n_labels = int(n), int(n_labels)
        self.seed, self.domain_mod = int(seed), int(domain_mod)
        self._h = _load().gsw_cl_new(seed, n, n_labels, beta, zipf_s, domain_mod)
        if not self._h:
            raise MemoryError("Chung-Lu generator tables")
        self._dev = None

    def _device_tables(self):
        """Device copies (torch tensors) of the generator's tables."""
        if self._dev is None:
            import torch
            p = [ctypes.c_void_p() for _ in range(5)]
            _load().gsw_cl_tables(self._h, *[ctypes.byref(x) for x in p])
            sizes = [self.n, self.n, self.n_labels, self.n_labels, self.n]
            types = [ctypes.c_uint32, ctypes.c_int32, ctypes.c_uint32, ctypes.c_int32, ctypes.c_int32]
            self._dev = [torch.from_numpy(np.ctypeslib.as_array(ctypes.cast(x, ctypes.POINTER(t)), (k,))
                                          .view(np.int32)).cuda()
                         for x, t, k in zip(p, types, sizes)]
        return self._dev

    def device_draws(self, first: int, count: int, out, stream=None) -> int:
        """Draws [first, first + count) into `out` (a device int32 tensor of count * 3 values,
        in draw order), computed on the device by the twin of the host draw; a draw whose object
        rejection failed is (-1, -1, -1). Returns the number of such failed draws."""
        import torch
        vthr, valias, lthr, lalias, perm = self._device_tables()
        st = stream if stream is not None else torch.cuda.current_stream().cuda_stream
        rc = _load_dev().gsw_dev_cl_draws(vthr.data_ptr(), valias.data_ptr(), self.n, lthr.data_ptr(),
                                          lalias.data_ptr(), self.n_labels, perm.data_ptr(), self.seed,
                                          self.domain_mod, first, count, out.data_ptr(), st)
        if rc != 0:
            raise RuntimeError(f"gsw_dev_cl_draws: HIP error {rc}")
        return int((out.view(-1, 3)[:, 0] < 0).sum().item())

    def device_graph(self, total: int):
        """Draws [0, total) as a device (k, 3) int32 tensor, failed draws left out."""
        import torch
        out = torch.empty(total * 3, dtype=torch.int32, device="cuda")
        chunk = 1 << 28
        bad = 0
        for a in range(0, total, chunk):
            k = min(chunk, total - a)
            bad += self.device_draws(a, k, out[3 * a:3 * (a + k)])
        t = out.view(-1, 3)
        return t[t[:, 0] >= 0] if bad else t

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.gsw_cl_free(self._h)
            self._h = None

    def draws(self, first: int, count: int, out: np.ndarray = None) -> np.ndarray:
        """Draws [first, first + count) as (k, 3) int32, draws whose object rejection failed
        left out (k <= count); `out` (count * 3 int32) is used as the buffer when given."""
        buf = out if out is not None else np.empty(count * 3, np.int32)
        k = _load().gsw_cl_draws(self._h, first, count, buf)
        return buf[:3 * k].reshape(k, 3)

    def chunks(self, total: int, chunk: int = 100_000_000):
        """Draws [0, total) in chunks (one buffer reused: consume each chunk before the next)."""
        buf = np.empty(min(chunk, total) * 3, np.int32)
        for a in range(0, total, chunk):
            yield self.draws(a, min(chunk, total - a), buf)


def _decode(rec: np.ndarray) -> dict:
    maxqv = 16
    nqv, ne = int(rec[0]), int(rec[1])
    consts = [int(x) for x in rec[2:2 + nqv]]
    e = rec[2 + maxqv:2 + maxqv + 3 * ne].reshape(ne, 3)
    return {"n_qv": nqv, "qv_const": consts, "edges": [tuple(int(v) for v in row) for row in e]}


def walk_queries(triples: np.ndarray, n: int, seed: int, shape: str, nq: int, const_prob: float = 0.5,
                 first: int = 0, max_consts: int = 2, n_consts: int = -1, const_max_deg: int = 0) -> list:
    """nq query graphs of the given shape from seeded walks (candidates first .. first+nq-1).
    n_consts >= 0: exactly that many non-centre constants (shapes chain4..triangle), chosen among
    walk vertices with at most const_max_deg incident triples when const_max_deg > 0."""
    lib = _load()
    w = lib.gsw_query_record_words()
    out = np.zeros(max(nq, 1) * w, np.int32)
    t = np.ascontiguousarray(triples, dtype=np.int32).reshape(-1)
    got = lib.gsw_walk_queries_ex(t, len(triples), n, seed, SHAPES[shape], first, nq, const_prob, max_consts,
                                  n_consts, const_max_deg, out)
    if got < 0:
        raise ValueError(f"gsw_walk_queries failed ({got})")
    return [_decode(out[i * w:(i + 1) * w]) for i in range(got)]


def c0_star_query(triples: np.ndarray, n: int, seed: int = 0) -> dict:
    """The 3-edge star (?x,p1,?a),(?x,p2,?b),(?x,p3,c) with c a constant, from a seeded walk."""
    return walk_queries(triples, n, seed, "c0star", 1)[0]


def poisson_arrivals(seed: int, rate: float, duration: float) -> np.ndarray:
    cap = int(rate * duration * 2 + 1000)
    out = np.zeros(cap, np.float64)
    k = _load().gsw_poisson_arrivals(seed, rate, duration, cap, out)
    return out[:k].copy()


# Workload recipes (sizes of the configurations the tests and the benchmark use).
C0 = dict(seed=0, n=10_000, n_labels=16, m=100_000)
C1 = dict(seed=1, n=10_000_000, n_labels=256, m=100_000_000, beta=2.1, zipf_s=1.1, domain_mod=5)


# The 2B-triple graph: the distinct triples among the first `draws` Chung-Lu draws (the draws
# are counted before duplicates are removed); its query walks run on the first `walk_draws`.
C4 = dict(seed=4, n=200_000_000, n_labels=1024, draws=2_000_000_000, walk_draws=200_000_000, beta=2.0,
          zipf_s=1.1, domain_mod=5)


def c4_stream(scale: float = 1.0) -> ChungLuStream:
    """The 2B-triple graph's draw stream; `scale` < 1 shrinks n and the draws together."""
    return ChungLuStream(C4["seed"], max(16, int(C4["n"] * scale)), C4["n_labels"], C4["beta"], C4["zipf_s"],
                         C4["domain_mod"])


def c4_sizes(scale: float = 1.0):
    """(n, draws, walk draws) of the 2B-triple graph at a scale."""
    return (max(16, int(C4["n"] * scale)), max(16, int(C4["draws"] * scale)),
            max(16, int(C4["walk_draws"] * scale)))


def c0_graph() -> np.ndarray:
    return uniform_graph(C0["seed"], C0["n"], C0["n_labels"], C0["m"])


def c1_graph(scale: float = 1.0) -> np.ndarray:
    """The power-law graph; `scale` < 1 shrinks n and m together (tests)."""
    n = max(16, int(C1["n"] * scale))
    m = max(16, int(C1["m"] * scale))
    return chunglu_graph(C1["seed"], n, C1["n_labels"], m, C1["beta"], C1["zipf_s"], C1["domain_mod"])
