"""Write the query sets of the power-law workload with their exact counts.

Candidates come from the seeded walk generator (``gen.c``); every count comes
from the oracle (message-passing count for acyclic queries, backtracking with a
work cap for cyclic ones). Queries whose count exceeds the cap, or that the
oracle cannot count within its work cap, are skipped; the next candidate of the
same stream is tried. Run from the repository root:

    python -m workload.make_querysets [--set c1|c2|c3] [--scale 1.0] [--per-shape 25] [--total 1024]
    python -m workload.make_querysets --set c1 --digests   (add row digests to an existing set)

c1: 25 queries per shape (chain-4, star-5, snowflake-8, triangle), counts in
[1, 1e9]; c2: the batched set, 256 queries per shape with random constants and
counts in [1, 1e7] (they spread over the decades; the histogram is printed); c3: the served set, mixed walk shapes with 1-12
edges and 0-2 constants, counts up to 1e7. Output:
workload/data/<set>[s<scale>]_queries.json.
"""
from __future__ import annotations

import argparse
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workload  # noqa: E402

SHAPES = ["chain4", "star5", "snowflake8", "triangle"]
_G = None


def _is_acyclic(q):
    parent = list(range(q["n_qv"]))

    def find(x):
        while parent[x] != x:
            x = parent[x]
        return x
    pairs = set()
    for a, _, b in q["edges"]:
        if a == b or q["qv_const"][a] >= 0 or q["qv_const"][b] >= 0:
            continue
        pairs.add((min(a, b), max(a, b)))
    for a, b in pairs:
        ra, rb = find(a), find(b)
        if ra == rb:
            return False
        parent[ra] = rb
    return True


def _count(q, work_cap):
    try:
        if _is_acyclic(q):
            return _G.count_acyclic(q)
        return _G.eval(q, rows=False, work_cap=work_cap)[0]
    except (oracle.OracleError, OverflowError):
        return -1


def _count_bt(q, work_cap):
    """Backtracking count with a work cap (-1 when the cap is reached)."""
    try:
        return _G.eval(q, rows=False, work_cap=work_cap)[0]
    except oracle.OracleError:
        return -1


def batched_set(trip, n, pool, args, t0):
    """Queries of the four shapes with random constants (0-2 per query; snowflakes
    with 2, else almost all of them exceed the count bound): per shape the first
    walk candidates whose exact count is in [1, 1e7], up to total/4 per shape or
    the shape's time budget; the remaining quota is filled by the shapes in order.
    Exact counts: message passing for acyclic queries, backtracking with the work
    cap for cyclic ones. The count histogram by decade is printed."""
    per = args.total // len(SHAPES)
    got = {sh: [] for sh in SHAPES}
    first = {sh: 0 for sh in SHAPES}

    def fill(shape, si, want, budget):
        ts = time.time()
        cp, mc = (1.0, 2) if shape == "snowflake8" else (args.const_prob, 2)
        while len(got[shape]) < want and first[shape] < args.max_candidates and time.time() - ts < budget:
            batch = workload.walk_queries(trip, n, 100 + si, shape, 64, const_prob=cp, first=first[shape],
                                          max_consts=mc)
            counts = pool.starmap(_count, [(q, args.work_cap) for q in batch])
            for i, (q, c) in enumerate(zip(batch, counts)):
                if 1 <= c <= 10_000_000 and len(got[shape]) < want:
                    got[shape].append({"shape": shape, "candidate": first[shape] + i, "count": int(c), "query": q})
            first[shape] += 64
            print(shape, first[shape], len(got[shape]), f"({time.time() - t0:.0f}s)", flush=True)

    for si, shape in enumerate(SHAPES):
        fill(shape, si, per, args.shape_budget)
    for si, shape in enumerate(SHAPES):   # top up from the shapes that yield
        short = args.total - sum(len(v) for v in got.values())
        if short <= 0:
            break
        fill(shape, si, len(got[shape]) + short, args.shape_budget)
    out = []
    for shape in SHAPES:
        hist = [0] * 8
        for g in got[shape]:
            hist[min(7, len(str(g["count"])) - 1)] += 1
        print(shape, len(got[shape]), "decades", hist, flush=True)
        out += got[shape]
    return out


def served_set(trip, n, pool, args, t0):
    """Mixed walk shapes, 1-12 edges, 0-2 constants, counts in [1, 1e7] (message passing for
    acyclic queries, backtracking with the work cap for cyclic ones)."""
    got, first = [], 0
    while len(got) < args.total and first < args.max_candidates * 4:
        batch = workload.walk_queries(trip, n, 200, "mixed", 64, first=first, max_consts=2)
        counts = pool.starmap(_count, [(q, args.work_cap) for q in batch])
        for i, (q, c) in enumerate(zip(batch, counts)):
            if 1 <= c <= 10_000_000 and len(got) < args.total:
                got.append({"shape": "mixed", "candidate": first + i, "count": int(c), "query": q})
        first += 64
        print(f"served: {len(got)} from {first} candidates ({time.time() - t0:.0f}s)", flush=True)
    return got


def add_digests(path, threads, t0):
    """Add the oracle's order-independent row digest (count, sum and XOR of the row
    hashes) to every query of an existing set file, evaluated by backtracking on
    `threads` host threads; the digest's count must equal the stored count."""
    with open(path) as f:
        out = json.load(f)
    for i, rec in enumerate(out["queries"]):
        q = dict(rec["query"])
        q["edges"] = [tuple(e) for e in q["edges"]]
        ts = time.time()
        cnt, hs, hx = _G.digest(q, threads=threads, support_filter=True)
        if cnt != rec["count"]:
            raise SystemExit(f"query {i}: backtracking count {cnt} != stored count {rec['count']}")
        rec["digest_sum"], rec["digest_xor"] = str(hs), str(hx)
        print(f"digest {i} {rec['shape']} count={cnt} {time.time() - ts:.1f}s ({time.time() - t0:.0f}s)", flush=True)
    out["digest"] = ("row digest: count, sum mod 2^64 and XOR of per-row hashes (oracle.c), rows listing the "
                     "variables in ascending query-vertex index")
    with open(path + ".tmp", "w") as f:
        json.dump(out, f)
    os.replace(path + ".tmp", path)
    print("wrote", path)


def main():
    global _G
    ap = argparse.ArgumentParser()
    ap.add_argument("--set", default="c1", choices=["c1", "c2", "c3"])
    ap.add_argument("--scale", type=float, default=1.0)
    ap.add_argument("--per-shape", type=int, default=25)
    ap.add_argument("--total", type=int, default=1024)
    ap.add_argument("--const-prob", type=float, default=0.5)
    ap.add_argument("--max-candidates", type=int, default=20000)
    ap.add_argument("--cap", type=int, default=1_000_000_000)
    ap.add_argument("--work-cap", type=int, default=300_000_000)
    ap.add_argument("--procs", type=int, default=min(8, os.cpu_count() or 1))
    ap.add_argument("--shape-budget", type=float, default=1200.0, help="seconds per shape (batched set)")
    ap.add_argument("--digests", action="store_true", help="add row digests to the existing set file")
    args = ap.parse_args()
    t0 = time.time()
    trip = workload.c1_graph(args.scale)
    n = max(16, int(workload.C1["n"] * args.scale))
    print(f"graph: {len(trip)} triples, {time.time() - t0:.1f}s", flush=True)
    _G = oracle.Graph(trip, n, workload.C1["n_labels"])
    print(f"oracle index: {time.time() - t0:.1f}s", flush=True)
    out = {"workload": "c1", "scale": args.scale, "n": n, "m": int(len(trip)), "n_labels": workload.C1["n_labels"],
           "seed": workload.C1["seed"], "count_cap": args.cap,
           "note": "counts written by the oracle (workload/make_querysets.py)", "queries": []}
    sc = "" if args.scale == 1.0 else f"s{args.scale:g}"
    if args.digests:
        add_digests(os.path.join(ROOT, "workload", "data", f"{args.set}{sc}_queries.json"), args.procs, t0)
        return
    ctx = mp.get_context("fork")
    if args.set != "c1":
        with ctx.Pool(args.procs) as pool:
            qs = batched_set(trip, n, pool, args, t0) if args.set == "c2" else served_set(trip, n, pool, args, t0)
        out["workload"] = args.set
        out["count_cap"] = 10_000_000
        out["queries"] = qs
        sc = "" if args.scale == 1.0 else f"s{args.scale:g}"
        path = os.path.join(ROOT, "workload", "data", f"{args.set}{sc}_queries.json")
        os.makedirs(os.path.dirname(path), exist_ok=True)
        with open(path, "w") as f:
            json.dump(out, f)
        print("wrote", path)
        return
    with ctx.Pool(args.procs) as pool:
        for shape in SHAPES:
            got, first = [], 0
            while len(got) < args.per_shape and first < 4000:
                batch = workload.walk_queries(trip, n, workload.C1["seed"], shape, 32, first=first)
                counts = pool.starmap(_count, [(q, args.work_cap) for q in batch])
                for i, (q, c) in enumerate(zip(batch, counts)):
                    if 1 <= c <= args.cap and len(got) < args.per_shape:
                        got.append({"shape": shape, "candidate": first + i, "count": int(c), "query": q})
                first += 32
            print(f"{shape}: {len(got)} queries from {first} candidates, counts "
                  f"{sorted(g['count'] for g in got)} ({time.time() - t0:.0f}s)", flush=True)
            out["queries"] += got
    name = "c1_queries.json" if args.scale == 1.0 else f"c1s{args.scale:g}_queries.json"
    path = os.path.join(ROOT, "workload", "data", name)
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w") as f:
        json.dump(out, f)
    print("wrote", path)


if __name__ == "__main__":
    main()
