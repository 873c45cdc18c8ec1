"""Write the query sets of the power-law workload with their exact counts.

Candidates come from the seeded walk generator (``gen.c``); every count comes
from the oracle (message-passing count for acyclic queries, backtracking with a
work cap for cyclic ones). Queries whose count exceeds the cap, or that the
oracle cannot count within its work cap, are skipped; the next candidate of the
same stream is tried. Run from the repository root:

    python -m workload.make_querysets [--set c1|c2|c3] [--scale 1.0] [--per-shape 25] [--total 1024]
    python -m workload.make_querysets --set c1 --digests   (add row digests to an existing set)
    python -m workload.make_querysets --set c2 --per-bucket 32 --shape-budget 900 --procs 3
    python -m workload.make_querysets --set c2 --digests --digest-timeout 300 --procs 6
    python -m workload.make_querysets --set c4 --work-cap 50000000 --per-shape 12 --shape-budget 1500 --procs 6

c1: 25 queries per shape (chain-4, star-5, snowflake-8, triangle), counts in
[1, 1e9]; c2: the batched set, 4 shapes x 8 count decades (1..1e8) x 32 queries with
0-2 constants; c3: the served set, mixed walk shapes with 1-12 edges and 0-2
constants, counts up to 1e7; c4: the 2B-triple graph's sets. Output:
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


def stratified_set(trip, n, pool, args, t0):
    """The batched set stratified by selectivity: for each of the four shapes, `per_bucket`
    queries in each of 8 count decades [10^d, 10^(d+1)), d = 0..7, with 0, 1 or 2 constants
    (uniformly) at non-centre walk positions (triangles: at most 1, the walk's three vertices
    being all there is). Candidates come from the seeded walk generator in stream order and
    are counted by the oracle (message passing for acyclic queries, backtracking with a work
    cap for cycles); a candidate fills a free place of its decade. A shape's search stops at
    its time budget; unfilled places are reported."""
    per = args.per_bucket
    buckets = {sh: [[] for _ in range(8)] for sh in SHAPES}
    for si, shape in enumerate(SHAPES):
        ts, first = time.time(), 0
        while time.time() - ts < args.shape_budget and any(len(b) < per for b in buckets[shape]):
            batch = []
            for nc in (0, 1, 2):
                if shape == "triangle" and nc == 2:
                    continue
                batch += [(nc, q) for q in workload.walk_queries(trip, n, 300 + si, shape, 32, first=first,
                                                                  n_consts=nc)]
            counts = pool.starmap(_count, [(q, args.work_cap) for _, q in batch])
            for (nc, q), c in zip(batch, counts):
                if 1 <= c < 10 ** 8:
                    d = len(str(c)) - 1
                    if len(buckets[shape][d]) < per:
                        buckets[shape][d].append({"shape": shape, "decade": d, "constants": nc, "candidate": first,
                                                  "count": int(c), "query": q})
            first += 32
            print(shape, first, [len(b) for b in buckets[shape]], f"({time.time() - t0:.0f}s)", flush=True)
    out = []
    for shape in SHAPES:
        print(shape, "per decade", [len(b) for b in buckets[shape]], flush=True)
        for b in buckets[shape]:
            out += b
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


def _digest_capped(q, work_cap):
    """Count and row digest by backtracking with a work cap; None when the cap is reached."""
    try:
        return _G.digest(q, work_cap=work_cap)
    except oracle.OracleError:
        return None


def c4_set(args, t0):
    """The 2B-triple graph's query set. The graph is the distinct triples among the first
    `draws` Chung-Lu draws (N = 2e8, beta 2.0, 1024 Zipf labels, typed domains); the oracle
    builds its index from the draw stream. Query walks run on the first `walk_draws` draws
    (every walk triple is a triple of the graph, so every query has a binding).

    - selective set (the batched leg, 256 queries): snowflake-8 with 2 constants, star-5 with 2
      constants and chain-4 with 1 constant, constants at walk vertices of at most 16 incident
      triples (in the walk sample); kept when the oracle's backtracking finishes within its
      work cap with a count in [1, 1e7]; count and row digest from that backtracking;
    - large set: chain-4 and star-5 with one constant, kept when the exact count (message
      passing) is in [1e7, 1e9]; row digest by backtracking over arc-consistent domains.
    """
    global _G
    n, D, Wd = workload.c4_sizes(args.scale)
    P = workload.C4["n_labels"]
    st = workload.c4_stream(args.scale)
    _G = oracle.Graph.from_chunks(lambda: st.chunks(D, 100_000_000), n, P, threads=args.procs)
    print(f"oracle index: n={n} draws={D} distinct={_G.m} ({time.time() - t0:.0f}s)", flush=True)
    wt = st.draws(0, Wd).copy()
    del st
    print(f"walk sample: {len(wt)} triples ({time.time() - t0:.0f}s)", flush=True)
    ctx = mp.get_context("fork")
    sel = {"snowflake8": [], "star5": [], "chain4": []}
    quota = {"snowflake8": 128, "star5": 64, "chain4": 64}
    nconst = {"snowflake8": 2, "star5": 2, "chain4": 1}
    first = {k: 0 for k in sel}
    with ctx.Pool(args.procs) as pool:
        def fill(shape, want, budget):
            ts = time.time()
            while len(sel[shape]) < want and time.time() - ts < budget:
                batch = workload.walk_queries(wt, n, 440 + list(sel).index(shape), shape, 64, first=first[shape],
                                              n_consts=nconst[shape], const_max_deg=16)
                res = pool.starmap(_digest_capped, [(q, args.work_cap) for q in batch])
                for i, (q, r) in enumerate(zip(batch, res)):
                    if r is not None and 1 <= r[0] <= 10_000_000 and len(sel[shape]) < want:
                        sel[shape].append({"shape": shape, "group": "selective", "candidate": first[shape] + i,
                                           "count": int(r[0]), "digest_sum": str(r[1]), "digest_xor": str(r[2]),
                                           "query": q})
                first[shape] += 64
                print(f"c4 selective {shape}: {len(sel[shape])} from {first[shape]} ({time.time() - t0:.0f}s)",
                      flush=True)
        for shape in sel:
            fill(shape, quota[shape], args.shape_budget)
        for shape in sel:   # top up to 256 from the shapes that yield
            short = 256 - sum(len(v) for v in sel.values())
            if short > 0:
                fill(shape, len(sel[shape]) + short, args.shape_budget / 2)
    large = []
    for si, shape in enumerate(("chain4", "star5")):
        got, fst, ts = 0, 0, time.time()
        while got < args.per_shape and time.time() - ts < args.shape_budget:
            for q in workload.walk_queries(wt, n, 460 + si, shape, 16, first=fst, n_consts=1):
                try:
                    c = _G.count_acyclic(q, threads=args.procs)
                except OverflowError:
                    c = -1
                if 10_000_000 <= c <= 1_000_000_000 and got < args.per_shape:
                    large.append({"shape": shape, "group": "large", "candidate": fst, "count": int(c), "query": q})
                    got += 1
                fst += 1
            print(f"c4 large {shape}: {got} from {fst} ({time.time() - t0:.0f}s)", flush=True)
    for rec in large:
        ts = time.time()
        cnt, hs, hx = _G.digest(rec["query"], threads=args.procs, support_filter=True)
        if cnt != rec["count"]:
            raise SystemExit(f"backtracking count {cnt} != message-passing count {rec['count']}")
        rec["digest_sum"], rec["digest_xor"] = str(hs), str(hx)
        print(f"c4 large digest {rec['shape']} count={cnt} {time.time() - ts:.0f}s", flush=True)
    out = {"workload": "c4", "scale": args.scale, "n": n, "draws": D, "m": int(_G.m), "n_labels": P,
           "seed": workload.C4["seed"], "walk_draws": Wd,
           "note": "counts and row digests written by the oracle (workload/make_querysets.py --set c4)",
           "digest": ("row digest: count, sum mod 2^64 and XOR of per-row hashes (oracle.c), rows listing the "
                      "variables in ascending query-vertex index"),
           "queries": sum(sel.values(), []) + large}
    sc = "" if args.scale == 1.0 else f"s{args.scale:g}"
    path = os.path.join(ROOT, "workload", "data", f"c4{sc}_queries.json")
    with open(path + ".tmp", "w") as f:
        json.dump(out, f)
    os.replace(path + ".tmp", path)
    print("wrote", path, {k: len(v) for k, v in sel.items()}, "large", len(large), flush=True)


def _digest_child(q, conn):
    try:
        conn.send(_G.digest(q, threads=1, support_filter=True))
    except Exception as e:   # noqa: BLE001 - reported to the parent
        conn.send(repr(e))
    conn.close()


def add_digests(path, procs, t0, timeout_s=0.0):
    """Add the oracle's order-independent row digest (count, sum and XOR of the row
    hashes) to every query of an existing set file, evaluated by backtracking; the
    digest's count must equal the stored count. timeout_s > 0: each query's
    backtracking runs in a forked child, `procs` at a time, and one that has not
    finished after timeout_s seconds is stopped: that query keeps its count without a
    digest, and the set lists it under "no_digest"."""
    with open(path) as f:
        out = json.load(f)
    recs = out["queries"]

    def finish(i, res, ts):
        rec = recs[i]
        if isinstance(res, str):
            raise SystemExit(f"query {i}: oracle error {res}")
        cnt, hs, hx = res
        if cnt != rec["count"]:
            raise SystemExit(f"query {i}: backtracking count {cnt} != stored count {rec['count']}")
        rec["digest_sum"], rec["digest_xor"] = str(hs), str(hx)
        print(f"digest {i} {rec['shape']} count={cnt} {time.time() - ts:.1f}s ({time.time() - t0:.0f}s)", flush=True)

    todo = [i for i, r in enumerate(recs) if "digest_sum" not in r]
    skipped = []
    if timeout_s <= 0:
        for i in todo:
            q = dict(recs[i]["query"])
            q["edges"] = [tuple(e) for e in q["edges"]]
            ts = time.time()
            finish(i, _G.digest(q, threads=procs, support_filter=True), ts)
    else:
        ctx = mp.get_context("fork")
        running = {}   # i -> (process, parent end of the pipe, start)
        while todo or running:
            while todo and len(running) < procs:
                i = todo.pop(0)
                q = dict(recs[i]["query"])
                q["edges"] = [tuple(e) for e in q["edges"]]
                a, b = ctx.Pipe(duplex=False)
                p = ctx.Process(target=_digest_child, args=(q, b))
                p.start()
                b.close()
                running[i] = (p, a, time.time())
            time.sleep(0.05)
            for i in list(running):
                p, a, ts = running[i]
                if a.poll():
                    res = a.recv()
                    p.join()
                    del running[i]
                    finish(i, res, ts)
                elif time.time() - ts > timeout_s:
                    p.kill()
                    p.join()
                    del running[i]
                    skipped.append(i)
                    print(f"digest {i} {recs[i]['shape']} count={recs[i]['count']}: stopped after {timeout_s:.0f}s",
                          flush=True)
    if skipped:
        out["no_digest"] = sorted(skipped)
        out["no_digest_note"] = (f"the oracle's backtracking did not finish within {timeout_s:.0f}s for these "
                                 "queries: their counts (message passing) stand without a row digest")
    out["digest"] = ("row digest: count, sum mod 2^64 and XOR of per-row hashes (oracle.c), rows listing the "
                     "variables in ascending query-vertex index")
    with open(path + ".tmp", "w") as f:
        json.dump(out, f)
    os.replace(path + ".tmp", path)
    print("wrote", path)


def main():
    global _G
    ap = argparse.ArgumentParser()
    ap.add_argument("--set", default="c1", choices=["c1", "c2", "c3", "c4"])
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
    ap.add_argument("--digest-timeout", type=float, default=0.0,
                    help="with --digests: seconds per query in a forked child (0: no limit, in process)")
    ap.add_argument("--per-bucket", type=int, default=32, help="batched set: queries per shape and count decade")
    args = ap.parse_args()
    t0 = time.time()
    if args.set == "c4":
        c4_set(args, t0)
        return
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
        add_digests(os.path.join(ROOT, "workload", "data", f"{args.set}{sc}_queries.json"), args.procs, t0,
                    args.digest_timeout)
        return
    ctx = mp.get_context("fork")
    if args.set != "c1":
        with ctx.Pool(args.procs) as pool:
            qs = stratified_set(trip, n, pool, args, t0) if args.set == "c2" else served_set(trip, n, pool, args, t0)
        out["workload"] = args.set
        out["count_cap"] = 100_000_000 if args.set == "c2" else 10_000_000
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
