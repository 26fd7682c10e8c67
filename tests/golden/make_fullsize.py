"""Writes tests/golden/fullsize.json: the oracle's row count and bag hash of
every full-size result the GPU parity tests check.

Only the seeded generators (``synth``) and the oracle (``oracle``) are
called; nothing here runs the library.  Each entry records the generator
arguments and facts of its input (sizes, chosen constants) so that a test
can tell when the inputs changed under it.

    python tests/golden/make_fullsize.py [cfg2] [cfg3] [cfg4] [cfg5] [--jobs N]

Sections:
  cfg2  the 2-pattern join over the 50M-triple store (whole result)
  cfg3  the 4-pattern query over the 200M-triple store (whole result)
  cfg4  each of the 512 batched subqueries: the first join and, for the
        chained half, the second (whole results)
  cfg5  served queries over the 500M-triple store: the first queries of the
        seeded random-walk stream whose oracle evaluation stays within a row
        cap, with their results; the others are listed as over the cap
Hash: ``oracle.multiset_hash`` of the columns in ascending variable order.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from multiprocessing import get_context

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from oracle.core import Table  # noqa: E402
import synth  # noqa: E402

OUT = os.path.join(HERE, "fullsize.json")
CFG5_ROW_CAP = 1 << 26        # served queries kept for parity: oracle result and intermediates within this
CFG5_STREAM = 700             # queries drawn from the seeded stream (the benchmark's warm-up + timed queries)
CFG5_PARITY = 64              # of those, the first this many within the cap get a stored hash


def bag(T: Table):
    vs = sorted(T.vars)
    n, h1, h2 = oracle.multiset_hash([T.col(v) for v in vs])
    return {"vars": vs, "rows": n, "h1": str(h1), "h2": str(h2)}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def do_cfg2():
    t0 = time.time()
    w = synth.store_cfg2()
    log(f"cfg2: store in {time.time() - t0:.0f} s; query {w.patterns}")
    exp = oracle.query(w.s, w.p, w.o, w.patterns)
    return {"args": {"seed": 1, "n": 50_000_000}, "meta": {k: int(v) for k, v in w.meta.items()},
            "patterns": [list(p) for p in w.patterns], "result": bag(exp)}


def do_cfg3():
    sel = json.load(open(os.path.join(ROOT, "synth", "cfg3_draw.json")))
    t0 = time.time()
    w = synth.store_cfg3(seed=sel["seed"])
    pats = synth.query_cfg3(w, sel["draw"])
    log(f"cfg3: store in {time.time() - t0:.0f} s; query {pats}")
    exp = oracle.query(w.s, w.p, w.o, pats)
    return {"args": {"seed": sel["seed"], "draw": sel["draw"], "n": 200_000_000},
            "patterns": [list(p) for p in pats], "result": bag(exp)}


_SUBS = None


def _cfg4_one(i):
    sub = _SUBS[i]
    v = synth.cfg4_vars(sub)
    t1 = Table(v["T1"], sub["T1"])
    t2 = Table(v["T2"], sub["T2"])
    r1 = oracle.join(t1, t2, 0)
    out = {"rows": [int(t1.n), int(t2.n)], "join1": bag(r1)}
    if "T3" in sub:
        t3 = Table(v["T3"], sub["T3"])
        out["rows"].append(int(t3.n))
        out["join2"] = bag(oracle.join(r1, t3, 20))
    return out


def do_cfg4(jobs):
    global _SUBS
    t0 = time.time()
    _SUBS = synth.batch_cfg4(seed=1, n_sub=512)
    log(f"cfg4: 512 subqueries in {time.time() - t0:.0f} s")
    with get_context("fork").Pool(jobs) as pool:
        res = pool.map(_cfg4_one, range(len(_SUBS)), chunksize=1)
    _SUBS = None
    return {"args": {"seed": 1, "n_sub": 512}, "subqueries": res}


_W5 = None


def _cfg5_one(q):
    try:
        exp = oracle.query(_W5.s, _W5.p, _W5.o, q, max_rows=CFG5_ROW_CAP)
    except OverflowError:
        return None
    if exp.n > CFG5_ROW_CAP:
        return None
    return bag(exp)


def do_cfg5(jobs):
    global _W5
    t0 = time.time()
    w = synth.store_cfg5()
    qs = synth.serving_cfg5(w, CFG5_STREAM, seed=1)
    log(f"cfg5: store and {len(qs)} queries in {time.time() - t0:.0f} s")
    _W5 = w
    with get_context("fork").Pool(jobs) as pool:
        res = pool.map(_cfg5_one, qs, chunksize=1)
    _W5 = None
    within = [i for i, r in enumerate(res) if r is not None]
    return {"args": {"seed": 1, "n": 500_000_000, "stream": CFG5_STREAM, "row_cap": CFG5_ROW_CAP},
            "within_cap": within,
            "parity": [{"index": i, "patterns": [list(p) for p in qs[i]], "result": res[i]}
                       for i in within[:CFG5_PARITY]]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("sections", nargs="*", default=["cfg2", "cfg3", "cfg4", "cfg5"])
    ap.add_argument("--jobs", type=int, default=max(1, min(8, os.cpu_count() or 1)))
    args = ap.parse_args()
    doc = json.load(open(OUT)) if os.path.exists(OUT) else {}
    doc["hash"] = "oracle.multiset_hash over the columns in ascending variable order"
    for sec in args.sections:
        t0 = time.time()
        if sec == "cfg2":
            doc["cfg2"] = do_cfg2()
        elif sec == "cfg3":
            doc["cfg3"] = do_cfg3()
        elif sec == "cfg4":
            doc["cfg4"] = do_cfg4(args.jobs)
        elif sec == "cfg5":
            doc["cfg5"] = do_cfg5(args.jobs)
        else:
            raise SystemExit(f"unknown section {sec}")
        log(f"{sec}: done in {time.time() - t0:.0f} s")
        with open(OUT + ".tmp", "w") as f:
            json.dump(doc, f, indent=1)
        os.replace(OUT + ".tmp", OUT)


if __name__ == "__main__":
    main()
