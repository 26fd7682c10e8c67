"""Benchmark of the MapSQ join path on one MI355X.

Workload (default): the plain 2-pattern join ``?x p1 ?y . ?y p2 c`` over
50M dictionary-encoded int32 triples (32 predicates, Zipf(1.0); subject and
object IDs Zipf(1.1) over 10M entities), about 194M output rows.  The store
and its indexes are built once and stay resident in HBM; one step is one
``mapsq_query`` call: map both patterns, group the records by key (here both
patterns come from the index sorted on the key, so the join pairs key runs
directly), count/scan, materialise the result table in HBM, free it.
``value`` is joined output rows per second.

The roofline entry is for the dominant kernel (materialisation): its
algorithmic bytes per launch divided by its average launch time, timed with
HIP events recorded by the library on the stream it launches on.

Two more measurements go into the same JSON line: "batched" (512
independent subqueries, plain one-join-per-call against one batched launch
per chain step, exact row-for-row agreement checked) and "serving" (a
resident 500M-triple store, random-walk queries, one query at a time against
continuous batching, saturated and at Poisson arrival rates, p50/p99).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
                       [--no-batched] [--no-serving]
       python bench.py --cfg4-only | --cfg5-only   (one of the two extra measurements)
       python bench.py --copy-calibration   (plain copy of a known size, for PMC scaling)
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "materialize_cfg2_traffic.json")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def traffic_from_profile():
    """HBM bytes per materialisation launch from the committed rocprofv3 PMC
    summary, or None if it is missing or was taken on another kernel source."""
    try:
        d = json.load(open(PROFILE_TRAFFIC))
    except (OSError, ValueError):
        return None
    from paper_1702_03484_amd.profile_summary import kernel_sha

    if d.get("kernel_source_sha256") != kernel_sha():
        return None
    return d.get("hbm_bytes_per_launch")


def copy_calibration(nbytes=1 << 30, reps=3):
    import torch

    a = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": nbytes, "reps": reps}), flush=True)


def cpu_baseline(w):
    """The oracle, as it stands, on the full workload (one run)."""
    import oracle

    t0 = time.perf_counter()
    p1 = oracle.pmt(w.s, w.p, w.o, w.patterns[0], key_var=1)
    p2 = oracle.pmt(w.s, w.p, w.o, w.patterns[1], key_var=1)
    rs = oracle.join(p1, p2, 1)
    el = time.perf_counter() - t0
    return {"value": rs.n / el, "unit": "rows/s", "cores": 1, "kind": "oracle",
            "sample": f"whole workload, one run: numpy map of both patterns + sort-merge join, "
                      f"{rs.n} rows in {el:.2f} s (numpy, single thread)"}, rs.n


def phase_table(prof):
    """Per-phase average launch time, algorithmic bytes and GB/s (fraction of peak)."""
    from paper_1702_03484_amd import binding as B

    out = {}
    for k, name in enumerate(B.PHASES):
        if name in ("index", "batch"):
            continue
        n = prof.launches[k]
        if n == 0:
            continue
        ms = prof.ms[k] / n
        by = prof.bytes[k] / n
        gbs = by / (ms * 1e-3) / 1e9 if ms > 0 else None
        out[name] = {"avg_ms": round(ms, 4), "bytes_per_launch": int(by),
                     "gbs": round(gbs, 1) if gbs else None,
                     "frac": round(gbs / HBM_PEAK_GBS, 4) if gbs else None}
    return out


def run_shuffle(n=16_000_000, key_bits=24, reps=5):
    """The shuffle path on its own: a join of two n-row tables with uniform
    random keys over 2^key_bits values and one value column each, with the
    merge join, the semi-join reduction and the exact count before sorting
    turned off, so every record goes through the histogram, radix passes,
    segment heads and counts, and nothing else is timed."""
    import numpy as np
    import torch

    from paper_1702_03484_amd import binding as B
    from paper_1702_03484_amd.engine import MapSQ

    r = np.random.default_rng(11)
    with MapSQ(arena_bytes=32 << 30) as sess:
        cols = [torch.from_numpy(r.integers(0, 1 << key_bits, n).astype(np.int32)).cuda() for _ in range(2)]
        vals = [torch.from_numpy(r.integers(0, 1 << 31, n).astype(np.int32)).cuda() for _ in range(2)]
        L = sess.table([0, 1], [cols[0], vals[0]], key_max=(1 << key_bits) - 1)
        R = sess.table([0, 2], [cols[1], vals[1]], key_max=(1 << key_bits) - 1)
        sess.set_join_options(semijoin=1, merge=1, precount=1)
        for _ in range(2):
            sess.free(sess.join(L, R, 0))
        torch.cuda.synchronize()
        B.mapsq_profile_enable(sess.ctx, True)
        t0 = time.perf_counter()
        for _ in range(reps):
            t = sess.join(L, R, 0)
            rows = int(t.nrows)
            sess.free(t)
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) / reps
        st = sess.stats()
        phases = phase_table(B.mapsq_profile_read(sess.ctx))
    return {"workload": f"join of two {n}-row tables, uniform keys over 2^{key_bits}, one value column each, "
                       "merge join, semi-join and exact pre-count off", "records": 2 * n, "rows": rows, "radix_bits": st.radix_bits,
            "passes": st.passes, "ms_per_join": round(el * 1e3, 3), "phases": phases}


def run_cfg4(seed=1, n_sub=512, reps=2):
    """Batched form vs plain one-join-per-call form on the 512-subquery
    batch workload; exactness: every batched result equals the plain result
    row for row (compared on the GPU)."""
    import numpy as np
    import torch

    from paper_1702_03484_amd import binding as B
    from paper_1702_03484_amd.engine import MapSQ
    from synth import batch_cfg4, cfg4_vars

    log(f"[cfg4] generating {n_sub} subqueries")
    t0 = time.perf_counter()
    subs = batch_cfg4(seed=seed, n_sub=n_sub)
    log(f"[cfg4] generated in {time.perf_counter() - t0:.1f} s")
    sess = MapSQ(arena_bytes=96 << 30)
    kmax = (1 << 31) - 2  # values span the whole ID range
    tabs = []
    in_rows = 0
    for s in subs:
        v = cfg4_vars(s)
        d = {}
        for name in ("T1", "T2", "T3"):
            if name in s:
                cols = [torch.from_numpy(c).cuda() for c in s[name]]
                d[name] = sess.table(v[name], cols, key_max=kmax)
                in_rows += len(s[name][0])
        tabs.append(d)
    del subs
    torch.cuda.synchronize()
    log(f"[cfg4] {in_rows} input rows resident")

    def plain_run(keep=False):
        outs = []
        for d in tabs:
            r1 = sess.join(d["T1"], d["T2"], 0)
            if "T3" in d:
                r2 = sess.join(r1, d["T3"], 20)
                if keep:
                    outs.append((r1, r2))
                else:
                    sess.free(r1)
                    sess.free(r2)
            elif keep:
                outs.append((r1, None))
            else:
                sess.free(r1)
        return outs

    def batch_run():
        first = sess.join_batch([(d["T1"], d["T2"], 0) for d in tabs])
        chain = [i for i, d in enumerate(tabs) if "T3" in d]
        second = sess.join_batch([(first[i], tabs[i]["T3"], 20) for i in chain])
        return first, dict(zip(chain, second))

    # warm up both forms (graph capture, status growth)
    for t in plain_run(keep=False):
        pass
    f, s2 = batch_run()
    rows = sum(int(f[i].nrows) if i not in s2 else int(s2[i].nrows) for i in range(len(tabs)))
    for t in list(f) + list(s2.values()):
        sess.free(t)
    torch.cuda.synchronize()

    tp, tb = [], []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plain_run()
        torch.cuda.synchronize()
        tp.append(time.perf_counter() - t0)
        B.mapsq_profile_enable(sess.ctx, True)
        t0 = time.perf_counter()
        f, s2 = batch_run()
        torch.cuda.synchronize()
        tb.append(time.perf_counter() - t0)
        prof = B.mapsq_profile_read(sess.ctx)
        for t in list(f) + list(s2.values()):
            sess.free(t)
    log(f"[cfg4] plain {min(tp):.3f} s, batched {min(tb):.3f} s")

    # exactness: batched == plain, row for row, every join
    f, s2 = batch_run()
    exact = True
    for i, d in enumerate(tabs):
        r1 = sess.join(d["T1"], d["T2"], 0)
        pairs = [(r1, f[i])]
        r2 = None
        if "T3" in d:
            r2 = sess.join(r1, d["T3"], 20)
            pairs.append((r2, s2[i]))
        for a, b in pairs:
            if a.nrows != b.nrows or a.vars != b.vars:
                exact = False
            else:
                for c in range(a.ncols):
                    if not torch.equal(sess.column(a, c), sess.column(b, c)):
                        exact = False
        sess.free(r1)
        if r2 is not None:
            sess.free(r2)
    for t in list(f) + list(s2.values()):
        sess.free(t)
    sess.close()
    n_q = len(tabs)
    bms = prof.ms[6] / max(1, prof.launches[6])
    bbytes = prof.bytes[6] / max(1, prof.launches[6])
    return {"workload": f"{n_q} subqueries (half 1 join, half 2 chained joins), tables log-uniform "
                        f"[1e3, 1e7] rows, key cardinality log-uniform [1e2, 1e6], output cap 2^24 per join",
            "input_rows": in_rows, "output_rows": rows,
            "plain_qps": n_q / min(tp), "batched_qps": n_q / min(tb), "speedup": min(tp) / min(tb),
            "batched_rows_per_s": rows / min(tb),
            "batched_launch_avg_ms": round(bms, 3),
            "batched_launch_gbs": round(bbytes / (bms * 1e-3) / 1e9, 1) if bms > 0 else None,
            "exact_vs_plain": exact}


def run_cfg5(n_triples=500_000_000, n_queries=600, warm=100, loads=(0.25, 0.5, 1.0, 2.0), seed=1):
    """Serving over the resident store: plain one-query-at-a-time vs
    continuous batching, Poisson arrivals at fractions of the plain form's
    saturated rate; p50/p99 latency and completed queries/s."""
    import numpy as np
    import torch

    from paper_1702_03484_amd import binding as B
    from paper_1702_03484_amd import serving
    from paper_1702_03484_amd.engine import MapSQ
    from synth import serving_cfg5, store_cfg5

    log(f"[cfg5] generating the {n_triples}-triple store")
    t0 = time.perf_counter()
    w = store_cfg5(n=n_triples, n_entities=max(1000, n_triples // 5))
    log(f"[cfg5] generated in {time.perf_counter() - t0:.1f} s; drawing queries")
    qs = serving_cfg5(w, warm + n_queries, seed=seed)
    sess = MapSQ(arena_bytes=160 << 30)
    info = sess.load(w.s, w.p, w.o)
    del w
    torch.cuda.synchronize()
    log(f"[cfg5] store resident: {info.n_triples} triples, {info.n_predicates} predicates")
    warm_q, qs = qs[:warm], qs[warm:]
    serving.run_plain(sess, warm_q, np.zeros(len(warm_q)))
    serving.run_continuous(sess, warm_q, np.zeros(len(warm_q)))
    sat_plain, lat_p, st_p = serving.run_plain(sess, qs, np.zeros(len(qs)))
    sat_cont, _, st_c = serving.run_continuous(sess, qs, np.zeros(len(qs)))
    # the same queries complete, and the same fail with the same status, in
    # both modes (serving reports every memory failure as TOO_LARGE)
    mem = np.where(st_p == B.MAPSQ_ERR_CAPACITY, B.MAPSQ_ERR_TOO_LARGE, st_p)
    sat_cont["same_outcomes_as_plain"] = bool((st_c == mem).all())
    # one query at a time from t = 0: the gaps between completions are service times
    order = np.argsort(lat_p)
    svc = np.diff(np.concatenate([[0.0], lat_p[order]]))
    svc_of = np.empty_like(svc)
    svc_of[order] = svc
    ok = st_p == 0
    log(f"[cfg5] plain service time: completed {svc_of[ok].sum():.3f} s over {ok.sum()} queries, "
        f"refused {svc_of[~ok].sum():.3f} s over {(~ok).sum()}")
    for j in np.argsort(-svc_of)[:8]:
        log(f"[cfg5]   {svc_of[j] * 1e3:8.2f} ms status {int(st_p[j])}: {qs[j]}")
    log(f"[cfg5] saturated: plain {sat_plain['qps']:.0f} q/s, continuous {sat_cont['qps']:.0f} q/s")
    rows = []
    for f in loads:
        qps = f * sat_plain["qps"]
        arr = serving.poisson_arrivals(seed, len(qs), qps)
        p, _, _ = serving.run_plain(sess, qs, arr)
        c, _, _ = serving.run_continuous(sess, qs, arr)
        rows.append({"load": f, "offered_qps": qps, "plain": p, "continuous": c})
        log(f"[cfg5] load {f}: plain p50 {p['p50_ms']:.2f} ms p99 {p['p99_ms']:.2f} ms {p['qps']:.0f} q/s; "
            f"continuous p50 {c['p50_ms']:.2f} ms p99 {c['p99_ms']:.2f} ms {c['qps']:.0f} q/s")
    sess.close()
    return {"workload": f"{info.n_triples}-triple resident store (128 predicates Zipf 1.0, entities Zipf 1.1 over "
                        f"{n_triples // 5}), {len(qs)} random-walk queries of 1-5 patterns with 0-2 constants each",
            "saturated_plain": sat_plain, "saturated_continuous": sat_cont, "poisson": rows}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--n", type=int, default=50_000_000, help="triples (default: the full workload)")
    ap.add_argument("--no-batched", action="store_true", help="leave out the 512-subquery batched-vs-plain measurement")
    ap.add_argument("--cfg4-only", action="store_true")
    ap.add_argument("--no-serving", action="store_true", help="leave out the serving measurement (500M-triple store)")
    ap.add_argument("--cfg5-only", action="store_true")
    ap.add_argument("--shuffle-only", action="store_true", help="only the 16M + 16M-record shuffle join")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (--gpus {args.gpus} requested): the join runs on a single "
              "MI355X and there is no multi-GPU path", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return
    if args.cfg4_only:
        print(json.dumps(run_cfg4()), flush=True)
        return
    if args.cfg5_only:
        print(json.dumps(run_cfg5()), flush=True)
        return
    if args.shuffle_only:
        print(json.dumps(run_shuffle()), flush=True)
        return

    import torch

    from paper_1702_03484_amd import binding as B
    from paper_1702_03484_amd.engine import MapSQ
    from synth import store_cfg2, var

    full = args.n == 50_000_000
    log(f"[bench] generating the workload ({args.n} triples)")
    t0 = time.perf_counter()
    w = store_cfg2() if full else store_cfg2(n=args.n, n_entities=max(1000, args.n // 5),
                                               row_cap=4 * args.n)
    log(f"[bench] generated in {time.perf_counter() - t0:.1f} s: {w.meta}")

    sess = MapSQ(arena_bytes=32 << 30)
    B.mapsq_profile_enable(sess.ctx, True)
    t0 = time.perf_counter()
    info = sess.load(w.s, w.p, w.o)
    torch.cuda.synchronize()
    load_s = time.perf_counter() - t0
    prof = B.mapsq_profile_read(sess.ctx)
    index_ms = prof.ms[5]
    log(f"[bench] store loaded: {info.n_triples} triples, {info.n_predicates} predicates, max id {info.max_id}, "
        f"load {load_s:.2f} s (index build {index_ms:.1f} ms on the GPU)")

    rows = 0
    for i in range(args.warmup):
        t = sess.query(w.patterns)
        rows = int(t.nrows)
        sess.free(t)
    torch.cuda.synchronize()
    log(f"[bench] warmup done: {rows} rows per step")

    B.mapsq_profile_enable(sess.ctx, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        t = sess.query(w.patterns)
        rows = int(t.nrows)
        sess.free(t)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    prof = B.mapsq_profile_read(sess.ctx)
    log(f"[bench] timed {args.steps} steps in {el:.4f} s")

    phases = phase_table(prof)
    # Map of a pattern with only a constant object over the whole store: a
    # scan of the raw columns with ballot compaction (the paper's Map)
    c = w.patterns[1][2]
    B.mapsq_profile_enable(sess.ctx, False)
    B.mapsq_profile_enable(sess.ctx, True)
    for _ in range(5):
        t = sess.map((var(0), var(1), c))
        sess.free(t)
    torch.cuda.synchronize()
    mp = phase_table(B.mapsq_profile_read(sess.ctx)).get("map")
    if mp:
        mp["pattern"] = "?s ?p c over the 50M-triple store (variable predicate: full scan + compaction)"
    mat = phases["materialize"]
    achieved = mat["gbs"]
    traffic = traffic_from_profile()
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": "materialize_kernel", "avg_ms": mat["avg_ms"],
                "bytes_per_launch": mat["bytes_per_launch"]}

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on the same workload")
        cpu, cpu_rows = cpu_baseline(w)
        if cpu_rows != rows:
            raise SystemExit(f"oracle row count {cpu_rows} != GPU row count {rows}")
        log(f"[bench] oracle: {cpu['value']:.3e} rows/s")

    sess.close()
    del sess
    torch.cuda.empty_cache()

    def guarded(fn, name):
        try:
            return fn()
        except Exception as e:  # the main line must still come out
            log(f"[bench] {name} failed: {e!r}")
            return {"error": repr(e)}
        finally:
            torch.cuda.empty_cache()

    shuffle = guarded(run_shuffle, "shuffle measurement")
    batched = None if args.no_batched else guarded(run_cfg4, "batched measurement")
    served = None if args.no_serving else guarded(run_cfg5, "serving measurement")
    out = {
        "metric": "joined output rows/s",
        "value": rows * args.steps / el,
        "unit": "rows/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": "plain 2-pattern join ?x p1 ?y . ?y p2 c over 50M int32 triples "
                               "(32 predicates Zipf 1.0, s/o Zipf 1.1 over 10M entities)" if full else
                               f"plain 2-pattern join, {args.n} triples (reduced)",
                   "triples": info.n_triples, "rows_per_step": rows, "left_rows": int(sess_stats_left(w)),
                   "index_build_ms": round(index_ms, 2)},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "phases": phases,
        "map": mp,
        "shuffle": shuffle,
        "batched": batched,
        "serving": served,
    }
    print(json.dumps(out), flush=True)


def sess_stats_left(w):
    import numpy as np

    return int(np.count_nonzero(w.p == w.patterns[0][1]))


if __name__ == "__main__":
    main()
