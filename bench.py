"""Benchmark of the MapSQ join path on one MI355X.

Workload (default line): the plain 2-pattern join ``?x p1 ?y . ?y p2 c``
over 50M dictionary-encoded int32 triples (32 predicates, Zipf(1.0); subject
and object IDs Zipf(1.1) over 10M entities), about 194M output rows.  The
store and its indexes are built once and stay resident in HBM; one step is
one ``mapsq_query`` call: map both patterns, group the records by key (here
both patterns come from the index sorted on the key, so the join pairs key
runs directly), count/scan, materialise the result table in HBM, free it.
``value`` is joined output rows per second.

Timing protocol: every timed repetition starts cold.  A 2 GiB device buffer
is read first (eight times the 256 MB last-level cache), the stream is
synchronised, and only then does the repetition's clock start; the
repetition ends with a synchronisation.  The headline times ``--steps``
such repetitions after ``--warmup`` untimed ones; the other legs report the
median of 5 after 2 warm-ups.

The roofline entry is for the dominant kernel (materialisation): its
algorithmic bytes per launch divided by its average launch time, timed with
HIP events recorded by the library on the stream it launches on.

Further legs in the same JSON line: the same join forced through the radix
sort ("cfg2_sort": every record shuffled, the paper's Sort), the
four-pattern query over 200M triples ("cfg3", whose last join shuffles), a
map scan with a variable predicate, a 16M + 16M-record shuffle join,
"batched" (512 independent subqueries, plain one-join-per-call against one
batched launch per chain step, exact row-for-row agreement checked) and
"serving" (a resident 500M-triple store, random-walk queries, one query at
a time against continuous batching, saturated and at Poisson arrival
rates, p50/p99).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
                       [--no-cfg3] [--no-batched] [--no-serving] [--warm]
       python bench.py --cfg3-only | --cfg4-only | --cfg5-only | --shuffle-only | --dict-only
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
FLUSH_BYTES = 2 << 30  # read before every timed repetition (the last-level cache is 256 MB)
COLD = True


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def traffic_from_profile(path=PROFILE_TRAFFIC):
    """HBM bytes per launch from a committed rocprofv3 PMC summary, or None
    if it is missing or was taken on other kernel sources."""
    try:
        d = json.load(open(path))
    except (OSError, ValueError):
        return None
    from paper_1702_03484_amd.profile_summary import kernel_sha

    if d.get("kernel_source_sha256") != kernel_sha():
        return None
    return d.get("hbm_bytes_per_launch")


_flush_buf = None


def cold():
    """Evict the caches by reading a 2 GiB buffer, then wait for the device.
    A read leaves the last-level cache holding clean lines of the buffer; a
    write would leave it full of dirty lines whose write-back then competes
    with the timed kernel's own traffic (a 2 GiB fill "finishes" in 155 us,
    far above HBM speed, and drains afterwards)."""
    global _flush_buf
    import torch

    if COLD:
        if _flush_buf is None:
            _flush_buf = torch.ones(FLUSH_BYTES // 8, dtype=torch.int64, device="cuda")
            torch.cuda.synchronize()
        _flush_buf.sum()
    torch.cuda.synchronize()


def timed_reps(fn, reps=5, warm=2, prof_ctx=None):
    """``warm`` untimed calls, then ``reps`` cold repetitions of ``fn``
    (each timed from after the cache flush to a synchronisation).  With
    ``prof_ctx``, the library's phase profile covers the timed repetitions
    only and is returned too."""
    import torch

    from paper_1702_03484_amd import binding as B

    out = None
    for _ in range(warm):
        out = fn()
    torch.cuda.synchronize()
    if prof_ctx is not None:
        B.mapsq_profile_enable(prof_ctx, False)
        B.mapsq_profile_enable(prof_ctx, True)
    ts = []
    for _ in range(reps):
        cold()
        t0 = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    prof = B.mapsq_profile_read(prof_ctx) if prof_ctx is not None else None
    if prof_ctx is not None:
        B.mapsq_profile_enable(prof_ctx, False)
    return ts, out, prof


def median(xs):
    xs = sorted(xs)
    n = len(xs)
    return xs[n // 2] if n % 2 else 0.5 * (xs[n // 2 - 1] + xs[n // 2])


def copy_calibration(nbytes=1 << 30, reps=3):
    import torch

    a = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": nbytes, "reps": reps}), flush=True)


def cpu_baseline(w, reps=3):
    """The oracle as it stands, on the whole workload: map of both patterns
    and the join, median of ``reps`` runs.  numpy runs on one thread; the
    oracle's C hash join (OpenMP) is timed beside it on all the cores this
    process may use, for the same map + join + output columns."""
    import numpy as np

    import oracle
    from oracle import hashjoin

    cores = len(os.sched_getaffinity(0))
    ts, n = [], 0
    for _ in range(reps):
        t0 = time.perf_counter()
        p1 = oracle.pmt(w.s, w.p, w.o, w.patterns[0], key_var=1)
        p2 = oracle.pmt(w.s, w.p, w.o, w.patterns[1], key_var=1)
        rs = oracle.join(p1, p2, 1)
        ts.append(time.perf_counter() - t0)
        n = rs.n
        del rs
    threads = int(os.environ.get("OMP_NUM_THREADS", cores))
    th, nh = [], 0
    for _ in range(reps):
        t0 = time.perf_counter()
        p1 = oracle.pmt(w.s, w.p, w.o, w.patterns[0], key_var=1)
        p2 = oracle.pmt(w.s, w.p, w.o, w.patterns[1], key_var=1)
        i, j = hashjoin.hj_pairs(p1.col(1), p2.col(1), nthreads=min(threads, cores))
        cols = [p1.col(1)[i], p1.col(0)[i]] + [p2.col(v)[j] for v in p2.vars if v != 1]
        th.append(time.perf_counter() - t0)
        nh = int(i.size)
        del i, j, cols
    el, eh = median(ts), median(th)
    return {"value": n / el, "unit": "rows/s", "cores": 1, "kind": "oracle",
            "sample": f"whole workload, median of {reps} runs: numpy map of both patterns + sort-merge join, "
                      f"{n} rows in {el:.2f} s on one thread (host has {cores} cores available)",
            "host_cores": cores,
            "allcore": {"value": nh / eh, "unit": "rows/s", "cores": min(threads, cores), "kind": "oracle",
                        "sample": f"whole workload, median of {reps} runs: numpy map + the oracle's C hash join "
                                  f"(OpenMP, {min(threads, cores)} threads) + output columns, {nh} rows in {eh:.2f} s"}}, n


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

        def one():
            t = sess.join(L, R, 0)
            rows = int(t.nrows)
            sess.free(t)
            return rows

        ts, rows, prof = timed_reps(one, reps=reps, prof_ctx=sess.ctx)
        el = median(ts)
        st = sess.stats()
        phases = phase_table(prof)
    return {"workload": f"join of two {n}-row tables, uniform keys over 2^{key_bits}, one value column each, "
                       "merge join, semi-join and exact pre-count off", "records": 2 * n, "rows": rows, "radix_bits": st.radix_bits,
            "passes": st.passes, "ms_per_join": round(el * 1e3, 3), "timing": "median of 5 cold repetitions",
            "phases": phases}


def run_cfg3(reps=5):
    """The four-pattern query over 200M triples (three joins; the last one
    shuffles), median of ``reps`` cold repetitions of ``mapsq_query``."""
    import torch

    from paper_1702_03484_amd import binding as B
    from paper_1702_03484_amd.engine import MapSQ
    from synth import query_cfg3, store_cfg3

    sel = json.load(open(os.path.join(ROOT, "synth", "cfg3_draw.json")))
    log("[cfg3] generating the 200M-triple store")
    t0 = time.perf_counter()
    w = store_cfg3(seed=sel["seed"])
    pats = [tuple(p) for p in query_cfg3(w, sel["draw"])]
    log(f"[cfg3] generated in {time.perf_counter() - t0:.1f} s; query {pats}")
    with MapSQ(arena_bytes=48 << 30) as sess:
        info = sess.load(w.s, w.p, w.o)
        del w
        torch.cuda.synchronize()

        def one():
            t = sess.query(pats)
            rows = int(t.nrows)
            sess.free(t)
            return rows

        ts, rows, prof = timed_reps(one, reps=reps, prof_ctx=sess.ctx)
        st = sess.stats()
        plan_sizes = sess.last_plan()
        # the same query planned on exact join sizes counted on the GPU
        sess.set_planner(True)
        try:
            tx, rows_x, _ = timed_reps(one, reps=reps)
            plan_exact = sess.last_plan()
        finally:
            sess.set_planner(False)
        assert rows_x == rows
    el = median(ts)
    log(f"[cfg3] {rows} rows in {el * 1e3:.3f} ms (median); exact-size plan {median(tx) * 1e3:.3f} ms")
    return {"workload": f"?x p1 ?y . ?x p2 ?z . ?x p3 c . ?w p4 ?y over {info.n_triples} int32 triples "
                        "(64 predicates Zipf 1.0, s uniform and o Zipf 1.2 over 50M entities)",
            "patterns": [list(p) for p in pats], "rows": rows, "ms_per_query": round(el * 1e3, 3),
            "rows_per_s": rows / el, "timing": f"median of {reps} cold repetitions",
            "last_join": {"path": int(st.path), "records_sorted": int(st.sorted_records), "radix_bits": int(st.radix_bits),
                          "passes": int(st.passes), "segments": int(st.segments)},
            "phases": phase_table(prof),
            "plans": {"step": "(pattern, key variable, rows, join sizes counted)",
                      "pattern_sizes": plan_sizes, "exact_join_sizes": plan_exact,
                      "ms_exact_join_sizes": round(median(tx) * 1e3, 3)}}


def run_dict(n_terms=10_000_000, n_vocab=2_000_000, reps=5):
    """Dictionary encoding of an RDF-shaped term stream resident in HBM
    (Zipf(1.1) frequencies over a 2M-term vocabulary of IRIs and literals):
    one encode of the whole batch into a fresh dictionary per repetition,
    and the decode of every identifier back to text; median of ``reps``
    cold repetitions.  Beside it, the oracle's dictionary (a Python dict)
    on the first 1M terms."""
    import numpy as np
    import torch

    from oracle import dictionary as D
    from paper_1702_03484_amd.engine import MapSQ
    from synth import rdf_terms

    log(f"[dict] drawing {n_terms} terms over {n_vocab}")
    data, off, _ = rdf_terms(1, n_terms, n_vocab)
    text = int(off[-1])
    with MapSQ(arena_bytes=16 << 30) as sess:
        dd = torch.from_numpy(data).cuda()
        do = torch.from_numpy(off).cuda()
        state = {}

        def enc():
            sess.dict_create(n_terms, 2 * text)
            ids, new = sess.dict_encode(dd, do)
            state["ids"], state["new"] = ids, new
            return new

        te, _, _ = timed_reps(enc, reps=reps)
        ids = state["ids"]

        def dec():
            b, o = sess.dict_decode(ids)
            state["dec"] = (b, o)
            return int(o[-1])

        td, back, _ = timed_reps(dec, reps=reps)
        assert back == text and torch.equal(state["dec"][0], dd) and torch.equal(state["dec"][1], do)
        distinct = state["new"]
    sample = 1_000_000
    terms = D.split_terms(data[:int(off[sample])].tobytes(), off[:sample + 1])
    t0 = time.perf_counter()
    D.encode(terms)
    cpu_s = time.perf_counter() - t0
    e, d = median(te), median(td)
    log(f"[dict] encode {n_terms / e / 1e6:.0f} M terms/s ({text / e / 1e9:.1f} GB/s of text), "
        f"decode {n_terms / d / 1e6:.0f} M terms/s; oracle {sample / cpu_s / 1e6:.2f} M terms/s")
    return {"workload": f"{n_terms} RDF-shaped terms (IRIs and literals), Zipf 1.1 over {n_vocab}, "
                        f"{text} bytes of text, device buffers",
            "distinct": distinct, "encode_ms": round(e * 1e3, 3), "encode_terms_per_s": n_terms / e,
            "encode_text_gbs": round(text / e / 1e9, 1), "decode_ms": round(d * 1e3, 3),
            "decode_terms_per_s": n_terms / d, "decode_text_gbs": round(text / d / 1e9, 1),
            "timing": f"median of {reps} cold repetitions; encode into a fresh dictionary each time, "
                      "decode includes its size read-back",
            "cpu_oracle": {"terms_per_s": sample / cpu_s, "sample": f"first {sample} terms, Python dict, 1 thread"}}


def run_cfg2_sort(sess, w, reps=5):
    """The headline join with the merge join and the semi-join reduction
    turned off: every record of both partial-match tables goes through the
    radix sort (Algorithm 1's Sort), then count, scan and materialisation."""
    from paper_1702_03484_amd import binding as B

    sess.set_join_options(semijoin=1, merge=1)
    try:
        def one():
            t = sess.query(w.patterns)
            rows = int(t.nrows)
            sess.free(t)
            return rows

        ts, rows, prof = timed_reps(one, reps=reps, prof_ctx=sess.ctx)
        st = sess.stats()
    finally:
        sess.set_join_options()
    el = median(ts)
    assert st.path == B.MAPSQ_PATH_SORT
    return {"workload": "the headline join with every record radix-sorted (merge join and semi-join off)",
            "rows": rows, "ms_per_query": round(el * 1e3, 3), "rows_per_s": rows / el,
            "timing": f"median of {reps} cold repetitions", "records_sorted": int(st.sorted_records),
            "radix_bits": int(st.radix_bits), "passes": int(st.passes), "phases": phase_table(prof)}


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


def run_cfg5(n_triples=500_000_000, n_queries=600, warm=100, loads=(0.25, 0.5, 1.0, 2.0, 4.0), seed=1,
             row_cap=1 << 26, stream=4000):
    """Serving over the resident store: plain one-query-at-a-time vs
    continuous batching, saturated and with Poisson arrivals at multiples of
    the plain form's saturated rate; p50/p99 latency and queries/s.

    The query mix is capped like the other workloads: the seeded random-walk
    stream is drawn, each query is answered once by ``mapsq_query``, and a
    query whose exact result has more than ``row_cap`` rows (or that cannot
    fit the arena) is redrawn, i.e. skipped for the next one in the stream;
    the skipped fraction is reported.  Saturated rates count every query
    processed (completed or refused) per second of wall time."""
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
    drawn = serving_cfg5(w, stream, seed=seed)
    sess = MapSQ(arena_bytes=160 << 30)
    info = sess.load(w.s, w.p, w.o)
    del w
    torch.cuda.synchronize()
    log(f"[cfg5] store resident: {info.n_triples} triples, {info.n_predicates} predicates")
    qs, over, examined, sizes = [], 0, 0, []
    for q in drawn:
        examined += 1
        try:
            t = B.mapsq_query(sess.ctx, q)
            n = int(t.nrows)
            B.mapsq_table_free(sess.ctx, t)
        except B.MapSQError:
            n = None
        if n is None or n > row_cap:
            over += 1
            continue
        qs.append(q)
        sizes.append(n)
        if len(qs) == warm + n_queries:
            break
    torch.cuda.synchronize()
    log(f"[cfg5] mix: {len(qs)} queries within {row_cap} rows; {over} of the first {examined} drawn were over")
    warm_q, qs = qs[:warm], qs[warm:]
    serving.run_plain(sess, warm_q, np.zeros(len(warm_q)))
    serving.run_continuous(sess, warm_q, np.zeros(len(warm_q)))
    sat_plain, lat_p, st_p = serving.run_plain(sess, qs, np.zeros(len(qs)))
    sat_cont, _, st_c = serving.run_continuous(sess, qs, np.zeros(len(qs)))
    # the same queries complete, and the same fail with the same status, in
    # both modes (serving reports every memory failure as TOO_LARGE)
    mem = np.where(st_p == B.MAPSQ_ERR_CAPACITY, B.MAPSQ_ERR_TOO_LARGE, st_p)
    sat_cont["same_outcomes_as_plain"] = bool((st_c == mem).all())
    log(f"[cfg5] saturated: plain {sat_plain['processed_qps']:.0f} q/s, continuous {sat_cont['processed_qps']:.0f} q/s")
    # the plain form with each query planned on exact join sizes counted on
    # the GPU (serving plans on pattern sizes): plans that differ, and rate
    plans = []
    for q in qs:
        t = B.mapsq_query(sess.ctx, q)
        B.mapsq_table_free(sess.ctx, t)
        plans.append(B.mapsq_last_plan(sess.ctx))
    sess.set_planner(True)
    try:
        sat_exact, _, st_x = serving.run_plain(sess, qs, np.zeros(len(qs)))
        differ, smaller = 0, 0
        for q, ps in zip(qs, plans):
            t = B.mapsq_query(sess.ctx, q)
            B.mapsq_table_free(sess.ctx, t)
            px = B.mapsq_last_plan(sess.ctx)
            if [s_[:2] for s_ in px] != [s_[:2] for s_ in ps]:
                differ += 1
                if max([s_[2] for s_ in px[1:-1]] or [0]) < max([s_[2] for s_ in ps[1:-1]] or [0]):
                    smaller += 1
    finally:
        sess.set_planner(False)
    sat_exact["same_outcomes_as_plain"] = bool((st_x == st_p).all())
    planner = {"plain_exact_join_sizes": sat_exact, "plans_differ": differ,
               "smaller_largest_intermediate": smaller, "queries": len(qs)}
    log(f"[cfg5] exact-size plans: {differ} of {len(qs)} differ ({smaller} with a smaller largest intermediate); "
        f"plain {sat_exact['processed_qps']:.0f} q/s")
    rows = []
    for f in loads:
        qps = f * sat_plain["processed_qps"]
        arr = serving.poisson_arrivals(seed, len(qs), qps)
        p, _, _ = serving.run_plain(sess, qs, arr)
        c, _, _ = serving.run_continuous(sess, qs, arr)
        rows.append({"load": f, "offered_qps": qps, "plain": p, "continuous": c})
        log(f"[cfg5] load {f}: plain p50 {p['p50_ms']:.2f} ms p99 {p['p99_ms']:.2f} ms {p['qps']:.0f} q/s "
            f"(saturated {p['saturated']}); continuous p50 {c['p50_ms']:.2f} ms p99 {c['p99_ms']:.2f} ms "
            f"{c['qps']:.0f} q/s (saturated {c['saturated']})")
    sess.close()
    return {"workload": f"{info.n_triples}-triple resident store (128 predicates Zipf 1.0, entities Zipf 1.1 over "
                        f"{n_triples // 5}), {len(qs)} random-walk queries of 1-5 patterns with 0-2 constants each, "
                        f"results capped at {row_cap} rows",
            "mix": {"examined": examined, "over_cap_or_refused": over, "redraw_rate": over / max(1, examined),
                    "rows_p50": float(np.percentile(sizes, 50)) if sizes else None,
                    "rows_max": int(max(sizes)) if sizes else None},
            "saturated_plain": sat_plain, "saturated_continuous": sat_cont, "planner": planner, "poisson": rows}


def main():
    global COLD
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--n", type=int, default=50_000_000, help="triples (default: the full workload)")
    ap.add_argument("--no-cfg3", action="store_true", help="leave out the 200M-triple four-pattern query")
    ap.add_argument("--cfg3-only", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="leave out the 512-subquery batched-vs-plain measurement")
    ap.add_argument("--cfg4-only", action="store_true")
    ap.add_argument("--no-serving", action="store_true", help="leave out the serving measurement (500M-triple store)")
    ap.add_argument("--cfg5-only", action="store_true")
    ap.add_argument("--shuffle-only", action="store_true", help="only the 16M + 16M-record shuffle join")
    ap.add_argument("--dict-only", action="store_true", help="only the term dictionary encode/decode")
    ap.add_argument("--no-dict", action="store_true", help="leave out the term dictionary measurement")
    ap.add_argument("--warm", action="store_true", help="no cache flush before timed repetitions")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (--gpus {args.gpus} requested): the join runs on a single "
              "MI355X and there is no multi-GPU path", file=sys.stderr)
        sys.exit(2)
    COLD = not args.warm
    if args.copy_calibration:
        copy_calibration()
        return
    if args.cfg3_only:
        print(json.dumps(run_cfg3()), flush=True)
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
    if args.dict_only:
        print(json.dumps(run_dict()), flush=True)
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
    left_rows = int((w.p == w.patterns[0][1]).sum())

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

    def step():
        t = sess.query(w.patterns)
        rows = int(t.nrows)
        sess.free(t)
        return rows

    # the headline: --steps cold repetitions after --warmup untimed ones
    ts, rows, prof = timed_reps(step, reps=args.steps, warm=args.warmup, prof_ctx=sess.ctx)
    el = sum(ts)
    log(f"[bench] {rows} rows per step; timed {args.steps} steps in {el:.4f} s (median {median(ts) * 1e3:.3f} ms)")
    phases = phase_table(prof)
    mat = phases["materialize"]
    achieved = mat["gbs"]
    traffic = traffic_from_profile()
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": "materialize_kernel", "avg_ms": mat["avg_ms"],
                "bytes_per_launch": mat["bytes_per_launch"]}

    # the same join with every record through the radix sort
    log("[bench] the same join forced through the radix sort")
    sort_leg = run_cfg2_sort(sess, w) if full else None
    # Map of a pattern with only a constant object over the whole store: a
    # scan of the raw columns with ballot compaction (the paper's Map)
    c = w.patterns[1][2]

    def scan():
        t = sess.map((var(0), var(1), c))
        n = int(t.nrows)
        sess.free(t)
        return n

    _, _, mprof = timed_reps(scan, prof_ctx=sess.ctx)
    mp = phase_table(mprof).get("map")
    if mp:
        mp["pattern"] = "?s ?p c over the 50M-triple store (variable predicate: full scan + compaction)"
        mp["timing"] = "average of 5 cold repetitions"

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on the same workload")
        cpu, cpu_rows = cpu_baseline(w)
        if cpu_rows != rows:
            raise SystemExit(f"oracle row count {cpu_rows} != GPU row count {rows}")
        log(f"[bench] oracle: {cpu['value']:.3e} rows/s (1 thread), {cpu['allcore']['value']:.3e} rows/s "
            f"({cpu['allcore']['cores']} threads)")

    sess.close()
    del sess, w
    torch.cuda.empty_cache()

    def guarded(fn, name):
        try:
            return fn()
        except Exception as e:  # the main line must still come out
            log(f"[bench] {name} failed: {e!r}")
            return {"error": repr(e)}
        finally:
            torch.cuda.empty_cache()

    cfg3 = None if (args.no_cfg3 or not full) else guarded(run_cfg3, "cfg3 measurement")
    shuffle = guarded(run_shuffle, "shuffle measurement")
    dictionary = None if args.no_dict else guarded(run_dict, "dictionary measurement")
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
                   "triples": info.n_triples, "rows_per_step": rows, "left_rows": left_rows,
                   "index_build_ms": round(index_ms, 2),
                   "timing": "each step cold (2 GiB cache flush before it, outside the clock)" if COLD else "warm"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "phases": phases,
        "cfg2_sort": sort_leg,
        "cfg3": cfg3,
        "map": mp,
        "shuffle": shuffle,
        "dictionary": dictionary,
        "batched": batched,
        "serving": served,
    }
    print(json.dumps(out), flush=True)



if __name__ == "__main__":
    main()
