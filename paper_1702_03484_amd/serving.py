"""Load generators of the serving API: Poisson arrivals, latency accounting.

``run_continuous`` drives mapsq_submit / mapsq_serve_step / mapsq_poll_next
(continuous batching inside the library); ``run_plain`` answers the same
arrivals one query at a time with mapsq_query.  Both only marshal calls and
record host clocks; every query runs in the library's HIP kernels.
"""
from __future__ import annotations

import time

import numpy as np
import torch

from . import binding as B


def poisson_arrivals(seed: int, n: int, qps: float) -> np.ndarray:
    """Arrival times (s) of a Poisson process of rate qps."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([5000, 2, seed])))
    return np.cumsum(rng.exponential(1.0 / qps, n))


def _summary(lat, status, t_end, arrivals):
    """Completed and processed (completed or refused) queries per second of
    the span from the first arrival to the end; ``saturated`` when the run
    ended more than 5% after the last arrival (the queue did not keep up)."""
    ok = status == 0
    done = lat[ok]
    first = arrivals[0] if len(arrivals) else 0.0
    span = max(t_end - first, 1e-9)
    last = arrivals[-1] if len(arrivals) else 0.0
    return {
        "queries": int(len(lat)),
        "completed": int(ok.sum()),
        "rejected": int((status == B.MAPSQ_ERR_TOO_LARGE).sum()),
        "failed": int((~ok & (status != B.MAPSQ_ERR_TOO_LARGE)).sum()),
        "wall_s": float(t_end),
        "arrival_span_s": float(last - first),
        "saturated": bool(t_end - first > 1.05 * (last - first)),
        "qps": float(ok.sum() / span),
        "processed_qps": float(len(lat) / span),
        "p50_ms": float(np.percentile(done, 50) * 1e3) if done.size else None,
        "p99_ms": float(np.percentile(done, 99) * 1e3) if done.size else None,
    }


def run_continuous(sess, queries, arrivals, budget_bytes=0, max_active=0, collect=None, max_idle_rounds=5000,
                   collect_hash=None):
    """Continuous batching: queries are submitted when they arrive; every
    scheduler round admits, maps and runs one batched join step.  Raises
    RuntimeError after ``max_idle_rounds`` rounds in a row in which no query
    ended (the library bounds its own rounds without progress as well).
    ``collect[j]`` gets query j's (vars, host columns); ``collect_hash(j,
    table)`` is called with each result table before it is freed."""
    B.mapsq_serve_config(sess.ctx, budget_bytes, max_active)
    n = len(queries)
    lat = np.full(n, np.nan)
    status = np.zeros(n, dtype=np.int64)
    pending = {}
    i = 0
    rounds = 0
    idle = 0
    t0 = time.perf_counter()
    while i < n or pending:
        now = time.perf_counter() - t0
        while i < n and arrivals[i] <= now:
            pending[B.mapsq_submit(sess.ctx, queries[i])] = i
            i += 1
        if not pending:
            time.sleep(max(0.0, arrivals[i] - now))
            continue
        B.mapsq_serve_step(sess.ctx)
        rounds += 1
        torch.cuda.current_stream(sess.device).synchronize()
        now = time.perf_counter() - t0
        idle += 1
        while True:  # the queries that ended this round, one call each
            tk, st, t = B.mapsq_poll_next(sess.ctx)
            if not tk:
                break
            idle = 0
            j = pending.pop(tk)
            status[j] = st
            lat[j] = now - arrivals[j]
            if t is not None:
                if collect is not None:
                    collect[j] = (list(t.vars), sess.to_numpy(t))
                if collect_hash is not None:
                    collect_hash(j, t)
                B.mapsq_table_free(sess.ctx, t)
        if idle > max_idle_rounds:
            raise RuntimeError(f"serving: no query ended in {max_idle_rounds} rounds ({len(pending)} pending)")
    out = _summary(lat, status, time.perf_counter() - t0, arrivals)
    out["rounds"] = rounds
    return out, lat, status


def run_plain(sess, queries, arrivals, collect=None):
    """One query at a time, in arrival order, with mapsq_query."""
    n = len(queries)
    lat = np.full(n, np.nan)
    status = np.zeros(n, dtype=np.int64)
    t0 = time.perf_counter()
    for j in range(n):
        now = time.perf_counter() - t0
        if arrivals[j] > now:
            time.sleep(arrivals[j] - now)
        try:
            t = B.mapsq_query(sess.ctx, queries[j])
        except B.MapSQError as e:
            status[j] = e.code
            lat[j] = time.perf_counter() - t0 - arrivals[j]
            continue
        torch.cuda.current_stream(sess.device).synchronize()
        lat[j] = time.perf_counter() - t0 - arrivals[j]
        if collect is not None:
            collect[j] = (list(t.vars), sess.to_numpy(t))
        B.mapsq_table_free(sess.ctx, t)
    return _summary(lat, status, time.perf_counter() - t0, arrivals), lat, status
