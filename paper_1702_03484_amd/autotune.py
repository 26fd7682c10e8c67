"""Autotuner of the radix sort's digit width and tile size.

For each (key bits, record count) class it times every candidate
(digit width 4..11, 8 or 16 keys per thread) on synthetic keys of that
shape, using the library's own HIP-event phase timing (the sort phase of a
join), records the fastest in the library with mapsq_tune_record, and keeps
the table in a JSON cache.  Every candidate sorts to the same order, so a
choice changes speed only.
"""
from __future__ import annotations

import json
import os

import torch

from . import binding as B

CANDIDATES = [(rb, kpt) for rb in range(4, 12) for kpt in (8, 16)]


def _bitlen(v: int) -> int:
    return int(v).bit_length()


def tune_class(sess, key_bits: int, nrec: int, reps: int = 3, seed: int = 0):
    """Best (rb, kpt) and the sort-phase times of every candidate."""
    g = torch.Generator(device="cuda").manual_seed(seed)
    hi = (1 << key_bits) if key_bits < 31 else (1 << 31) - 1
    nl = nrec * 3 // 4
    lk = torch.randint(0, hi, (nl,), generator=g, device="cuda", dtype=torch.int64).to(torch.int32)
    # a small right side with few matches keeps the materialisation out of the timing
    rk = torch.full((max(1, nrec - nl),), hi - 1, device="cuda", dtype=torch.int32)
    L = sess.table([0], [lk], key_max=hi - 1)
    R = sess.table([0], [rk], key_max=hi - 1)
    # every record through the shuffle: no semi-join reduction, no merge join
    sess.set_join_options(semijoin=1, merge=1)
    times = {}
    for rb, kpt in CANDIDATES:
        sess.set_tuning(rb, kpt)
        t = sess.join(L, R, 0)
        sess.free(t)
        B.mapsq_profile_enable(sess.ctx, True)
        for _ in range(reps):
            t = sess.join(L, R, 0)
            sess.free(t)
        prof = B.mapsq_profile_read(sess.ctx)
        times[(rb, kpt)] = prof.ms[1] / max(1, prof.launches[1])
    sess.set_tuning(0, 0)
    sess.set_join_options(0, 0)
    B.mapsq_profile_enable(sess.ctx, False)
    best = min(times, key=times.get)
    return best, times


def autotune(sess, classes, cache_path=None):
    """classes: iterable of (key_bits, record count).  Records the choices in
    the library and, if cache_path is given, merges them into that JSON."""
    table = load_cache(cache_path) if cache_path else {}
    for key_bits, nrec in classes:
        (rb, kpt), times = tune_class(sess, key_bits, nrec)
        lg = _bitlen(nrec)
        B.mapsq_tune_record(sess.ctx, key_bits, lg, rb, kpt)
        table[f"{key_bits}:{lg}"] = {"radix_bits": rb, "keys_per_thread": kpt,
                                     "sort_ms": {f"{a}/{b}": round(v, 4) for (a, b), v in times.items()}}
    if cache_path:
        with open(cache_path, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
    return table


def load_cache(path):
    if not path or not os.path.exists(path):
        return {}
    return json.load(open(path))


def install(sess, path):
    """Record a cached table in the library (no timing)."""
    for k, v in load_cache(path).items():
        kb, lg = (int(x) for x in k.split(":"))
        B.mapsq_tune_record(sess.ctx, kb, lg, v["radix_bits"], v["keys_per_thread"])


DEFAULT_TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning.json")
DEFAULT_CLASSES = [(kb, 3 << (lg - 2)) for kb in (20, 24, 26, 31) for lg in range(11, 26)]


def main(argv=None):
    import argparse

    from .engine import MapSQ

    ap = argparse.ArgumentParser(description="time every (digit width, keys per thread) per size class")
    ap.add_argument("--out", default=DEFAULT_TABLE)
    ap.add_argument("--arena-gb", type=float, default=16.0)
    args = ap.parse_args(argv)
    with MapSQ(arena_bytes=int(args.arena_gb * (1 << 30)), tuning=None) as sess:
        for kb, n in DEFAULT_CLASSES:
            autotune(sess, [(kb, n)], cache_path=args.out)
            e = load_cache(args.out)[f"{kb}:{_bitlen(n)}"]
            print(f"key bits {kb:2d}  records {n:9d}  ->  {e['radix_bits']} bits x {e['keys_per_thread']} keys/thread",
                  flush=True)


if __name__ == "__main__":
    main()
