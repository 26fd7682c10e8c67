"""Autotuner of the join's launch shapes.

Sort: for each (key bits, record count) class it times every candidate
digit width (4..11) and tile size (8 or 16 keys per thread) on synthetic keys
of that shape.  Materialisation: for each output size class it times the
grid cap of the materialisation launch (its waves stride over the work
items).  Times come from the library's own HIP-event phase timing; the
fastest choice of each class is recorded in the library (mapsq_tune_record,
mapsq_tune_record_mat) and kept in a JSON table.  Every candidate gives the
same rows in the same order, so a choice changes speed only.

The table carries the SHA-256 of the device sources it was measured on;
``install`` refuses a table taken on other kernel code (the library then
uses its built-in choices).
"""
from __future__ import annotations

import json
import os
import sys

import torch

from . import binding as B
from .profile_summary import kernel_sha

SORT_CANDIDATES = [(rb, kpt) for rb in range(4, 12) for kpt in (8, 16)]
MAT_CANDIDATES = [1024, 2048, 4096, 8192, 16384]


def _bitlen(v: int) -> int:
    return int(v).bit_length()


def _phase_ms(sess, run, phase: int, reps: int) -> float:
    run()
    B.mapsq_profile_enable(sess.ctx, True)
    for _ in range(reps):
        run()
    prof = B.mapsq_profile_read(sess.ctx)
    B.mapsq_profile_enable(sess.ctx, False)
    return prof.ms[phase] / max(1, prof.launches[phase])


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

    def one():
        sess.free(sess.join(L, R, 0))

    times = {}
    try:
        for rb, kpt in SORT_CANDIDATES:
            sess.set_tuning(rb, kpt)
            times[(rb, kpt)] = _phase_ms(sess, one, 1, reps)
    finally:
        sess.set_tuning(0, 0)
        sess.set_join_options()
    best = min(times, key=times.get)
    return best, times


def tune_mat_class(sess, rows: int, reps: int = 3, seed: int = 0):
    """Best materialisation grid cap for an output of about `rows` rows: a
    join whose keys each pair 64 LEFT with 64 RIGHT rows (one value column
    per side), timed for every candidate cap."""
    g = torch.Generator(device="cuda").manual_seed(seed)
    nkeys = max(1, rows // 4096)
    lk = torch.arange(nkeys, device="cuda", dtype=torch.int32).repeat_interleave(64)
    lv = torch.randint(0, 1 << 30, (lk.numel(),), generator=g, device="cuda", dtype=torch.int64).to(torch.int32)
    rv = torch.randint(0, 1 << 30, (lk.numel(),), generator=g, device="cuda", dtype=torch.int64).to(torch.int32)
    L = sess.table([0, 1], [lk, lv], key_max=nkeys, sorted_col=1)
    R = sess.table([0, 2], [lk.clone(), rv], key_max=nkeys, sorted_col=1)

    def one():
        sess.free(sess.join(L, R, 0))

    times = {}
    try:
        for cap in MAT_CANDIDATES:
            B.mapsq_set_mat_tuning(sess.ctx, cap)
            times[cap] = _phase_ms(sess, one, 3, reps)
    finally:
        B.mapsq_set_mat_tuning(sess.ctx, 0)
    best = min(times, key=times.get)
    return best, times


def load_cache(path):
    if not path or not os.path.exists(path):
        return {}
    return json.load(open(path))


def _fresh(table) -> bool:
    return table.get("kernel_source_sha256") == kernel_sha()


def install(sess, path) -> bool:
    """Record a cached table in the library (no timing).  A table measured
    on other kernel sources is refused (False): its choices may no longer
    be the fastest, and the library's built-in choices apply."""
    table = load_cache(path)
    if not table:
        return False
    if not _fresh(table):
        print(f"autotune: {path} was measured on other kernel sources; not installed", file=sys.stderr)
        return False
    for k, v in table.get("sort", {}).items():
        kb, lg = (int(x) for x in k.split(":"))
        B.mapsq_tune_record(sess.ctx, kb, lg, v["radix_bits"], v["keys_per_thread"])
    for k, v in table.get("materialize", {}).items():
        B.mapsq_tune_record_mat(sess.ctx, int(k), v["max_blocks"])
    return True


DEFAULT_TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning.json")
DEFAULT_CLASSES = [(kb, 3 << (lg - 2)) for kb in (20, 24, 26, 31) for lg in range(11, 26)]
DEFAULT_MAT_CLASSES = [1 << lg for lg in range(16, 29, 2)]


def autotune(sess, classes, mat_classes=(), cache_path=None):
    """classes: (key_bits, record count) pairs; mat_classes: output row
    counts.  Records the choices in the library and, with cache_path,
    writes the table (stamped with the device-source hash)."""
    table = load_cache(cache_path) if cache_path else {}
    if not _fresh(table):
        table = {}
    table["kernel_source_sha256"] = kernel_sha()
    sort = table.setdefault("sort", {})
    for key_bits, nrec in classes:
        (rb, kpt), times = tune_class(sess, key_bits, nrec)
        lg = _bitlen(nrec)
        B.mapsq_tune_record(sess.ctx, key_bits, lg, rb, kpt)
        sort[f"{key_bits}:{lg}"] = {"radix_bits": rb, "keys_per_thread": kpt,
                                    "sort_ms": {f"{a}/{b}": round(v, 4) for (a, b), v in times.items()}}
    mat = table.setdefault("materialize", {})
    for rows in mat_classes:
        cap, times = tune_mat_class(sess, rows)
        lg = _bitlen(rows)
        B.mapsq_tune_record_mat(sess.ctx, lg, cap)
        mat[str(lg)] = {"max_blocks": cap, "materialize_ms": {str(c): round(v, 4) for c, v in times.items()}}
    if cache_path:
        with open(cache_path, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
    return table


def main(argv=None):
    import argparse

    from .engine import MapSQ

    ap = argparse.ArgumentParser(description="time the sort's digit widths and tiles, and the "
                                             "materialisation grid, per size class")
    ap.add_argument("--out", default=DEFAULT_TABLE)
    ap.add_argument("--arena-gb", type=float, default=16.0)
    args = ap.parse_args(argv)
    with MapSQ(arena_bytes=int(args.arena_gb * (1 << 30)), tuning=None) as sess:
        for kb, n in DEFAULT_CLASSES:
            autotune(sess, [(kb, n)], cache_path=args.out)
            e = load_cache(args.out)["sort"][f"{kb}:{_bitlen(n)}"]
            print(f"sort: key bits {kb:2d}  records {n:9d}  ->  {e['radix_bits']} bits x "
                  f"{e['keys_per_thread']} keys/thread", flush=True)
        for rows in DEFAULT_MAT_CLASSES:
            autotune(sess, [], [rows], cache_path=args.out)
            e = load_cache(args.out)["materialize"][str(_bitlen(rows))]
            print(f"materialize: rows {rows:11d}  ->  {e['max_blocks']} blocks", flush=True)


if __name__ == "__main__":
    main()
