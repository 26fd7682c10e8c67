"""Summaries of rocprofv3 output (CSV) for the records kept under profiles/.

  python -m paper_1702_03484_amd.profile_summary stats DIR
      per-kernel calls / average / total duration from *_kernel_stats.csv
  python -m paper_1702_03484_amd.profile_summary pmc DIR COUNTER [REGEX [FIRST]]
      mean value of COUNTER per dispatch of the kernels matching REGEX, from
      *_counter_collection.csv (with FIRST: over the first FIRST matching
      dispatches in dispatch order only, e.g. one leg of a run whose later
      legs launch the same kernel)
  python -m paper_1702_03484_amd.profile_summary traffic K_FETCH K_WRITE COPY_FETCH COPY_WRITE COPY_BYTES OUT
      HBM bytes per launch of a kernel: FETCH_SIZE and WRITE_SIZE (KiB per
      dispatch, from two ``pmc`` summaries) each scaled by what the same
      counter reads for a plain copy of COPY_BYTES, written as JSON together
      with the SHA-256 of the device sources the counters were taken on
"""
from __future__ import annotations

import csv
import glob
import hashlib
import json
import os
import re
import sys

HERE = os.path.dirname(os.path.abspath(__file__))


def kernel_sources():
    """Every device source of the library (kernels and the headers they include)."""
    d = os.path.join(HERE, "csrc")
    return sorted(os.path.join(d, f) for f in os.listdir(d) if f.endswith((".hip", ".h")))


def kernel_sha() -> str:
    """SHA-256 over every device source: a counter record taken on other
    kernel code no longer matches."""
    h = hashlib.sha256()
    for p in kernel_sources():
        h.update(os.path.basename(p).encode())
        h.update(open(p, "rb").read())
    return h.hexdigest()


def _one(d, pattern):
    files = sorted(glob.glob(os.path.join(d, "**", pattern), recursive=True))
    if not files:
        raise SystemExit(f"no {pattern} under {d}")
    return files[0]


def stats(d):
    rows = list(csv.DictReader(open(_one(d, "*kernel_stats.csv"))))
    out = []
    for r in rows:
        out.append({"kernel": r["Name"], "calls": int(r["Calls"]), "avg_us": float(r["AverageNs"]) / 1e3,
                    "total_ms": float(r["TotalDurationNs"]) / 1e6, "pct": float(r["Percentage"])})
    return out


def pmc(d, counter, regex=".*", first=None):
    rows = list(csv.DictReader(open(_one(d, "*counter_collection.csv"))))
    rx = re.compile(regex)
    sel = [r for r in rows if r.get("Counter_Name") == counter and rx.search(r.get("Kernel_Name", ""))]
    sel.sort(key=lambda r: int(r.get("Dispatch_Id", 0)))
    if first is not None:
        sel = sel[:first]
    per = {}
    for r in sel:
        per.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
    return {k: {"dispatches": len(v), "mean": sum(v) / len(v)} for k, v in per.items()}


def main(argv):
    cmd = argv[0]
    if cmd == "stats":
        for r in stats(argv[1]):
            print(f"{r['kernel'][:100]:100s} {r['calls']:6d} {r['avg_us']:12.1f} us {r['total_ms']:10.3f} ms {r['pct']:6.2f}%")
    elif cmd == "pmc":
        print(json.dumps(pmc(argv[1], argv[2], argv[3] if len(argv) > 3 else ".*",
                             int(argv[4]) if len(argv) > 4 else None), indent=1))
    elif cmd == "traffic":
        mf, mw, cf, cw = (json.load(open(p)) for p in argv[1:5])
        copy_bytes = float(argv[5])

        def mean(d):
            v = list(d.values())
            return sum(x["mean"] * x["dispatches"] for x in v) / sum(x["dispatches"] for x in v)

        sf = copy_bytes / (mean(cf) * 1024.0)
        sw = copy_bytes / (mean(cw) * 1024.0)
        out = {"fetch_kib_per_launch": mean(mf), "write_kib_per_launch": mean(mw),
               "copy_fetch_scale": sf, "copy_write_scale": sw,
               "hbm_bytes_per_launch": mean(mf) * 1024.0 * sf + mean(mw) * 1024.0 * sw,
               "kernel_source_sha256": kernel_sha()}
        json.dump(out, open(argv[6], "w"), indent=1)
        print(json.dumps(out, indent=1))
    else:
        raise SystemExit(__doc__)


if __name__ == "__main__":
    main(sys.argv[1:])
