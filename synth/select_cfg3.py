"""Pick the config-3 query draw (run offline; writes synth/cfg3_draw.json).

Tries the seeded draws of ``query_cfg3`` in order and keeps the first whose
exact output size, computed by the oracle, lies in [20M, 400M] rows.  Only
the oracle computes sizes here.  Usage: python -m synth.select_cfg3
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

import oracle  # noqa: E402
from synth.gen import query_cfg3, store_cfg3  # noqa: E402

LO, HI = 20_000_000, 400_000_000


def main(max_draws: int = 200):
    w = store_cfg3()
    by_pred = {}
    for d in range(max_draws):
        pats = query_cfg3(w, d)
        preds = [p for _, p, _ in pats]
        for p in preds:
            if p not in by_pred:
                m = w.p == p
                by_pred[p] = (w.s[m], w.o[m])

        def sub(ps):
            ss = np.concatenate([by_pred[p][0] for p in ps])
            oo = np.concatenate([by_pred[p][1] for p in ps])
            pp = np.concatenate([np.full(by_pred[p][0].size, p, np.int32) for p in ps])
            return ss, pp, oo

        s3, p3, o3 = sub(sorted(set(preds[:3])))
        j2 = oracle.query(s3, p3, o3, pats[:3])
        s4, p4, o4 = sub([preds[3]])
        t4 = oracle.match_pattern(s4, p4, o4, pats[3])
        n3 = oracle.join_cardinality(j2, t4, 1)
        print(f"draw {d}: |J2| = {j2.n}, |P4| = {t4.n}, |J3| = {n3}", flush=True)
        if LO <= n3 <= HI:
            out = {"seed": w.meta["seed"], "draw": d, "patterns": pats, "j3_rows": int(n3),
                   "note": "first draw of query_cfg3 with an oracle-computed output in [20M, 400M] rows"}
            json.dump(out, open(os.path.join(HERE, "cfg3_draw.json"), "w"), indent=1)
            print(json.dumps(out))
            return out
    raise SystemExit("no draw in range")


if __name__ == "__main__":
    main()
