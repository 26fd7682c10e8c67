"""Seeded cases run through the bounds-checked build (test infrastructure).

``inputs()`` builds the host inputs of every case; ``python
tests/debug_workload.py OUT_DIR`` (run with MAPSQ_LIB=debug) loads them on
the GPU, runs each case through the library and saves every result table
to OUT_DIR/<case>.npz (its variables and columns).  The calling test
compares them with the oracle and checks that the run printed no bounds
report.
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from synth import random_store, random_table, var  # noqa: E402


def _pair(seed, nl, nr, card, vl, vr):
    keys = np.arange(card, dtype=np.int64) * 3 + 2
    lc = random_table(seed, nl, card, vl, key_ids=keys)
    rc = random_table(seed + 1, nr, card, vr, key_ids=keys)
    return ([0] + [10 + k for k in range(vl)], lc), ([0] + [20 + k for k in range(vr)], rc)


def inputs():
    """{case: description}: joins are ((lvars, lcols), (rvars, rcols), key,
    options); 'store' cases hold the triples and the patterns."""
    c = {}
    c["shuffle"] = _pair(301, 60_000, 40_000, 3_000, 2, 1) + (0, {})
    c["semijoin"] = _pair(303, 200_000, 3_000, 100_000, 1, 2) + (0, {"semijoin": 2})
    (lv, lc), (rv, rc) = _pair(305, 50_000, 30_000, 4_000, 1, 1)
    ol, orr = np.argsort(lc[0], kind="stable"), np.argsort(rc[0], kind="stable")
    c["merge"] = ((lv, [x[ol] for x in lc]), (rv, [x[orr] for x in rc]), 0, {"sorted": True})
    (lv, lc), (rv, rc) = _pair(307, 40_000, 30_000, 2_000, 2, 1)
    lc[1] = lc[1] % 50  # the second shared variable over few values, so pairs agree on it often
    rv = [0, 10]
    rc[1] = lc[1][np.random.default_rng(307).integers(0, len(lc[1]), len(rc[1]))]
    c["composite"] = ((lv, lc), (rv, rc), 0, {})
    c["batch"] = [_pair(400 + 2 * i, 2_000 + 9_000 * i, 30_000 - 3_000 * i, 300 + 700 * i, i % 3, (i + 2) % 3)
                  for i in range(8)]
    w = random_store(41, 300_000, 30_000, 6)
    p0, p1, p2 = 30_000, 30_001, 30_002
    c["store"] = (w.s, w.p, w.o)
    c["map"] = (var(0), var(1), int(w.o[17]))
    c["query"] = [(var(0), p0, var(1)), (var(1), p1, var(2)), (var(0), p2, var(3))]
    return c


def main(out_dir):
    import torch

    from paper_1702_03484_amd.engine import MapSQ

    c = inputs()
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).cuda()  # noqa: E731

    def save(name, sess, t):
        cols = sess.to_numpy(t)
        np.savez(os.path.join(out_dir, name + ".npz"), vars=np.array(list(t.vars)), *cols)
        sess.free(t)

    with MapSQ(arena_bytes=4 << 30, tuning=None) as sess:
        for name in ("shuffle", "semijoin", "merge", "composite"):
            (lv, lc), (rv, rc), key, opt = c[name]
            so = 1 if opt.get("sorted") else 0
            L = sess.table(lv, [dev(x) for x in lc], key_max=int(max(lc[0].max(), rc[0].max())), sorted_col=so)
            R = sess.table(rv, [dev(x) for x in rc], key_max=int(max(lc[0].max(), rc[0].max())), sorted_col=so)
            sess.set_join_options(semijoin=opt.get("semijoin", 0))
            save(name, sess, sess.join(L, R, key))
            sess.set_join_options()
        joins = []
        for (lv, lc), (rv, rc) in c["batch"]:
            km = int(max(lc[0].max(), rc[0].max()))
            joins.append((sess.table(lv, [dev(x) for x in lc], key_max=km),
                          sess.table(rv, [dev(x) for x in rc], key_max=km), 0))
        for i, t in enumerate(sess.join_batch(joins)):
            save(f"batch{i}", sess, t)
        sess.load(*c["store"])
        save("map", sess, sess.map(c["map"]))
        save("query", sess, sess.query(c["query"]))
    print("workload done", flush=True)


if __name__ == "__main__":
    main(sys.argv[1])
