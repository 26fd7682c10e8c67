"""Full-size parity: the benchmark's 50M-triple join and the 200M-triple
four-pattern query, checked against the oracle by the row count of every
key (exact, all keys) and by the exact rows of sampled keys."""
import json
import os

import numpy as np
import pytest

import oracle
from oracle.core import Table
from synth import query_cfg3, store_cfg2, store_cfg3
from tests.conftest import announce

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


def runs(sorted_keys):
    """(distinct keys, run lengths) of a sorted key column."""
    if sorted_keys.size == 0:
        return sorted_keys, np.zeros(0, np.int64)
    starts = np.concatenate([[0], np.flatnonzero(np.diff(sorted_keys)) + 1])
    lens = np.diff(np.concatenate([starts, [sorted_keys.size]]))
    return sorted_keys[starts], lens.astype(np.int64)


def test_cfg2_full_size(sess):
    w = store_cfg2()
    announce(f"cfg2 full size: 50M triples, query {w.patterns}")
    sess.load(w.s, w.p, w.o)
    t = sess.query(w.patterns)
    x, y = sess.to_numpy(t)  # projection [?x, ?y]; rows grouped by the join key ?y
    assert t.vars == [0, 1]
    P1 = oracle.pmt(w.s, w.p, w.o, w.patterns[0], key_var=1)
    P2 = oracle.pmt(w.s, w.p, w.o, w.patterns[1], key_var=1)
    keys, cl, cr = oracle.join_key_counts(P1, P2, 1)
    assert int(t.nrows) == int(cl @ cr) == w.meta["predicted_rows"]
    gk, glen = runs(y)
    assert np.array_equal(gk, keys) and np.array_equal(glen, cl * cr)
    # exact rows of sampled keys, and the hottest key (a cL x cR block)
    r = np.random.default_rng(0)
    starts = np.concatenate([[0], np.cumsum(glen)[:-1]])
    pick = list(r.choice(keys.size, size=min(25, keys.size), replace=False)) + [int(np.argmax(cl * cr))]
    for i in pick:
        k = keys[i]
        xs = x[starts[i]: starts[i] + glen[i]]
        lx = np.sort(P1.col(0)[P1.col(1) == k])
        # the key's rows are the product of its P1 rows and P2 rows, one
        # block per row of whichever table the planner put on the left
        a = xs.reshape(cl[i], cr[i])       # P1 on the left: rows constant
        b = xs.reshape(cr[i], cl[i])       # P2 on the left: rows identical
        ok_a = np.all(a == a[:, :1]) and np.array_equal(np.sort(a[:, 0]), lx)
        ok_b = np.all(b == b[:1, :]) and np.array_equal(np.sort(b[0]), lx)
        assert ok_a or ok_b, f"key {k}"
    sess.free(t)


def test_cfg3_full_size(sess):
    sel = json.load(open(os.path.join(os.path.dirname(HERE), "synth", "cfg3_draw.json")))
    w = store_cfg3(seed=sel["seed"])
    pats = [tuple(p) for p in query_cfg3(w, sel["draw"])]
    assert pats == [tuple(p) for p in sel["patterns"]]
    announce(f"cfg3 full size: 200M triples, query {pats}")
    sess.load(w.s, w.p, w.o)
    t = sess.query(pats)
    assert t.vars == [0, 1, 2, 3] and int(t.nrows) == sel["j3_rows"]
    cols = sess.to_numpy(t)
    sess.free(t)
    # plan-agnostic checks: every value of ?x and of ?y gets exactly as many
    # rows as the oracle's counting says, and sampled ?x values get exactly
    # the oracle's rows.  Rows with a given (x, y) from P1 number
    # cnt_P2(x) * cnt_P3(x) * cnt_P4(y).
    x, y = cols[0].astype(np.int64), cols[1].astype(np.int64)
    p1 = oracle.pmt(w.s, w.p, w.o, pats[0])
    p2 = oracle.pmt(w.s, w.p, w.o, pats[1])
    p3 = oracle.pmt(w.s, w.p, w.o, pats[2])
    p4 = oracle.pmt(w.s, w.p, w.o, pats[3], key_var=1)
    E = w.n_entities
    c2 = np.bincount(p2.col(0), minlength=E).astype(np.int64)
    c3 = np.bincount(p3.col(0), minlength=E).astype(np.int64)
    c4 = np.bincount(p4.col(1), minlength=E).astype(np.int64)
    wgt = c2[p1.col(0)] * c3[p1.col(0)] * c4[p1.col(1)]
    assert int(wgt.sum()) == sel["j3_rows"]
    assert np.array_equal(np.bincount(x, minlength=E), np.bincount(p1.col(0), weights=wgt, minlength=E).astype(np.int64))
    assert np.array_equal(np.bincount(y, minlength=E), np.bincount(p1.col(1), weights=wgt, minlength=E).astype(np.int64))
    j2 = oracle.query(w.s, w.p, w.o, pats[:3])
    xs = np.unique(x)
    r = np.random.default_rng(1)
    for k in r.choice(xs, size=min(25, xs.size), replace=False):
        m = x == k
        got = Table([0, 1, 2, 3], [c[m] for c in cols])
        a = Table(j2.vars, [c[j2.col(0) == k] for c in j2.cols])
        exp = oracle.join(a, p4, 1)
        assert np.array_equal(oracle.canonical_rows(got, [0, 1, 2, 3]), oracle.canonical_rows(exp, [0, 1, 2, 3]))
