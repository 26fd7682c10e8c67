"""Full-size parity: every result of the five workloads at their full size
against the oracle, as whole bags.

The oracle's row count and bag hash of each result are stored in
``tests/golden/fullsize.json`` by ``tests/golden/make_fullsize.py`` (which
calls only the seeded generators and the oracle).  Here the same inputs are
generated again, run through the library, and each result table is hashed
where it lies in device memory (``tests/bag_hash.py``, the oracle's hash
written with torch and pinned to it).  Equal row counts and equal 128-bit
hashes of every result: the 50M-triple join (index-merge and forced-shuffle
paths), the 200M-triple four-pattern query, both joins of every one of the
512 batched subqueries (batched and one join per call), and the served
queries of the 500M-triple store (served together and one at a time).
"""
import json
import os

import numpy as np
import pytest
import torch

import oracle
from paper_1702_03484_amd import binding as B
from paper_1702_03484_amd import serving
from paper_1702_03484_amd.engine import MapSQ
from synth import batch_cfg4, cfg4_vars, query_cfg3, serving_cfg5, store_cfg2, store_cfg3, store_cfg5
from tests.bag_hash import table_hash
from tests.conftest import announce

pytestmark = [pytest.mark.gpu, pytest.mark.slow]
HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = json.load(open(os.path.join(HERE, "golden", "fullsize.json")))


def expect(entry):
    r = entry["result"] if "result" in entry else entry
    return r["vars"], (r["rows"], int(r["h1"]), int(r["h2"]))


def runs(sorted_keys):
    """(distinct keys, run lengths) of a sorted key column."""
    if sorted_keys.size == 0:
        return sorted_keys, np.zeros(0, np.int64)
    starts = np.concatenate([[0], np.flatnonzero(np.diff(sorted_keys)) + 1])
    lens = np.diff(np.concatenate([starts, [sorted_keys.size]]))
    return sorted_keys[starts], lens.astype(np.int64)


def test_cfg2_full_size(sess):
    g = GOLDEN["cfg2"]
    w = store_cfg2()
    assert [list(p) for p in w.patterns] == g["patterns"] and w.meta["c"] == g["meta"]["c"]
    announce(f"cfg2 full size: 50M triples, query {w.patterns}; merge path, semi-join + sort, sort")
    sess.load(w.s, w.p, w.o)
    vs, exp = expect(g)
    try:
        # index views paired directly; the larger side filtered by the
        # smaller's keys, then sorted; every record through the radix sort
        for merge, semi, path in ((0, 0, B.MAPSQ_PATH_MERGE), (1, 0, B.MAPSQ_PATH_SEMIJOIN), (1, 1, B.MAPSQ_PATH_SORT)):
            sess.set_join_options(semijoin=semi, merge=merge)
            t = sess.query(w.patterns)
            assert sess.stats().path == path
            got = table_hash(sess, t, vs)
            y = sess.column(t, list(t.vars).index(1)).cpu().numpy()
            sess.free(t)
            assert got == exp, f"path {path}: {got} != {exp}"
        # the rows of every key (a readable check beside the hash)
        P1 = oracle.pmt(w.s, w.p, w.o, w.patterns[0], key_var=1)
        P2 = oracle.pmt(w.s, w.p, w.o, w.patterns[1], key_var=1)
        keys, cl, cr = oracle.join_key_counts(P1, P2, 1)
        gk, glen = runs(y)
        assert np.array_equal(gk, keys) and np.array_equal(glen, cl * cr)
    finally:
        sess.set_join_options()


def test_cfg3_full_size(sess):
    g = GOLDEN["cfg3"]
    sel = json.load(open(os.path.join(os.path.dirname(HERE), "synth", "cfg3_draw.json")))
    w = store_cfg3(seed=sel["seed"])
    pats = [tuple(p) for p in query_cfg3(w, sel["draw"])]
    assert [list(p) for p in pats] == g["patterns"]
    announce(f"cfg3 full size: 200M triples, query {pats}")
    sess.load(w.s, w.p, w.o)
    del w
    t = sess.query(pats)
    vs, exp = expect(g)
    got = table_hash(sess, t, vs)
    sess.free(t)
    assert got == exp and exp[0] == sel["j3_rows"]


@pytest.fixture(scope="module")
def cfg4():
    """The 512 subqueries resident in a session of their own."""
    g = GOLDEN["cfg4"]
    subs = batch_cfg4(seed=g["args"]["seed"], n_sub=g["args"]["n_sub"])
    s = MapSQ(arena_bytes=96 << 30)
    kmax = (1 << 31) - 2
    tabs = []
    for sub, gs in zip(subs, g["subqueries"]):
        v = cfg4_vars(sub)
        d = {}
        for name in ("T1", "T2", "T3"):
            if name in sub:
                d[name] = s.table(v[name], [torch.from_numpy(c).cuda() for c in sub[name]], key_max=kmax)
        assert [int(d[k].nrows) for k in ("T1", "T2", "T3") if k in d] == gs["rows"]
        tabs.append(d)
    del subs
    yield s, tabs, g["subqueries"]
    s.close()


def test_cfg4_batched_full_size(cfg4):
    s, tabs, gold = cfg4
    announce("cfg4 full size: 512 subqueries, two batched launches, every result hashed against the oracle")
    first = s.join_batch([(d["T1"], d["T2"], 0) for d in tabs])
    chain = [i for i, d in enumerate(tabs) if "T3" in d]
    second = dict(zip(chain, s.join_batch([(first[i], tabs[i]["T3"], 20) for i in chain])))
    bad = []
    for i, gs in enumerate(gold):
        vs, exp = expect(gs["join1"])
        if table_hash(s, first[i], vs) != exp:
            bad.append((i, "join1"))
        if i in second:
            vs, exp = expect(gs["join2"])
            if table_hash(s, second[i], vs) != exp:
                bad.append((i, "join2"))
    for t in list(first) + list(second.values()):
        s.free(t)
    assert not bad, f"{len(bad)} results differ from the oracle, first {bad[:5]}"


def test_cfg4_plain_full_size(cfg4):
    s, tabs, gold = cfg4
    announce("cfg4 full size: 512 subqueries one join per call, every result hashed against the oracle")
    bad = []
    for i, (d, gs) in enumerate(zip(tabs, gold)):
        r1 = s.join(d["T1"], d["T2"], 0)
        vs, exp = expect(gs["join1"])
        if table_hash(s, r1, vs) != exp:
            bad.append((i, "join1"))
        if "T3" in d:
            r2 = s.join(r1, d["T3"], 20)
            vs, exp = expect(gs["join2"])
            if table_hash(s, r2, vs) != exp:
                bad.append((i, "join2"))
            s.free(r2)
        s.free(r1)
    assert not bad, f"{len(bad)} results differ from the oracle, first {bad[:5]}"


def test_cfg5_served_full_size():
    """The served queries of the 500M-triple store whose oracle result stays
    within the stored row cap: each result, served together with the
    others (continuous batching) and one at a time (mapsq_query), has the
    oracle's bag."""
    g = GOLDEN["cfg5"]
    a = g["args"]
    announce(f"cfg5 full size: {a['n']}-triple store, {len(g['parity'])} served queries within {a['row_cap']} rows")
    w = store_cfg5(seed=a["seed"], n=a["n"])
    qs = serving_cfg5(w, a["stream"], seed=a["seed"])
    picked = [e["index"] for e in g["parity"]]
    queries = [qs[i] for i in picked]
    assert [[list(p) for p in q] for q in queries] == [e["patterns"] for e in g["parity"]]
    with MapSQ(arena_bytes=128 << 30) as s:
        s.load(w.s, w.p, w.o)
        del w
        exp = [expect(e) for e in g["parity"]]
        got = {}
        serving.run_continuous(s, queries, np.zeros(len(queries)), collect_hash=lambda j, t: got.__setitem__(
            j, table_hash(s, t, exp[j][0])))
        bad = [j for j in range(len(queries)) if got.get(j) != exp[j][1]]
        assert not bad, f"served: queries {[picked[j] for j in bad]} differ from the oracle"
        for j, q in enumerate(queries):
            t = s.query(q)
            h = table_hash(s, t, exp[j][0])
            s.free(t)
            assert h == exp[j][1], f"query {picked[j]} alone differs from the oracle"
