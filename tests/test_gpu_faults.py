"""Error paths under injected arena-allocation failures.

mapsq_debug_fail_alloc(ctx, k) makes the context's (k+1)-th arena
allocation from then on fail as if the arena were full.  For every k from 0
to past the last allocation a call makes, the call must end either with the
fault-free result (an allocation that has a fallback, such as the
sorted-order copy of the value cells, may fail without changing anything)
or with a memory status (CAPACITY or TOO_LARGE); it must give back every
arena byte it took; and the context must stay usable.  The failure is forced
from the host: every kernel that runs, runs to its normal end.
"""
import os

import numpy as np
import pytest
import torch

from paper_1702_03484_amd import binding as B
from paper_1702_03484_amd import serving
from paper_1702_03484_amd.engine import MapSQ
from synth import random_store, random_table, var
from tests.conftest import announce

pytestmark = pytest.mark.gpu
MEMORY = (B.MAPSQ_ERR_CAPACITY, B.MAPSQ_ERR_TOO_LARGE)


@pytest.fixture(scope="module")
def fs():
    s = MapSQ(arena_bytes=2 << 30)
    yield s
    s.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).cuda()


def snap(sess, t):
    return list(t.vars), [np.array(c) for c in sess.to_numpy(t)]


def same(a, b):
    return a[0] == b[0] and len(a[1]) == len(b[1]) and all(np.array_equal(x, y) for x, y in zip(a[1], b[1]))


def free_bytes(sess):
    torch.cuda.synchronize()
    return B.mapsq_arena_free_bytes(sess.ctx)[0]


def sweep(sess, run, limit):
    """run() returns host snapshots of its results (freeing them); the
    fault-free run first (it also creates whatever the context keeps), then
    one run per fault position.  Returns how many runs failed."""
    ref = run()
    free0 = free_bytes(sess)
    failed, last_ok = 0, False
    for k in range(limit):
        B.mapsq_debug_fail_alloc(sess.ctx, k)
        try:
            got = run()
        except B.MapSQError as e:
            assert e.code in MEMORY, (k, e.code, str(e))
            failed += 1
            last_ok = False
        else:
            assert len(got) == len(ref) and all(same(a, b) for a, b in zip(got, ref)), f"fault at allocation {k}"
            last_ok = True
        finally:
            B.mapsq_debug_fail_alloc(sess.ctx, -1)
        assert free_bytes(sess) == free0, f"fault at allocation {k}: arena bytes not returned"
    assert failed >= 1 and last_ok, (failed, last_ok)
    return failed


def _join_tables(sess, seed, nl, nr, card, vl, vr, extra=False):
    keys = np.arange(card, dtype=np.int64) * 5 + 1
    lc = random_table(seed, nl, card, vl, key_ids=keys)
    rc = random_table(seed + 1, nr, card, vr, key_ids=keys)
    lv = [0] + [10 + k for k in range(vl)]
    rv = [0] + [20 + k for k in range(vr)]
    if extra:  # a second shared variable: a composite-key join
        rv[1] = lv[1]
        rc[1] = lc[1][np.random.default_rng(seed).integers(0, nl, nr)]
    L = sess.table(lv, [dev(c) for c in lc], key_max=int(keys.max()))
    R = sess.table(rv, [dev(c) for c in rc], key_max=int(keys.max()))
    return L, R


@pytest.mark.parametrize("case", ["shuffle", "semijoin", "merge", "composite"])
def test_join_under_alloc_faults(fs, case):
    announce(f"alloc faults: join ({case})")
    if case == "composite":
        L, R = _join_tables(fs, 11, 60_000, 40_000, 3_000, 2, 1, extra=True)
    elif case == "semijoin":
        L, R = _join_tables(fs, 13, 300_000, 2_000, 200_000, 1, 2)
    elif case == "merge":
        L, R = _join_tables(fs, 15, 50_000, 30_000, 4_000, 1, 1)
        keys_l = fs.to_numpy(L)
        order_l = np.argsort(keys_l[0], kind="stable")
        keys_r = fs.to_numpy(R)
        order_r = np.argsort(keys_r[0], kind="stable")
        L = fs.table(list(L.vars), [dev(c[order_l]) for c in keys_l], key_max=L.key_max, sorted_col=1)
        R = fs.table(list(R.vars), [dev(c[order_r]) for c in keys_r], key_max=R.key_max, sorted_col=1)
    else:
        L, R = _join_tables(fs, 17, 100_000, 60_000, 5_000, 2, 1)
    if case == "semijoin":
        fs.set_join_options(semijoin=2)
    try:
        def run():
            t = fs.join(L, R, 0)
            s = snap(fs, t)
            fs.free(t)
            return [s]

        sweep(fs, run, 30)
    finally:
        fs.set_join_options()


def test_query_under_alloc_faults(fs):
    announce("alloc faults: three-pattern query on a 200k-triple store")
    w = random_store(31, 200_000, 20_000, 6)
    fs.load(w.s, w.p, w.o)
    p0, p1, p2 = 20_000, 20_001, 20_002
    pats = [(var(0), p0, var(1)), (var(1), p1, var(2)), (var(0), p2, var(3))]

    def run():
        t = fs.query(pats)
        s = snap(fs, t)
        fs.free(t)
        return [s]

    sweep(fs, run, 60)


def test_batch_under_alloc_faults(fs):
    announce("alloc faults: batch of 10 joins")
    joins = []
    for i in range(10):
        L, R = _join_tables(fs, 100 + 2 * i, 3_000 + 7_000 * i, 20_000 - 1_500 * i, 500 + 300 * i, i % 3, (i + 1) % 3)
        joins.append((L, R, 0))

    def run():
        outs = fs.join_batch(joins)
        s = [snap(fs, t) for t in outs]
        for t in outs:
            fs.free(t)
        return s

    sweep(fs, run, 30)


def test_serving_under_alloc_faults(fs):
    """Served queries under a fault: each one ends with its alone result or
    a memory status; the loop ends and every byte comes back.  (A step that
    finds no memory is retried in a later round, so a single failed
    allocation usually costs a round, not a query.)"""
    announce("alloc faults: serving 5 queries")
    w = random_store(37, 150_000, 15_000, 5)
    fs.load(w.s, w.p, w.o)
    p = [15_000 + k for k in range(5)]
    qs = [[(var(0), p[0], var(1)), (var(1), p[1], var(2))],
          [(var(0), p[2], var(1)), (var(0), p[3], var(2))],
          [(var(0), p[1], var(1)), (var(1), p[4], var(2)), (var(0), p[0], var(3))],
          [(var(0), p[3], var(1))],
          [(var(1), p[2], var(0)), (var(1), p[4], var(2))]]
    alone = []
    for q in qs:
        t = fs.query(q)
        alone.append(snap(fs, t))
        fs.free(t)
    arrivals = np.zeros(len(qs))
    got = {}
    serving.run_continuous(fs, qs, arrivals, collect=got)  # creates the server state
    free0 = free_bytes(fs)
    for k in range(40):
        got = {}
        B.mapsq_debug_fail_alloc(fs.ctx, k)
        try:
            _, _, status = serving.run_continuous(fs, qs, arrivals, collect=got)
        finally:
            B.mapsq_debug_fail_alloc(fs.ctx, -1)
        for j in range(len(qs)):
            if status[j] == 0:
                assert same((got[j][0], got[j][1]), alone[j]), (k, j)
            else:
                assert status[j] in MEMORY, (k, j, status[j])
        assert free_bytes(fs) == free0, f"fault at allocation {k}: arena bytes not returned"


def test_fault_from_the_environment():
    """MAPSQ_FAULT=alloc:0 makes the first allocation after mapsq_create
    fail; the next call runs normally."""
    announce("alloc faults: MAPSQ_FAULT environment variable")
    os.environ["MAPSQ_FAULT"] = "alloc:0"
    try:
        s = MapSQ(arena_bytes=512 << 20)
    finally:
        del os.environ["MAPSQ_FAULT"]
    try:
        L, R = _join_tables(s, 51, 20_000, 10_000, 1_000, 1, 1)
        free0 = free_bytes(s)
        with pytest.raises(B.MapSQError) as e:
            s.join(L, R, 0)
        assert e.value.code in MEMORY
        assert free_bytes(s) == free0
        t = s.join(L, R, 0)
        assert t.nrows > 0
        s.free(t)
        assert free_bytes(s) == free0
    finally:
        s.close()
