"""GPU parity of mapsq_join_batch: every join of a batch equals the oracle
(as a bag) and the plain mapsq_join (row for row), with and without graph
capture, on replays, and for joins that fall back to the plain path."""
import os

import numpy as np
import pytest
import torch

import oracle
from oracle.core import Table
from paper_1702_03484_amd import binding as B
from synth import random_table
from tests.conftest import announce
from tests.gpu_util import assert_same_bag, host_table

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).cuda()


def make_batch(sess, seed, count, max_rows=300_000):
    """Joins of uneven sizes (log-uniform), 0-3 value columns a side, key
    cardinality log-uniform; some empty sides and disjoint key sets."""
    r = np.random.default_rng(seed)
    joins, host = [], []
    for i in range(count):
        nl = int(np.exp(r.uniform(0, np.log(max_rows))))
        nr = int(np.exp(r.uniform(0, np.log(max_rows))))
        if i % 13 == 5:
            nl = 0
        card = int(np.exp(r.uniform(0, np.log(50_000))))
        card = max(card, nl * nr // 2_000_000 + 1)  # expected output at most ~2M rows
        vl, vr = int(r.integers(0, 4)), int(r.integers(0, 4))
        keys = np.unique(r.integers(0, (1 << 31) - 1, size=card * 2))[:card]
        rkeys = keys if i % 11 != 7 else keys + 1  # disjoint now and then
        lc = random_table(seed * 1000 + 2 * i, nl, card, vl, key_ids=keys)
        rc = random_table(seed * 1000 + 2 * i + 1, nr, card, vr, key_ids=rkeys)
        lv = [0] + [10 + k for k in range(vl)]
        rv = [0] + [20 + k for k in range(vr)]
        km = int(max(keys.max(), rkeys.max())) if i % 2 else -1
        L = sess.table(lv, [dev(c) for c in lc], key_max=km)
        R = sess.table(rv, [dev(c) for c in rc], key_max=km)
        joins.append((L, R, 0))
        host.append((Table(lv, lc), Table(rv, rc)))
    return joins, host


def check_against_plain_and_oracle(sess, joins, host, outs):
    for i, ((L, R, k), (hl, hr), t) in enumerate(zip(joins, host, outs)):
        exp = oracle.join(hl, hr, 0)
        assert t.vars == exp.vars, i
        got = host_table(sess, t)
        assert_same_bag(got, exp)
        p = sess.join(L, R, k)
        pc = sess.to_numpy(p)
        assert all(np.array_equal(a, b) for a, b in zip(got.cols, pc)), f"join {i}: row order differs from mapsq_join"
        sess.free(p)


def test_batch_matches_oracle_and_plain(sess):
    announce("batch of 40 uneven joins (graph)")
    joins, host = make_batch(sess, 1, 40)
    outs = sess.join_batch(joins)
    check_against_plain_and_oracle(sess, joins, host, outs)
    for t in outs:
        sess.free(t)


def test_batch_sparse_joins_segment_major(sess):
    """Sparse joins (about one output row per key; segment-major work items)
    beside one with a 65-row key (row chunks), 0-3 value columns a side,
    against the oracle and row for row against mapsq_join."""
    announce("batch of sparse joins (segment-major work items)")
    r = np.random.default_rng(5)
    joins, host = [], []
    for i, (n, hot, vl, vr) in enumerate([(50_000, (8, 8), 1, 1), (120_000, (5, 13), 2, 1), (3_000, (1, 1), 0, 3),
                                          (70_001, (8, 8), 3, 2), (999, (2, 3), 1, 0)]):
        keys = r.permutation(np.arange(1, 4 * n, 2))[:n].astype(np.int32)
        lk = np.concatenate([keys, np.zeros(hot[0], np.int32)])
        rk = np.concatenate([r.permutation(keys)[: n - n // 10], np.zeros(hot[1], np.int32)])
        lc = [lk] + [r.integers(0, 1 << 31, lk.size).astype(np.int32) for _ in range(vl)]
        rc = [rk] + [r.integers(0, 1 << 31, rk.size).astype(np.int32) for _ in range(vr)]
        lv = [0] + [10 + k for k in range(vl)]
        rv = [0] + [20 + k for k in range(vr)]
        joins.append((sess.table(lv, [dev(c) for c in lc]), sess.table(rv, [dev(c) for c in rc]), 0))
        host.append((Table(lv, lc), Table(rv, rc)))
    outs = sess.join_batch(joins)
    check_against_plain_and_oracle(sess, joins, host, outs)
    for t in outs:
        sess.free(t)


def test_batch_graph_replay_and_direct_launch_agree(sess, monkeypatch):
    announce("batch: graph replays and direct launches agree")
    joins, host = make_batch(sess, 2, 25, max_rows=100_000)
    runs = []
    for mode in ["1", "1", "0", "1"]:
        monkeypatch.setenv("MAPSQ_BATCH_GRAPH", mode)
        outs = sess.join_batch(joins)
        runs.append([sess.to_numpy(t) for t in outs])
        for t in outs:
            sess.free(t)
    for r in runs[1:]:
        for a, b in zip(runs[0], r):
            assert all(np.array_equal(x, y) for x, y in zip(a, b))
    outs = sess.join_batch(joins)
    check_against_plain_and_oracle(sess, joins, host, outs)
    for t in outs:
        sess.free(t)


def test_batch_fallbacks_and_freeing(sess):
    announce("batch: plain-path fallbacks, shared block release")
    free0 = B.mapsq_arena_free_bytes(sess.ctx)[0]
    keys = np.arange(1000, 1300)
    lc = random_table(70, 5000, 300, 2, key_ids=keys, val_hi=7)
    rc = random_table(71, 3000, 300, 2, key_ids=keys, val_hi=7)
    L = sess.table([0, 1, 2], [dev(c) for c in lc], key_max=1299)
    R = sess.table([0, 3, 1], [dev(c) for c in rc], key_max=1299)   # shares variable 1: plain path
    wide_l = random_table(72, 4000, 300, 5, key_ids=keys)
    wide_r = random_table(73, 4000, 300, 4, key_ids=keys)
    WL = sess.table([0] + list(range(30, 35)), [dev(c) for c in wide_l])
    WR = sess.table([0] + list(range(40, 44)), [dev(c) for c in wide_r])  # 10 columns: plain path
    R2 = sess.table([0, 9], [dev(rc[0]), dev(rc[1])], key_max=1299)
    joins = [(L, R, 0), (WL, WR, 0), (L, R2, 0)]
    outs = sess.join_batch(joins)
    exps = [oracle.join(Table([0, 1, 2], lc), Table([0, 3, 1], rc), 0),
            oracle.join(Table([0] + list(range(30, 35)), wide_l), Table([0] + list(range(40, 44)), wide_r), 0),
            oracle.join(Table([0, 1, 2], lc), Table([0, 9], rc[:2]), 0)]
    for t, e in zip(outs, exps):
        assert t.vars == e.vars
        assert_same_bag(host_table(sess, t), e)
    for t in outs:
        sess.free(t)
    torch.cuda.synchronize()
    # status words may have grown once; everything else is returned
    assert B.mapsq_arena_free_bytes(sess.ctx)[0] >= free0 - (64 << 20)


def test_batch_chain(sess):
    announce("batch: chained second stage keyed on a value column of the first")
    r = np.random.default_rng(5)
    k1 = np.unique(r.integers(0, 1 << 30, 4000))[:3000]
    k2 = np.unique(r.integers(0, 1 << 30, 3000))[:2000]
    stage1, hosts = [], []
    for i in range(12):
        t1 = random_table(100 + i, int(r.integers(100, 50_000)), 3000, 1, key_ids=k1)
        n2 = int(r.integers(100, 50_000))
        t2 = [k1[r.integers(0, k1.size, n2)].astype(np.int32), k2[r.integers(0, k2.size, n2)].astype(np.int32)]
        t3 = random_table(300 + i, int(r.integers(100, 4_000)), 2000, 2, key_ids=k2)
        A = sess.table([0, 1], [dev(c) for c in t1], key_max=int(k1.max()))
        Bt = sess.table([0, 2], [dev(c) for c in t2], key_max=int(max(k1.max(), k2.max())))
        C = sess.table([2, 3, 4], [dev(c) for c in t3], key_max=int(k2.max()))
        stage1.append((A, Bt, 0))
        hosts.append((Table([0, 1], t1), Table([0, 2], t2), Table([2, 3, 4], t3), C))
    outs1 = sess.join_batch(stage1)
    stage2 = [(o, h[3], 2) for o, h in zip(outs1, hosts)]
    outs2 = sess.join_batch(stage2)
    for o2, (a, b, c, _) in zip(outs2, hosts):
        exp = oracle.join(oracle.join(a, b, 0), c, 2)
        assert_same_bag(host_table(sess, o2), exp)
    for t in outs1 + outs2:
        sess.free(t)


def test_batch_full_int32_keys_unknown_bound(sess):
    """Caller tables whose keys span the whole int32 range (negative keys
    included) and whose key bound is unknown (key_max = -1): each batched
    join equals the oracle as a bag and mapsq_join row for row (the plain
    path rebases on the keys' minimum; the batched one sorts all 32 bits)."""
    announce("batch of joins with keys over [INT32_MIN, INT32_MAX], key_max unknown")
    r = np.random.default_rng(23)
    joins, host = [], []
    for i, (nl, nr, card, vl, vr) in enumerate([(5_000, 7_000, 300, 1, 1), (40_000, 900, 2_000, 2, 0),
                                                 (1, 1, 1, 0, 1), (12_345, 12_345, 12_000, 1, 2)]):
        keys = np.unique(r.integers(-(1 << 31), (1 << 31) - 1, size=card * 2, dtype=np.int64))[:card]
        keys[0] = -(1 << 31)  # the extremes always take part
        keys[-1] = (1 << 31) - 1
        keys = keys.astype(np.int32)
        lc = [keys[r.integers(0, card, nl)]] + [r.integers(-(1 << 31), (1 << 31) - 1, nl, dtype=np.int64).astype(np.int32)
                                              for _ in range(vl)]
        rc = [keys[r.integers(0, card, nr)]] + [r.integers(-(1 << 31), (1 << 31) - 1, nr, dtype=np.int64).astype(np.int32)
                                              for _ in range(vr)]
        lv = [0] + [10 + k for k in range(vl)]
        rv = [0] + [20 + k for k in range(vr)]
        L = sess.table(lv, [dev(c) for c in lc], key_max=-1)
        R = sess.table(rv, [dev(c) for c in rc], key_max=-1)
        joins.append((L, R, 0))
        host.append((Table(lv, lc), Table(rv, rc)))
    outs = sess.join_batch(joins)
    assert any(t.nrows > 0 for t in outs)
    check_against_plain_and_oracle(sess, joins, host, outs)
    for t in outs:
        sess.free(t)


def test_batch_semijoin_filter(sess):
    """The batched semi-join reduction (a Bloom filter of the smaller side's
    keys drops the larger side's records without a partner before the sort)
    gives the same rows in the same order with the filter off, automatic and
    forced, equal to the oracle and to mapsq_join: mostly unmatched larger
    sides on either side, a larger side with no partner at all, sides that
    the automatic rule leaves unfiltered, record counts at tile edges."""
    announce("batch: semi-join filter off, automatic and forced")
    specs = [  # (nl, nr, key universe, vl, vr, disjoint)
        (200_000, 2_000, 1_000_000, 1, 2, False),
        (3_000, 150_001, 500_000, 2, 0, False),
        (4096 * 8 + 1, 4096 - 1, 100_000, 1, 1, False),
        (50_000, 30_000, 1_000, 3, 1, False),
        (80_000, 1_000, 50_000, 0, 2, True),
        (4096 * 4, 4096 * 2, 20_000, 1, 0, False),
        (1, 70_000, 10, 1, 1, False),
    ]
    joins, host = [], []
    for i, (nl, nr, U, vl, vr, disjoint) in enumerate(specs):
        keys = np.arange(U, dtype=np.int64) * 7 + 3
        rkeys = keys + 1 if disjoint else keys
        lc = random_table(700 + 2 * i, nl, U, vl, key_ids=keys)
        rc = random_table(701 + 2 * i, nr, U, vr, key_ids=rkeys)
        lv = [0] + [10 + k for k in range(vl)]
        rv = [0] + [20 + k for k in range(vr)]
        km = int(max(keys.max(), rkeys.max())) if i % 2 else -1
        joins.append((sess.table(lv, [dev(c) for c in lc], key_max=km),
                      sess.table(rv, [dev(c) for c in rc], key_max=km), 0))
        host.append((Table(lv, lc), Table(rv, rc)))
    outs, stats = {}, {}
    for mode in (1, 0, 2):
        sess.set_join_options(semijoin=mode)
        try:
            outs[mode] = sess.join_batch(joins)
            stats[mode] = sess.stats()
        finally:
            sess.set_join_options()
    allrec = sum(nl + nr for nl, nr, *_ in specs)
    assert stats[1].sorted_records == allrec and stats[1].path == B.MAPSQ_PATH_SORT
    assert stats[0].path == B.MAPSQ_PATH_SEMIJOIN and stats[0].sorted_records < allrec // 2
    assert stats[2].sorted_records <= stats[0].sorted_records
    for mode in (0, 2):
        assert stats[mode].out_rows == stats[1].out_rows
        for i, (a, b) in enumerate(zip(outs[1], outs[mode])):
            assert a.nrows == b.nrows and a.vars == b.vars, (mode, i)
            for c in range(a.ncols):
                assert torch.equal(sess.column(a, c), sess.column(b, c)), (mode, i, c)
    check_against_plain_and_oracle(sess, joins, host, outs[0])
    for ts in outs.values():
        for t in ts:
            sess.free(t)


def test_batch_keys_per_thread_agree(sess):
    """The batched launch at 8, 16 and 32 keys per thread (tiles of 2,048,
    4,096 and 8,192 records; 32 is the default) gives the same rows in the
    same order, equal to the oracle and to mapsq_join; the joins' record
    counts fall below, on and just past tile edges of every size, and the
    filtered (semi-join) and unfiltered paths both run."""
    announce("batch: 8, 16 and 32 keys per thread agree")
    joins, host = make_batch(sess, 5, 24, max_rows=120_000)
    for i, (nl, nr) in enumerate([(8192, 8191), (8193, 2048), (4096, 12_289), (2047, 40_000)]):
        keys = np.arange(3_000, dtype=np.int64) * 5 + 1
        lc = random_table(900 + 2 * i, nl, 3_000, 1, key_ids=keys)
        rc = random_table(901 + 2 * i, nr, 3_000, 2, key_ids=keys)
        lv, rv = [0, 10], [0, 20, 21]
        joins.append((sess.table(lv, [dev(c) for c in lc], key_max=-1),
                      sess.table(rv, [dev(c) for c in rc], key_max=-1), 0))
        host.append((Table(lv, lc), Table(rv, rc)))
    outs = {}
    try:
        for kpt in (8, 16, 0):
            sess.set_tuning(0, kpt)
            outs[kpt] = sess.join_batch(joins)
    finally:
        sess.set_tuning(0, 0)
    for kpt in (8, 16):
        for i, (a, b) in enumerate(zip(outs[0], outs[kpt])):
            assert a.nrows == b.nrows and a.vars == b.vars, (kpt, i)
            for c in range(a.ncols):
                assert torch.equal(sess.column(a, c), sess.column(b, c)), (kpt, i, c)
    check_against_plain_and_oracle(sess, joins, host, outs[0])
    for ts in outs.values():
        for t in ts:
            sess.free(t)
