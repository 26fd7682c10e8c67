"""GPU parity of the whole join path (map, sort, count/scan, materialise)
against the oracle, through the C ABI.  Integer work: results must be the
same bag of int32 rows exactly."""
import numpy as np
import pytest
import torch

import oracle
from oracle.core import Table
from paper_1702_03484_amd import binding as B
from synth import random_store, random_table, store_cfg1, var
from tests.conftest import announce
from tests.fixtures import load_table1
from tests.gpu_util import assert_same_bag, host_table

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).cuda()


def keyset(seed, card, lo=0, hi=(1 << 31) - 1):
    r = np.random.default_rng(seed)
    return np.unique(r.integers(lo, hi, size=card * 3))[:card]


# ------------------------------------------------------------ worked example

def test_table1_on_gpu(sess):
    announce("table1 map/join/query")
    f = load_table1()
    sess.load(f["s"], f["p"], f["o"])
    t1 = sess.map(f["P1"], key_var=1)
    t2 = sess.map(f["P2"], key_var=1)
    assert t1.vars == [1, 0] and t2.vars == [1]
    assert sorted(map(tuple, np.stack(sess.to_numpy(t1), 1).tolist())) == sorted(f["Tp1"][0])
    assert sorted(map(tuple, np.stack(sess.to_numpy(t2), 1).tolist())) == sorted(f["Tp2"][0])
    rs = sess.join(t1, t2, 1)
    assert rs.vars == [1, 0]
    assert sorted(map(tuple, np.stack(sess.to_numpy(rs), 1).tolist())) == sorted(f["RS"][0])
    st = sess.stats()
    assert st.out_rows == 2 and st.left_rows == 3 and st.right_rows == 2
    sess.free(rs)
    q = sess.query([f["P1"], f["P2"]], select=[0])
    assert sorted(map(tuple, np.stack(sess.to_numpy(q), 1).tolist())) == sorted(f["SELECT"][0])
    sess.free(q)


# ---------------------------------------------------------------- plain joins

JOIN_CASES = [
    # (nL, nR, key cardinality, left value cols, right value cols, key_max known)
    (1, 1, 1, 1, 0, True),
    (3, 5, 2, 0, 0, True),
    (4096, 4096, 300, 1, 1, True),            # exactly one sort tile per side
    (65536, 65536 - 1, 4000, 2, 1, False),    # tile multiples and a ragged tail
    (100_003, 77_777, 5000, 2, 1, False),
    (300_001, 17, 50, 1, 0, True),            # skewed: few keys, big left side
    (3001, 2999, 1, 1, 1, True),              # a single key: |L| x |R| rows
    (250_000, 250_000, 200_000, 1, 2, False), # mostly unique keys
    (1_000_003, 1000, 900, 3, 3, False),      # many columns
]


@pytest.mark.parametrize("hot", [(8, 8), (5, 13)])
@pytest.mark.parametrize("vl,vr", [(1, 1), (2, 1)])
def test_sparse_join_around_the_segment_major_bound(sess, hot, vl, vr):
    """A sparse shuffled join (about one row per key) plus one hot key whose
    product is 64 rows (segment-major materialisation) or 65 (row-chunk
    kernel); value-carrying (1 + 1 columns) and id-payload (2 + 1) records."""
    announce(f"sparse join, hot key {hot[0]}x{hot[1]}, vl={vl} vr={vr}")
    r = np.random.default_rng(hot[0] * 100 + vl)
    n = 200_003
    keys = r.permutation(np.arange(1, 4 * n, 2))[:n].astype(np.int32)
    lk = np.concatenate([keys, np.zeros(hot[0], np.int32)])
    rk = np.concatenate([r.permutation(keys)[: n - 1000], np.zeros(hot[1], np.int32)])
    lc = [lk] + [r.integers(0, 1 << 31, lk.size).astype(np.int32) for _ in range(vl)]
    rc = [rk] + [r.integers(0, 1 << 31, rk.size).astype(np.int32) for _ in range(vr)]
    lvars = [0] + list(range(10, 10 + vl))
    rvars = [0] + list(range(20, 20 + vr))
    sess.set_join_options(semijoin=1, merge=1)
    try:
        out = sess.join(sess.table(lvars, [dev(c) for c in lc]), sess.table(rvars, [dev(c) for c in rc]), 0)
        exp = oracle.join(Table(lvars, lc), Table(rvars, rc), 0)
        assert out.nrows == exp.n == n - 1000 + hot[0] * hot[1]
        assert_same_bag(host_table(sess, out), exp)
        sess.free(out)
    finally:
        sess.set_join_options(0, 0)


@pytest.mark.parametrize("nl,nr,card,vl,vr,known", JOIN_CASES)
def test_join_matches_oracle(sess, nl, nr, card, vl, vr, known):
    announce(f"join nl={nl} nr={nr} card={card} vl={vl} vr={vr} known={known}")
    keys = keyset(nl * 7 + nr, card)
    lc = random_table(nl, nl, card, vl, key_ids=keys)
    rc = random_table(nr + 1, nr, card, vr, key_ids=keys)
    lvars = [0] + list(range(10, 10 + vl))
    rvars = [0] + list(range(20, 20 + vr))
    kmax = int(keys.max()) if known else -1
    L = sess.table(lvars, [dev(c) for c in lc], key_max=kmax)
    R = sess.table(rvars, [dev(c) for c in rc], key_max=kmax)
    out = sess.join(L, R, 0)
    exp = oracle.join(Table(lvars, lc), Table(rvars, rc), 0)
    assert out.vars == exp.vars
    assert_same_bag(host_table(sess, out), exp)
    st = sess.stats()
    assert st.out_rows == exp.n
    sess.free(out)


def test_join_high_ids_and_negative_base(sess):
    announce("join ids near 2^31-2")
    keys = (1 << 31) - 2 - np.arange(0, 700 * 13, 13)
    lc = random_table(5, 20000, 700, 1, key_ids=keys)
    rc = random_table(6, 9000, 700, 1, key_ids=keys)
    L = sess.table([0, 1], [dev(c) for c in lc])
    R = sess.table([0, 2], [dev(c) for c in rc])
    out = sess.join(L, R, 0)
    assert_same_bag(host_table(sess, out), oracle.join(Table([0, 1], lc), Table([0, 2], rc), 0))
    sess.free(out)


@pytest.mark.parametrize("lo,hi", [(0, (1 << 31) - 2), (-(1 << 31), (1 << 31) - 1), (-5, 4)])
@pytest.mark.parametrize("vl,vr", [(1, 1), (0, 2)])
def test_join_key_range_extremes(sess, lo, hi, vl, vr):
    """Key ranges of 31 bits (values carried, 32-bit sort keys with the side
    bit), the full 32 bits (record positions instead) and a tiny negative
    range; keys at both ends of the range occur on both sides."""
    announce(f"join keys in [{lo}, {hi}] vl={vl} vr={vr}")
    r = np.random.default_rng(abs(lo) % 1000 + hi % 1000 + vl)
    mid = r.integers(lo, hi, size=3000, endpoint=True)
    keys = np.unique(np.concatenate([[lo, hi, lo + 1, hi - 1], mid])).astype(np.int64)
    nl, nr = (40_000, 30_000) if keys.size > 1000 else (2_000, 1_500)  # about 0.4-0.3M output rows
    lc = random_table(11 + vl, nl, keys.size, vl, key_ids=keys.astype(np.int32))
    rc = random_table(12 + vr, nr, keys.size, vr, key_ids=keys.astype(np.int32))
    lc[0][:2] = [lo, hi]
    rc[0][:2] = [hi, lo]
    lv = [0] + [10 + k for k in range(vl)]
    rv = [0] + [20 + k for k in range(vr)]
    sess.set_join_options(semijoin=1, merge=1)
    try:
        out = sess.join(sess.table(lv, [dev(c) for c in lc]), sess.table(rv, [dev(c) for c in rc]), 0)
        exp = oracle.join(Table(lv, lc), Table(rv, rc), 0)
        assert out.nrows == exp.n
        assert_same_bag(host_table(sess, out), exp)
        sess.free(out)
    finally:
        sess.set_join_options(0, 0)


def test_join_further_shared_variable(sess):
    announce("join with a second shared variable (equality filter)")
    keys = keyset(3, 500)
    lc = random_table(7, 30000, 500, 2, key_ids=keys, val_hi=5)
    rc = random_table(8, 20000, 500, 2, key_ids=keys, val_hi=5)
    L = sess.table([0, 1, 2], [dev(c) for c in lc])
    R = sess.table([0, 3, 1], [dev(c) for c in rc])  # variable 1 on both sides
    out = sess.join(L, R, 0)
    exp = oracle.join(Table([0, 1, 2], lc), Table([0, 3, 1], rc), 0)
    assert out.vars == exp.vars == [0, 1, 2, 3]
    assert_same_bag(host_table(sess, out), exp)
    sess.free(out)


def test_join_empty_and_disjoint(sess):
    announce("empty and disjoint joins")
    a = sess.table([0, 1], [dev(np.arange(10)), dev(np.arange(10))])
    e = sess.table([0, 2], [dev(np.zeros(0)), dev(np.zeros(0))])
    d = sess.table([0, 2], [dev(np.arange(100, 110)), dev(np.arange(10))])
    for r in (e, d):
        out = sess.join(a, r, 0)
        assert out.nrows == 0 and out.vars == [0, 1, 2]
        sess.free(out)


def test_join_order_is_deterministic_and_tuning_invariant(sess):
    announce("determinism and radix digit width / tile invariance")
    keys = keyset(11, 3000)
    lc = random_table(12, 150_000, 3000, 1, key_ids=keys)
    rc = random_table(13, 60_000, 3000, 1, key_ids=keys)
    L = sess.table([0, 1], [dev(c) for c in lc])
    R = sess.table([0, 2], [dev(c) for c in rc])
    ref = sess.join(L, R, 0)
    ref_cols = sess.to_numpy(ref)
    # rows grouped by ascending key
    k = ref_cols[0]
    assert np.all(k[1:] >= k[:-1])
    for rb in range(4, 12):
        for kpt in (8, 16):
            sess.set_tuning(rb, kpt)
            out = sess.join(L, R, 0)
            cols = sess.to_numpy(out)
            assert all(np.array_equal(a, b) for a, b in zip(cols, ref_cols)), (rb, kpt)
            assert sess.stats().radix_bits == rb
            sess.free(out)
    sess.set_tuning(0, 0)
    sess.free(ref)


SEMI_CASES = [
    # (nL, nR, LEFT key cardinality, RIGHT key cardinality, shared fraction of RIGHT keys, vl, vr, high IDs)
    (300_000, 5_000, 20_000, 800, 0.5, 1, 1, False),   # big LEFT
    (4_000, 250_001, 500, 30_000, 0.3, 2, 1, True),    # big RIGHT, IDs near 2^31
    (200_000, 3_000, 5_000, 200, 0.0, 1, 0, False),    # no key in common
    (100_000, 100_000, 1000, 1000, 1.0, 1, 1, False),  # equal sizes, every key shared
    (70_000, 9, 3, 2, 1.0, 0, 2, False),               # tiny RIGHT, hot keys
]


@pytest.mark.parametrize("nl,nr,cl,cr,shared,vl,vr,high", SEMI_CASES)
def test_semijoin_keeps_rows_and_order(sess, nl, nr, cl, cr, shared, vl, vr, high):
    announce(f"semi-join nl={nl} nr={nr} cl={cl} cr={cr} shared={shared}")
    lo = (1 << 31) - 20_000_000 if high else 0
    pool = keyset(nl + 3 * nr, cl + cr, lo=lo)
    kl = pool[:cl]
    ns = int(round(shared * cr))
    kr = np.concatenate([kl[:ns], pool[cl:cl + cr - ns]])
    lc = random_table(nl + 1, nl, cl, vl, key_ids=kl)
    rc = random_table(nr + 2, nr, len(kr), vr, key_ids=kr)
    lvars = [0] + list(range(10, 10 + vl))
    rvars = [0] + list(range(20, 20 + vr))
    L = sess.table(lvars, [dev(c) for c in lc])
    R = sess.table(rvars, [dev(c) for c in rc])
    cols = {}
    try:
        for mode in (1, 2, 0):
            sess.set_join_options(semijoin=mode, merge=1)
            out = sess.join(L, R, 0)
            st = sess.stats()
            cols[mode] = sess.to_numpy(out)
            if mode == 2:
                big, small = (lc[0], rc[0]) if nl >= nr else (rc[0], lc[0])
                assert st.path == B.MAPSQ_PATH_SEMIJOIN
                assert st.sorted_records == int(np.isin(big, small).sum()) + len(small)
            if mode == 1:
                assert st.path == B.MAPSQ_PATH_SORT and st.sorted_records == nl + nr
                assert_same_bag(host_table(sess, out), oracle.join(Table(lvars, lc), Table(rvars, rc), 0))
            sess.free(out)
    finally:
        sess.set_join_options(0, 0)
    for mode in (2, 0):
        assert all(np.array_equal(a, b) for a, b in zip(cols[mode], cols[1])), f"mode {mode} changed the rows"


MERGE_CASES = [
    # (nL, nR, key cardinality, left value cols, right value cols, extreme keys)
    (1, 1, 1, 1, 0, False),
    (5000, 5000, 1, 1, 1, False),              # one key: a 5000 x 5000 block
    (300_001, 1_588, 700, 0, 1, False),        # big sorted side, hot keys
    (1_588, 300_001, 700, 1, 0, True),         # the same mirrored, keys at INT32_MIN/MAX
    (200_000, 150_000, 120_000, 2, 1, False),  # mostly distinct keys
    (65_536, 1023, 5_000, 1, 2, True),
]


def _sorted_table(seed, n, card, nv, extreme):
    r = np.random.default_rng(seed)
    ids = keyset(seed, card, lo=-(1 << 31) + 1 if extreme else 0)
    if extreme:
        ids = np.unique(np.concatenate([ids[: max(card - 2, 0)], [-(1 << 31), (1 << 31) - 1]]))[:card]
    keys = np.sort(ids[r.integers(0, ids.size, size=n)]).astype(np.int32)
    return [keys] + [r.integers(0, 1 << 31, size=n).astype(np.int32) for _ in range(nv)]


@pytest.mark.parametrize("nl,nr,card,vl,vr,extreme", MERGE_CASES)
def test_merge_join_equals_the_shuffle(sess, nl, nr, card, vl, vr, extreme):
    announce(f"merge join nl={nl} nr={nr} card={card} vl={vl} vr={vr} extreme={extreme}")
    lc = _sorted_table(nl + 5, nl, card, vl, extreme)
    rc = _sorted_table(nr + 6, nr, card, vr, extreme)
    lvars = [0] + list(range(10, 10 + vl))
    rvars = [0] + list(range(20, 20 + vr))
    L = sess.table(lvars, [dev(c) for c in lc], sorted_col=1)
    R = sess.table(rvars, [dev(c) for c in rc], sorted_col=1)
    got = {}
    try:
        for merge in (0, 1):
            sess.set_join_options(semijoin=1, merge=merge)
            out = sess.join(L, R, 0)
            st = sess.stats()
            assert st.path == (B.MAPSQ_PATH_MERGE if merge == 0 else B.MAPSQ_PATH_SORT)
            assert out.sorted_col == 1
            got[merge] = sess.to_numpy(out)
            if merge == 0:
                exp = oracle.join(Table(lvars, lc), Table(rvars, rc), 0)
                assert st.out_rows == exp.n
                assert_same_bag(host_table(sess, out), exp)
            sess.free(out)
    finally:
        sess.set_join_options(0, 0)
    assert all(np.array_equal(a, b) for a, b in zip(got[0], got[1]))
    assert np.all(got[0][0][1:] >= got[0][0][:-1])


def test_views_claim_only_true_orders(sess):
    announce("sorted_col of index views and map outputs")
    w = random_store(31, 200_000, 3000, 40)
    sess.load(w.s, w.p, w.o)
    p1 = int(w.p[0])
    o1 = int(w.o[0])
    s1 = int(w.s[0])
    cases = [((var(0), p1, var(1)), 0), ((var(0), p1, var(1)), 1), ((var(0), p1, var(1)), -1),
             ((s1, p1, var(1)), 1), ((var(0), p1, o1), 0), ((var(0), p1, var(0)), 0),
             ((var(0), var(1), var(2)), 0)]
    claimed = 0
    for pat, key in cases:
        t = sess.map(pat, key_var=key)
        cols = sess.to_numpy(t)
        if t.sorted_col:
            c = cols[t.sorted_col - 1]
            assert np.all(c[1:] >= c[:-1]), (pat, key)
            claimed += 1
        if key >= 0 and t.vars[0] == key and pat[1] >= 0 and pat.count(var(key)) == 1:
            assert t.sorted_col == 1, (pat, key)  # an index order exists for the key
        sess.free(t)
    assert claimed >= 5


def test_query_merge_path_equals_shuffle(sess):
    announce("queries with and without the merge join")
    w = random_store(32, 300_000, 5000, 24)
    sess.load(w.s, w.p, w.o)
    r = np.random.default_rng(33)
    preds = np.unique(w.p)
    queries = []
    for _ in range(12):
        a, b, c = (int(x) for x in r.choice(preds, 3))
        o = int(w.o[r.integers(0, w.n)])
        queries += [[(var(0), a, var(1)), (var(1), b, o)],
                    [(var(0), a, var(1)), (var(0), b, var(2)), (var(0), c, var(3))],
                    [(var(0), a, var(1)), (var(1), b, var(2))]]
    merged = 0
    try:
        for q in queries:
            res = {}
            for merge in (0, 1):
                sess.set_join_options(0, merge)
                try:
                    t = sess.query(q)
                except B.MapSQError as e:
                    res[merge] = e.code
                    continue
                merged += merge == 0 and sess.stats().path == B.MAPSQ_PATH_MERGE
                res[merge] = (t.vars, sess.to_numpy(t))
                sess.free(t)
            if isinstance(res[0], int) or isinstance(res[1], int):
                assert res[0] == res[1]
                continue
            assert res[0][0] == res[1][0]
            assert all(np.array_equal(x, y) for x, y in zip(res[0][1], res[1][1])), q
    finally:
        sess.set_join_options(0, 0)
    assert merged >= 12


def test_large_join_counts_exactly_before_sorting(sess):
    announce("joins of 2^24+ records: exact count first (normal, empty, too large)")
    r = np.random.default_rng(41)
    n_big, n_small = (1 << 24) + 12345, 1_000_003
    kl = r.integers(0, 1 << 20, size=n_big).astype(np.int32)
    kr = r.integers(0, 1 << 20, size=n_small).astype(np.int32)
    vl = r.integers(0, 1 << 31, size=n_big).astype(np.int32)
    vr = r.integers(0, 1 << 31, size=n_small).astype(np.int32)
    L = sess.table([0, 1], [dev(kl), dev(vl)])
    R = sess.table([0, 2], [dev(kr), dev(vr)])
    sess.set_join_options(semijoin=1, merge=1, precount=2)
    try:
        out = sess.join(L, R, 0)
        exp_rows = int(np.bincount(kl, minlength=1 << 20).astype(np.int64) @ np.bincount(kr, minlength=1 << 20))
        assert out.nrows == exp_rows == sess.stats().out_rows
        k, a, b = sess.to_numpy(out)
        assert np.array_equal(np.bincount(k, minlength=1 << 20),
                              np.bincount(kl, minlength=1 << 20) * np.bincount(kr, minlength=1 << 20))
        # exact rows of a few keys
        for key in r.choice(np.unique(kr), 5, replace=False):
            got = Table([0, 1, 2], [k[k == key], a[k == key], b[k == key]])
            exp = oracle.join(Table([0, 1], [kl[kl == key], vl[kl == key]]), Table([0, 2], [kr[kr == key], vr[kr == key]]), 0)
            assert np.array_equal(oracle.canonical_rows(got), oracle.canonical_rows(exp))
        sess.free(out)
        # no key in common: empty, nothing sorted
        R2 = sess.table([0, 2], [dev(kr + (1 << 20)), dev(vr)])
        out = sess.join(L, R2, 0)
        assert out.nrows == 0 and sess.stats().out_rows == 0 and sess.stats().sorted_records == 0
        sess.free(out)
        # one hot key on both sides: far more rows than the arena holds
        free0 = B.mapsq_arena_free_bytes(sess.ctx)[0]
        L3 = sess.table([0, 1], [dev(np.zeros(n_big, np.int32)), dev(vl)])
        R3 = sess.table([0, 2], [dev(np.zeros(3000, np.int32)), dev(vr[:3000])])
        with pytest.raises(B.MapSQError) as ei:
            sess.join(L3, R3, 0)
        assert ei.value.code == B.MAPSQ_ERR_TOO_LARGE
        assert sess.stats().out_rows == n_big * 3000
        assert B.mapsq_arena_free_bytes(sess.ctx)[0] == free0
        # without the count first: the same outcomes, found after the sort
        # (sorting may grow the context's persistent look-back status words,
        # so the free space is taken again after it)
        sess.set_join_options(semijoin=1, merge=1, precount=1)
        out = sess.join(L, R2, 0)
        assert out.nrows == 0 and sess.stats().out_rows == 0 and sess.stats().sorted_records == n_big + n_small
        sess.free(out)
        free0 = B.mapsq_arena_free_bytes(sess.ctx)[0]
        with pytest.raises(B.MapSQError) as ei:
            sess.join(L3, R3, 0)
        assert ei.value.code == B.MAPSQ_ERR_TOO_LARGE
        assert sess.stats().out_rows == n_big * 3000
        assert B.mapsq_arena_free_bytes(sess.ctx)[0] == free0
    finally:
        sess.set_join_options(0, 0)


@pytest.mark.parametrize("nl,nr,card,vl,vr,known", [JOIN_CASES[i] for i in (0, 2, 5, 6, 7)])
def test_exact_count_first_on_small_joins(sess, nl, nr, card, vl, vr, known):
    """precount=2: the dense per-key count runs before every shuffle, small
    and skewed ones included; the rows stay those of the oracle."""
    announce(f"join with the count first nl={nl} nr={nr} card={card}")
    keys = keyset(nl * 7 + nr, card)
    lc = random_table(nl, nl, card, vl, key_ids=keys)
    rc = random_table(nr + 1, nr, card, vr, key_ids=keys)
    lvars = [0] + list(range(10, 10 + vl))
    rvars = [0] + list(range(20, 20 + vr))
    kmax = int(keys.max()) if known else -1
    sess.set_join_options(semijoin=1, merge=1, precount=2)
    try:
        out = sess.join(sess.table(lvars, [dev(c) for c in lc], key_max=kmax),
                        sess.table(rvars, [dev(c) for c in rc], key_max=kmax), 0)
        exp = oracle.join(Table(lvars, lc), Table(rvars, rc), 0)
        assert out.nrows == exp.n == sess.stats().out_rows
        assert_same_bag(host_table(sess, out), exp)
        sess.free(out)
    finally:
        sess.set_join_options(0, 0)


def test_join_too_large_is_refused_without_leak(sess):
    announce("TOO_LARGE: over 2^40 rows and over the arena")
    free0 = None
    for n in (1_100_000, 1_100_000, 400_000):  # 1.2e12 rows > 2^40 ; 1.6e11 rows > arena
        L = sess.table([0, 1], [dev(np.zeros(n)), dev(np.arange(n))], key_max=0)
        R = sess.table([0, 2], [dev(np.zeros(n)), dev(np.arange(n))], key_max=0)
        with pytest.raises(B.MapSQError) as ei:
            sess.join(L, R, 0)
        assert ei.value.code == B.MAPSQ_ERR_TOO_LARGE
        assert sess.stats().out_rows in (n * n, (1 << 40) - 1)
        if free0 is None:  # after the first call (the status words may grow once)
            free0 = B.mapsq_arena_free_bytes(sess.ctx)[0]
    assert B.mapsq_arena_free_bytes(sess.ctx)[0] == free0


def test_invalid_arguments(sess):
    announce("argument errors")
    a = sess.table([0, 1], [dev(np.arange(10)), dev(np.arange(10))])
    b = sess.table([2, 3], [dev(np.arange(10)), dev(np.arange(10))])
    with pytest.raises(B.MapSQError) as ei:
        sess.join(a, b, 0)
    assert ei.value.code == B.MAPSQ_ERR_INVALID_ARG
    with pytest.raises(B.MapSQError) as ei:
        sess.map((5, 6, 7))
    assert ei.value.code in (B.MAPSQ_ERR_UNSUPPORTED, B.MAPSQ_ERR_STATE)
    with pytest.raises(B.MapSQError) as ei:
        B.mapsq_set_tuning(sess.ctx, 3, 0)
    assert ei.value.code == B.MAPSQ_ERR_INVALID_ARG
    for bad in [(3, 0, 0), (0, 2, 0), (0, 0, 3), (-1, 0, 0), (0, 0, -1)]:
        with pytest.raises(B.MapSQError) as ei:
            B.mapsq_set_join_options(sess.ctx, *bad)
        assert ei.value.code == B.MAPSQ_ERR_INVALID_ARG, bad
    B.mapsq_set_join_options(sess.ctx, 0, 0, 0)


# ----------------------------------------------------------------------- map

def _store_with_repeats(seed, n, ne, npred):
    w = random_store(seed, n, ne, npred)
    w.o[: n // 10] = w.s[: n // 10]
    w.s[n // 10: n // 8] = w.p[n // 10: n // 8]
    w.o[n // 10: n // 8] = w.p[n // 10: n // 8]
    return w


MAP_SHAPES = [
    (var(0), "P", var(1)), (var(0), "P", "O"), ("S", "P", var(1)), (var(0), var(1), var(2)),
    (var(0), var(1), "O"), ("S", var(0), var(1)), (var(0), "P", var(0)), (var(0), var(0), var(0)),
    (var(0), var(1), var(0)), ("S", var(0), "O"), (var(0), "Q", var(1)),
]


def test_map_matches_oracle(sess):
    w = _store_with_repeats(21, 300_007, 3000, 6)
    sess.load(w.s, w.p, w.o)
    info = B.mapsq_store_info(sess.ctx)
    assert info.n_triples == w.n and info.n_predicates == 6 and info.max_id == int(max(w.s.max(), w.p.max(), w.o.max()))
    r = np.random.default_rng(0)
    for shape in MAP_SHAPES:
        for _ in range(3):
            t = int(r.integers(0, w.n))
            const = {"S": int(w.s[t]), "P": int(w.p[t]), "O": int(w.o[t]), "Q": 10**9}
            pat = tuple(const[x] if isinstance(x, str) else x for x in shape)
            announce(f"map {pat}")
            exp = oracle.match_pattern(w.s, w.p, w.o, pat)
            for key in [-1] + exp.vars:
                got = sess.map(pat, key_var=key)
                if key >= 0:
                    assert got.vars[0] == key
                assert_same_bag(host_table(sess, got), exp)
                sess.free(got)


def test_map_large_scans(sess):
    """Scans longer than one tile per block (the map's blocks then own runs of
    several tiles) with a ragged tail: dense, sparse, two-test and empty
    selections must each give exactly the oracle's bag."""
    w = _store_with_repeats(23, 9_000_037, 200_000, 5)
    sess.load(w.s, w.p, w.o)
    hot = int(np.bincount(w.o).argmax())
    for pat in [(var(0), var(1), hot), (var(0), var(1), var(0)), (var(0), var(0), var(1)),
                (var(0), var(1), int(w.p[0])), (var(0), var(0), 10**9)]:
        announce(f"map over 9M triples {pat}")
        exp = oracle.match_pattern(w.s, w.p, w.o, pat)
        got = sess.map(pat)
        assert int(got.nrows) == exp.n
        assert_same_bag(host_table(sess, got), exp)
        sess.free(got)


def test_map_dedup_load(sess):
    announce("load with MAPSQ_LOAD_DEDUP")
    w = random_store(31, 50_000, 50, 3)
    sess.load(w.s, w.p, w.o, dedup=True)
    ds, dp, do = oracle.core.dedup_triples(w.s, w.p, w.o)
    assert B.mapsq_store_info(sess.ctx).n_triples == ds.size
    pat = (var(0), var(1), var(2))
    got = sess.map(pat)
    assert_same_bag(host_table(sess, got), oracle.match_pattern(ds, dp, do, pat))
    pat2 = (var(0), int(w.p[0]), var(1))
    got = sess.map(pat2)
    assert_same_bag(host_table(sess, got), oracle.match_pattern(ds, dp, do, pat2))


# --------------------------------------------------------------------- query

def test_cfg1_query(sess):
    w = store_cfg1()
    announce(f"cfg1 query {w.patterns}")
    sess.load(w.s, w.p, w.o)
    got = sess.query(w.patterns)
    exp = oracle.query(w.s, w.p, w.o, w.patterns)
    assert exp.n >= 1
    assert_same_bag(host_table(sess, got), exp)
    sess.free(got)


def _random_queries(w, seed, count):
    """Connected BGPs of 1-4 patterns: every pattern after the first reuses a
    bound variable; constants, variable predicates and repeated variables
    appear at random."""
    r = np.random.default_rng(seed)
    preds = np.unique(w.p)
    out = []
    for _ in range(count):
        m = int(r.integers(1, 5))
        pats, used, nxt = [], [], 0
        for i in range(m):
            t = int(r.integers(0, w.n))
            if i == 0:
                a = nxt
                nxt += 1
            else:
                a = int(r.choice(used))
            used.append(a) if a not in used else None
            u = r.random()
            if u < 0.3:
                b = int(w.o[t])                # constant
            elif u < 0.4:
                b = var(a)                     # repeated variable
            elif u < 0.6 and len(used) > 1:
                b = var(int(r.choice(used)))
            else:
                b = var(nxt)
                used.append(nxt)
                nxt += 1
            p = int(r.choice(preds)) if r.random() < 0.85 else var(10 + i)
            s_, o_ = (var(a), b) if r.random() < 0.5 else (b, var(a))
            if s_ >= 0 and o_ >= 0 and p >= 0:
                o_ = var(a)
            pats.append((s_, p, o_))
        out.append(pats)
    return out


def test_random_queries_match_oracle(sess):
    w = random_store(41, 20_000, 400, 5)
    sess.load(w.s, w.p, w.o)
    done = 0
    for pats in _random_queries(w, 5, 60):
        exp_n = None
        try:
            exp = oracle.query(w.s, w.p, w.o, pats)
            exp_n = exp.n
        except MemoryError:
            continue
        if exp_n > 5_000_000:
            continue
        announce(f"query {pats}")
        got = sess.query(pats)
        assert_same_bag(host_table(sess, got), exp)
        sess.free(got)
        done += 1
    assert done >= 40


def test_query_select_projection(sess):
    w = random_store(42, 5000, 80, 3)
    sess.load(w.s, w.p, w.o)
    e = w.n_entities
    pats = [(var(0), e, var(1)), (var(1), e + 1, var(2)), (var(2), e + 2, var(3))]
    announce(f"projection {pats}")
    for sel in ([3, 0], [1], [2, 1, 0, 3]):
        got = sess.query(pats, select=sel)
        exp = oracle.query(w.s, w.p, w.o, pats, select=sel)
        assert got.vars == sel
        assert_same_bag(host_table(sess, got), exp, var_order=sel)
        sess.free(got)
