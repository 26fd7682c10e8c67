"""GPU parity of the composite-key join: two tables that bind two common
variables are joined on both at once (packed into one 32-bit sort word when
the two ranges fit, else sorted on the second word and then stably on the
first), and cyclic basic graph patterns, whose closing pattern shares two
variables with the running result, are answered through it.  Compared with
the oracle's join on both variables (``oracle.join_on``), with the
single-variable join plus equality filter (the library's other mode) and,
for queries on tiny stores, with brute-force enumeration of witnesses."""
import numpy as np
import pytest
import torch

import oracle
from oracle.core import Table
from paper_1702_03484_amd import binding as B
from synth import random_store, var
from tests.conftest import announce
from tests.gpu_util import assert_same_bag, host_table

pytestmark = pytest.mark.gpu

I32_MIN, I32_MAX = -(1 << 31), (1 << 31) - 1


def pair_tables(seed, nl, nr, k1_ids, k2_ids, npairs, vl, vr, stray=0.2):
    """Left (k1, v.., k2) and right (k2, w.., k1) tables whose rows take a
    (k1, k2) pair from a seeded pool of npairs pairs; a `stray` fraction of
    rows keeps the pool's k1 with a random k2 from k2_ids (they meet partners
    on k1 only, which the second variable must turn away)."""
    r = np.random.default_rng(seed)
    pool1 = k1_ids[r.integers(0, k1_ids.size, npairs)]
    pool2 = k2_ids[r.integers(0, k2_ids.size, npairs)]
    if npairs >= 2:  # the extremes of both id sets are in the pool
        pool1[:2] = k1_ids.min(), k1_ids.max()
        pool2[:2] = k2_ids.min(), k2_ids.max()

    def side(n):
        pick = r.integers(0, npairs, n)
        k1, k2 = pool1[pick].copy(), pool2[pick].copy()
        odd = r.random(n) < stray
        k2[odd] = k2_ids[r.integers(0, k2_ids.size, int(odd.sum()))]
        return k1.astype(np.int32), k2.astype(np.int32)

    lk1, lk2 = side(nl)
    rk1, rk2 = side(nr)
    lvals = [r.integers(I32_MIN, I32_MAX, nl, dtype=np.int64).astype(np.int32) for _ in range(vl)]
    rvals = [r.integers(I32_MIN, I32_MAX, nr, dtype=np.int64).astype(np.int32) for _ in range(vr)]
    L = Table([0] + list(range(10, 10 + vl)) + [1], [lk1] + lvals + [lk2])
    R = Table([1] + list(range(20, 20 + vr)) + [0], [rk2] + rvals + [rk1])
    return L, R


def ids(seed, card, lo=0, hi=I32_MAX):
    r = np.random.default_rng(seed)
    return np.unique(r.integers(lo, hi, card * 2, dtype=np.int64))[:card]


def dev_table(sess, T, key_max=-1):
    return sess.table(T.vars, [torch.from_numpy(c).cuda() for c in T.cols], key_max=key_max)


CASES = [
    # name, nL, nR, k1 ids, k2 ids, pairs, left / right value columns, packed into one word
    ("tiny", 5, 7, np.arange(3), np.arange(2), 4, 1, 1, True),
    ("packed", 300_001, 200_003, ids(1, 4000, 0, 5000), ids(2, 900, 0, 1000), 20_000, 1, 1, True),
    ("packed_32_bits", 250_000, 260_000, ids(3, 30_000, 0, 1 << 16), ids(4, 30_000, 0, 1 << 16), 50_000, 2, 1, True),
    ("two_words", 400_000, 350_000, ids(5, 30_000), ids(6, 50), 60_000, 1, 2, False),
    # one k1 for every row (its single-variable product is 9e9 rows) and k2
    # over the whole int32 range: 32 bits of key in the second word alone
    ("k2_full_range", 100_000, 90_000, np.array([7]),
     np.concatenate([[I32_MIN, I32_MAX], ids(9, 5000, I32_MIN, I32_MAX)]), 20_000, 1, 0, False),
    ("negative_keys", 70_000, 80_000, ids(7, 500, I32_MIN, -1), ids(8, 700, I32_MIN, I32_MAX), 3000, 3, 3, False),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_composite_join_matches_oracle(sess, case):
    name, nl, nr, k1, k2, npairs, vl, vr, packed = case
    announce(f"composite join {name}: {nl} x {nr} rows")
    L, R = pair_tables(len(name), nl, nr, k1, k2, npairs, vl, vr)
    exp = oracle.join_on(L, R, [0, 1])
    dl, dr = dev_table(sess, L), dev_table(sess, R)
    t = sess.join(dl, dr, 0)
    st = sess.stats()
    assert st.path == B.MAPSQ_PATH_COMPOSITE and st.out_rows == exp.n
    b1, b2 = (int(np.int64(k.max()) - np.int64(k.min())).bit_length() for k in (
        np.concatenate([L.col(0), R.col(0)]), np.concatenate([L.col(1), R.col(1)])))
    assert st.key_bits == b1 + b2 and (b1 + b2 <= 32 and b2 <= 31) == packed
    assert t.vars == exp.vars
    got = host_table(sess, t)
    sess.free(t)
    assert_same_bag(got, exp)
    # the same bag from the single-variable join and the equality filter,
    # where its intermediate (every pair agreeing on k1) is small enough
    if oracle.join_cardinality(L, R, 0) > 50_000_000:
        return
    sess.set_join_options(composite=1)
    try:
        t = sess.join(dl, dr, 0)
        assert sess.stats().path != B.MAPSQ_PATH_COMPOSITE
        assert_same_bag(host_table(sess, t), exp)
        sess.free(t)
    finally:
        sess.set_join_options()


@pytest.mark.parametrize("packed", [True, False], ids=["packed", "two_words"])
def test_composite_join_ten_million_rows(sess, packed):
    """10M input rows (6M + 4M): ids over 20 + 10 bits (one packed word) or
    over the whole 31-bit range (two words)."""
    announce(f"composite join, 6M x 4M rows, {'packed' if packed else 'two words'}")
    if packed:
        k1, k2 = ids(11, 600_000, 0, 1 << 20), ids(12, 1000, 0, 1 << 10)
    else:
        k1, k2 = ids(13, 600_000), ids(14, 1000)
    L, R = pair_tables(20 + packed, 6_000_000, 4_000_000, k1, k2, 2_000_000, 1, 1)
    exp = oracle.join_on(L, R, [0, 1])
    t = sess.join(dev_table(sess, L), dev_table(sess, R), 0)
    st = sess.stats()
    assert st.path == B.MAPSQ_PATH_COMPOSITE and st.out_rows == exp.n
    assert (st.key_bits <= 32) == packed
    got = host_table(sess, t)
    sess.free(t)
    assert_same_bag(got, exp)


@pytest.mark.parametrize("wide", [False, True], ids=["packed", "three_words"])
def test_composite_join_three_variables(sess, wide):
    """Tables that share three variables: the key is (k1, k2, k3), packed
    when the three ranges fit 32 bits, else sorted word by word."""
    announce(f"composite join on three variables, {'three words' if wide else 'packed'}")
    r = np.random.default_rng(40 + wide)
    hi = (1 << 31) - 1 if wide else 1 << 9
    npairs, nl, nr = 30_000, 500_000, 400_000
    pool = [r.integers(0, hi, npairs).astype(np.int32) for _ in range(3)]

    def side(n):
        pick = r.integers(0, npairs, n)
        cols = [p[pick].copy() for p in pool]
        odd = r.random(n) < 0.3  # agree on two variables, not the third
        cols[r.integers(0, 3)][odd] = r.integers(0, hi, int(odd.sum())).astype(np.int32)
        return cols

    a, b = side(nl), side(nr)
    L = Table([5, 0, 6, 1], [a[0], r.integers(0, 1 << 30, nl).astype(np.int32), a[1], a[2]])
    R = Table([1, 5, 6, 2], [b[2], b[0], b[1], r.integers(0, 1 << 30, nr).astype(np.int32)])
    exp = oracle.join_on(L, R, [5, 6, 1])
    t = sess.join(dev_table(sess, L), dev_table(sess, R), 5)
    st = sess.stats()
    assert st.path == B.MAPSQ_PATH_COMPOSITE and st.out_rows == exp.n and (st.key_bits <= 32) != wide
    assert t.vars == exp.vars == [5, 0, 6, 1, 2]
    got = host_table(sess, t)
    sess.free(t)
    assert_same_bag(got, exp)


def test_composite_join_empty_and_no_common_pair(sess):
    announce("composite join: empty side, no common pair")
    L, R = pair_tables(31, 1000, 800, np.arange(50), np.arange(40), 300, 1, 1, stray=0.0)
    E = Table(R.vars, [c[:0] for c in R.cols])
    t = sess.join(dev_table(sess, L), dev_table(sess, E), 0)
    assert int(t.nrows) == 0 and t.vars == [0, 10, 1, 20]
    sess.free(t)
    # every right row keeps a left k1 but takes a k2 no left row has
    R2 = Table(R.vars, [R.cols[0] + 1000, R.cols[1], R.cols[2]])
    t = sess.join(dev_table(sess, L), dev_table(sess, R2), 0)
    assert int(t.nrows) == 0 and sess.stats().path == B.MAPSQ_PATH_COMPOSITE
    sess.free(t)
    assert oracle.join_on(L, R2, [0, 1]).n == 0


CYCLIC = [
    # triangle: the closing pattern shares ?a and ?c with the running result
    lambda e: [(var(0), e, var(1)), (var(1), e + 1, var(2)), (var(2), e + 2, var(0))],
    # two patterns over the same pair of variables
    lambda e: [(var(0), e, var(1)), (var(0), e + 1, var(1))],
    # a four-cycle
    lambda e: [(var(0), e, var(1)), (var(1), e + 1, var(2)), (var(2), e, var(3)), (var(3), e + 1, var(0))],
    # a triangle with a pendant edge and a variable predicate shared by two patterns
    lambda e: [(var(0), var(4), var(1)), (var(1), var(4), var(2)), (var(2), e, var(0)), (var(2), e + 1, var(3))],
    # three variables shared by the last pattern (two in the key, one filtered)
    lambda e: [(var(0), var(1), var(2)), (var(2), e, var(0)), (var(0), var(1), var(2))],
]


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_cyclic_queries_match_bruteforce(sess, seed):
    announce(f"cyclic queries on tiny stores, seed {seed}")
    w = random_store(100 + seed, 40, 5, 3)
    sess.load(w.s, w.p, w.o)
    for make in CYCLIC:
        pats = make(w.n_entities)
        t = sess.query(pats)
        got = host_table(sess, t)
        sess.free(t)
        exp = oracle.query_bruteforce(w.s, w.p, w.o, pats)
        assert_same_bag(got, exp)


def test_cyclic_queries_match_oracle_on_a_larger_store(sess):
    announce("cyclic queries on a 300k-triple store")
    w = random_store(7, 300_000, 4000, 4)
    sess.load(w.s, w.p, w.o)
    for make in CYCLIC:
        pats = make(w.n_entities)
        exp = oracle.query(w.s, w.p, w.o, pats)
        t = sess.query(pats)
        got = host_table(sess, t)
        sess.free(t)
        assert_same_bag(got, exp)
