"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Table 1 of the paper, brute force, sqlite3, closed forms and special cases.
CPU only.
"""
import sqlite3

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st, HealthCheck

import oracle
from oracle import hashjoin
from oracle.core import Table, cross, dedup_triples, pattern_vars
from synth import random_store, random_table, var
from tests.fixtures import load_table1


def rows_set(T, vs=None):
    return sorted(map(tuple, oracle.canonical_rows(T, vs).tolist()))


# ---------------------------------------------------------------- Table 1 ---

def test_table1_partial_matches():
    f = load_table1()
    exp1, vars1 = f["Tp1"]
    t1 = oracle.pmt(f["s"], f["p"], f["o"], f["P1"], key_var=1)
    assert t1.vars == vars1
    assert sorted(map(tuple, t1.rows().tolist())) == sorted(exp1)
    exp2, vars2 = f["Tp2"]
    t2 = oracle.pmt(f["s"], f["p"], f["o"], f["P2"], key_var=1)
    assert t2.vars == vars2
    assert sorted(map(tuple, t2.rows().tolist())) == sorted(exp2)
    # Table 1(b) prints the constant "Hospital" beside each key: every row of
    # Tp2 is indeed a store triple with that object.
    trip = set(zip(f["s"].tolist(), f["p"].tolist(), f["o"].tolist()))
    for (job,) in exp2:
        assert (job, f["dict"]["workAt"], f["dict"]['"Hospital"']) in trip


def test_table1_join_result():
    f = load_table1()
    t1 = oracle.pmt(f["s"], f["p"], f["o"], f["P1"], key_var=1)
    t2 = oracle.pmt(f["s"], f["p"], f["o"], f["P2"], key_var=1)
    rs = oracle.join(t1, t2, 1)
    exp, vs = f["RS"]
    assert rs.vars == vs
    assert sorted(map(tuple, rs.rows().tolist())) == sorted(exp)
    assert sorted(map(tuple, oracle.join_nested_loop(t1, t2, 1).rows().tolist())) == sorted(exp)


def test_table1_select_person():
    f = load_table1()
    q = oracle.query(f["s"], f["p"], f["o"], [f["P1"], f["P2"]], select=[0])
    exp, _ = f["SELECT"]
    assert sorted(map(tuple, q.rows().tolist())) == sorted(exp)
    d = {v: k for k, v in f["dict"].items()}
    assert sorted(d[r[0]] for r in q.rows().tolist()) == ["Jim", "Susan"]


# ------------------------------------------------------------------- map ---

def _bruteforce_map(s, p, o, pat):
    rows = []
    vs = pattern_vars(pat)
    for g in zip(s.tolist(), p.tolist(), o.tolist()):
        b = {}
        ok = True
        for t, val in zip(pat, g):
            if t >= 0:
                ok &= t == val
            else:
                v = -t - 1
                if v in b and b[v] != val:
                    ok = False
                b.setdefault(v, val)
        if ok:
            rows.append(tuple(b[v] for v in vs))
    return rows


PATTERNS = [
    (var(0), "P", var(1)),
    (var(0), "P", "O"),
    ("S", "P", var(1)),
    (var(0), var(1), var(2)),
    (var(0), var(1), "O"),
    ("S", var(0), var(1)),
    (var(0), "P", var(0)),
    (var(0), var(0), var(0)),
    (var(0), var(1), var(0)),
]


@pytest.mark.parametrize("shape", PATTERNS)
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_map_matches_bruteforce(shape, seed):
    w = random_store(seed, 400, 12, 3)
    # make repeated-variable patterns hit: add some s == o and s == p rows
    w.o[:40] = w.s[:40]
    w.s[40:50] = w.p[40:50]
    w.o[40:50] = w.p[40:50]
    r = np.random.default_rng(seed)
    trip = r.integers(0, w.n)
    const = {"S": int(w.s[trip]), "P": int(w.p[trip]), "O": int(w.o[trip])}
    pat = tuple(const[t] if isinstance(t, str) else t for t in shape)
    got = oracle.match_pattern(w.s, w.p, w.o, pat)
    exp = _bruteforce_map(w.s, w.p, w.o, pat)
    assert got.n == len(exp)
    if got.vars:
        assert list(map(tuple, got.rows().tolist())) == exp  # same order: store order


def test_map_partition_invariant():
    w = random_store(5, 5000, 300, 7)
    total = 0
    for pid in np.unique(w.p):
        total += oracle.match_pattern(w.s, w.p, w.o, (var(0), int(pid), var(1))).n
    assert total == w.n


# ------------------------------------------------------------------ join ---

def _tiny_tables(data):
    kcard = data.draw(st.integers(1, 6))
    nl = data.draw(st.integers(0, 25))
    nr = data.draw(st.integers(0, 25))
    lk = data.draw(st.lists(st.integers(0, kcard), min_size=nl, max_size=nl))
    rk = data.draw(st.lists(st.integers(0, kcard), min_size=nr, max_size=nr))
    lv = data.draw(st.lists(st.integers(-3, 100), min_size=nl, max_size=nl))
    rv = data.draw(st.lists(st.integers(-3, 100), min_size=nr, max_size=nr))
    L = Table([1, 0], [np.array(lk, np.int32), np.array(lv, np.int32)])
    R = Table([1, 2], [np.array(rk, np.int32), np.array(rv, np.int32)])
    return L, R


@settings(max_examples=200, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(st.data())
def test_join_equals_nested_loops(data):
    L, R = _tiny_tables(data)
    a = oracle.join(L, R, 1)
    b = oracle.join_nested_loop(L, R, 1)
    assert a.vars == b.vars == [1, 0, 2]
    assert rows_set(a) == rows_set(b)


@settings(max_examples=100, deadline=None)
@given(st.data())
def test_join_extra_shared_variable_is_filtered(data):
    L, R = _tiny_tables(data)
    R2 = Table([1, 0], [R.cols[0], (R.cols[1] % 4).astype(np.int32)])
    L2 = Table([1, 0], [L.cols[0], (L.cols[1] % 4).astype(np.int32)])
    a = oracle.join(L2, R2, 1)
    assert a.vars == [1, 0]
    assert rows_set(a) == rows_set(oracle.join_nested_loop(L2, R2, 1))


def _tiny_two_key_tables(data):
    """Tables binding variables 1 and 3 on both sides (plus 0 on the left,
    2 on the right), values drawn from small ranges so that pairs agree on
    one shared variable but not the other often."""
    nl = data.draw(st.integers(0, 30))
    nr = data.draw(st.integers(0, 30))

    def col(n, hi):
        return np.array(data.draw(st.lists(st.integers(-2, hi), min_size=n, max_size=n)), np.int32)

    L = Table([1, 0, 3], [col(nl, 4), col(nl, 50), col(nl, 3)])
    R = Table([3, 2, 1], [col(nr, 3), col(nr, 50), col(nr, 4)])
    return L, R


@settings(max_examples=200, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(st.data())
def test_join_on_two_keys_equals_nested_loops(data):
    """The two-variable join is the bag of row pairs that agree on both
    variables, enumerated here by plain nested loops."""
    L, R = _tiny_two_key_tables(data)
    got = oracle.join_on(L, R, [1, 3])
    assert got.vars == [1, 0, 3, 2]
    exp = []
    for a in range(L.n):
        for b in range(R.n):
            if L.col(1)[a] == R.col(1)[b] and L.col(3)[a] == R.col(3)[b]:
                exp.append((int(L.col(1)[a]), int(L.col(0)[a]), int(L.col(3)[a]), int(R.col(2)[b])))
    assert rows_set(got) == sorted(exp)
    # joining on the first variable and filtering the second gives the same bag
    assert rows_set(oracle.join(L, R, 1)) == sorted(exp)
    # key order only changes which variable leads the columns
    swapped = oracle.join_on(L, R, [3, 1])
    assert sorted(swapped.vars) == sorted(got.vars)
    assert rows_set(swapped, got.vars) == sorted(exp)


def test_join_on_equals_sqlite():
    r = np.random.default_rng(8)
    n1, n2 = 4000, 3000
    L = Table([0, 5, 1], [r.integers(0, 40, n1), r.integers(0, 30, n1), r.integers(0, 1000, n1)])
    R = Table([5, 2, 0], [r.integers(0, 30, n2), r.integers(0, 1000, n2), r.integers(0, 40, n2)])
    con = sqlite3.connect(":memory:")
    con.execute("create table L(x int, y int, a int)")
    con.execute("create table R(y int, b int, x int)")
    con.executemany("insert into L values(?,?,?)", L.rows().tolist())
    con.executemany("insert into R values(?,?,?)", R.rows().tolist())
    exp = sorted(con.execute("select L.x, L.y, L.a, R.b from L join R on L.x = R.x and L.y = R.y").fetchall())
    got = oracle.join_on(L, R, [0, 5])
    assert got.vars == [0, 5, 1, 2]
    assert rows_set(got) == exp
    assert oracle.join_on_cardinality(L, R, [0, 5]) == len(exp)
    # an empty side: no rows, every column
    E = Table([5, 2, 0], [np.zeros(0, np.int32)] * 3)
    assert oracle.join_on(L, E, [0, 5]).n == 0 and oracle.join_on(L, E, [0, 5]).vars == [0, 5, 1, 2]


def test_cardinality_closed_form():
    # |RS| = sum_k cL(k) * cR(k), computed here from two bincounts
    L = Table([0, 1], random_table(1, 20000, 500, 1, key_ids=np.arange(700)))
    R = Table([0, 2], random_table(2, 7000, 500, 1, key_ids=np.arange(300, 1000)))
    cl = np.bincount(L.col(0), minlength=1000).astype(np.int64)
    cr = np.bincount(R.col(0), minlength=1000).astype(np.int64)
    expect = int(cl @ cr)
    assert oracle.join(L, R, 0).n == expect
    assert oracle.join_cardinality(L, R, 0) == expect
    keys, a, b = oracle.join_key_counts(L, R, 0)
    assert np.array_equal(a, cl[keys]) and np.array_equal(b, cr[keys])


def test_join_equals_sqlite():
    L = Table([0, 1, 3], random_table(3, 3000, 200, 2, key_ids=np.arange(1000, 1300), val_hi=50))
    R = Table([0, 2], random_table(4, 2000, 200, 1, key_ids=np.arange(1100, 1400), val_hi=50))
    con = sqlite3.connect(":memory:")
    con.execute("create table L(k int, a int, b int)")
    con.execute("create table R(k int, c int)")
    con.executemany("insert into L values(?,?,?)", L.rows().tolist())
    con.executemany("insert into R values(?,?)", R.rows().tolist())
    exp = sorted(con.execute("select L.k, L.a, L.b, R.c from L join R on L.k = R.k").fetchall())
    got = oracle.join(L, R, 0)
    assert got.vars == [0, 1, 3, 2]
    assert rows_set(got) == exp


def test_special_cases():
    r = np.random.default_rng(0)
    # all keys distinct on both sides -> rows are the key intersection
    lk = r.permutation(1000)[:600].astype(np.int32)
    rk = r.permutation(1000)[:500].astype(np.int32)
    rs = oracle.join(Table([0], [lk]), Table([0], [rk]), 0)
    assert sorted(rs.col(0).tolist()) == sorted(set(lk.tolist()) & set(rk.tolist()))
    # one key -> |L| x |R| rows, each pairing once
    L = Table([0, 1], [np.full(37, 5, np.int32), np.arange(37, dtype=np.int32)])
    R = Table([0, 2], [np.full(11, 5, np.int32), np.arange(100, 111, dtype=np.int32)])
    rs = oracle.join(L, R, 0)
    assert rs.n == 37 * 11
    assert rows_set(rs) == sorted((5, a, b) for a in range(37) for b in range(100, 111))
    # an empty side -> empty result with the full column list
    E = Table([0, 2], [np.zeros(0, np.int32), np.zeros(0, np.int32)])
    rs = oracle.join(L, E, 0)
    assert rs.n == 0 and rs.vars == [0, 1, 2]
    # self-join -> sum_k c(k)^2
    k = r.integers(0, 50, 3000).astype(np.int32)
    T = Table([0], [k])
    assert oracle.join(T, T, 0).n == int((np.bincount(k).astype(np.int64) ** 2).sum())


def test_hash_join_witness():
    L = Table([0, 1], random_table(5, 50000, 3000, 1))
    keys = np.unique(L.col(0))
    R = Table([0, 2], random_table(6, 20000, 0, 1, key_ids=np.concatenate([keys[::3], np.arange(50)])))
    i, j = hashjoin.hj_pairs(L.col(0), R.col(0), nthreads=4)
    got = sorted(zip(L.col(0)[i].tolist(), L.col(1)[i].tolist(), R.col(2)[j].tolist()))
    assert got == rows_set(oracle.join(L, R, 0))


# ----------------------------------------------------------------- query ---

@st.composite
def tiny_query(draw):
    n_ent = draw(st.integers(2, 5))
    n_pred = draw(st.integers(1, 3))
    n = draw(st.integers(0, 14))
    trip = draw(st.lists(st.tuples(st.integers(0, n_ent - 1), st.integers(n_ent, n_ent + n_pred - 1),
                                   st.integers(0, n_ent - 1)), min_size=n, max_size=n))
    m = draw(st.integers(1, 3))
    nv = draw(st.integers(1, 4))
    pats = []
    for _ in range(m):
        pat = []
        for pos in range(3):
            if draw(st.booleans()) or pos == 1 and draw(st.booleans()):
                pat.append(-draw(st.integers(1, nv)))
            elif pos == 1:
                pat.append(draw(st.integers(n_ent, n_ent + n_pred - 1)))
            else:
                pat.append(draw(st.integers(0, n_ent - 1)))
        pats.append(tuple(pat))
    arr = np.array(trip, dtype=np.int32).reshape(-1, 3)
    return arr[:, 0].copy(), arr[:, 1].copy(), arr[:, 2].copy(), pats


@settings(max_examples=300, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(tiny_query())
def test_query_equals_bruteforce(q):
    s, p, o, pats = q
    a = oracle.query(s, p, o, pats)
    b = oracle.query_bruteforce(s, p, o, pats)
    assert a.vars == b.vars
    assert a.n == b.n
    assert rows_set(a) == rows_set(b)


@settings(max_examples=100, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(tiny_query(), st.randoms())
def test_query_order_independent(q, rnd):
    s, p, o, pats = q
    perm = list(pats)
    rnd.shuffle(perm)
    a = oracle.query(s, p, o, pats)
    b = oracle.query(s, p, o, perm)
    assert sorted(a.vars) == sorted(b.vars)
    assert rows_set(a, sorted(a.vars)) == rows_set(b, sorted(a.vars))


def test_chain_query_equals_sqlite():
    w = random_store(11, 3000, 60, 4)
    P = [w.n_entities + i for i in range(4)]
    x, y, z, u = var(0), var(1), var(2), var(3)
    pats = [(x, P[0], y), (x, P[1], z), (x, P[2], int(w.o[7])), (u, P[3], y)]
    con = sqlite3.connect(":memory:")
    con.execute("create table T(s int, p int, o int)")
    con.executemany("insert into T values(?,?,?)", zip(w.s.tolist(), w.p.tolist(), w.o.tolist()))
    sql = (f"select a.s, a.o, b.o, d.s from T a, T b, T c, T d where a.p={P[0]} and b.p={P[1]} "
           f"and c.p={P[2]} and c.o={int(w.o[7])} and d.p={P[3]} and b.s=a.s and c.s=a.s and d.o=a.o")
    exp = sorted(con.execute(sql).fetchall())
    got = oracle.query(w.s, w.p, w.o, pats)
    assert got.vars == [0, 1, 2, 3]
    assert rows_set(got) == exp
    assert len(exp) > 0


def test_dedup_triples():
    s = np.array([1, 1, 2, 1], np.int32)
    p = np.array([5, 5, 5, 5], np.int32)
    o = np.array([3, 3, 3, 4], np.int32)
    a, b, c = dedup_triples(s, p, o)
    assert list(zip(a, b, c)) == [(1, 5, 3), (2, 5, 3), (1, 5, 4)]


def test_cross_product():
    L = Table([0], [np.arange(3, dtype=np.int32)])
    R = Table([1], [np.arange(10, 14, dtype=np.int32)])
    assert rows_set(cross(L, R)) == sorted((a, b) for a in range(3) for b in range(10, 14))


def test_multiset_hash_is_order_free():
    r = np.random.default_rng(1)
    cols = [r.integers(0, 100, 1000).astype(np.int32) for _ in range(3)]
    perm = r.permutation(1000)
    assert oracle.multiset_hash(cols) == oracle.multiset_hash([c[perm] for c in cols])
    cols2 = [c.copy() for c in cols]
    cols2[1][5] += 1
    assert oracle.multiset_hash(cols) != oracle.multiset_hash(cols2)
    # swapping two columns changes the hash (columns are ordered)
    assert oracle.multiset_hash(cols) != oracle.multiset_hash([cols[1], cols[0], cols[2]])
