"""Plain numpy oracle of MapSQ's join path (test infrastructure only).

TEST INFRASTRUCTURE ONLY: only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may use this module.

What is computed (Feng, Zhang and Feng, arXiv 1702.03484):

* Section 1 (the running example and Table 1): every triple pattern maps to
  a table of partial matches whose key is the variable it shares with the
  other pattern and whose value is its other variables; the query result is
  the join of those tables.
* Section 2, Algorithm 1: the join emits, for every key, each pairing of a
  row labelled LEFT (from the first table) with a row labelled RIGHT (from
  the second).  That is exactly the per-key cross product, i.e. a relational
  equi-join on the key, so the oracle writes out the equi-join by its plain
  definition and never imitates the map/sort/reduce steps.
* Section 2, text after Algorithm 1: results are merged pattern by pattern,
  on one shared variable at a time.

Readings where the paper is silent (each is listed with its reason in the
design notes of the repository): bag semantics with no implicit
de-duplication; only variables become columns (constants such as
"Hospital" in Table 1 are not materialised); output columns are
``[key, left values in left order, right values in right order]`` as in
Table 1(c); when two tables share more than one variable, every shared
variable must agree (``join_on`` joins on all of them; ``join`` joins on one
and filters the others, the same bag); a pattern that shares nothing with
the bound variables joins by cross product; row order is not part of the
result (compare as multisets).

Pins (tests marked ``not gpu``): Table 1 of the paper as a golden fixture;
nested loops on tiny inputs; brute-force enumeration of query witnesses;
sqlite3 joins; the closed form |RS| = sum_k cL(k) cR(k); special cases
(distinct keys -> set intersection, one key -> |L| x |R|, empty side ->
empty, self-join -> sum_k c(k)^2); the C hash join in ``hashjoin.c``.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

_M64 = (1 << 64) - 1


@dataclass
class Table:
    """A binding table: one int32 column per variable (SoA), ``n`` rows."""

    vars: list
    cols: list
    n: int = field(default=-1)

    def __post_init__(self):
        self.vars = [int(v) for v in self.vars]
        self.cols = [np.ascontiguousarray(c, dtype=np.int32) for c in self.cols]
        if self.cols:
            n = int(self.cols[0].shape[0])
            assert all(int(c.shape[0]) == n for c in self.cols)
            assert self.n in (-1, n)
            self.n = n
        assert self.n >= 0, "a table with no columns needs an explicit row count"
        assert len(set(self.vars)) == len(self.vars), "one column per variable"

    def col(self, v: int) -> np.ndarray:
        return self.cols[self.vars.index(v)]

    def rows(self) -> np.ndarray:
        if not self.cols:
            return np.zeros((self.n, 0), dtype=np.int32)
        return np.stack(self.cols, axis=1)


def _is_var(t: int) -> bool:
    return t < 0


def _var_no(t: int) -> int:
    return -t - 1


def pattern_vars(pattern) -> list:
    """Variables of a triple pattern in first-appearance order over (s, p, o)."""
    out = []
    for t in pattern:
        if _is_var(t) and _var_no(t) not in out:
            out.append(_var_no(t))
    return out


def match_pattern(s, p, o, pattern) -> Table:
    """Partial matches of one triple pattern (Section 1, P1/P2 and Table 1(a),(b)).

    A triple matches when every constant position holds that constant and
    every repeated variable takes one value.  Rows keep store order; every
    matching triple gives one row (bag).  Only variables become columns.
    """
    cols = (np.asarray(s), np.asarray(p), np.asarray(o))
    mask = np.ones(cols[0].shape[0], dtype=bool)
    first_pos = {}
    for pos, t in enumerate(pattern):
        if _is_var(t):
            v = _var_no(t)
            if v in first_pos:
                mask &= cols[pos] == cols[first_pos[v]]
            else:
                first_pos[v] = pos
        else:
            mask &= cols[pos] == t
    vs = pattern_vars(pattern)
    if not vs:
        return Table([], [], n=int(mask.sum()))
    return Table(vs, [cols[first_pos[v]][mask] for v in vs])


def pmt(s, p, o, pattern, key_var=None) -> Table:
    """Partial-match table with the key variable first, then the other
    variables (Section 1: key = shared variable, value = other variables)."""
    t = match_pattern(s, p, o, pattern)
    if key_var is None or key_var < 0:
        return t
    order = [key_var] + [v for v in t.vars if v != key_var]
    return Table(order, [t.col(v) for v in order])


def _out_vars(L: Table, R: Table, key: int):
    lv = [v for v in L.vars if v != key]
    rv = [v for v in R.vars if v != key and v not in L.vars]
    extra = [v for v in R.vars if v != key and v in L.vars]
    return lv, rv, extra


def join_key_counts(L: Table, R: Table, key: int):
    """For every key on both sides: (key, cL = rows of L, cR = rows of R)."""
    kl, cl = np.unique(L.col(key), return_counts=True)
    kr, cr = np.unique(R.col(key), return_counts=True)
    common, il, ir = np.intersect1d(kl, kr, assume_unique=True, return_indices=True)
    return common.astype(np.int32), cl[il].astype(np.int64), cr[ir].astype(np.int64)


def join_cardinality(L: Table, R: Table, key: int) -> int:
    """|L join_key R| before any further equality filter: sum_k cL(k) cR(k)."""
    _, cl, cr = join_key_counts(L, R, key)
    return int(np.dot(cl, cr))


def _pairs_sort_merge(lk: np.ndarray, rk: np.ndarray, chunk_rows: int = 1 << 25):
    """Row-index pairs (i, j) with lk[i] == rk[j], by sorting both key columns.

    For every common key with left rows A (ascending row order) and right
    rows B, the pairs are A x B enumerated left-major: pair t of the group is
    (A[t // |B|], B[t % |B|]).
    """
    lo = np.argsort(lk, kind="stable")
    ro = np.argsort(rk, kind="stable")
    ukl, l_start, l_cnt = np.unique(lk[lo], return_index=True, return_counts=True)
    ukr, r_start, r_cnt = np.unique(rk[ro], return_index=True, return_counts=True)
    _, il, ir = np.intersect1d(ukl, ukr, assume_unique=True, return_indices=True)
    ls, lc, rs, rc = l_start[il], l_cnt[il].astype(np.int64), r_start[ir], r_cnt[ir].astype(np.int64)
    tot = lc * rc
    out_i, out_j = [], []
    g0 = 0
    while g0 < tot.size:  # groups in chunks to bound the temporaries
        acc = np.cumsum(tot[g0:])
        g1 = g0 + max(1, int(np.searchsorted(acc, chunk_rows, side="right")))
        t_g = tot[g0:g1]
        n = int(t_g.sum())
        g = np.repeat(np.arange(g0, g1), t_g)
        t = np.arange(n, dtype=np.int64) - np.repeat(np.cumsum(t_g) - t_g, t_g)
        a = t // rc[g]
        b = t - a * rc[g]
        out_i.append(lo[ls[g] + a])
        out_j.append(ro[rs[g] + b])
        g0 = g1
    if not out_i:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    return np.concatenate(out_i), np.concatenate(out_j)


def join(L: Table, R: Table, key: int) -> Table:
    """Sort-merge join of two partial-match tables on ``key`` (Algorithm 1).

    Output columns: key, L's other variables in L's order, then R's
    variables that L does not have, in R's order (Table 1(c)).  Variables
    other than the key that both sides bind must agree (equality filter
    after the key join).
    """
    assert key in L.vars and key in R.vars
    lv, rv, extra = _out_vars(L, R, key)
    i, j = _pairs_sort_merge(L.col(key), R.col(key))
    if extra:
        keep = np.ones(i.shape[0], dtype=bool)
        for v in extra:
            keep &= L.col(v)[i] == R.col(v)[j]
        i, j = i[keep], j[keep]
    cols = [L.col(key)[i]] + [L.col(v)[i] for v in lv] + [R.col(v)[j] for v in rv]
    return Table([key] + lv + rv, cols)


def join_on(L: Table, R: Table, keys) -> Table:
    """Equi-join of two tables on every variable in ``keys`` at once: the bag
    of (L row, R row) pairs that agree on all of them, i.e. their natural
    join when ``keys`` lists every variable both bind.  This is the
    relational meaning of merging partial matches that share more than one
    variable (Section 2 merges on one shared variable; the second one must
    then agree too).  Columns as :func:`join` with key ``keys[0]``; shared
    variables outside ``keys`` are filtered for equality.

    Each row's tuple of key values is numbered (equal tuples get equal
    numbers, by ``np.unique`` over the rows of both tables), and the pairs
    are those of the sort-merge join on that number.
    """
    keys = [int(v) for v in keys]
    assert keys and all(v in L.vars and v in R.vars for v in keys)
    lv, rv, extra = _out_vars(L, R, keys[0])
    if L.n == 0 or R.n == 0:
        i = j = np.zeros(0, np.int64)
    else:
        both = np.concatenate([np.stack([L.col(v) for v in keys], axis=1),
                               np.stack([R.col(v) for v in keys], axis=1)])
        _, tid = np.unique(both, axis=0, return_inverse=True)
        tid = tid.reshape(-1)
        i, j = _pairs_sort_merge(tid[:L.n], tid[L.n:])
    rest = [v for v in extra if v not in keys]
    if rest:
        keep = np.ones(i.shape[0], dtype=bool)
        for v in rest:
            keep &= L.col(v)[i] == R.col(v)[j]
        i, j = i[keep], j[keep]
    cols = [L.col(keys[0])[i]] + [L.col(v)[i] for v in lv] + [R.col(v)[j] for v in rv]
    return Table([keys[0]] + lv + rv, cols)


def join_on_cardinality(L: Table, R: Table, keys) -> int:
    """|join_on(L, R, keys)| before any further equality filter: the sum over
    key tuples of (rows of L with the tuple) x (rows of R with it)."""
    keys = [int(v) for v in keys]
    if L.n == 0 or R.n == 0:
        return 0
    both = np.concatenate([np.stack([L.col(v) for v in keys], axis=1),
                           np.stack([R.col(v) for v in keys], axis=1)])
    _, tid = np.unique(both, axis=0, return_inverse=True)
    tid = tid.reshape(-1)
    m = int(tid.max()) + 1
    cl = np.bincount(tid[:L.n], minlength=m).astype(np.int64)
    cr = np.bincount(tid[L.n:], minlength=m).astype(np.int64)
    return int(cl @ cr)


def join_nested_loop(L: Table, R: Table, key: int) -> Table:
    """Nested-loop join (named in Section 2 as the plain join): every pair of
    rows is tested.  Pure Python; tiny inputs only."""
    lv, rv, extra = _out_vars(L, R, key)
    lk, rk = L.col(key), R.col(key)
    out = []
    for i in range(L.n):
        for j in range(R.n):
            if lk[i] != rk[j]:
                continue
            if any(L.col(v)[i] != R.col(v)[j] for v in extra):
                continue
            out.append([lk[i]] + [L.col(v)[i] for v in lv] + [R.col(v)[j] for v in rv])
    vs = [key] + lv + rv
    if not out:
        return Table(vs, [np.zeros(0, np.int32) for _ in vs])
    arr = np.array(out, dtype=np.int64)
    return Table(vs, [arr[:, c] for c in range(len(vs))])


def cross(L: Table, R: Table) -> Table:
    """Cartesian product (a pattern that shares no variable with the rest)."""
    i = np.repeat(np.arange(L.n, dtype=np.int64), R.n)
    j = np.tile(np.arange(R.n, dtype=np.int64), L.n)
    rv = [v for v in R.vars if v not in L.vars]
    assert len(rv) == len(R.vars)
    return Table(L.vars + rv, [c[i] for c in L.cols] + [R.col(v)[j] for v in rv], n=L.n * R.n)


def equality_filter(T: Table, va: int, cols_b: np.ndarray) -> Table:
    keep = T.col(va) == cols_b
    return Table(T.vars, [c[keep] for c in T.cols], n=int(keep.sum()))


def query_vars(patterns) -> list:
    out = []
    for pat in patterns:
        for v in pattern_vars(pat):
            if v not in out:
                out.append(v)
    return out


def project(T: Table, select) -> Table:
    """SELECT as a bag projection (no DISTINCT), in the order given."""
    if select is None:
        return T
    return Table(list(select), [T.col(v) for v in select], n=T.n)


def query(s, p, o, patterns, select=None, max_rows=None) -> Table:
    """Basic graph pattern evaluation by pattern-by-pattern merging (Section 2).

    Fixed oracle order: start from pattern 0, then repeatedly take the
    lowest-index remaining pattern that shares a variable with the bound
    ones and join on every shared variable at once (:func:`join_on`, the
    same bag as joining on the first shared one and filtering the others
    for equality, without the larger intermediate); with none connected,
    take the lowest-index one by cross product.  Columns end in
    first-appearance order, then ``select`` projects.  With ``max_rows``,
    an intermediate that would exceed it raises OverflowError before it is
    built (a guard on the oracle's memory; results are unchanged).
    """
    order = query_vars(patterns)
    tabs = [match_pattern(s, p, o, pat) for pat in patterns]
    cur = tabs[0]
    left = list(range(1, len(patterns)))
    while left:
        pick = None
        for i in left:
            if set(tabs[i].vars) & set(cur.vars):
                pick = i
                break
        if pick is None:
            pick = left[0]
            nxt = tabs[pick]
            if max_rows is not None and cur.n * nxt.n > max_rows:
                raise OverflowError("intermediate over max_rows")
            if not nxt.vars:
                cur = Table(cur.vars, [np.tile(c, nxt.n) for c in cur.cols], n=cur.n * nxt.n)
            else:
                cur = cross(cur, nxt)
        else:
            nxt = tabs[pick]
            shared = [v for v in order if v in cur.vars and v in nxt.vars]
            if max_rows is not None and join_on_cardinality(cur, nxt, shared) > max_rows:
                raise OverflowError("intermediate over max_rows")
            cur = join_on(cur, nxt, shared)
        left.remove(pick)
    vs = [v for v in order if v in cur.vars]
    cur = Table(vs, [cur.col(v) for v in vs], n=cur.n)
    return project(cur, select)


def query_bruteforce(s, p, o, patterns, select=None) -> Table:
    """Every witness tuple (g_1..g_m) of store triples with g_i matching
    pattern i under one variable binding gives one mapping (bag).  Pure
    Python backtracking over all triples; tiny stores only."""
    order = query_vars(patterns)
    trip = list(zip(np.asarray(s).tolist(), np.asarray(p).tolist(), np.asarray(o).tolist()))
    rows = []

    def rec(i, binding):
        if i == len(patterns):
            rows.append([binding[v] for v in order])
            return
        for g in trip:
            b = dict(binding)
            ok = True
            for t, val in zip(patterns[i], g):
                if t >= 0:
                    if t != val:
                        ok = False
                        break
                else:
                    v = -t - 1
                    if v in b and b[v] != val:
                        ok = False
                        break
                    b[v] = val
            if ok:
                rec(i + 1, b)

    rec(0, {})
    if not order:
        return Table([], [], n=len(rows))
    arr = np.array(rows, dtype=np.int64).reshape(len(rows), len(order))
    return project(Table(order, [arr[:, c] for c in range(len(order))]), select)


def canonical_rows(T: Table, var_order=None) -> np.ndarray:
    """Rows with columns in ``var_order``, sorted lexicographically (int64)."""
    vs = T.vars if var_order is None else list(var_order)
    if not vs:
        return np.zeros((T.n, 0), dtype=np.int64)
    arr = np.stack([T.col(v).astype(np.int64) for v in vs], axis=1)
    if arr.shape[0] == 0:
        return arr
    idx = np.lexsort(arr.T[::-1])
    return arr[idx]


def _splitmix64(x: np.ndarray) -> np.ndarray:
    # SplitMix64 finaliser (Steele, Lea and Flood, OOPSLA 2014).
    x = x + np.uint64(0x9E3779B97F4A7C15)
    x = (x ^ (x >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
    x = (x ^ (x >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return x ^ (x >> np.uint64(31))


def multiset_hash(cols, chunk: int = 1 << 24):
    """Order-independent hash of a bag of rows given as a list of equal-length
    integer columns: (row count, sum of two independent row mixes mod 2^64)."""
    n = int(cols[0].shape[0]) if cols else 0
    h1 = 0
    h2 = 0
    with np.errstate(over="ignore"):
        for lo in range(0, n, chunk):
            hi = min(n, lo + chunk)
            a = np.full(hi - lo, 0x1234567, dtype=np.uint64)
            b = np.full(hi - lo, 0x7654321, dtype=np.uint64)
            for c in cols:
                v = c[lo:hi].astype(np.int64).astype(np.uint64)
                a = _splitmix64(a ^ v)
                b = _splitmix64(b + v * np.uint64(0x2545F4914F6CDD1D))
            h1 = (h1 + int(a.sum(dtype=np.uint64))) & _M64
            h2 = (h2 + int(b.sum(dtype=np.uint64))) & _M64
    return n, h1, h2


def dedup_triples(s, p, o):
    """RDF set semantics: keep the first occurrence of every distinct triple."""
    arr = np.stack([np.asarray(s), np.asarray(p), np.asarray(o)], axis=1)
    _, first = np.unique(arr, axis=0, return_index=True)
    first.sort()
    return arr[first, 0], arr[first, 1], arr[first, 2]
