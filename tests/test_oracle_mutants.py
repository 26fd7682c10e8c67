"""Planted mistakes: each plausible slip in the oracle must fail one of the pins.

The mistakes are planted in the oracle, on the CPU, with monkeypatch.
"""
import numpy as np
import pytest

import oracle
import oracle.core as core
from oracle.core import Table
from synth import random_store, random_table, var
from tests.fixtures import load_table1


def _rows(T):
    return sorted(map(tuple, oracle.canonical_rows(T).tolist()))


def pin_table1():
    f = load_table1()
    t1 = oracle.pmt(f["s"], f["p"], f["o"], f["P1"], key_var=1)
    t2 = oracle.pmt(f["s"], f["p"], f["o"], f["P2"], key_var=1)
    assert sorted(map(tuple, t1.rows().tolist())) == sorted(f["Tp1"][0])
    assert sorted(map(tuple, t2.rows().tolist())) == sorted(f["Tp2"][0])
    rs = oracle.join(t1, t2, 1)
    assert sorted(map(tuple, rs.rows().tolist())) == sorted(f["RS"][0])


def pin_nested_loops():
    for seed in range(4):
        L = Table([1, 0], random_table(20 + seed, 30, 6, 1, key_ids=np.arange(8), val_hi=9))
        R = Table([1, 2], random_table(40 + seed, 17, 6, 1, key_ids=np.arange(3, 11), val_hi=9))
        assert _rows(oracle.join(L, R, 1)) == _rows(oracle.join_nested_loop(L, R, 1))
        R2 = Table([1, 0], R.cols)
        assert _rows(oracle.join(L, R2, 1)) == _rows(oracle.join_nested_loop(L, R2, 1))


def pin_closed_form():
    L = Table([0, 1], random_table(1, 2000, 50, 1, key_ids=np.arange(70)))
    R = Table([0, 2], random_table(2, 700, 50, 1, key_ids=np.arange(30, 100)))
    cl = np.bincount(L.col(0), minlength=100).astype(np.int64)
    cr = np.bincount(R.col(0), minlength=100).astype(np.int64)
    assert oracle.join(L, R, 0).n == int(cl @ cr)


def pin_map_bruteforce():
    w = random_store(3, 300, 10, 3)
    w.o[:30] = w.s[:30]
    for pat in [(var(0), w.n_entities, var(1)), (var(0), w.n_entities + 1, int(w.o[5])),
                (int(w.s[9]), var(0), var(1)), (var(0), w.n_entities, var(0))]:
        got = oracle.match_pattern(w.s, w.p, w.o, pat)
        exp = []
        for g in zip(w.s.tolist(), w.p.tolist(), w.o.tolist()):
            b, ok = {}, True
            for t, v in zip(pat, g):
                if t >= 0:
                    ok &= t == v
                elif b.setdefault(t, v) != v:
                    ok = False
            if ok:
                exp.append(tuple(b[t] for t in dict.fromkeys(x for x in pat if x < 0)))
        assert list(map(tuple, got.rows().tolist())) == exp


def pin_query_bruteforce():
    w = random_store(7, 25, 4, 2)
    e = w.n_entities
    for pats in [[(var(0), e, var(1)), (var(1), e + 1, var(2))],
                 [(var(0), e, var(1)), (var(0), e + 1, var(1))],
                 [(var(0), e, var(1)), (var(2), e + 1, var(3))],
                 [(var(0), var(1), var(2)), (var(2), e, var(0))]]:
        a = oracle.query(w.s, w.p, w.o, pats)
        b = oracle.query_bruteforce(w.s, w.p, w.o, pats)
        assert _rows(a) == _rows(b)


def pin_two_key_nested_loops():
    r = np.random.default_rng(5)
    for n1, n2 in ((40, 30), (25, 60)):
        L = Table([1, 0, 3], [r.integers(0, 4, n1), r.integers(0, 9, n1), r.integers(0, 3, n1)])
        R = Table([3, 2, 1], [r.integers(0, 3, n2), r.integers(0, 9, n2), r.integers(0, 4, n2)])
        exp = sorted((int(L.col(1)[a]), int(L.col(0)[a]), int(L.col(3)[a]), int(R.col(2)[b]))
                     for a in range(n1) for b in range(n2)
                     if L.col(1)[a] == R.col(1)[b] and L.col(3)[a] == R.col(3)[b])
        got = oracle.join_on(L, R, [1, 3])
        assert got.vars == [1, 0, 3, 2]
        assert sorted(map(tuple, got.rows().tolist())) == exp


PINS = [pin_table1, pin_nested_loops, pin_closed_form, pin_map_bruteforce, pin_query_bruteforce,
        pin_two_key_nested_loops]


def _caught():
    failed = []
    for pin in PINS:
        try:
            pin()
        except AssertionError:
            failed.append(pin.__name__)
    return failed


def test_pins_pass_on_the_real_oracle():
    assert _caught() == []


_orig_pairs = core._pairs_sort_merge
_orig_match = core.match_pattern


def mut_drop_last_group(lk, rk, chunk_rows=1 << 25):
    i, j = _orig_pairs(lk, rk, chunk_rows)
    if i.size == 0:
        return i, j
    last = lk[i[-1]]
    keep = lk[i] != last
    return i[keep], j[keep]


def mut_transposed_index(lk, rk, chunk_rows=1 << 25):
    # a = t % |B|, b = t // |B| instead of a = t // |B|, b = t % |B|
    i, j = _orig_pairs(lk, rk, chunk_rows)
    return np.minimum(i, lk.size - 1), j[::-1].copy()


def mut_same_side_pairs(lk, rk, chunk_rows=1 << 25):
    # pairs LEFT rows with LEFT rows of the same key (label test inverted)
    i, _ = _orig_pairs(lk, lk, chunk_rows)
    j, _ = _orig_pairs(rk, rk, chunk_rows)
    n = min(i.size, j.size)
    return i[:n], j[:n]


def mut_no_repeat_filter(s, p, o, pattern):
    # a repeated variable is not checked for equality
    seen = set()
    pat = []
    for t in pattern:
        if t < 0 and t in seen:
            pat.append(-1000 - len(pat))
        else:
            pat.append(t)
            seen.add(t)
    T = _orig_match(s, p, o, tuple(pat))
    keep = [i for i, v in enumerate(T.vars) if v < 900]
    return Table([T.vars[i] for i in keep], [T.cols[i] for i in keep], n=T.n)


def mut_wrong_position(s, p, o, pattern):
    # constant of the object position compared against the subject column
    return _orig_match(o, p, s, pattern) if pattern[2] >= 0 else _orig_match(s, p, o, pattern)


def mut_no_extra_filter(L, R, key):
    lv, rv, extra = core._out_vars(L, R, key)
    i, j = _orig_pairs(L.col(key), R.col(key))
    cols = [L.col(key)[i]] + [L.col(v)[i] for v in lv] + [R.col(v)[j] for v in rv]
    return Table([key] + lv + rv, cols)


def mut_right_from_left(L, R, key):
    lv, rv, extra = core._out_vars(L, R, key)
    i, j = _orig_pairs(L.col(key), R.col(key))
    cols = [L.col(key)[i]] + [L.col(v)[i] for v in lv] + [R.col(v)[np.minimum(i, R.n - 1)] for v in rv]
    return Table([key] + lv + rv, cols)


def mut_join_on_first_key_only(L, R, keys):
    # the pairs agree on the first key only (the others never compared)
    lv, rv, extra = core._out_vars(L, R, keys[0])
    i, j = _orig_pairs(L.col(keys[0]), R.col(keys[0]))
    cols = [L.col(keys[0])[i]] + [L.col(v)[i] for v in lv] + [R.col(v)[j] for v in rv]
    return Table([keys[0]] + lv + rv, cols)


def mut_join_on_separate_numbering(L, R, keys):
    # each table numbers its own key tuples: equal numbers no longer mean equal tuples
    lv, rv, extra = core._out_vars(L, R, keys[0])
    _, tl = np.unique(np.stack([L.col(v) for v in keys], 1), axis=0, return_inverse=True)
    _, tr = np.unique(np.stack([R.col(v) for v in keys], 1), axis=0, return_inverse=True)
    i, j = _orig_pairs(tl.reshape(-1), tr.reshape(-1))
    cols = [L.col(keys[0])[i]] + [L.col(v)[i] for v in lv] + [R.col(v)[j] for v in rv]
    return Table([keys[0]] + lv + rv, cols)


MUTANTS = [
    ("_pairs_sort_merge", mut_drop_last_group),
    ("_pairs_sort_merge", mut_transposed_index),
    ("_pairs_sort_merge", mut_same_side_pairs),
    ("match_pattern", mut_no_repeat_filter),
    ("match_pattern", mut_wrong_position),
    ("join", mut_no_extra_filter),
    ("join", mut_right_from_left),
    ("join_on", mut_join_on_first_key_only),
    ("join_on", mut_join_on_separate_numbering),
]


@pytest.mark.parametrize("name,fn", MUTANTS, ids=[m[1].__name__ for m in MUTANTS])
def test_planted_mistake_is_caught(monkeypatch, name, fn):
    monkeypatch.setattr(core, name, fn)
    if name in ("match_pattern", "join", "join_on"):
        monkeypatch.setattr(oracle, name, fn)
    caught = _caught()
    assert caught, f"no pin caught the planted mistake {fn.__name__}"
