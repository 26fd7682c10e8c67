"""Pins of the oracle's dictionary encoding: Table 1's terms, brute force on
small inputs, numpy's first-occurrence numbering as a second witness,
round trips, incremental growth, and planted mistakes caught."""
import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings, strategies as st

from oracle import dictionary as D
from tests.fixtures import load_table1


def brute_ids(terms):
    """Identifier of each term: the number of distinct terms whose first
    appearance comes before this term's first appearance."""
    firsts = [i for i, t in enumerate(terms) if terms.index(t) == i]
    return [sum(1 for f in firsts if f < terms.index(t)) for t in terms]


def test_table1_terms():
    f = load_table1()
    names = {v: k for k, v in f["dict"].items()}
    triples = [(names[s], names[p], names[o]) for s, p, o in zip(f["s"], f["p"], f["o"])]
    flat = [t.encode() for tr in triples for t in tr]
    ids, table = D.encode(flat)
    # every term of the example gets one identifier, decoding gives it back
    assert len(table) == len(set(flat)) and D.decode(ids, table) == flat
    assert table[0] == triples[0][0].encode() and ids[0] == 0
    # the join of Table 1 carried out on identifiers decodes to Table 1(c)'s names
    enc = ids.reshape(-1, 3)
    job, works = table.index(b"hasJob"), table.index(b"workAt")
    hosp = table.index(b'"Hospital"')
    rs = sorted((D.decode([a[2]], table)[0], D.decode([a[0]], table)[0])
                for a in enc if a[1] == job for b in enc if b[1] == works and b[2] == hosp and b[0] == a[2])
    assert rs == [(b"Doctor", b"Jim"), (b"Nurse", b"Susan")]


@settings(max_examples=200, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(st.lists(st.binary(min_size=0, max_size=4), max_size=40))
def test_encode_equals_brute_force(terms):
    ids, table = D.encode(terms)
    assert ids.tolist() == brute_ids(terms)
    assert D.decode(ids, table) == terms
    assert len(table) == len(set(terms))


@settings(max_examples=100, deadline=None)
@given(st.lists(st.binary(min_size=0, max_size=3), max_size=30), st.lists(st.binary(min_size=0, max_size=3), max_size=30))
def test_incremental_encoding(a, b):
    """Encoding a then b equals encoding a + b at once; lookups never grow."""
    ia, ta = D.encode(a)
    ib, tb = D.encode(b, ta)
    iab, tab = D.encode(a + b)
    assert ia.tolist() + ib.tolist() == iab.tolist() and tb == tab
    assert D.lookup(b, ta).tolist() == [ta.index(t) if t in ta else -1 for t in b]


def test_numpy_first_occurrence_witness():
    r = np.random.default_rng(3)
    words = [f"<http://example.org/r{k}>".encode() for k in range(5000)]
    terms = [words[k] for k in r.zipf(1.3, 20000) % 5000]
    ids, table = D.encode(terms)
    # np.unique numbers terms in sorted order; re-rank by first occurrence
    u, first, inv = np.unique(np.array(terms, dtype=object).astype(bytes), return_index=True, return_inverse=True)
    rank = np.empty(u.size, dtype=np.int64)
    rank[np.argsort(first, kind="stable")] = np.arange(u.size)
    assert np.array_equal(ids, rank[inv.reshape(-1)])
    data, off = D.join_terms(terms)
    assert D.split_terms(data, off) == terms


def _mut_last_seen(terms, known=None):
    # identifiers in order of last appearance instead of first
    ids, table = D.encode(list(reversed(terms)), known)
    return ids[::-1].copy(), table


def _mut_sorted(terms, known=None):
    # identifiers in byte order instead of appearance order
    table = list(known or []) + sorted(set(terms) - set(known or []))
    index = {t: i for i, t in enumerate(table)}
    return np.array([index[t] for t in terms], dtype=np.int32), table


@pytest.mark.parametrize("mut", [_mut_last_seen, _mut_sorted])
def test_planted_mistake_is_caught(mut):
    terms = [b"b", b"a", b"b", b"c", b"a", b"d"]
    ids, _ = mut(terms)
    assert ids.tolist() != brute_ids(terms)
