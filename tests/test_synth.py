"""The seeded generators: exact Zipf law, determinism, and workload shape."""
import hashlib

import numpy as np
from scipy import stats

import oracle
from synth import gen, store_cfg1, store_cfg2, scramble_ids, zipf_bounded


def _sha(*arrs):
    h = hashlib.sha256()
    for a in arrs:
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def test_zipf_matches_pmf():
    for q, n in [(1.0, 32), (1.1, 200), (1.2, 50), (0.7, 10)]:
        rng = np.random.Generator(np.random.PCG64(123))
        x = zipf_bounded(rng, 400_000, n, q)
        assert x.min() >= 1 and x.max() <= n
        k = np.arange(1, n + 1)
        pmf = k ** -q / np.sum(k ** -q)
        obs = np.bincount(x, minlength=n + 1)[1:]
        chi = stats.chisquare(obs, pmf * x.size)
        assert chi.pvalue > 1e-4, (q, n, chi)


def test_scramble_is_bijection():
    for n in [20000, 10_000_000 // 1000, 50_000]:
        ids = scramble_ids(np.arange(1, n + 1), n)
        assert np.array_equal(np.sort(ids), np.arange(n))


def test_chunking_is_thread_independent(monkeypatch):
    a = gen._zipf_ids(3 * gen.CHUNK // 2, (7, 0, 0), 1000, 1.1)
    monkeypatch.setattr(gen, "_threads", lambda: 1)
    b = gen._zipf_ids(3 * gen.CHUNK // 2, (7, 0, 0), 1000, 1.1)
    assert np.array_equal(a, b)


def test_cfg1_shape_and_determinism():
    w = store_cfg1()
    w2 = store_cfg1()
    assert _sha(w.s, w.p, w.o) == _sha(w2.s, w2.p, w2.o)
    assert w.n == 100_000
    assert w.s.min() >= 0 and w.s.max() < 20000 and w.o.max() < 20000
    assert set(np.unique(w.p).tolist()) == set(range(20000, 20008))
    res = oracle.query(w.s, w.p, w.o, w.patterns)
    assert res.n >= 1


def test_cfg2_small_scale_shape():
    w = store_cfg2(n=2_000_000, n_entities=400_000, row_cap=2_000_000)
    assert w.n == 2_000_000 and w.p.min() >= 400_000 and w.p.max() < 400_032
    # predicates are Zipf(1.0): the top one carries about 1/H_32 of the triples
    top = np.mean(w.p == 400_000)
    assert abs(top - 1 / np.sum(1 / np.arange(1, 33))) < 0.01
    res = oracle.query(w.s, w.p, w.o, w.patterns)
    assert res.n == w.meta["predicted_rows"] and 0 < res.n <= 2_000_000
