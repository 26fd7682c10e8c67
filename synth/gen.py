"""Seeded generators of RDF-shaped synthetic workloads.

Term encoding used everywhere in this repository: a term of a triple pattern
is a constant ID when it is >= 0 and the variable number ``-t-1`` when it is
< 0 (``var(0) == -1``).  Entities take the IDs ``[0, n_entities)`` and
predicates the IDs ``[n_entities, n_entities + n_pred)``, one dictionary for
both, as an RDF dictionary encoding would give.

Every random stream is ``numpy.random.Generator(PCG64(SeedSequence(key)))``
with ``key = [config, stream, chunk]``; the chunk size is fixed, so the data
does not depend on how many threads draw it.  Streams: 0 = triples,
1 = choice of predicates and constants, 2 = arrivals and query mix.
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np

KNUTH_MUL = 2654435761  # Knuth's multiplicative-hash constant (odd, not a multiple of 5)
CHUNK = 1 << 22
ID_LIMIT = (1 << 31) - 1  # IDs live in [0, 2^31 - 1)


def var(v: int) -> int:
    """Pattern term for variable number ``v``."""
    return -v - 1


@dataclass
class Workload:
    name: str
    s: np.ndarray
    p: np.ndarray
    o: np.ndarray
    n_entities: int
    n_pred: int
    patterns: list = field(default_factory=list)  # list of (s, p, o) term triples
    select: list | None = None  # projected variables, None = all
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.s.shape[0])

    def pred_id(self, rank: int) -> int:
        """ID of the predicate of Zipf rank ``rank`` (1 = most frequent)."""
        return self.n_entities + rank - 1


def _rng(*key: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(k) for k in key])))


def _threads() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        n = os.cpu_count() or 1
    return max(1, min(16, n))


# ---------------------------------------------------------------------------
# Bounded Zipf sampling: rejection-inversion of Hoermann and Derflinger,
# "Rejection-inversion to generate variates from monotone discrete
# distributions" (ACM TOMACS 6(3), 1996).  P(k) is proportional to k^-q for
# k = 1..N.  Exact, O(1) expected work per draw, vectorised by redrawing the
# rejected lanes.
# ---------------------------------------------------------------------------

def _h(x, q):
    return np.exp(-q * np.log(x))


def _H(x, q):
    # integral of h: (x^(1-q) - 1) / (1-q), log(x) at q == 1, in a form stable near q = 1
    lx = np.log(x)
    t = (1.0 - q) * lx
    with np.errstate(invalid="ignore", divide="ignore"):
        f = np.where(np.abs(t) > 1e-8, np.expm1(t) / np.where(t == 0, 1.0, t), 1.0 + t / 2.0)
    return lx * f


def _Hinv(y, q):
    t = (1.0 - q) * y
    with np.errstate(invalid="ignore", divide="ignore"):
        f = np.where(np.abs(t) > 1e-8, np.log1p(t) / np.where(t == 0, 1.0, t), 1.0 - t / 2.0)
    return np.exp(y * f)


def zipf_bounded(rng: np.random.Generator, size: int, n_values: int, q: float) -> np.ndarray:
    """``size`` draws of a Zipf(q) rank in ``[1, n_values]`` as int64."""
    q = float(q)
    hx1 = float(_H(np.float64(1.5), q)) - 1.0
    hN = float(_H(np.float64(n_values + 0.5), q))
    sq = 2.0 - float(_Hinv(_H(np.float64(2.5), q) - _h(np.float64(2.0), q), q))
    out = np.empty(size, dtype=np.int64)
    todo = np.arange(size)
    while todo.size:
        u = hN + rng.random(todo.size) * (hx1 - hN)
        x = _Hinv(u, q)
        k = np.clip(np.floor(x + 0.5), 1, n_values)
        ok = (k - x <= sq) | (u >= _H(k + 0.5, q) - _h(k, q))
        out[todo[ok]] = k[ok].astype(np.int64)
        todo = todo[~ok]
    return out


def scramble_ids(rank: np.ndarray, n_values: int) -> np.ndarray:
    """Bijection rank (1-based) -> ID in [0, n_values): ((rank-1) * KNUTH_MUL) mod n_values.

    Spreads the hot ranks over all bits of the ID space.
    """
    assert math.gcd(KNUTH_MUL, n_values) == 1, "multiplier must be coprime to the ID range"
    r = rank.astype(np.uint64) - np.uint64(1)
    return ((r * np.uint64(KNUTH_MUL)) % np.uint64(n_values)).astype(np.int32)


def _chunked(n: int, key: tuple, draw) -> np.ndarray:
    """Fill an int32 array of length n chunk by chunk; chunk c uses rng(key + (c,))."""
    out = np.empty(n, dtype=np.int32)
    nchunks = (n + CHUNK - 1) // CHUNK

    def work(c):
        lo = c * CHUNK
        hi = min(n, lo + CHUNK)
        out[lo:hi] = draw(_rng(*key, c), hi - lo)

    if nchunks <= 1:
        for c in range(nchunks):
            work(c)
    else:
        with ThreadPoolExecutor(_threads()) as ex:
            list(ex.map(work, range(nchunks)))
    return out


def _uniform_ids(n, key, lo, hi):
    return _chunked(n, key, lambda r, m: r.integers(lo, hi, size=m, dtype=np.int64).astype(np.int32))


def _zipf_ids(n, key, n_values, q, offset=0, scramble=True):
    def draw(r, m):
        k = zipf_bounded(r, m, n_values, q)
        if scramble:
            return scramble_ids(k, n_values) + np.int32(offset)
        return (k - 1 + offset).astype(np.int32)

    return _chunked(n, key, draw)


# ---------------------------------------------------------------------------
# Config 1: 100k triples, 8 uniform predicates, s and o uniform over 20k IDs,
# query ?x p1 ?y . ?y p2 c.
# ---------------------------------------------------------------------------

def store_cfg1(seed: int = 1) -> Workload:
    n, ne, npred = 100_000, 20_000, 8
    cfg = 1000 + seed
    s = _uniform_ids(n, (cfg, 0, 0), 0, ne)
    p = _uniform_ids(n, (cfg, 0, 1), ne, ne + npred)
    o = _uniform_ids(n, (cfg, 0, 2), 0, ne)
    r = _rng(cfg, 1)
    p1 = int(ne + r.integers(0, npred))
    p2 = int(ne + r.integers(0, npred))
    # c: walk the triples of p2 in a seeded order and take the object of the
    # first one whose subject also occurs as an object of p1 (so the result is
    # not empty).
    objs_p1 = np.zeros(ne, dtype=bool)
    objs_p1[o[p == p1]] = True
    idx2 = np.flatnonzero(p == p2)
    c = None
    for i in idx2[r.permutation(idx2.size)]:
        if objs_p1[s[i]]:
            c = int(o[i])
            break
    assert c is not None
    x, y = var(0), var(1)
    return Workload("cfg1", s, p, o, ne, npred, patterns=[(x, p1, y), (y, p2, c)],
                    meta={"p1": p1, "p2": p2, "c": c, "seed": seed})


# ---------------------------------------------------------------------------
# Config 2: 50M triples, predicates Zipf(1.0) over 32, s and o Zipf(1.1) over
# 10M entities (one rank->ID map for both roles), query ?x p1 ?y . ?y p2 c.
# ---------------------------------------------------------------------------

def _store_zipf(cfg, n, ne, npred, q_pred, q_s, q_o, s_uniform=False):
    p = _zipf_ids(n, (cfg, 0, 1), npred, q_pred, offset=ne, scramble=False)
    if s_uniform:
        s = _uniform_ids(n, (cfg, 0, 0), 0, ne)
    else:
        s = _zipf_ids(n, (cfg, 0, 0), ne, q_s)
    o = _zipf_ids(n, (cfg, 0, 2), ne, q_o)
    return s, p, o


def store_cfg2(seed: int = 1, n: int = 50_000_000, n_entities: int = 10_000_000,
               row_cap: int = 200_000_000) -> Workload:
    """``n`` and ``n_entities`` can be scaled down for tests; the defaults are the full size.

    The constant c is workload shaping: among the objects of p2 it is the
    one with the largest predicted output that does not exceed ``row_cap``,
    predicted from two histograms (how often each entity is an object of p1,
    and how often each (subject, c) pair occurs under p2).  Nothing checks a
    join result against this prediction.
    """
    npred = 32
    cfg = 2000 + seed
    s, p, o = _store_zipf(cfg, n, n_entities, npred, 1.0, 1.1, 1.1)
    r = _rng(cfg, 1)
    p1 = n_entities + int(r.integers(0, 8))
    p2 = n_entities + int(r.integers(0, 8))
    hist_obj_p1 = np.bincount(o[p == p1], minlength=n_entities).astype(np.float64)
    m2 = p == p2
    pred = np.bincount(o[m2], weights=hist_obj_p1[s[m2]], minlength=n_entities)
    pred[pred > row_cap] = -1.0
    c = int(np.argmax(pred))  # ties -> smallest ID
    x, y = var(0), var(1)
    return Workload("cfg2", s, p, o, n_entities, npred, patterns=[(x, p1, y), (y, p2, c)],
                    meta={"p1": p1, "p2": p2, "c": c, "seed": seed,
                          "predicted_rows": int(pred[c])})


# ---------------------------------------------------------------------------
# Config 3: 200M triples, 64 predicates Zipf(1.0), s uniform over 50M,
# o Zipf(1.2) over 50M; query ?x p1 ?y . ?x p2 ?z . ?x p3 c . ?w p4 ?y.
# ---------------------------------------------------------------------------

def store_cfg3(seed: int = 1, n: int = 200_000_000, n_entities: int = 50_000_000) -> Workload:
    """Store of config 3 (no query yet; see ``query_cfg3``)."""
    npred = 64
    cfg = 3000 + seed
    s, p, o = _store_zipf(cfg, n, n_entities, npred, 1.0, None, 1.2, s_uniform=True)
    return Workload("cfg3", s, p, o, n_entities, npred, meta={"seed": seed})


def query_cfg3(w: Workload, draw: int = 0) -> list:
    """One seeded draw of ``?x p1 ?y . ?x p2 ?z . ?x p3 c . ?w p4 ?y``.

    p1..p4 are distinct predicates among the 8 most frequent; c is an object
    of p3 whose frequency rank under p3 is drawn uniformly from [50, 1000)
    (the hottest objects make the output billions of rows).  Callers that
    need the output inside a size band try successive draws.
    """
    r = _rng(3000 + w.meta["seed"], 1, draw)
    preds = w.n_entities + r.permutation(8)[:4]
    p1, p2, p3, p4 = (int(v) for v in preds)
    vals, cnts = np.unique(w.o[w.p == p3], return_counts=True)
    ranked = vals[np.argsort(-cnts, kind="stable")[:1000]]
    c = int(ranked[int(r.integers(50, ranked.size))])
    x, y, z, u = var(0), var(1), var(2), var(3)
    return [(x, p1, y), (x, p2, z), (x, p3, c), (u, p4, y)]


# ---------------------------------------------------------------------------
# Small random stores and tables for property tests.
# ---------------------------------------------------------------------------

def random_store(seed: int, n: int, n_entities: int, n_pred: int) -> Workload:
    r = _rng(9000, seed)
    s = r.integers(0, n_entities, size=n, dtype=np.int64).astype(np.int32)
    p = r.integers(n_entities, n_entities + n_pred, size=n, dtype=np.int64).astype(np.int32)
    o = r.integers(0, n_entities, size=n, dtype=np.int64).astype(np.int32)
    return Workload(f"random{seed}", s, p, o, n_entities, n_pred, meta={"seed": seed})


def random_table(seed: int, nrows: int, key_card: int, nvals: int, key_ids: np.ndarray | None = None,
                 val_hi: int = ID_LIMIT) -> list:
    """Key column drawn uniformly from ``key_card`` distinct IDs plus ``nvals``
    value columns uniform in ``[0, val_hi)``; returns a list of int32 arrays."""
    r = _rng(9100, seed)
    if key_ids is None:
        key_ids = np.unique(r.integers(0, ID_LIMIT, size=key_card * 2, dtype=np.int64))[:key_card]
        key_ids = r.permutation(key_ids)
    keys = key_ids[r.integers(0, key_ids.size, size=nrows)].astype(np.int32)
    cols = [keys]
    for _ in range(nvals):
        cols.append(r.integers(0, val_hi, size=nrows, dtype=np.int64).astype(np.int32))
    return cols


def _loguniform(r, lo, hi):
    return int(np.exp(r.uniform(np.log(lo), np.log(hi))))


def _distinct_ids(r, k):
    ids = np.unique(r.integers(0, ID_LIMIT, size=int(k * 1.1) + 16, dtype=np.int64))
    while ids.size < k:
        ids = np.unique(np.concatenate([ids, r.integers(0, ID_LIMIT, size=k, dtype=np.int64)]))
    return r.permutation(ids[:k]).astype(np.int32)


def batch_cfg4(seed: int = 1, n_sub: int = 512, size_lo: float = 1e3, size_hi: float = 1e7,
               card_lo: float = 1e2, card_hi: float = 1e6, cap: float = 2.0 ** 24) -> list:
    """Config 4: ``n_sub`` independent subqueries, half of them one join
    (T1 JOIN T2 on variable 0), half a chain of two (then JOIN T3 on T2's
    first value column, variable 20).  Every table has log-uniform
    [size_lo, size_hi] rows, 1-3 value columns uniform in [0, 2^31-1), and
    keys drawn uniformly from a seeded set of K distinct IDs, K log-uniform
    in [card_lo, card_hi].  A join is redrawn while |L|*|R|/K exceeds ``cap``
    (the expected output); for a chain the cap also holds for the second join.
    Variables: T1 = [0, 10..], T2 = [0, 20, 21..], T3 = [20, 30..].

    Returns a list of dicts with 'kind' (2 or 3 patterns) and 'T1', 'T2'
    (and 'T3') as lists of int32 columns (key first).  Sizes are drawn first
    and the columns afterwards, one seeded stream per table, in parallel.
    """
    r = _rng(4000 + seed, 1)
    specs = []
    for q in range(n_sub):
        kind = 2 if q % 2 == 0 else 3
        while True:
            n1, n2 = _loguniform(r, size_lo, size_hi), _loguniform(r, size_lo, size_hi)
            k1 = _loguniform(r, card_lo, card_hi)
            v1, v2 = int(r.integers(1, 4)), int(r.integers(1, 4))
            est = n1 * n2 / k1
            if est > cap:
                continue
            if kind == 3:
                n3 = _loguniform(r, size_lo, size_hi)
                k2 = _loguniform(r, card_lo, card_hi)
                v3 = int(r.integers(1, 4))
                if est * n3 / k2 > cap:
                    continue
            break
        spec = {"kind": kind, "n1": n1, "n2": n2, "k1": k1, "v1": v1, "v2": v2}
        if kind == 3:
            spec.update({"n3": n3, "k2": k2, "v3": v3})
        specs.append(spec)

    def build(q):
        sp = specs[q]
        rq = _rng(4000 + seed, 2, q)
        keys1 = _distinct_ids(rq, sp["k1"])
        keys2 = _distinct_ids(rq, sp["k2"]) if sp["kind"] == 3 else None

        def table(n, keyset, nv, first_from=None):
            cols = [keyset[rq.integers(0, keyset.size, size=n)]]
            for c in range(nv):
                if c == 0 and first_from is not None:
                    cols.append(first_from[rq.integers(0, first_from.size, size=n)])
                else:
                    cols.append(rq.integers(0, ID_LIMIT, size=n, dtype=np.int64).astype(np.int32))
            return cols

        out = {"kind": sp["kind"], "T1": table(sp["n1"], keys1, sp["v1"]),
               "T2": table(sp["n2"], keys1, sp["v2"], first_from=keys2)}
        if sp["kind"] == 3:
            out["T3"] = table(sp["n3"], keys2, sp["v3"])
        return out

    with ThreadPoolExecutor(_threads()) as ex:
        return list(ex.map(build, range(n_sub)))


def cfg4_vars(sub: dict):
    """Variables of the tables of one config-4 subquery."""
    v = {"T1": [0] + [10 + c for c in range(len(sub["T1"]) - 1)],
         "T2": [0] + [20 + c for c in range(len(sub["T2"]) - 1)]}
    if "T3" in sub:
        v["T3"] = [20] + [30 + c for c in range(len(sub["T3"]) - 1)]
    return v


def store_cfg5(seed: int = 1, n: int = 500_000_000, n_entities: int = 100_000_000, n_pred: int = 128) -> Workload:
    """Config 5 store: predicates Zipf(1.0) over 128, subjects and objects
    Zipf(1.1) over 100M entities with one rank->ID map for both roles."""
    cfg = 5000 + seed
    s, p, o = _store_zipf(cfg, n, n_entities, n_pred, 1.0, 1.1, 1.1)
    return Workload("cfg5", s, p, o, n_entities, n_pred, meta={"seed": seed})


def serving_cfg5(w: Workload, n_queries: int, seed: int = 1, sample: int = 20_000_000) -> list:
    """Queries of 1-5 triple patterns, each a seeded random walk over the
    store's first ``sample`` triples (so every query has at least one
    answer): start at a random triple, then repeatedly step from a visited
    entity to a random triple that has it as subject or object.  Each
    pattern keeps 0, 1 or 2 of its positions constant (probabilities 0.05,
    0.45, 0.5; a kept position is the predicate with probability 0.8 when
    it is free) and turns the rest into variables, one variable per distinct
    value of the walk, so consecutive patterns share variables.
    """
    m = min(sample, w.n)
    S, P, O = w.s[:m], w.p[:m], w.o[:m]
    by_s = np.argsort(S, kind="stable")
    by_o = np.argsort(O, kind="stable")
    s_sorted, o_sorted = S[by_s], O[by_o]
    r = _rng(5000 + seed, 2)
    out = []
    for _ in range(n_queries):
        npat = int(r.integers(1, 6))
        walk = [int(r.integers(0, m))]
        nodes = [int(S[walk[0]]), int(O[walk[0]])]
        tries = 0
        while len(walk) < npat and tries < 50:
            tries += 1
            e = nodes[int(r.integers(0, len(nodes)))]
            use_s = bool(r.integers(0, 2))
            arr, order = (s_sorted, by_s) if use_s else (o_sorted, by_o)
            ev = np.int32(e)  # a typed scalar: no conversion of the whole array
            lo, hi = int(np.searchsorted(arr, ev, "left")), int(np.searchsorted(arr, ev, "right"))
            if hi <= lo:
                continue
            t = int(order[lo + int(r.integers(0, hi - lo))])
            if t in walk:
                continue
            walk.append(t)
            nodes += [int(S[t]), int(O[t])]
        varof = {}
        pats = []
        for t in walk:
            trip = [int(S[t]), int(P[t]), int(O[t])]
            k = int(r.choice(3, p=[0.05, 0.45, 0.5]))
            keep = set()
            while len(keep) < k:
                if 1 not in keep and r.random() < 0.8:
                    keep.add(1)
                else:
                    keep.add(int(r.integers(0, 3)))
            pat = []
            for pos in range(3):
                if pos in keep:
                    pat.append(trip[pos])
                else:
                    v = varof.setdefault(trip[pos], len(varof))
                    pat.append(var(v))
            pats.append(tuple(pat))
        out.append(pats)
    return out


def rdf_terms(seed: int, n_terms: int, n_vocab: int, q: float = 1.1, max_literal: int = 80) -> tuple:
    """A stream of ``n_terms`` RDF-shaped byte-string terms drawn from a
    vocabulary of ``n_vocab`` distinct terms with Zipf(q) frequencies: IRIs
    ``<http://example.org/{kind}/{k}>`` (kinds by class of rank) and, for one
    rank in five, quoted literals of 0..max_literal random lowercase bytes.
    Returns (uint8 bytes, int64 offsets of n_terms + 1, the vocabulary as a
    list of bytes in rank order)."""
    r = _rng(7000 + seed, 0)
    kinds = [b"person", b"org", b"pub", b"course", b"dept"]
    vocab = []
    lens = r.integers(0, max_literal + 1, n_vocab)
    for k in range(n_vocab):
        if k % 5 == 4:
            lit = r.integers(97, 123, int(lens[k]), dtype=np.int64).astype(np.uint8).tobytes()
            vocab.append(b'"' + lit + b'"')
        else:
            vocab.append(b"<http://example.org/" + kinds[k % 5] + b"/" + str(k).encode() + b">")
    ranks = zipf_bounded(r, n_terms, n_vocab, q) - 1
    # a random bijection of ranks to vocabulary entries (hot terms of every kind)
    perm = r.permutation(n_vocab)
    picks = perm[ranks]
    vlen = np.array([len(v) for v in vocab], dtype=np.int64)
    voff = np.zeros(n_vocab + 1, dtype=np.int64)
    voff[1:] = np.cumsum(vlen)
    vbytes = np.frombuffer(b"".join(vocab), dtype=np.uint8)
    off = np.zeros(n_terms + 1, dtype=np.int64)
    off[1:] = np.cumsum(vlen[picks])
    # gather every picked term's bytes: position j of the output takes byte
    # (j - off[i]) of term i
    owner = np.repeat(np.arange(n_terms, dtype=np.int64), vlen[picks])
    src = voff[picks][owner] + (np.arange(off[-1], dtype=np.int64) - off[:-1][owner])
    return vbytes[src].copy(), off, vocab
