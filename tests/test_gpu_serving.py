"""Serving: each result is the same alone and in the mix (exact, row for
row), admission by predicted bytes, and agreement with the oracle."""
import numpy as np
import pytest

import oracle
from paper_1702_03484_amd import binding as B
from paper_1702_03484_amd import serving
from synth import serving_cfg5, store_cfg5
from tests.conftest import announce
from tests.gpu_util import assert_same_bag
from oracle.core import Table

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def served(sess):
    w = store_cfg5(n=4_000_000, n_entities=800_000)
    sess.load(w.s, w.p, w.o)
    qs = serving_cfg5(w, 120, sample=2_000_000)
    return w, qs


def _alone(sess, qs):
    out = {}
    for j, q in enumerate(qs):
        try:
            t = B.mapsq_query(sess.ctx, q)
        except B.MapSQError as e:
            out[j] = e.code
            continue
        out[j] = (list(t.vars), sess.to_numpy(t))
        B.mapsq_table_free(sess.ctx, t)
    return out


def test_results_alone_equal_results_in_the_mix(sess, served):
    w, qs = served
    announce(f"serving: {len(qs)} queries alone vs all at once vs Poisson arrivals")
    alone = _alone(sess, qs)
    ok = [j for j in alone if not isinstance(alone[j], int)]
    assert len(ok) >= len(qs) // 2
    for arrivals in (np.zeros(len(qs)), serving.poisson_arrivals(1, len(qs), 2000.0)):
        got = {}
        summ, lat, status = serving.run_continuous(sess, qs, arrivals, collect=got)
        assert summ["rounds"] >= 1
        for j in ok:
            assert status[j] == 0, (j, status[j])
            gv, gc = got[j]
            av, ac = alone[j]
            assert gv == av
            if not all(np.array_equal(a, b) for a, b in zip(gc, ac)):
                same_bag = np.array_equal(oracle.canonical_rows(Table(gv, gc, n=len(gc[0]))),
                                          oracle.canonical_rows(Table(av, ac, n=len(ac[0]))))
                raise AssertionError(f"query {j} {qs[j]} differs in the mix: rows {len(gc[0])} vs {len(ac[0])}, "
                                     f"same bag: {same_bag}")


def test_served_results_match_the_oracle(sess, served):
    w, qs = served
    announce("serving: results up to 5M rows against the oracle")
    got = {}
    serving.run_continuous(sess, qs[:60], np.zeros(60), collect=got)
    checked = 0
    for j, (vs, cols) in got.items():
        if cols and len(cols[0]) > 5_000_000:
            continue
        try:
            exp = oracle.query(w.s, w.p, w.o, qs[j], max_rows=20_000_000)
        except OverflowError:  # the oracle's fixed order would build a huge intermediate
            continue
        assert_same_bag(Table(vs, cols, n=len(cols[0]) if cols else 0), exp)
        checked += 1
    assert checked >= 20


def test_admission_budget_rejects_only_what_cannot_fit(sess, served):
    w, qs = served
    announce("serving: tiny admission budget")
    summ, lat, status = serving.run_continuous(sess, qs[:40], np.zeros(40), budget_bytes=1 << 20, max_active=4)
    assert summ["completed"] + summ["rejected"] == 40
    assert summ["completed"] > 0
    B.mapsq_serve_config(sess.ctx, 0, 0)


def test_plain_and_continuous_agree(sess, served):
    w, qs = served
    announce("serving: plain form vs continuous batching")
    a, b = {}, {}
    serving.run_plain(sess, qs[:50], np.zeros(50), collect=a)
    serving.run_continuous(sess, qs[:50], np.zeros(50), collect=b)
    assert a.keys() == b.keys()
    for j in a:
        assert a[j][0] == b[j][0]
        assert all(np.array_equal(x, y) for x, y in zip(a[j][1], b[j][1]))


def test_tight_arena_mix_completes_what_completes_alone(sess, served):
    """In an arena where the largest result fits alone but not beside the
    others, every query that completes alone completes in the saturated mix
    with the same rows (it waits for memory instead of failing)."""
    from paper_1702_03484_amd.engine import MapSQ

    w, qs = served
    big_alone = _alone(sess, qs)
    size = {j: 4 * len(v[1][0]) * len(v[1]) for j, v in big_alone.items() if not isinstance(v, int) and v[1]}
    big = max(size.values())
    free, _ = B.mapsq_arena_free_bytes(sess.ctx)
    footprint = (48 << 30) - free
    arena = footprint + 2 * big + (256 << 20)
    announce(f"serving: tight arena of {arena >> 20} MiB, largest result {big >> 20} MiB")
    with MapSQ(arena_bytes=arena) as tight:
        tight.load(w.s, w.p, w.o)
        alone = _alone(tight, qs)
        ok = [j for j in alone if not isinstance(alone[j], int)]
        assert any(size.get(j, 0) >= big // 2 for j in ok)
        got = {}
        summ, lat, status = serving.run_continuous(tight, qs, np.zeros(len(qs)), collect=got)
        announce(f"serving: tight arena: {len(ok)} complete alone, {summ['completed']} in the mix")
        for j in ok:
            assert status[j] == 0, (j, int(status[j]), qs[j])
            assert got[j][0] == alone[j][0]
            assert all(np.array_equal(a, b) for a, b in zip(got[j][1], alone[j][1])), j
        memory = (B.MAPSQ_ERR_CAPACITY, B.MAPSQ_ERR_TOO_LARGE)
        for j in range(len(qs)):
            if j not in ok:  # serving reports every memory failure as TOO_LARGE
                want = B.MAPSQ_ERR_TOO_LARGE if alone[j] in memory else alone[j]
                assert status[j] == want, (j, int(status[j]), alone[j])


def test_poll_next_returns_each_finished_query_once(sess, served):
    w, qs = served
    announce("serving: mapsq_poll_next after mapsq_poll")
    tickets = [B.mapsq_submit(sess.ctx, q) for q in qs[:12]]
    for _ in range(10_000):
        active, waiting = B.mapsq_serve_step(sess.ctx)
        if active == 0 and waiting == 0:
            break
    assert active == 0 and waiting == 0
    try:  # retired here: poll_next skips it
        done, t = B.mapsq_poll(sess.ctx, tickets[3])
    except B.MapSQError:  # a query that failed is retired too
        done, t = True, None
    assert done
    if t is not None:
        B.mapsq_table_free(sess.ctx, t)
    seen = []
    while True:
        tk, st, t = B.mapsq_poll_next(sess.ctx)
        if not tk:
            break
        seen.append(tk)
        assert (st == 0) == (t is not None)
        if t is not None:
            B.mapsq_table_free(sess.ctx, t)
    assert sorted(seen) == sorted(tickets[:3] + tickets[4:])
    assert B.mapsq_poll_next(sess.ctx) == (0, 0, None)
