"""The join-order planners of mapsq_query on the GPU: the plan from pattern
sizes (default) and the plan from exact join sizes counted on the GPU.
Both must give the oracle's bag; the exact planner's every step must be a
candidate whose exact |RS| (recomputed here with the oracle) is the
smallest, and the reported plan must name every pattern once with the row
count each step produced."""
import numpy as np
import pytest

import oracle
from oracle.core import Table
from synth import random_store, var
from tests.conftest import announce
from tests.gpu_util import assert_same_bag, host_table
from tests.test_gpu_join import _random_queries

pytestmark = pytest.mark.gpu


def shared_in_order(qvars, a, b):
    return [v for v in qvars if v in a.vars and v in b.vars]


def check_exact_plan(w, pats, plan):
    """Replays the plan with the oracle: step 0 is the start pattern, and at
    every join step the picked pattern's exact |RS| with the running result
    is the smallest over the connected candidates (the first step: over all
    connected pairs), and equals the rows the step reported."""
    qvars = oracle.core.query_vars(pats)
    tabs = [oracle.match_pattern(w.s, w.p, w.o, p) for p in pats]
    m = len(pats)
    assert sorted(s[0] for s in plan) == list(range(m))
    start = plan[0][0]
    assert plan[0][2] == tabs[start].n
    if m > 2 and len(plan) > 1 and plan[1][1] >= 0:
        sizes = [oracle.join_on_cardinality(tabs[i], tabs[j], shared_in_order(qvars, tabs[i], tabs[j]))
                 for i in range(m) for j in range(i + 1, m) if shared_in_order(qvars, tabs[i], tabs[j])]
        assert plan[1][2] == min(sizes), (plan, sizes)
    cur = tabs[start]
    done = {start}
    for k, (pick, key, rows, cand) in enumerate(plan[1:], 1):
        if key >= 0:
            sh = shared_in_order(qvars, cur, tabs[pick])
            assert sh and sh[0] == key
            if k > 1:
                sizes = [oracle.join_on_cardinality(cur, tabs[j], shared_in_order(qvars, cur, tabs[j]))
                         for j in range(m) if j not in done and shared_in_order(qvars, cur, tabs[j])]
                assert cand == len(sizes) and rows == min(sizes), (plan, sizes)
            cur = oracle.join_on(cur, tabs[pick], sh)
        else:
            assert not any(shared_in_order(qvars, cur, tabs[j]) for j in range(m) if j not in done)
            cur = oracle.core.cross(cur, tabs[pick])
        assert rows == cur.n
        done.add(pick)


def test_exact_planner_picks_the_smallest_join_and_matches_the_oracle(sess):
    w = random_store(43, 20_000, 400, 5)
    sess.load(w.s, w.p, w.o)
    sess.set_planner(True)
    done = 0
    try:
        for pats in _random_queries(w, 6, 60):
            if len(pats) < 3:
                continue
            exp = oracle.query(w.s, w.p, w.o, pats)
            if exp.n > 5_000_000:
                continue
            announce(f"exact planner: query {pats}")
            got = sess.query(pats)
            plan = sess.last_plan()
            assert_same_bag(host_table(sess, got), exp)
            sess.free(got)
            check_exact_plan(w, pats, plan)
            assert any(s[3] > 0 for s in plan[1:])
            done += 1
    finally:
        sess.set_planner(False)
    assert done >= 15


def test_size_planner_reports_its_plan(sess):
    """The default plan starts from the smallest partial-match table and
    takes the smallest connected table next; nothing is counted."""
    w = random_store(44, 5000, 80, 3)
    sess.load(w.s, w.p, w.o)
    e = w.n_entities
    pats = [(var(0), e, var(1)), (var(1), e + 1, var(2)), (var(2), e + 2, int(w.o[w.p == e + 2][0]))]
    announce(f"size planner plan of {pats}")
    t = sess.query(pats)
    plan = sess.last_plan()
    exp = oracle.query(w.s, w.p, w.o, pats)
    assert_same_bag(host_table(sess, t), exp)
    sess.free(t)
    sizes = [oracle.match_pattern(w.s, w.p, w.o, p).n for p in pats]
    assert plan[0] == (int(np.argmin(sizes)), -1, min(sizes), 0)
    assert [s[3] for s in plan] == [0, 0, 0] and plan[-1][2] == exp.n


def test_exact_planner_on_a_star_and_link_query(sess):
    """cfg-3-shaped query on a small store: a subject star on ?x and an
    object-object link on ?y.  Both plans give the bag; the exact plan's
    first join is the smallest connected pair, so it is never larger than
    the size plan's first join."""
    w = random_store(45, 200_000, 3000, 6)
    sess.load(w.s, w.p, w.o)
    e = w.n_entities
    c = int(np.bincount(w.o[w.p == e + 2]).argmax())
    pats = [(var(0), e, var(1)), (var(0), e + 1, var(2)), (var(0), e + 2, c), (var(3), e + 3, var(1))]
    announce(f"star + link: {pats}")
    exp = oracle.query(w.s, w.p, w.o, pats)
    res = {}
    for exact in (False, True):
        sess.set_planner(exact)
        t = sess.query(pats)
        res[exact] = sess.last_plan()
        assert_same_bag(host_table(sess, t), exp)
        sess.free(t)
    sess.set_planner(False)
    check_exact_plan(w, pats, res[True])
    assert res[True][1][2] <= res[False][1][2], res
