"""The bounds-checked build (libmapsq_debug.so, compiled with -DMQ_DEBUG).

Seeded cases of every path (shuffled, semi-join, merge and composite-key
joins, a batch with filtered joins, a map scan and a three-pattern query)
run through the debug library in a child process (the binding loads it
when MAPSQ_LIB=debug).  The run must print no bounds report, and every
result must equal the oracle's as a bag: the checks see only in-range
indices and change nothing.
"""
import os
import subprocess
import sys

import numpy as np
import pytest

import oracle
from oracle.core import Table
from tests import debug_workload as W
from tests.conftest import ROOT, announce
from tests.gpu_util import assert_same_bag

pytestmark = pytest.mark.gpu
LIB = os.path.join(ROOT, "paper_1702_03484_amd", "libmapsq_debug.so")


def _load(d, name) -> Table:
    z = np.load(os.path.join(d, name + ".npz"))
    vs = [int(v) for v in z["vars"]]
    cols = [z[f"arr_{i}"] for i in range(len(vs))]
    return Table(vs, cols, n=len(cols[0]) if cols else 0)


def test_debug_build_runs_clean(tmp_path):
    if not os.path.exists(LIB):
        pytest.skip("libmapsq_debug.so is not built (python -m paper_1702_03484_amd.build --debug)")
    announce("bounds-checked build: every path on seeded cases (child process)")
    env = dict(os.environ, MAPSQ_LIB="debug")
    r = subprocess.run([sys.executable, "-u", os.path.join(ROOT, "tests", "debug_workload.py"), str(tmp_path)],
                       env=env, capture_output=True, text=True, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-3000:]
    assert "workload done" in out, out[-3000:]
    assert "mapsq bounds check" not in out, out[-3000:]
    c = W.inputs()
    for name in ("shuffle", "semijoin", "merge"):
        (lv, lc), (rv, rc), key, _ = c[name]
        assert_same_bag(_load(tmp_path, name), oracle.join(Table(lv, lc), Table(rv, rc), key))
    (lv, lc), (rv, rc), key, _ = c["composite"]
    assert_same_bag(_load(tmp_path, "composite"), oracle.join_on(Table(lv, lc), Table(rv, rc), [0, 10]))
    for i, ((lv, lc), (rv, rc)) in enumerate(c["batch"]):
        assert_same_bag(_load(tmp_path, f"batch{i}"), oracle.join(Table(lv, lc), Table(rv, rc), 0))
    s, p, o = c["store"]
    assert_same_bag(_load(tmp_path, "map"), oracle.match_pattern(s, p, o, c["map"]))
    assert_same_bag(_load(tmp_path, "query"), oracle.query(s, p, o, c["query"]))
