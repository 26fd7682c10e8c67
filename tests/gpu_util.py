"""Helpers of the GPU parity tests: bring a library table to the host and
compare it with the oracle as a bag of rows (exact, int32)."""
import numpy as np

import oracle
from oracle.core import Table


def host_table(sess, t) -> Table:
    cols = sess.to_numpy(t)
    return Table(list(t.vars), cols, n=int(t.nrows))


def assert_same_bag(got: Table, exp: Table, var_order=None):
    vs = list(exp.vars) if var_order is None else list(var_order)
    assert sorted(got.vars) == sorted(exp.vars), (got.vars, exp.vars)
    assert got.n == exp.n, f"row count {got.n} != {exp.n}"
    a = oracle.canonical_rows(got, vs)
    b = oracle.canonical_rows(exp, vs)
    assert np.array_equal(a, b)


def oracle_table_of(vars, cols) -> Table:
    return Table(list(vars), [np.asarray(c) for c in cols])
