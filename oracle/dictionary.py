"""Dictionary encoding of RDF terms (test infrastructure only).

TEST INFRASTRUCTURE ONLY: only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may use this module.

Table 1 of the paper writes the running example with string terms (Anny,
Jim, Susan, hasJob, workAt, "Hospital", ...) while the join works on their
identifiers: a dictionary maps every distinct term to one integer and back.
This is its plain definition, with the reading the library takes: a term is
a byte string, identifiers are dense (0, 1, 2, ...) and given in order of
first appearance, and a dictionary grows by appending the terms it has not
seen, in the order they first appear in the new batch.
"""
from __future__ import annotations

import numpy as np


def split_terms(data: bytes, offsets) -> list:
    """The byte strings data[offsets[i]:offsets[i+1]]."""
    off = [int(x) for x in offsets]
    return [bytes(data[off[i]:off[i + 1]]) for i in range(len(off) - 1)]


def join_terms(terms) -> tuple:
    """(bytes, int64 offsets) of a list of byte strings, back to back."""
    off = np.zeros(len(terms) + 1, dtype=np.int64)
    off[1:] = np.cumsum([len(t) for t in terms], dtype=np.int64)
    return b"".join(terms), off


def encode(terms, known: list | None = None) -> tuple:
    """Identifiers of ``terms`` under the dictionary ``known`` (a list whose
    index is the identifier), extended by every term it lacks in order of
    first appearance.  Returns (ids as int32, the extended dictionary)."""
    table = list(known or [])
    index = {t: i for i, t in enumerate(table)}
    ids = np.empty(len(terms), dtype=np.int32)
    for i, t in enumerate(terms):
        if t not in index:
            index[t] = len(table)
            table.append(t)
        ids[i] = index[t]
    return ids, table


def lookup(terms, known: list) -> np.ndarray:
    """Identifiers of ``terms`` in ``known`` without adding any (-1: absent)."""
    index = {t: i for i, t in enumerate(known)}
    return np.array([index.get(t, -1) for t in terms], dtype=np.int32)


def decode(ids, known: list) -> list:
    """The terms of the identifiers ``ids``."""
    return [known[int(i)] for i in ids]
