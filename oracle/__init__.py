"""CPU oracle for the MapReduce-based join of SPARQL partial-match tables.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import, call, link or run
anything in this package.  The product path (``paper_1702_03484_amd`` and
``libmapsq.so``) never touches it and shares no code with it.

Contents
--------
``core``      plain numpy definitions: pattern matching (map), sort-merge
              join, nested-loop join, per-key counts, query evaluation,
              brute-force query evaluation, canonical row order and an
              order-independent multiset hash.
``hashjoin``  a plain C hash join (``hashjoin.c``, OpenMP) used as a second,
              independently written witness and for host timing.
``dictionary`` term <-> identifier encoding by its plain definition (a Python
              dict; identifiers dense, in order of first appearance).

Every function cites the passage of the paper it follows (Feng, Zhang and
Feng, "MapSQ: A MapReduce-based Framework for SPARQL Queries on GPU",
arXiv 1702.03484).  Parity pins: see the header of ``core``.
"""
from .core import (  # noqa: F401
    Table,
    match_pattern,
    pmt,
    join,
    join_on,
    join_on_cardinality,
    join_nested_loop,
    join_key_counts,
    join_cardinality,
    equality_filter,
    query,
    query_bruteforce,
    project,
    canonical_rows,
    multiset_hash,
)
