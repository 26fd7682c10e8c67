"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the
benchmark.

This package only draws data: dictionary-encoded int32 triple stores, the
triple patterns of the queries run over them, random partial-match tables,
and streams of RDF-shaped string terms.  It contains none of the join's arithmetic (no map, no sort, no
per-key counting of the join itself), so that neither side of a parity test
can inherit a mistake from it.
"""
from .gen import (  # noqa: F401
    Workload,
    zipf_bounded,
    scramble_ids,
    store_cfg1,
    store_cfg2,
    store_cfg3,
    query_cfg3,
    random_store,
    random_table,
    batch_cfg4,
    cfg4_vars,
    serving_cfg5,
    store_cfg5,
    var,
    rdf_terms,
)
