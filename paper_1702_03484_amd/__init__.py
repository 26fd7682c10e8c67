"""MI355X (gfx950) implementation of MapSQ's MapReduce-based join of SPARQL
partial-match tables (Feng, Zhang and Feng, arXiv 1702.03484).

``binding`` is the ctypes layer over ``libmapsq.so`` (C ABI in
``include/mapsq.h``); ``engine.MapSQ`` is a session that owns the torch
arena.  Importing ``engine`` needs torch; ``binding`` does not.
"""
from . import binding  # noqa: F401
