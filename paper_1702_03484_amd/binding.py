"""ctypes binding of libmapsq.so (include/mapsq.h).

Argument marshalling only: every step of the join runs in the library's HIP
kernels.  The functions keep the C names; a status other than MAPSQ_OK
raises :class:`MapSQError` carrying the code and the context's message.
PyTorch is used for device memory (the arena tensor) and the stream.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# MAPSQ_LIB=debug selects the bounds-checked build (libmapsq_debug.so); any
# other value is the path of another build of the library
_ENV_LIB = os.environ.get("MAPSQ_LIB", "")
LIB_PATH = (os.path.join(HERE, "libmapsq_debug.so") if _ENV_LIB == "debug"
            else _ENV_LIB or os.path.join(HERE, "libmapsq.so"))
MAX_COLS = 16

MAPSQ_OK = 0
MAPSQ_ERR_INVALID_ARG = -1
MAPSQ_ERR_UNSUPPORTED = -2
MAPSQ_ERR_CAPACITY = -3
MAPSQ_ERR_TOO_LARGE = -4
MAPSQ_ERR_HIP = -5
MAPSQ_ERR_STATE = -6
MAPSQ_PATH_SORT, MAPSQ_PATH_SEMIJOIN, MAPSQ_PATH_MERGE, MAPSQ_PATH_COMPOSITE = 0, 1, 2, 3
MAPSQ_LOAD_DEVICE_PTRS = 1
MAPSQ_LOAD_DEDUP = 2
MAPSQ_JOIN_INTO_SCRATCH_BYTES = 64 << 20
MAPSQ_JOIN_INTO_MAX_RECORDS = 1 << 21

ERROR_NAMES = {
    -1: "INVALID_ARG", -2: "UNSUPPORTED", -3: "CAPACITY", -4: "TOO_LARGE", -5: "HIP", -6: "STATE",
}


class mapsq_pattern(ctypes.Structure):
    _fields_ = [("s", ctypes.c_int32), ("p", ctypes.c_int32), ("o", ctypes.c_int32)]


class mapsq_table(ctypes.Structure):
    _fields_ = [
        ("nrows", ctypes.c_int64),
        ("ncols", ctypes.c_int32),
        ("owned", ctypes.c_int32),
        ("var", ctypes.c_int32 * MAX_COLS),
        ("col", ctypes.c_void_p * MAX_COLS),
        ("block", ctypes.c_uint64),
        ("key_max", ctypes.c_int32),
        ("sorted_col", ctypes.c_int32),
    ]

    @property
    def vars(self):
        return [int(self.var[i]) for i in range(self.ncols)]


class mapsq_store_facts(ctypes.Structure):
    _fields_ = [
        ("n_triples", ctypes.c_int64),
        ("n_predicates", ctypes.c_int64),
        ("max_id", ctypes.c_int32),
        ("id_bits", ctypes.c_int32),
        ("device_bytes", ctypes.c_uint64),
    ]


class mapsq_join_stats(ctypes.Structure):
    _fields_ = [
        ("left_rows", ctypes.c_int64),
        ("right_rows", ctypes.c_int64),
        ("segments", ctypes.c_int64),
        ("out_rows", ctypes.c_int64),
        ("radix_bits", ctypes.c_int32),
        ("passes", ctypes.c_int32),
        ("key_bits", ctypes.c_int32),
        ("path", ctypes.c_int32),
        ("sorted_records", ctypes.c_int64),
    ]


NPHASES = 9
PHASES = ["map", "sort", "count", "materialize", "filter", "index", "batch", "gather", "semijoin"]


class mapsq_profile(ctypes.Structure):
    _fields_ = [
        ("ms", ctypes.c_double * NPHASES),
        ("bytes", ctypes.c_double * NPHASES),
        ("launches", ctypes.c_int64 * NPHASES),
        ("joins", ctypes.c_int64),
        ("rows_out", ctypes.c_int64),
    ]


class mapsq_plan_step(ctypes.Structure):
    _fields_ = [
        ("pattern", ctypes.c_int32),
        ("key_var", ctypes.c_int32),
        ("rows", ctypes.c_int64),
        ("candidates", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]


MAPSQ_PLAN_SIZES, MAPSQ_PLAN_EXACT = 0, 1


class mapsq_join_desc(ctypes.Structure):
    _fields_ = [
        ("left", ctypes.POINTER(mapsq_table)),
        ("right", ctypes.POINTER(mapsq_table)),
        ("key_var", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]


class MapSQError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"mapsq {ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


_lib = None

# (name, restype, argtypes) of every exported symbol
_P = ctypes.c_void_p
_SIGS = [
    ("mapsq_create", ctypes.c_int32, [ctypes.c_int, _P, ctypes.c_size_t, _P, ctypes.POINTER(_P)]),
    ("mapsq_destroy", ctypes.c_int32, [_P]),
    ("mapsq_last_error", ctypes.c_char_p, [_P]),
    ("mapsq_load_triples", ctypes.c_int32, [_P, _P, _P, _P, ctypes.c_int64, ctypes.c_uint32]),
    ("mapsq_store_info", ctypes.c_int32, [_P, ctypes.POINTER(mapsq_store_facts)]),
    ("mapsq_predicate_stats", ctypes.c_int32,
     [_P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
      ctypes.POINTER(ctypes.c_int64)]),
    ("mapsq_map_pattern", ctypes.c_int32,
     [_P, ctypes.POINTER(mapsq_pattern), ctypes.c_int32, ctypes.POINTER(mapsq_table)]),
    ("mapsq_join", ctypes.c_int32,
     [_P, ctypes.POINTER(mapsq_table), ctypes.POINTER(mapsq_table), ctypes.c_int32, ctypes.POINTER(mapsq_table)]),
    ("mapsq_join_into", ctypes.c_int32,
     [_P, ctypes.POINTER(mapsq_table), ctypes.POINTER(mapsq_table), ctypes.c_int32, ctypes.POINTER(_P),
      ctypes.c_int64, ctypes.POINTER(mapsq_table)]),
    ("mapsq_query", ctypes.c_int32,
     [_P, ctypes.POINTER(mapsq_pattern), ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), ctypes.c_int32,
      ctypes.POINTER(mapsq_table)]),
    ("mapsq_join_batch", ctypes.c_int32,
     [_P, ctypes.POINTER(mapsq_join_desc), ctypes.c_int32, ctypes.POINTER(mapsq_table)]),
    ("mapsq_serve_config", ctypes.c_int32, [_P, ctypes.c_uint64, ctypes.c_int32]),
    ("mapsq_submit", ctypes.c_int32,
     [_P, ctypes.POINTER(mapsq_pattern), ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), ctypes.c_int32,
      ctypes.POINTER(ctypes.c_uint64)]),
    ("mapsq_serve_step", ctypes.c_int32, [_P, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]),
    ("mapsq_poll", ctypes.c_int32, [_P, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(mapsq_table)]),
    ("mapsq_poll_next", ctypes.c_int32,
     [_P, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(mapsq_table)]),
    ("mapsq_table_free", ctypes.c_int32, [_P, ctypes.POINTER(mapsq_table)]),
    ("mapsq_last_join_stats", ctypes.c_int32, [_P, ctypes.POINTER(mapsq_join_stats)]),
    ("mapsq_dict_create", ctypes.c_int32, [_P, ctypes.c_int64, ctypes.c_int64]),
    ("mapsq_dict_encode", ctypes.c_int32,
     [_P, _P, _P, ctypes.c_int64, ctypes.c_uint32, _P, ctypes.POINTER(ctypes.c_int64)]),
    ("mapsq_dict_decode", ctypes.c_int32,
     [_P, _P, ctypes.c_int64, ctypes.c_uint32, _P, _P, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]),
    ("mapsq_dict_info", ctypes.c_int32, [_P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]),
    ("mapsq_set_planner", ctypes.c_int32, [_P, ctypes.c_int32]),
    ("mapsq_last_plan", ctypes.c_int32,
     [_P, ctypes.POINTER(mapsq_plan_step), ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]),
    ("mapsq_set_tuning", ctypes.c_int32, [_P, ctypes.c_int32, ctypes.c_int32]),
    ("mapsq_set_join_options", ctypes.c_int32, [_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
    ("mapsq_profile_enable", ctypes.c_int32, [_P, ctypes.c_int32]),
    ("mapsq_profile_read", ctypes.c_int32, [_P, ctypes.POINTER(mapsq_profile)]),
    ("mapsq_tune_record", ctypes.c_int32, [_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
    ("mapsq_set_mat_tuning", ctypes.c_int32, [_P, ctypes.c_int32]),
    ("mapsq_tune_record_mat", ctypes.c_int32, [_P, ctypes.c_int32, ctypes.c_int32]),
    ("mapsq_arena_free_bytes", ctypes.c_int32, [_P, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64)]),
    ("mapsq_debug_fail_alloc", ctypes.c_int32, [_P, ctypes.c_int64]),
]
EXPORTED = [s[0] for s in _SIGS]


def lib():
    """The loaded library; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build the HIP library first "
                               "(python -c 'import __graft_entry__ as g; g.build()')")
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in _SIGS:
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(ctx, st):
    if st != MAPSQ_OK:
        msg = lib().mapsq_last_error(ctx).decode() if ctx else ""
        raise MapSQError(int(st), msg)


def mapsq_create(device: int, arena_ptr: int, arena_bytes: int, stream_ptr: int):
    out = _P()
    st = lib().mapsq_create(device, arena_ptr, arena_bytes, stream_ptr, ctypes.byref(out))
    if st != MAPSQ_OK:
        raise MapSQError(int(st), "mapsq_create failed")
    return out


def mapsq_destroy(ctx):
    _check(ctx, lib().mapsq_destroy(ctx))


def mapsq_last_error(ctx) -> str:
    return lib().mapsq_last_error(ctx).decode()


def mapsq_load_triples(ctx, s_ptr: int, p_ptr: int, o_ptr: int, n: int, flags: int = 0):
    _check(ctx, lib().mapsq_load_triples(ctx, s_ptr, p_ptr, o_ptr, n, flags))


def mapsq_store_info(ctx) -> mapsq_store_facts:
    out = mapsq_store_facts()
    _check(ctx, lib().mapsq_store_info(ctx, ctypes.byref(out)))
    return out


def mapsq_predicate_stats(ctx, predicate: int):
    """(triples, distinct subjects, distinct objects) of one predicate."""
    a, s, o = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    _check(ctx, lib().mapsq_predicate_stats(ctx, predicate, ctypes.byref(a), ctypes.byref(s), ctypes.byref(o)))
    return int(a.value), int(s.value), int(o.value)


def mapsq_map_pattern(ctx, pattern, key_var: int = -1) -> mapsq_table:
    pat = mapsq_pattern(*pattern)
    out = mapsq_table()
    _check(ctx, lib().mapsq_map_pattern(ctx, ctypes.byref(pat), key_var, ctypes.byref(out)))
    return out


def mapsq_join(ctx, left: mapsq_table, right: mapsq_table, key_var: int) -> mapsq_table:
    out = mapsq_table()
    _check(ctx, lib().mapsq_join(ctx, ctypes.byref(left), ctypes.byref(right), key_var, ctypes.byref(out)))
    return out


def mapsq_join_into(ctx, left: mapsq_table, right: mapsq_table, key_var: int, out_col_ptrs, out_capacity: int) -> mapsq_table:
    """out_col_ptrs: device addresses of the caller's output columns."""
    ptrs = (_P * max(1, len(out_col_ptrs)))(*out_col_ptrs)
    out = mapsq_table()
    _check(ctx, lib().mapsq_join_into(ctx, ctypes.byref(left), ctypes.byref(right), key_var, ptrs, out_capacity,
                                      ctypes.byref(out)))
    return out


def mapsq_query(ctx, patterns, select=None) -> mapsq_table:
    arr = (mapsq_pattern * len(patterns))(*[mapsq_pattern(*p) for p in patterns])
    sel = list(select or [])
    sarr = (ctypes.c_int32 * max(1, len(sel)))(*sel)
    out = mapsq_table()
    _check(ctx, lib().mapsq_query(ctx, arr, len(patterns), sarr, len(sel), ctypes.byref(out)))
    return out


def mapsq_join_batch(ctx, joins) -> list:
    """joins: list of (left table, right table, key variable)."""
    n = len(joins)
    descs = (mapsq_join_desc * max(1, n))()
    for i, (L, R, k) in enumerate(joins):
        descs[i].left = ctypes.pointer(L)
        descs[i].right = ctypes.pointer(R)
        descs[i].key_var = k
    outs = (mapsq_table * max(1, n))()
    _check(ctx, lib().mapsq_join_batch(ctx, descs, n, outs))
    return [outs[i] for i in range(n)]


def mapsq_serve_config(ctx, budget_bytes: int = 0, max_active: int = 0):
    _check(ctx, lib().mapsq_serve_config(ctx, budget_bytes, max_active))


def mapsq_submit(ctx, patterns, select=None) -> int:
    arr = (mapsq_pattern * len(patterns))(*[mapsq_pattern(*p) for p in patterns])
    sel = list(select or [])
    sarr = (ctypes.c_int32 * max(1, len(sel)))(*sel)
    t = ctypes.c_uint64()
    _check(ctx, lib().mapsq_submit(ctx, arr, len(patterns), sarr, len(sel), ctypes.byref(t)))
    return int(t.value)


def mapsq_serve_step(ctx):
    a, w = ctypes.c_int32(), ctypes.c_int32()
    _check(ctx, lib().mapsq_serve_step(ctx, ctypes.byref(a), ctypes.byref(w)))
    return int(a.value), int(w.value)


def mapsq_poll(ctx, ticket: int):
    """(done, table or None); raises MapSQError if the query failed."""
    d = ctypes.c_int32()
    out = mapsq_table()
    _check(ctx, lib().mapsq_poll(ctx, ticket, ctypes.byref(d), ctypes.byref(out)))
    return bool(d.value), (out if d.value else None)


def mapsq_poll_next(ctx):
    """(ticket, status, table or None) of the next query to end; ticket 0
    when none has.  A failed query comes back with its error status (no
    exception); invalid arguments raise MapSQError."""
    tk = ctypes.c_uint64()
    d = ctypes.c_int32()
    out = mapsq_table()
    st = lib().mapsq_poll_next(ctx, ctypes.byref(tk), ctypes.byref(d), ctypes.byref(out))
    if not d.value:
        _check(ctx, st)
        return 0, 0, None
    return int(tk.value), int(st), (out if st == 0 else None)


def mapsq_table_free(ctx, t: mapsq_table):
    _check(ctx, lib().mapsq_table_free(ctx, ctypes.byref(t)))


def mapsq_last_join_stats(ctx) -> mapsq_join_stats:
    out = mapsq_join_stats()
    _check(ctx, lib().mapsq_last_join_stats(ctx, ctypes.byref(out)))
    return out


def mapsq_set_join_options(ctx, semijoin: int = 0, merge: int = 0, precount: int = 0, composite: int = 0):
    """semijoin: 0 automatic, 1 never, 2 always; merge: 0 when both sides are
    sorted on the key, 1 never; precount (exact |RS| before sorting): 0 for
    shuffles of 2^24+ records unless a planned step's expected output is
    small, 1 never, 2 always; composite: 0 a second
    shared variable is part of the join key, 1 it is filtered afterwards."""
    _check(ctx, lib().mapsq_set_join_options(ctx, semijoin, merge, precount, composite))


MAPSQ_DICT_DEVICE_PTRS = 1
MAPSQ_DICT_LOOKUP = 2


def mapsq_dict_create(ctx, max_terms: int, max_bytes: int):
    _check(ctx, lib().mapsq_dict_create(ctx, max_terms, max_bytes))


def mapsq_dict_encode(ctx, bytes_ptr: int, offsets_ptr: int, n: int, flags: int, ids_ptr: int) -> int:
    """Pointers are host or device addresses (flags); returns the number of new terms."""
    nn = ctypes.c_int64(0)
    _check(ctx, lib().mapsq_dict_encode(ctx, bytes_ptr, offsets_ptr, n, flags, ids_ptr, ctypes.byref(nn)))
    return nn.value


def mapsq_dict_decode(ctx, ids_ptr: int, n: int, flags: int, offsets_ptr: int, bytes_ptr: int, cap_bytes: int) -> int:
    """Returns the byte count written (raises TOO_LARGE with the need in the message)."""
    need = ctypes.c_int64(0)
    _check(ctx, lib().mapsq_dict_decode(ctx, ids_ptr, n, flags, offsets_ptr, bytes_ptr, cap_bytes, ctypes.byref(need)))
    return need.value


def mapsq_dict_need(ctx, ids_ptr: int, n: int, flags: int, offsets_ptr: int) -> int:
    """Bytes a decode of these identifiers needs (a decode with no room)."""
    need = ctypes.c_int64(0)
    st = lib().mapsq_dict_decode(ctx, ids_ptr, n, flags, offsets_ptr, None, 0, ctypes.byref(need))
    if st not in (MAPSQ_OK, MAPSQ_ERR_TOO_LARGE):
        _check(ctx, st)
    return need.value


def mapsq_dict_info(ctx):
    t, b = ctypes.c_int64(0), ctypes.c_int64(0)
    _check(ctx, lib().mapsq_dict_info(ctx, ctypes.byref(t), ctypes.byref(b)))
    return t.value, b.value


def mapsq_set_planner(ctx, mode: int):
    _check(ctx, lib().mapsq_set_planner(ctx, mode))


def mapsq_last_plan(ctx) -> list:
    """The last query's plan: [(pattern, key_var, rows, candidates counted), ...]."""
    n = ctypes.c_int32(0)
    _check(ctx, lib().mapsq_last_plan(ctx, None, 0, ctypes.byref(n)))
    steps = (mapsq_plan_step * max(1, n.value))()
    _check(ctx, lib().mapsq_last_plan(ctx, steps, n.value, ctypes.byref(n)))
    return [(s.pattern, s.key_var, int(s.rows), s.candidates) for s in steps[:n.value]]


def mapsq_set_tuning(ctx, radix_bits: int = 0, keys_per_thread: int = 0):
    _check(ctx, lib().mapsq_set_tuning(ctx, radix_bits, keys_per_thread))


def mapsq_profile_enable(ctx, on: bool = True):
    _check(ctx, lib().mapsq_profile_enable(ctx, 1 if on else 0))


def mapsq_profile_read(ctx) -> mapsq_profile:
    out = mapsq_profile()
    _check(ctx, lib().mapsq_profile_read(ctx, ctypes.byref(out)))
    return out


def mapsq_tune_record(ctx, key_bits: int, log2_records: int, radix_bits: int, keys_per_thread: int):
    _check(ctx, lib().mapsq_tune_record(ctx, key_bits, log2_records, radix_bits, keys_per_thread))


def mapsq_set_mat_tuning(ctx, max_blocks: int = 0):
    _check(ctx, lib().mapsq_set_mat_tuning(ctx, max_blocks))


def mapsq_tune_record_mat(ctx, log2_rows: int, max_blocks: int):
    _check(ctx, lib().mapsq_tune_record_mat(ctx, log2_rows, max_blocks))


def mapsq_arena_free_bytes(ctx):
    a = ctypes.c_uint64()
    b = ctypes.c_uint64()
    _check(ctx, lib().mapsq_arena_free_bytes(ctx, ctypes.byref(a), ctypes.byref(b)))
    return int(a.value), int(b.value)


def mapsq_debug_fail_alloc(ctx, after: int):
    _check(ctx, lib().mapsq_debug_fail_alloc(ctx, after))


def make_table(vars, col_ptrs, nrows: int, key_max: int = -1, sorted_col: int = 0) -> mapsq_table:
    """A caller-owned table (owned = 0) over existing device columns;
    sorted_col = 1 + a column the caller guarantees to be ascending, or 0."""
    t = mapsq_table()
    t.nrows = nrows
    t.ncols = len(vars)
    t.owned = 0
    t.key_max = key_max
    t.sorted_col = sorted_col
    for i, (v, p) in enumerate(zip(vars, col_ptrs)):
        t.var[i] = v
        t.col[i] = p
    return t
