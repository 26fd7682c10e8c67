"""The C-ABI library loads and exports every entry point that include/mapsq.h declares (no GPU needed)."""
import ctypes
import os
import re

from paper_1702_03484_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    txt = open(os.path.join(ROOT, "include", "mapsq.h")).read()
    return sorted(set(re.findall(r"^(?:mapsq_status|const char\*)\s+(mapsq_\w+)\(", txt, re.M)))


def test_header_declares_the_boundary():
    names = declared()
    for n in ["mapsq_load_triples", "mapsq_map_pattern", "mapsq_join", "mapsq_query"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(binding.LIB_PATH)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(declared()) == sorted(binding.EXPORTED)


def test_struct_layout_matches_header():
    # mapsq_table: int64 + 2*int32 + 16*int32 + 16*ptr + uint64 + 2*int32
    assert ctypes.sizeof(binding.mapsq_table) == 8 + 8 + 64 + 128 + 8 + 8
    assert ctypes.sizeof(binding.mapsq_pattern) == 12
    assert ctypes.sizeof(binding.mapsq_join_stats) == 4 * 8 + 4 * 4 + 8


def test_null_context_is_rejected_without_gpu_work():
    lib = binding.lib()
    assert lib.mapsq_destroy(None) == 0
    assert lib.mapsq_join(None, None, None, 0, None) == binding.MAPSQ_ERR_INVALID_ARG
    assert lib.mapsq_last_error(None) == b"null context"
    out = ctypes.c_void_p(1)
    # NULL arena: INVALID_ARG before any device call
    assert lib.mapsq_create(0, None, 1 << 30, None, ctypes.byref(out)) == binding.MAPSQ_ERR_INVALID_ARG
    assert out.value is None


def test_every_context_call_rejects_a_null_context():
    """Each call that takes a context returns INVALID_ARG for NULL before any
    device work (all other arguments zero or NULL)."""
    lib = binding.lib()
    checked = 0
    for name, res, args in binding._SIGS:
        if args[:1] != [binding._P] or name in ("mapsq_destroy", "mapsq_last_error"):
            continue
        fn = getattr(lib, name)
        vals = [None] + [0 if a in (ctypes.c_int, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32,
                                    ctypes.c_uint64, ctypes.c_size_t, ctypes.c_double) else None
                         for a in args[1:]]
        assert fn(*vals) == binding.MAPSQ_ERR_INVALID_ARG, name
        checked += 1
    assert checked >= 20
