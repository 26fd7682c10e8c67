"""A small session object over the C ABI: it owns the torch arena tensor and
uses torch's current HIP stream, and turns result columns into tensors.

Every computation is a libmapsq.so call; this module only marshals.
"""
from __future__ import annotations

import numpy as np
import torch

from . import binding as B


_DEFAULT_TUNING = "default"


class MapSQ:
    def __init__(self, arena_bytes: int = 8 << 30, device: int = 0, stream: torch.cuda.Stream | None = None,
                 tuning: str | None = _DEFAULT_TUNING):
        """tuning: a JSON table written by ``python -m paper_1702_03484_amd.autotune``
        (default: the one shipped with the package, if present; None: no table)."""
        if not torch.cuda.is_available():
            raise RuntimeError("MapSQ needs a GPU (gfx950); there is no CPU path")
        self.device = device
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=f"cuda:{device}")
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        self.ctx = B.mapsq_create(device, self.arena.data_ptr(), self.arena.numel(), self.stream.cuda_stream)
        self._keep = []
        if tuning is not None:
            from . import autotune

            autotune.install(self, autotune.DEFAULT_TABLE if tuning == _DEFAULT_TUNING else tuning)

    def close(self):
        """Destroy the context and drop the arena and kept tensors (returned
        to the device, not kept in torch's cache: arenas are large)."""
        if self.ctx is not None:
            B.mapsq_destroy(self.ctx)
            self.ctx = None
        self.arena = None
        self._keep.clear()
        torch.cuda.empty_cache()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # ---- store ------------------------------------------------------------
    def load(self, s, p, o, dedup: bool = False):
        flags = B.MAPSQ_LOAD_DEDUP if dedup else 0
        if isinstance(s, torch.Tensor) and s.is_cuda:
            cols = [x.contiguous().to(torch.int32) for x in (s, p, o)]
            flags |= B.MAPSQ_LOAD_DEVICE_PTRS
            ptrs = [c.data_ptr() for c in cols]
            n = cols[0].numel()
        else:
            cols = [np.ascontiguousarray(x, dtype=np.int32) for x in (s, p, o)]
            ptrs = [c.ctypes.data for c in cols]
            n = cols[0].size
        B.mapsq_load_triples(self.ctx, *ptrs, n, flags)
        return B.mapsq_store_info(self.ctx)

    # ---- the path ---------------------------------------------------------
    def map(self, pattern, key_var: int = -1) -> B.mapsq_table:
        return B.mapsq_map_pattern(self.ctx, pattern, key_var)

    def join(self, left: B.mapsq_table, right: B.mapsq_table, key_var: int) -> B.mapsq_table:
        return B.mapsq_join(self.ctx, left, right, key_var)

    def query(self, patterns, select=None) -> B.mapsq_table:
        return B.mapsq_query(self.ctx, patterns, select)

    def join_batch(self, joins) -> list:
        """joins: list of (left, right, key_var); one batched launch."""
        return B.mapsq_join_batch(self.ctx, joins)

    def free(self, t: B.mapsq_table):
        B.mapsq_table_free(self.ctx, t)

    def stats(self) -> B.mapsq_join_stats:
        return B.mapsq_last_join_stats(self.ctx)

    # ---- term dictionary -----------------------------------------------------
    def dict_create(self, max_terms: int, max_bytes: int):
        B.mapsq_dict_create(self.ctx, max_terms, max_bytes)

    def dict_encode(self, data, offsets, lookup: bool = False):
        """Identifiers of the terms data[offsets[i]:offsets[i+1]]: numpy
        buffers (host path, returns numpy) or device tensors (uint8 data,
        int64 offsets; returns an int32 tensor).  Returns (ids, new terms)."""
        flags = B.MAPSQ_DICT_LOOKUP if lookup else 0
        if isinstance(offsets, torch.Tensor):
            assert offsets.is_cuda and offsets.dtype == torch.int64 and data.dtype == torch.uint8
            n = offsets.numel() - 1
            ids = torch.empty(max(n, 1), dtype=torch.int32, device=offsets.device)
            new = B.mapsq_dict_encode(self.ctx, data.data_ptr(), offsets.data_ptr(), n,
                                      flags | B.MAPSQ_DICT_DEVICE_PTRS, ids.data_ptr())
            return ids[:n], new
        if isinstance(data, (bytes, bytearray)):
            data = np.frombuffer(data, dtype=np.uint8)
        data = np.ascontiguousarray(data, dtype=np.uint8)
        offsets = np.ascontiguousarray(offsets, dtype=np.int64)
        n = offsets.size - 1
        ids = np.empty(max(n, 1), dtype=np.int32)
        new = B.mapsq_dict_encode(self.ctx, data.ctypes.data if data.size else None, offsets.ctypes.data, n, flags,
                                  ids.ctypes.data)
        return ids[:n], new

    def dict_decode(self, ids):
        """(bytes, int64 offsets) of the terms of `ids` (numpy int32 on the
        host, or an int32 device tensor: then device tensors come back)."""
        if isinstance(ids, torch.Tensor):
            ids = ids.contiguous()
            n = ids.numel()
            off = torch.empty(n + 1, dtype=torch.int64, device=ids.device)
            need = B.mapsq_dict_need(self.ctx, ids.data_ptr(), n, B.MAPSQ_DICT_DEVICE_PTRS, off.data_ptr())
            out = torch.empty(max(need, 1), dtype=torch.uint8, device=ids.device)
            B.mapsq_dict_decode(self.ctx, ids.data_ptr(), n, B.MAPSQ_DICT_DEVICE_PTRS, off.data_ptr(), out.data_ptr(),
                                need)
            return out[:need], off
        ids = np.ascontiguousarray(ids, dtype=np.int32)
        n = ids.size
        off = np.empty(n + 1, dtype=np.int64)
        need = B.mapsq_dict_need(self.ctx, ids.ctypes.data, n, 0, off.ctypes.data)
        out = np.empty(max(need, 1), dtype=np.uint8)
        B.mapsq_dict_decode(self.ctx, ids.ctypes.data, n, 0, off.ctypes.data, out.ctypes.data, need)
        return out[:need].tobytes(), off

    def dict_info(self):
        return B.mapsq_dict_info(self.ctx)

    def set_planner(self, exact: bool):
        """mapsq_query join order from exact join sizes counted on the GPU
        (True) or from pattern sizes (False, the default)."""
        B.mapsq_set_planner(self.ctx, B.MAPSQ_PLAN_EXACT if exact else B.MAPSQ_PLAN_SIZES)

    def last_plan(self) -> list:
        return B.mapsq_last_plan(self.ctx)

    def set_tuning(self, radix_bits: int = 0, keys_per_thread: int = 0):
        B.mapsq_set_tuning(self.ctx, radix_bits, keys_per_thread)

    # ---- tables <-> tensors -------------------------------------------------

    def set_join_options(self, semijoin: int = 0, merge: int = 0, precount: int = 0, composite: int = 0):
        """semijoin 0 automatic / 1 never / 2 always; merge 0 automatic / 1 never;
        precount 0 shuffles of 2^24+ records (not planned steps with a small
        expected output) / 1 never / 2 always; composite 0
        a second shared variable joins as part of the key / 1 filtered after."""
        B.mapsq_set_join_options(self.ctx, semijoin, merge, precount, composite)


    def table(self, vars, tensors, key_max: int = -1, sorted_col: int = 0) -> B.mapsq_table:
        """Wrap caller-owned int32 device tensors (kept alive by this session);
        sorted_col = 1 + a column the caller guarantees to be ascending."""
        ts = [t.contiguous() for t in tensors]
        assert all(t.dtype == torch.int32 and t.is_cuda for t in ts)
        n = ts[0].numel() if ts else 0
        self._keep.extend(ts)
        return B.make_table(vars, [t.data_ptr() for t in ts], n, key_max, sorted_col)

    def column(self, t: B.mapsq_table, c: int) -> torch.Tensor:
        """Column c of a table as an int32 tensor view (no copy)."""
        n = int(t.nrows)
        if n == 0:
            return torch.empty(0, dtype=torch.int32, device=self.arena.device)
        ptr = int(t.col[c])
        off = ptr - self.arena.data_ptr()
        if 0 <= off and off + 4 * n <= self.arena.numel():
            return self.arena[off:off + 4 * n].view(torch.int32)
        for k in self._keep:
            if k.data_ptr() <= ptr and ptr + 4 * n <= k.data_ptr() + 4 * k.numel():
                i = (ptr - k.data_ptr()) // 4
                return k[i:i + n]
        raise ValueError("column is outside the arena and the wrapped tensors")

    def to_numpy(self, t: B.mapsq_table):
        torch.cuda.current_stream(self.device).synchronize()
        return [self.column(t, c).cpu().numpy() for c in range(t.ncols)]
