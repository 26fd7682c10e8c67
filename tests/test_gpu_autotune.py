"""The autotuner on the GPU: a tuned class is recorded and every candidate
launch shape gives the same rows in the same order."""
import json

import pytest
import torch

from paper_1702_03484_amd import autotune
from paper_1702_03484_amd import binding as B
from paper_1702_03484_amd.engine import MapSQ
from tests.conftest import announce

pytestmark = pytest.mark.gpu


def test_tuned_table_round_trip_and_same_rows(tmp_path):
    announce("autotune: one sort class and one materialisation class")
    out = tmp_path / "t.json"
    with MapSQ(arena_bytes=4 << 30, tuning=None) as s:
        table = autotune.autotune(s, [(20, 3 << 14)], [1 << 16], cache_path=str(out))
        assert set(table["sort"]) == {"20:16"} and set(table["materialize"]) == {"17"}
        assert autotune.install(s, str(out)) is True
        # a join materialised under every grid cap: identical columns
        g = torch.Generator(device="cuda").manual_seed(3)
        lk = torch.randint(0, 3000, (200_000,), generator=g, device="cuda", dtype=torch.int64).to(torch.int32)
        rk = torch.randint(0, 3000, (50_000,), generator=g, device="cuda", dtype=torch.int64).to(torch.int32)
        L = s.table([0, 1], [lk, torch.arange(lk.numel(), device="cuda", dtype=torch.int32)], key_max=2999)
        R = s.table([0, 2], [rk, torch.arange(rk.numel(), device="cuda", dtype=torch.int32)], key_max=2999)
        ref = None
        for cap in autotune.MAT_CANDIDATES:
            B.mapsq_set_mat_tuning(s.ctx, cap)
            t = s.join(L, R, 0)
            cols = [s.column(t, c).clone() for c in range(t.ncols)]
            s.free(t)
            if ref is None:
                ref = cols
            assert all(torch.equal(a, b) for a, b in zip(ref, cols)), cap
        B.mapsq_set_mat_tuning(s.ctx, 0)
    assert json.load(open(out))["kernel_source_sha256"]
