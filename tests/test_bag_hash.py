"""The torch bag hash used by the full-size parity tests equals the
oracle's multiset_hash (CPU here; on the device in the GPU variant)."""
import numpy as np
import pytest
import torch

import oracle
from tests.bag_hash import bag_hash


def _cols(seed, n, k):
    r = np.random.default_rng(seed)
    cols = [r.integers(-(1 << 31), (1 << 31) - 1, n, dtype=np.int64).astype(np.int32) for _ in range(k)]
    if n >= 4:
        for c in cols:
            c[:4] = [-(1 << 31), (1 << 31) - 1, 0, -1]
    return cols


@pytest.mark.parametrize("n,k,chunk", [(0, 2, 1 << 25), (1, 1, 1 << 25), (1000, 3, 1 << 25), (100_003, 4, 4096),
                                       (70_000, 7, 65_536)])
def test_torch_hash_equals_oracle_cpu(n, k, chunk):
    cols = _cols(n + k, n, k)
    assert bag_hash([torch.from_numpy(c) for c in cols], chunk=chunk) == oracle.multiset_hash(cols)


def test_torch_hash_is_order_free_and_column_order_aware():
    cols = _cols(3, 5000, 3)
    perm = np.random.default_rng(4).permutation(5000)
    t = [torch.from_numpy(c) for c in cols]
    assert bag_hash(t) == bag_hash([x[torch.from_numpy(perm)] for x in t])
    assert bag_hash(t) != bag_hash([t[1], t[0], t[2]])


@pytest.mark.gpu
def test_torch_hash_equals_oracle_on_device():
    for n, k in [(0, 1), (12_345, 2), (3_000_001, 5)]:
        cols = _cols(n, n, k)
        assert bag_hash([torch.from_numpy(c).cuda() for c in cols], chunk=1 << 20) == oracle.multiset_hash(cols)
