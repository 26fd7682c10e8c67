"""The oracle's order-independent bag hash, computed with torch so that a
result table resident in device memory can be hashed where it lies.

It is the same function as ``oracle.multiset_hash`` (row count, and two
sums mod 2^64 of per-row SplitMix64 mixes over the columns in the given
order), written with int64 tensors: additions, products and sums wrap mod
2^64, and a right shift is made logical by masking.  ``test_bag_hash`` pins
it to ``oracle.multiset_hash`` on the CPU and, where a GPU is present, on
the device.
"""
import torch

_M64 = (1 << 64) - 1


def _s64(c: int) -> int:
    """A 64-bit constant as the int64 with the same bits."""
    return c - (1 << 64) if c >= (1 << 63) else c


_GOLDEN = _s64(0x9E3779B97F4A7C15)
_MUL1 = _s64(0xBF58476D1CE4E5B9)
_MUL2 = _s64(0x94D049BB133111EB)
_MULV = _s64(0x2545F4914F6CDD1D)


def _srl(x: torch.Tensor, k: int) -> torch.Tensor:
    return (x >> k) & ((1 << (64 - k)) - 1)


def _mix(x: torch.Tensor) -> torch.Tensor:
    x = x + _GOLDEN
    x = (x ^ _srl(x, 30)) * _MUL1
    x = (x ^ _srl(x, 27)) * _MUL2
    return x ^ _srl(x, 31)


def bag_hash(cols, chunk: int = 1 << 25):
    """(rows, h1, h2) of the bag of rows given as equal-length int32 columns
    (tensors on any device), in the order given."""
    n = int(cols[0].numel()) if cols else 0
    h1 = 0
    h2 = 0
    for lo in range(0, n, chunk):
        hi = min(n, lo + chunk)
        dev = cols[0].device
        a = torch.full((hi - lo,), 0x1234567, dtype=torch.int64, device=dev)
        b = torch.full((hi - lo,), 0x7654321, dtype=torch.int64, device=dev)
        for c in cols:
            v = c[lo:hi].to(torch.int64)
            a = _mix(a ^ v)
            b = _mix(b + v * _MULV)
        h1 = (h1 + int(a.sum())) & _M64
        h2 = (h2 + int(b.sum())) & _M64
    return n, h1, h2


def table_hash(sess, t, var_order):
    """bag_hash of a library table's columns, taken in ``var_order``."""
    vs = list(t.vars)
    assert sorted(vs) == sorted(var_order), (vs, var_order)
    return bag_hash([sess.column(t, vs.index(v)) for v in var_order])
