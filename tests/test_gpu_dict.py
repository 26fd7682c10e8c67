"""GPU dictionary encoding of terms against the oracle's plain definition
(identifiers dense, in order of first appearance; integer results, so
bit-exact), through the C ABI on both the host and the device path."""
import numpy as np
import pytest
import torch

import oracle
from oracle import dictionary as D
from paper_1702_03484_amd import binding as B
from paper_1702_03484_amd.engine import MapSQ
from synth import rdf_terms
from tests.conftest import announce
from tests.fixtures import load_table1

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def s():
    with MapSQ(arena_bytes=4 << 30) as m:
        yield m


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def test_table1_through_the_dictionary(s):
    """The worked example end to end on strings: encode the store's terms,
    load the identifiers, run the query, decode the answer."""
    announce("dictionary: Table 1 on strings")
    f = load_table1()
    names = {v: k for k, v in f["dict"].items()}
    flat = [names[int(x)].encode() for tr in zip(f["s"], f["p"], f["o"]) for x in tr]
    data, off = D.join_terms(flat)
    s.dict_create(64, 4096)
    ids, new = s.dict_encode(np.frombuffer(data, np.uint8), off)
    exp, table = D.encode(flat)
    assert np.array_equal(ids, exp) and new == len(table)
    enc = ids.reshape(-1, 3)
    s.load(enc[:, 0].copy(), enc[:, 1].copy(), enc[:, 2].copy())
    q_ids, _ = s.dict_encode(*(D.join_terms([b"hasJob", b"workAt", b'"Hospital"'])), lookup=True)
    job, works, hosp = (int(x) for x in q_ids)
    t = s.query([(-1, job, -2), (-2, works, hosp)], select=[0, 1])
    cols = s.to_numpy(t)
    s.free(t)
    person, jobs = (D.split_terms(*s.dict_decode(c)) for c in cols)
    assert sorted(zip(jobs, person)) == [(b"Doctor", b"Jim"), (b"Nurse", b"Susan")]


@pytest.mark.parametrize("path", ["host", "device"])
def test_encode_batches_match_the_oracle(s, path):
    """Three batches of RDF-shaped terms (Zipf frequencies, empty and long
    literals, bytes that differ only late) encoded one after another: every
    identifier equals the oracle's, and decoding gives the bytes back."""
    announce(f"dictionary: three batches, {path} buffers")
    s.dict_create(400_000, 40 << 20)
    known = []
    for k, (n, vocab) in enumerate(((200_000, 50_000), (150_000, 120_000), (300_000, 80_000))):
        data, off, _ = rdf_terms(10 * k + (path == "device"), n, vocab, max_literal=200)
        terms = D.split_terms(data.tobytes(), off)
        if k == 1:  # the empty term, a long one and two that differ only in their last byte
            extra = [b"", b"x" * 5000, b"<http://example.org/a" + b"b" * 300 + b"1>",
                     b"<http://example.org/a" + b"b" * 300 + b"2>"]
            terms = terms + extra + terms[:10] + extra
            data, off = D.join_terms(terms)
            data = np.frombuffer(data, np.uint8)
        exp, known2 = D.encode(terms, known)
        if path == "device":
            got, new = s.dict_encode(dev(data), dev(off))
            got = got.cpu().numpy()
        else:
            got, new = s.dict_encode(data, off)
        assert np.array_equal(got, exp), f"batch {k}: {np.flatnonzero(got != exp)[:5]}"
        assert new == len(known2) - len(known)
        known = known2
        assert s.dict_info() == (len(known), sum(len(t) for t in known))
    # every identifier decodes to its term, host and device path
    ids = np.random.default_rng(5).integers(0, len(known), 100_000).astype(np.int32)
    want = D.decode(ids, known)
    data, off = s.dict_decode(ids)
    assert D.split_terms(data, off) == want
    ddata, doff = s.dict_decode(dev(ids))
    assert D.split_terms(ddata.cpu().numpy().tobytes(), doff.cpu().numpy()) == want


def test_lookup_capacity_and_errors(s):
    announce("dictionary: lookup, capacity, bad offsets, bad identifiers")
    s.dict_create(100, 10_000)
    a = [b"a", b"bb", b"a", b"ccc"]
    ids, new = s.dict_encode(*(D.join_terms(a)))
    assert ids.tolist() == [0, 1, 0, 2] and new == 3
    # lookups add nothing; unknown terms give -1
    ids, new = s.dict_encode(*(D.join_terms([b"bb", b"zz", b"ccc"])), lookup=True)
    assert ids.tolist() == [1, -1, 2] and new == 0 and s.dict_info() == (3, 6)
    # a batch whose new terms overflow the dictionary leaves it as it was
    over = [f"t{k}".encode() for k in range(100)]
    with pytest.raises(B.MapSQError) as e:
        s.dict_encode(*(D.join_terms(over)))
    assert e.value.code == B.MAPSQ_ERR_CAPACITY and s.dict_info() == (3, 6)
    ids, new = s.dict_encode(*(D.join_terms([b"ccc", b"d", b"a"])))
    assert ids.tolist() == [2, 3, 0] and new == 1
    # offsets that decrease, or do not start at 0: refused before any byte is read
    data = np.frombuffer(b"abcdef", np.uint8)
    for bad in ([0, 3, 2, 6], [1, 3, 6]):
        with pytest.raises(B.MapSQError) as e:
            s.dict_encode(data, np.array(bad, np.int64))
        assert e.value.code == B.MAPSQ_ERR_INVALID_ARG
        with pytest.raises(B.MapSQError) as e:
            s.dict_encode(dev(data), dev(np.array(bad, np.int64)))
        assert e.value.code == B.MAPSQ_ERR_INVALID_ARG
    assert s.dict_info() == (4, 7)
    # identifiers outside the dictionary; too little room for the text
    with pytest.raises(B.MapSQError) as e:
        s.dict_decode(np.array([0, 4], np.int32))
    assert e.value.code == B.MAPSQ_ERR_INVALID_ARG
    ids = np.array([2, 2], np.int32)
    off = np.zeros(3, np.int64)
    buf = np.zeros(5, np.uint8)
    with pytest.raises(B.MapSQError) as e:
        B.mapsq_dict_decode(s.ctx, ids.ctypes.data, 2, 0, off.ctypes.data, buf.ctypes.data, 5)
    assert e.value.code == B.MAPSQ_ERR_TOO_LARGE and not buf.any()


def test_four_million_terms(s):
    """4M terms over a 1M-term vocabulary in one device batch (the table at
    about half load), then the same stream again: nothing new."""
    announce("dictionary: 4M terms, 1M distinct")
    data, off, _ = rdf_terms(3, 4_000_000, 1_000_000)
    terms = D.split_terms(data.tobytes(), off)
    exp, known = D.encode(terms)
    s.dict_create(4_000_000, 256 << 20)
    got, new = s.dict_encode(dev(data), dev(off))
    assert new == len(known) and np.array_equal(got.cpu().numpy(), exp)
    again, new = s.dict_encode(dev(data), dev(off))
    assert new == 0 and np.array_equal(again.cpu().numpy(), exp)
