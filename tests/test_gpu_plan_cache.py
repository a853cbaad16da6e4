"""The on-disk plan cache (PB3_PLAN_CACHE): the triangle counts T of every
candidate triplet and the multipole mixing blocks are read from a file
keyed by the geometry instead of being recomputed, and a file whose key,
length or checksum does not match is ignored and rewritten."""

import struct
import sys

import numpy as np
import pytest

from synthetic import kf_edges, quadratic_field

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _fnv1a(data: bytes, h: int = 1469598103934665603) -> int:
    for c in data:
        h = ((h ^ c) * 1099511628211) & 0xFFFFFFFFFFFFFFFF
    return h


def _parse(blob: bytes):
    """(key, what, values) of a cache file: three text lines, a u64 length,
    the FP64 values and a u64 FNV-1a checksum of key and values."""
    magic, key, what, rest = blob.split(b"\n", 3)
    assert magic == b"PB3PLAN1"
    (n,) = struct.unpack_from("<Q", rest, 0)
    vals = np.frombuffer(rest, dtype="<f8", count=n, offset=8).copy()
    (cs,) = struct.unpack_from("<Q", rest, 8 + 8 * n)
    assert cs == _fnv1a(vals.tobytes(), _fnv1a(key))
    return key, what, vals


def _build(key: bytes, what: bytes, vals: np.ndarray) -> bytes:
    body = vals.astype("<f8").tobytes()
    return b"PB3PLAN1\n" + key + b"\n" + what + b"\n" + struct.pack("<Q", vals.size) + body + \
        struct.pack("<Q", _fnv1a(body, _fnv1a(key)))


def test_counts_are_cached_and_checked(torch_cuda, tmp_path, monkeypatch):
    import paper_2404_07249_amd as pb3

    torch = torch_cuda
    n, box, edges = 48, 900.0, kf_edges(8)
    _say("[case] plan cache: counts")
    d = torch.from_numpy(quadratic_field(n, box, 1.0, 81).astype(np.float32)).cuda()
    monkeypatch.setenv("PB3_PLAN_CACHE", str(tmp_path))
    a = pb3.Plan(n, box, edges)  # computes T and writes the file
    files = sorted(tmp_path.glob("pb3_counts_*.bin"))
    assert len(files) == 1
    blob = files[0].read_bytes()
    key, what, vals = _parse(blob)
    assert what == b"counts" and b"N48x48x48" in key
    T = a.norm()[1]
    cnt = np.rint(vals)  # FP64 sums of the count pass, within rounding of integers
    assert np.array_equal(np.sort(cnt[cnt > 0]), np.sort(T))  # every kept triplet's count
    b = pb3.Plan(n, box, edges)  # reads it
    assert np.array_equal(b.norm()[1], T)
    ra, rb = a.polyspectra(d), b.polyspectra(d)
    assert torch.equal(ra[0], rb[0]) and torch.equal(ra[1], rb[1])
    # the file is what plan creation reads: a valid file with other values gives other counts
    files[0].write_bytes(_build(key, what, 2.0 * vals))
    assert np.array_equal(pb3.Plan(n, box, edges).norm()[1], 2.0 * T)
    # a damaged file is ignored, and rewritten with the computed counts
    bad = bytearray(_build(key, what, 2.0 * vals))
    bad[-1] ^= 1
    files[0].write_bytes(bytes(bad))
    assert np.array_equal(pb3.Plan(n, box, edges).norm()[1], T)
    assert files[0].read_bytes() == blob
    # a file written for another key (same name) is ignored too
    files[0].write_bytes(_build(key + b" other", what, 2.0 * vals))
    assert np.array_equal(pb3.Plan(n, box, edges).norm()[1], T)
    # other geometries have files of their own; without the variable nothing is read or written
    pb3.Plan(n, box, kf_edges(7))
    assert len(list(tmp_path.glob("pb3_counts_*.bin"))) == 2
    files[0].write_bytes(_build(key, what, 2.0 * vals))
    monkeypatch.delenv("PB3_PLAN_CACHE")
    assert np.array_equal(pb3.Plan(n, box, edges).norm()[1], T)
    assert not list(tmp_path.glob("*.tmp*"))


def test_mixing_blocks_are_cached(torch_cuda, tmp_path, monkeypatch):
    import paper_2404_07249_amd as pb3

    torch = torch_cuda
    n, box, edges = 32, 1000.0, kf_edges(8)
    _say("[case] plan cache: multipole mixing blocks")
    d = torch.from_numpy(quadratic_field(n, box, 1.0, 82).astype(np.float32)).cuda()
    ref = pb3.Plan(n, box, edges, lmax=2, bk_fisher=True)  # no cache
    monkeypatch.setenv("PB3_PLAN_CACHE", str(tmp_path))
    a = pb3.Plan(n, box, edges, lmax=2, bk_fisher=True)
    (mf,) = tmp_path.glob("pb3_mixing_*.bin")
    assert len(list(tmp_path.glob("pb3_counts_*.bin"))) == 1
    b = pb3.Plan(n, box, edges, lmax=2, bk_fisher=True)
    for p in (a, b):
        assert np.array_equal(p.multipole_mixing(), ref.multipole_mixing())
        got, want = p.multipoles(d), ref.multipoles(d)
        assert torch.equal(got[0], want[0]) and torch.equal(got[1], want[1])
    key, what, vals = _parse(mf.read_bytes())
    assert what == b"mixing" and key.endswith(b" lmax2") and vals.size == ref.multipole_mixing().size
