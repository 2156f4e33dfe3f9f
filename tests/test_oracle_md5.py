"""Pins of the oracle's MD5, direct hashing, batch and per-chunk digests.

MD5 is pinned against two implementations that share nothing with the oracle:
Python's hashlib (OpenSSL) and the coreutils ``md5sum`` binary.  Direct
hashing is pinned by composing the library routine by hand.
"""
import hashlib
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

import gen
import oracle


def _h(b):
    return hashlib.md5(bytes(b)).digest()


def test_md5_every_length_to_1100():
    data = gen.random_bytes(0xA11, 1100)
    for n in range(0, 1101):
        assert oracle.md5(data[:n]) == _h(data[:n]), n


@pytest.mark.parametrize("n", [55, 56, 57, 63, 64, 65, 119, 120, 121, 127, 128,
                               4095, 4096, 4097, 1 << 20, (1 << 20) + 13])
def test_md5_padding_edges_and_large(n):
    data = gen.random_bytes(n, n)
    assert oracle.md5(data) == _h(data)


def test_md5_structured_inputs():
    for data in (b"", b"\x00" * 1000, b"\xff" * 1000, bytes(range(256)) * 9):
        assert oracle.md5(data) == _h(data)


@pytest.mark.skipif(shutil.which("md5sum") is None, reason="md5sum not present")
def test_md5_against_md5sum():
    with tempfile.TemporaryDirectory() as d:
        for n in (0, 1, 64, 4096, 100003):
            data = gen.random_bytes(n + 5, n)
            p = os.path.join(d, "x.bin")
            data.tofile(p)
            hexd = subprocess.check_output(["md5sum", p]).split()[0].decode()
            assert oracle.md5(data).hex() == hexd


@pytest.mark.parametrize("n", [0, 1, 100, 4095, 4096, 4097, 8192, 3 * 4096 + 5,
                               1 << 20])
def test_direct_is_digest_of_digests(n):
    data = gen.random_bytes(n * 3 + 1, n)
    seg, root = oracle.direct(data, 4096)
    pieces = [bytes(data[i:i + 4096]) for i in range(0, n, 4096)]
    assert seg.shape == (len(pieces), 16)
    for j, p in enumerate(pieces):
        assert bytes(seg[j]) == _h(p)
    assert root == _h(b"".join(_h(p) for p in pieces))


def test_direct_single_segment_root_is_md5_of_digest():
    data = gen.random_bytes(9, 1000)
    seg, root = oracle.direct(data)
    assert root == _h(_h(data))
    assert root != _h(data)


def test_direct_empty():
    seg, root = oracle.direct(b"")
    assert seg.shape == (0, 16) and root == _h(b"")


@pytest.mark.parametrize("segment", [64, 128, 1000, 65536])
def test_direct_other_segment_sizes(segment):
    data = gen.random_bytes(segment, 70000)
    seg, root = oracle.direct(data, segment)
    pieces = [bytes(data[i:i + segment]) for i in range(0, len(data), segment)]
    assert [bytes(r) for r in seg] == [_h(p) for p in pieces]
    assert root == _h(b"".join(_h(p) for p in pieces))


def test_batch_matches_hashlib():
    off, ln, arena, seed = gen.batch_small(n_buf=300)
    data = gen.random_bytes(seed, arena)
    out = oracle.md5_batch(data, off, ln)
    for m in range(300):
        o, l = int(off[m]), int(ln[m])
        assert bytes(out[m]) == _h(data[o:o + l])


def test_chunks_match_hashlib():
    data = gen.random_bytes(5, 10000)
    ends = np.array([1, 64, 65, 4000, 9999, 10000], dtype=np.uint64)
    out = oracle.md5_chunks(data, ends)
    lo = 0
    for k, e in enumerate(ends):
        assert bytes(out[k]) == _h(data[lo:int(e)])
        lo = int(e)
