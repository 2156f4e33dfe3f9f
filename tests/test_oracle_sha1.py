"""Pins of the oracle's SHA-1 and SHA-1 direct hashing.

SHA-1 is pinned against two implementations that share nothing with the
oracle: Python's hashlib (OpenSSL) and the coreutils ``sha1sum`` binary.
Direct hashing with SHA-1 is pinned by composing hashlib by hand.
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
    return hashlib.sha1(bytes(b)).digest()


def test_sha1_every_length_to_1100():
    data = gen.random_bytes(0x5A1, 1100)
    for n in range(0, 1101):
        assert oracle.sha1(data[:n]) == _h(data[:n]), n


@pytest.mark.parametrize("n", [55, 56, 57, 63, 64, 65, 119, 120, 121, 127, 128,
                               4095, 4096, 4097, 1 << 20, (1 << 20) + 13])
def test_sha1_padding_edges_and_large(n):
    data = gen.random_bytes(n + 77, n)
    assert oracle.sha1(data) == _h(data)


def test_sha1_structured_inputs():
    for data in (b"", b"\x00" * 1000, b"\xff" * 1000, bytes(range(256)) * 9):
        assert oracle.sha1(data) == _h(data)


@pytest.mark.skipif(shutil.which("sha1sum") is None, reason="sha1sum not present")
def test_sha1_against_sha1sum():
    with tempfile.TemporaryDirectory() as d:
        for n in (0, 1, 64, 4096, 100003):
            data = gen.random_bytes(n + 9, n)
            p = os.path.join(d, "x.bin")
            data.tofile(p)
            hexd = subprocess.check_output(["sha1sum", p]).split()[0].decode()
            assert oracle.sha1(data).hex() == hexd


@pytest.mark.parametrize("n", [0, 1, 100, 4095, 4096, 4097, 8192, 3 * 4096 + 5, 1 << 20])
def test_sha1_direct_is_digest_of_digests(n):
    data = gen.random_bytes(n * 5 + 3, n)
    seg, root = oracle.sha1_direct(data, 4096)
    pieces = [bytes(data[i:i + 4096]) for i in range(0, n, 4096)]
    assert seg.shape == (len(pieces), 20)
    for j, p in enumerate(pieces):
        assert seg[j].tobytes() == _h(p), j
    assert root == _h(b"".join(_h(p) for p in pieces))


@pytest.mark.parametrize("segment", [64, 128, 1000, 65536])
def test_sha1_direct_other_segment_sizes(segment):
    data = gen.random_bytes(segment, 200003)
    seg, root = oracle.sha1_direct(data, segment)
    pieces = [bytes(data[i:i + segment]) for i in range(0, len(data), segment)]
    assert [s.tobytes() for s in seg] == [_h(p) for p in pieces]
    assert root == _h(b"".join(_h(p) for p in pieces))


def test_sha1_direct_differs_from_md5_direct():
    data = gen.random_bytes(7, 10000)
    assert oracle.sha1_direct(data)[1] != oracle.direct(data)[1]
