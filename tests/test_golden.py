"""The stored fixtures under tests/golden/: each is what the oracle writes
for its seeded input (so a change to the oracle's arithmetic shows here), and
each is pinned independently of the oracle by hashlib and the chunk rule."""
import hashlib
import os
import sys

import numpy as np

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
import make_golden as mg  # noqa: E402


def test_direct_fixture_matches_oracle(tmp_path):
    p = tmp_path / "d.txt"
    mg.write_direct(str(p))
    assert p.read_text() == open(mg.DIRECT_FILE).read()


def test_cdc_fixture_matches_oracle(tmp_path):
    p = tmp_path / "c.txt"
    mg.write_cdc(str(p))
    assert p.read_text() == open(mg.CDC_FILE).read()


def test_direct_fixture_pinned_by_hashlib():
    data = mg.direct_input().tobytes()
    seg, root = mg.read_direct()
    assert len(seg) == len(data) // 4096 == 256
    for i, d in enumerate(seg):
        assert d == hashlib.md5(data[4096 * i:4096 * (i + 1)]).digest(), i
    assert root == hashlib.md5(b"".join(seg)).digest()


def test_cdc_fixture_pinned_by_hashlib_and_rule():
    data, base = mg.cdc_input()
    ends, dig = mg.read_cdc()
    assert ends[-1] == len(data) and all(b > a for a, b in zip(ends, ends[1:]))
    start = 0
    for k, (e, d) in enumerate(zip(ends, dig)):
        n = e - start
        assert n <= 65536 and (n >= 2048 or k == len(ends) - 1), k
        assert d == hashlib.md5(data[start:e].tobytes()).digest(), k
        start = e
    # a cut below the maximum length sits where the window hash has its low
    # 13 bits zero: W = sum of the last 48 bytes times powers of the base
    M = (1 << 64) - 1
    for k, e in enumerate(ends[:-1]):
        n = e - (ends[k - 1] if k else 0)
        if n == 65536:
            continue
        w = 0
        for b in data[e - 48:e].tolist():
            w = (w * base + b) & M
        assert w & 0x1FFF == 0, k
