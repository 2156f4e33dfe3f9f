"""Pins of the oracle's window hash, candidate test and chunk rule.

Pins used (none of them re-types the oracle's own loop):
* the window hash against the 48-term polynomial evaluated with Python
  integers, at every offset, for several bases;
* the closed forms: all-zero input hashes to 0 everywhere, so it cuts every
  `min` bytes; a 64-bit mask on random data never hits, so it cuts every `max`;
* the chunk rule stated as properties that determine it uniquely (bounds,
  cause of each cut, minimality) and as an independent search from each start;
* split invariance of the streaming form at random cut points, inside the
  first window and exactly at chunk ends.
"""
import hashlib
import random

import numpy as np
import pytest

import gen
import oracle

M64 = (1 << 64) - 1


def _brute_py(data, base):
    out = []
    for i in range(len(data)):
        if i < 47:
            out.append(0)
            continue
        s = 0
        for k in range(48):
            s += int(data[i - 47 + k]) * pow(base, 47 - k, 1 << 64)
        out.append(s & M64)
    return out


@pytest.mark.parametrize("base", [3, 257, 0x100000001B3, 0x9E3779B97F4A7C15,
                                  gen.cdc_base(), 2, (1 << 64) - 1])
def test_window_hash_against_python_polynomial(base):
    data = gen.random_bytes(base & 0xFFFF, 300)
    w = oracle.window_hash(data, base)
    assert [int(x) for x in w] == _brute_py(data, base)


@pytest.mark.parametrize("base", [5, gen.cdc_base(), 0xDEADBEEFCAFEBABF])
def test_window_hash_rolling_equals_sum_4096(base):
    data = gen.random_bytes(base & 0xFFF, 4096)
    assert np.array_equal(oracle.window_hash(data, base),
                          oracle.window_hash(data, base, brute=True))


def test_window_hash_zero_input():
    w = oracle.window_hash(np.zeros(500, np.uint8), gen.cdc_base())
    assert not w.any()


def test_window_hash_single_byte_weights():
    # One nonzero byte v at position p: W_i = v * B^(i-p) for p <= i < p+48.
    base = gen.cdc_base()
    data = np.zeros(200, np.uint8)
    data[100] = 7
    w = oracle.window_hash(data, base)
    for i in range(47, 200):
        exp = (7 * pow(base, i - 100, 1 << 64)) & M64 if 100 <= i < 148 else 0
        assert int(w[i]) == exp, i


def test_candidates_definition():
    base = gen.cdc_base()
    data = gen.random_bytes(11, 200000)
    w = oracle.window_hash(data, base)
    idx = np.arange(len(data))
    exp = idx[(idx >= 47) & ((w & np.uint64(0x1FFF)) == 0)]
    got = oracle.candidates(data, base, 13)
    assert np.array_equal(got, exp.astype(np.uint64))
    # density ~ 2^-13
    assert 5 < len(got) < 60


def test_all_zero_cuts_every_min():
    n = 10 * 2048 + 777
    ends, dig = oracle.cdc(np.zeros(n, np.uint8), gen.cdc_base())
    exp = list(range(2048, n, 2048)) + [n]
    assert [int(e) for e in ends] == exp
    z = hashlib.md5(b"\0" * 2048).digest()
    assert all(bytes(d) == z for d in dig[:-1])


@pytest.mark.parametrize("n", [1, 2048, 2049, 4097])
def test_all_zero_short_tail(n):
    base = gen.cdc_base()
    z = np.zeros(n, np.uint8)
    exp = list(range(2048, n, 2048)) + [n]
    assert [int(e) for e in oracle.select(oracle.candidates(z, base), n)] == exp
    assert [int(e) for e in oracle.cdc(z, base)[0]] == exp


def test_no_hit_mask_cuts_every_max():
    n = 5 * 65536 + 1234
    data = gen.random_bytes(42, n)
    ends, dig = oracle.cdc(data, gen.cdc_base(), mask_bits=64)
    assert [int(e) for e in ends] == [65536 * k for k in range(1, 6)] + [n]


def _rule_by_search(C, n, mn, mx):
    """Chunk ends from an independent search: from each start, the first end
    e in (s, min(s+mx, n)] whose last byte is a candidate with length >= mn,
    or whose length is exactly mx; the input end otherwise."""
    cset = set(int(c) for c in C)
    ends, s = [], 0
    while s < n:
        e = None
        for cand_end in range(s + 1, min(s + mx, n) + 1):
            ln = cand_end - s
            if (ln >= mn and (cand_end - 1) in cset) or ln == mx:
                e = cand_end
                break
        e = n if e is None else e
        ends.append(e)
        s = e
    return ends


def _check_properties(ends, C, n, mn, mx):
    cset = set(int(c) for c in C)
    Cs = np.asarray(C, dtype=np.int64)
    ends = [int(e) for e in ends]
    if n == 0:
        assert ends == []
        return
    assert ends[-1] == n
    assert all(b > a for a, b in zip(ends, ends[1:]))
    s = 0
    for k, e in enumerate(ends):
        ln = e - s
        assert 1 <= ln <= mx
        last = k == len(ends) - 1
        if not last:
            assert ln >= mn
            assert (e - 1) in cset or ln == mx
        # minimality: no earlier admissible cut inside this chunk, i.e. no
        # candidate i with s + mn - 1 <= i < e - 1
        lo = np.searchsorted(Cs, s + mn - 1, side="left")
        hi = np.searchsorted(Cs, e - 1, side="left")
        assert hi <= lo, (s, e, Cs[lo:hi][:3])
        s = e


@pytest.mark.parametrize("seed", range(12))
def test_rule_small_params_against_search(seed):
    rng = random.Random(seed)
    n = rng.randrange(0, 10000)
    mn = rng.choice([1, 2, 16, 64, 100])
    mx = mn + rng.choice([0, 1, 50, 200, 1000])
    bits = rng.choice([2, 3, 4, 6])
    base = gen.cdc_base(seed) if seed % 2 else rng.randrange(1, 1 << 64) | 1
    data = gen.random_bytes(seed + 100, n)
    C = oracle.candidates(data, base, bits)
    ends = oracle.select(C, n, mn, mx)
    assert [int(e) for e in ends] == _rule_by_search(C, n, mn, mx)
    _check_properties(ends, C, n, mn, mx)
    e2, d2 = oracle.cdc(data, base, bits, mn, mx)
    assert np.array_equal(e2, ends)
    lo = 0
    for k, e in enumerate(ends):
        assert bytes(d2[k]) == hashlib.md5(bytes(data[lo:int(e)])).digest()
        lo = int(e)


def test_rule_properties_default_params():
    base = gen.cdc_base()
    data = gen.cdc_input(n_blocks=64, block=65536, repeat_frac=0.2, seed=5)
    n = len(data)
    C = oracle.candidates(data, base)
    ends = oracle.select(C, n)
    _check_properties(ends, C, n, 2048, 65536)
    e2, d2 = oracle.cdc(data, base)
    assert np.array_equal(e2, ends)
    assert 250 < len(ends) < 600  # E[len] ~ 10 KiB


def test_dedup_sanity_repeated_blocks_share_digests():
    base = gen.cdc_base()
    data = gen.cdc_input(n_blocks=64, block=65536, repeat_frac=0.25, seed=9)
    ends, dig = oracle.cdc(data, base)
    lens = np.diff(np.concatenate([[0], ends.astype(np.int64)]))
    seen, dup_bytes = {}, 0
    for k in range(len(ends)):
        key = bytes(dig[k])
        if key in seen:
            dup_bytes += int(lens[k])
        seen[key] = k
    frac = dup_bytes / len(data)
    assert 0.08 < frac < 0.30


@pytest.mark.parametrize("seed", range(6))
def test_split_invariance(seed):
    rng = random.Random(1000 + seed)
    mn, mx, bits = (64, 512, 5) if seed % 2 else (2048, 65536, 13)
    n = rng.randrange(50000, 300000)
    base = gen.cdc_base(seed)
    data = gen.random_bytes(seed, n)
    whole_e, whole_d = oracle.cdc(data, base, bits, mn, mx)
    cuts = set(rng.sample(range(1, n), 30))
    cuts |= {1, 20, 47, 48, 49}
    cuts |= {int(e) for e in whole_e[:10]}
    cuts |= {int(e) + d for e in whole_e[:10] for d in (-1, 1)}
    cuts = sorted(c for c in cuts if 0 < c < n)
    ch = oracle.StreamingChunker(base, bits, mn, mx)
    prev = 0
    for c in cuts + [n]:
        ch.feed(data[prev:c])
        prev = c
    e, d = ch.finish()
    assert np.array_equal(e, whole_e)
    assert np.array_equal(d, whole_d)


def test_split_invariance_bytewise_small():
    base = gen.cdc_base()
    data = gen.random_bytes(3, 3000)
    whole = oracle.cdc(data, base, 4, 32, 200)
    ch = oracle.StreamingChunker(base, 4, 32, 200)
    for i in range(len(data)):
        ch.feed(data[i:i + 1])
    e, d = ch.finish()
    assert np.array_equal(e, whole[0]) and np.array_equal(d, whole[1])


@pytest.mark.parametrize("n", [0, 1, 47, 48, 2047, 2048, 65535, 65536, 65537])
def test_degenerate_lengths(n):
    base = gen.cdc_base()
    data = gen.random_bytes(n + 1, n)
    C = oracle.candidates(data, base)
    ends, dig = oracle.cdc(data, base)
    _check_properties(ends, C, n, 2048, 65536)
    assert [int(e) for e in ends] == _rule_by_search(C, n, 2048, 65536)
    if n == 0:
        assert len(ends) == 0
