"""The oracle's pins are sensitive: plausible slips planted into a copy of
oracle.c (on the CPU only) must each make at least one pin fail."""
import ctypes
import hashlib
import os
import subprocess
import tempfile

import numpy as np
import pytest

import gen
import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.c")

MUTANTS = {
    "round2_index": ("k = (1 + 5 * j) % 16", "k = (5 * j) % 16"),
    "round3_index": ("k = (5 + 3 * j) % 16", "k = (3 * j + 3) % 16"),
    "shift_swap": ("{7, 12, 17, 22}", "{7, 12, 22, 17}"),
    "F_function": ("f = (b & c) | (~b & d)", "f = (b & c) | (b & d)"),
    "I_function": ("f = c ^ (b | ~d)", "f = c ^ (b | d)"),
    "pad_position": ("while (c->npend != 56)", "while (c->npend != 48)"),
    "length_big_endian": ("len[i] = (uint8_t)(bits >> (8 * i));",
                          "len[i] = (uint8_t)(bits >> (8 * (7 - i)));"),
    "init_constant": ("c->st[2] = 0x98badcfeu;", "c->st[2] = 0x98badcfdu;"),
    "rolling_sign": ("            w -= (uint64_t)buf[i - OW] * b48;\n        W[i]",
                     "            w += (uint64_t)buf[i - OW] * b48;\n        W[i]"),
    "window_width": ("uint64_t b48 = pow64(base, OW), w = 0;\n    for (size_t i = 0; i < n; i++) {\n        w = w * base + buf[i];\n        if (i >= OW)\n            w -= (uint64_t)buf[i - OW] * b48;\n        W[i]",
                     "uint64_t b48 = pow64(base, OW - 1), w = 0;\n    for (size_t i = 0; i < n; i++) {\n        w = w * base + buf[i];\n        if (i >= OW)\n            w -= (uint64_t)buf[i - OW] * b48;\n        W[i]"),
    "select_min_strict": ("if ((len >= min_len && is_cand) || len == max_len) {\n            if (cnt < cap)",
                          "if ((len > min_len && is_cand) || len == max_len) {\n            if (cnt < cap)"),
    "select_eof": ("    if (s < n) {\n        if (cnt < cap)\n            ends[cnt] = n;",
                   "    if (s + 1 < n) {\n        if (cnt < cap)\n            ends[cnt] = n;"),
    "stream_max": ("if ((len >= c->min_len && is_cand) || len == c->max_len)",
                   "if ((len >= c->min_len && is_cand) || len == c->max_len + 1)"),
    "stream_ring": ("c->ring[i % OW] = b;", "c->ring[(i + 1) % OW] = b;"),
    "direct_root_over_data": ("oracle_md5(seg_digests, 16 * nseg, root);",
                              "oracle_md5(buf, n, root);"),
    "candidate_early": ("if (i + 1 >= OW && (w & m) == 0) {", "if ((w & m) == 0) {"),
    "sha1_schedule_rot": ("W[t] = rotl32(W[t - 3] ^ W[t - 8] ^ W[t - 14] ^ W[t - 16], 1);",
                          "W[t] = W[t - 3] ^ W[t - 8] ^ W[t - 14] ^ W[t - 16];"),
    "sha1_maj": ("return (x & y) ^ (x & z) ^ (y & z);  /* Maj */",
                 "return (x & y) ^ (x & z);  /* Maj */"),
    "sha1_k3": ("return 0x8f1bbcdcu;", "return 0x8f1bbcdbu;"),
    "sha1_rot30": ("c = rotl32(b, 30);", "c = rotl32(b, 2);"),
    "sha1_little_endian_len": ("last[total - 1 - k] = (uint8_t)(bits >> (8 * k));",
                               "last[total - 8 + k] = (uint8_t)(bits >> (8 * k));"),
    "sha1_pad_boundary": ("size_t total = r + 1 + 8 <= 64 ? 64 : 128;",
                          "size_t total = r + 8 <= 64 ? 64 : 128;"),
    "sha1_direct_root_width": ("oracle_sha1(seg_digests, 20 * nseg, root);",
                               "oracle_sha1(seg_digests, 16 * nseg, root);"),
}


def _build_mutant(old, new, d):
    src = open(SRC).read()
    assert src.count(old) == 1, old
    path = os.path.join(d, "m.c")
    open(path, "w").write(src.replace(old, new))
    so = os.path.join(d, "m.so")
    subprocess.check_call(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", "-o",
                           so, path, "-lm"])
    return so


def _pins_pass():
    """A quick battery of the same pins the full suite uses."""
    h = lambda b: hashlib.md5(bytes(b)).digest()
    data = gen.random_bytes(1, 5000)
    for n in (0, 3, 55, 56, 64, 100, 1000, 5000):
        if oracle.md5(data[:n]) != h(data[:n]):
            return False
    seg, root = oracle.direct(data[:9000] if len(data) >= 9000 else
                              gen.random_bytes(2, 9000))
    d9 = gen.random_bytes(2, 9000)
    seg, root = oracle.direct(d9)
    pieces = [bytes(d9[i:i + 4096]) for i in range(0, 9000, 4096)]
    if root != h(b"".join(h(p) for p in pieces)):
        return False
    base = gen.cdc_base()
    small = gen.random_bytes(3, 200)
    w = oracle.window_hash(small, base)
    for i in (47, 48, 120, 199):
        s = sum(int(small[i - 47 + k]) * pow(base, 47 - k, 1 << 64) for k in range(48))
        if int(w[i]) != s % (1 << 64):
            return False
    z = np.zeros(5000, np.uint8)
    if [int(c) for c in oracle.candidates(z, base)] != list(range(47, 5000)):
        return False
    if [int(e) for e in oracle.select(oracle.candidates(z, base), 5000)] != [2048, 4096, 5000]:
        return False
    e, dg = oracle.cdc(z, base)
    if [int(x) for x in e] != [2048, 4096, 5000]:
        return False
    z1 = np.zeros(4097, np.uint8)  # last chunk of exactly one byte
    if [int(x) for x in oracle.select(oracle.candidates(z1, base), 4097)] != [2048, 4096, 4097]:
        return False
    r = gen.random_bytes(7, 3 * 65536 + 5)
    e, dg = oracle.cdc(r, base, mask_bits=64)
    if [int(x) for x in e] != [65536, 131072, 196608, 3 * 65536 + 5]:
        return False
    mid = gen.random_bytes(8, 6000)
    e, dg = oracle.cdc(mid, base, 4, 32, 200)
    C = oracle.candidates(mid, base, 4)
    if not np.array_equal(e, oracle.select(C, 6000, 32, 200)):
        return False
    lo = 0
    for k, x in enumerate(e):
        if bytes(dg[k]) != h(mid[lo:int(x)]):
            return False
        lo = int(x)
    h1 = lambda b: hashlib.sha1(bytes(b)).digest()
    for n in (0, 3, 55, 56, 64, 100, 1000, 5000):
        if oracle.sha1(data[:n]) != h1(data[:n]):
            return False
    seg1, root1 = oracle.sha1_direct(d9)
    if root1 != h1(b"".join(h1(p) for p in pieces)):
        return False
    return True


def test_unmutated_passes_battery():
    assert _pins_pass()


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name):
    old, new = MUTANTS[name]
    with tempfile.TemporaryDirectory() as d:
        so = _build_mutant(old, new, d)
        saved = oracle._lib
        try:
            oracle._lib = None
            real = oracle._LIB_PATH
            oracle._LIB_PATH = so
            oracle._L()
            caught = not _pins_pass()
        finally:
            oracle._LIB_PATH = real
            oracle._lib = saved
    assert caught, f"mutant {name} survived the pins"
