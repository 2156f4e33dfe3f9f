"""CPU oracle of the hashing hot path -- TEST INFRASTRUCTURE ONLY.

Thin ctypes wrapper over ``oracle.c`` (plain single-threaded C).  Only the
test suite, ``__graft_entry__.smoke()`` and the benchmark's ``cpu_baseline``
leg may import this package; the GPU library never does, and the two share no
code.  Definitions and their sources are listed in the header of ``oracle.c``
(RFC 1321 for MD5, FIPS 180-4 for SHA-1; the paper's direct-hashing and content-addressable
chunking primitives, Sec. 2.2 and Sec. 5.2).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

WINDOW = 48
DEFAULT_SEGMENT = 4096
DEFAULT_MASK_BITS = 13
DEFAULT_MIN = 2048
DEFAULT_MAX = 65536


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so (plain gcc, no vectorisation)."""
    if force or not os.path.exists(_LIB_PATH):
        src = os.path.join(_HERE, "oracle.c")
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fno-tree-vectorize", "-std=c11",
                               "-fPIC", "-shared", "-o", tmp, src, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def _L():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        vp, sz, u64, i32 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_uint64, ctypes.c_int
        sigs = {
            "oracle_md5": ([vp, sz, vp], None),
            "oracle_sha1": ([vp, sz, vp], None),
            "oracle_sha1_direct": ([vp, sz, sz, vp, vp], sz),
            "oracle_direct": ([vp, sz, sz, vp, vp], sz),
            "oracle_md5_batch": ([vp, vp, vp, sz, vp], None),
            "oracle_md5_chunks": ([vp, vp, sz, vp], None),
            "oracle_window_hash": ([vp, sz, u64, vp], None),
            "oracle_window_hash_brute": ([vp, sz, u64, vp], None),
            "oracle_candidates": ([vp, sz, u64, i32, vp, sz], sz),
            "oracle_select": ([vp, sz, u64, u64, u64, vp, sz], sz),
            "oracle_cdc_new": ([u64, i32, u64, u64], vp),
            "oracle_cdc_free": ([vp], None),
            "oracle_cdc_feed": ([vp, vp, sz, vp, vp, sz], sz),
            "oracle_cdc_finish": ([vp, vp, vp, sz], sz),
        }
        for name, (args, res) in sigs.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = res
        _lib = lib
    return _lib


def _u8(a) -> np.ndarray:
    if isinstance(a, (bytes, bytearray, memoryview)):
        return np.frombuffer(bytes(a), dtype=np.uint8)
    return np.ascontiguousarray(a, dtype=np.uint8)


def _p(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data if a.size else 0)


def md5(data) -> bytes:
    buf = _u8(data)
    out = np.zeros(16, dtype=np.uint8)
    _L().oracle_md5(_p(buf), buf.size, _p(out))
    return out.tobytes()


def direct(data, segment: int = DEFAULT_SEGMENT):
    """(segment digests as uint8[n_seg, 16], root digest bytes)."""
    buf = _u8(data)
    nseg = (buf.size + segment - 1) // segment
    seg = np.zeros((max(nseg, 1), 16), dtype=np.uint8)
    root = np.zeros(16, dtype=np.uint8)
    got = _L().oracle_direct(_p(buf), buf.size, segment, _p(seg), _p(root))
    assert got == nseg
    return seg[:nseg], root.tobytes()


def sha1(data) -> bytes:
    buf = _u8(data)
    out = np.zeros(20, dtype=np.uint8)
    _L().oracle_sha1(_p(buf), buf.size, _p(out))
    return out.tobytes()


def sha1_direct(data, segment: int = DEFAULT_SEGMENT):
    """(segment SHA-1 digests as uint8[n_seg, 20], root digest bytes)."""
    buf = _u8(data)
    nseg = (buf.size + segment - 1) // segment
    seg = np.zeros((max(nseg, 1), 20), dtype=np.uint8)
    root = np.zeros(20, dtype=np.uint8)
    got = _L().oracle_sha1_direct(_p(buf), buf.size, segment, _p(seg), _p(root))
    assert got == nseg
    return seg[:nseg], root.tobytes()


def md5_batch(arena, offsets, lengths) -> np.ndarray:
    a = _u8(arena)
    off = np.ascontiguousarray(offsets, dtype=np.uint64)
    ln = np.ascontiguousarray(lengths, dtype=np.uint32)
    out = np.zeros((len(off), 16), dtype=np.uint8)
    _L().oracle_md5_batch(_p(a), _p(off), _p(ln), len(off), _p(out))
    return out


def md5_chunks(data, ends) -> np.ndarray:
    buf = _u8(data)
    e = np.ascontiguousarray(ends, dtype=np.uint64)
    out = np.zeros((len(e), 16), dtype=np.uint8)
    _L().oracle_md5_chunks(_p(buf), _p(e), len(e), _p(out))
    return out


def window_hash(data, base: int, brute: bool = False) -> np.ndarray:
    buf = _u8(data)
    w = np.zeros(buf.size, dtype=np.uint64)
    fn = _L().oracle_window_hash_brute if brute else _L().oracle_window_hash
    fn(_p(buf), buf.size, base, _p(w))
    return w


def candidates(data, base: int, mask_bits: int = DEFAULT_MASK_BITS) -> np.ndarray:
    buf = _u8(data)
    cnt = _L().oracle_candidates(_p(buf), buf.size, base, mask_bits, None, 0)
    out = np.zeros(max(cnt, 1), dtype=np.uint64)
    got = _L().oracle_candidates(_p(buf), buf.size, base, mask_bits, _p(out), cnt)
    assert got == cnt
    return out[:cnt]


def select(cands, n: int, min_len: int = DEFAULT_MIN,
           max_len: int = DEFAULT_MAX) -> np.ndarray:
    c = np.ascontiguousarray(cands, dtype=np.uint64)
    cap = n // max(min_len, 1) + 2 if min_len else n + 1
    cap = max(cap, n // max_len + 2)
    out = np.zeros(cap, dtype=np.uint64)
    cnt = _L().oracle_select(_p(c), len(c), n, min_len, max_len, _p(out), cap)
    assert cnt <= cap
    return out[:cnt]


class StreamingChunker:
    """Chunker that accepts its input in pieces (state carried between calls)."""

    def __init__(self, base: int, mask_bits: int = DEFAULT_MASK_BITS,
                 min_len: int = DEFAULT_MIN, max_len: int = DEFAULT_MAX):
        self._h = _L().oracle_cdc_new(base, mask_bits, min_len, max_len)
        self._min = max(min_len, 1)
        self.ends: list[int] = []
        self.digests: list[bytes] = []

    def feed(self, data) -> None:
        buf = _u8(data)
        cap = buf.size // self._min + 2
        e = np.zeros(cap, dtype=np.uint64)
        d = np.zeros((cap, 16), dtype=np.uint8)
        cnt = _L().oracle_cdc_feed(self._h, _p(buf), buf.size, _p(e), _p(d), cap)
        assert cnt <= cap
        self.ends.extend(int(x) for x in e[:cnt])
        self.digests.extend(bytes(r) for r in d[:cnt])

    def finish(self):
        e = np.zeros(1, dtype=np.uint64)
        d = np.zeros((1, 16), dtype=np.uint8)
        cnt = _L().oracle_cdc_finish(self._h, _p(e), _p(d), 1)
        if cnt:
            self.ends.append(int(e[0]))
            self.digests.append(d[0].tobytes())
        _L().oracle_cdc_free(self._h)
        self._h = None
        return (np.array(self.ends, dtype=np.uint64),
                np.frombuffer(b"".join(self.digests), dtype=np.uint8).reshape(-1, 16))


def cdc(data, base: int, mask_bits: int = DEFAULT_MASK_BITS,
        min_len: int = DEFAULT_MIN, max_len: int = DEFAULT_MAX):
    """Whole-input chunking: (ends uint64[n], digests uint8[n, 16])."""
    ch = StreamingChunker(base, mask_bits, min_len, max_len)
    ch.feed(data)
    return ch.finish()
