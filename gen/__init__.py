"""Seeded synthetic inputs for the five hashing workloads.

This module produces input bytes, sizes, offsets and arrival times only; it
holds none of the hashing arithmetic.  Both the CPU oracle and the GPU path
consume what it produces, so the same seed always means the same bytes.

Random source: SplitMix64 (Steele, Lea, Flood, OOPSLA 2014), implemented in
``gen.c``.  A uniform double in [0, 1) is ``(x >> 11) * 2**-53`` of one 64-bit
draw.  Sub-streams are derived as ``sub(seed, tag) = splitmix64_at(seed, tag)``.

Workload recipes (sizes as the paper's storage workloads are framed: a
stream of data blocks to hash, Sec. 2.2 and Sec. 5.2):

* ``direct_one``   -- 1 MiB of seeded bytes, hashed as 256 segments of 4 KiB.
* ``direct_stream``-- 256 jobs of 8 MiB, job j drawing bytes from its own seed.
* ``cdc_input``    -- 256 MiB built from 4096 blocks of 64 KiB; 819 of them
  (20 %) are exact copies of a uniformly chosen earlier block.
* ``serving_jobs`` -- 20 000 jobs, sizes log-uniform in [4 KiB, 64 MiB], 70 %
  direct / 30 % chunking, Poisson arrivals at an offered load in GB/s, each job
  a 4 KiB-aligned slice of a seeded arena.
* ``batch_small``  -- 1 000 000 buffers, lengths log-uniform in [512 B, 16 KiB],
  16-byte-aligned starts in one seeded arena.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libgen.so")

SEED_BASE = 0x10051695
MASK64 = (1 << 64) - 1


def build(force: bool = True) -> str:
    """Compile gen.c into libgen.so next to it (plain gcc, no GPU code)."""
    if force or not os.path.exists(_LIB_PATH):
        src = os.path.join(_HERE, "gen.c")
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared",
                               "-o", tmp, src])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def _L():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        u64, vp, sz = ctypes.c_uint64, ctypes.c_void_p, ctypes.c_size_t
        lib.gen_splitmix64_at.argtypes = [u64, u64]
        lib.gen_splitmix64_at.restype = u64
        lib.gen_u64.argtypes = [u64, u64, vp, sz]
        lib.gen_u64.restype = None
        lib.gen_bytes.argtypes = [u64, vp, sz]
        lib.gen_bytes.restype = None
        lib.gen_bytes_multi.argtypes = [vp, vp, vp, sz, vp]
        lib.gen_bytes_multi.restype = None
        _lib = lib
    return _lib


# ---------------------------------------------------------------- primitives

def splitmix64_at(seed: int, k: int) -> int:
    return int(_L().gen_splitmix64_at(seed & MASK64, k & MASK64))


def sub_seed(seed: int, tag: int) -> int:
    return splitmix64_at(seed, tag)


def config_seed(k: int) -> int:
    """Seed of workload k (1..5): first SplitMix64 output of state base+k."""
    return splitmix64_at(SEED_BASE + k, 0)


def u64(seed: int, n: int, first: int = 0) -> np.ndarray:
    out = np.empty(n, dtype=np.uint64)
    if n:
        _L().gen_u64(seed & MASK64, first, out.ctypes.data, n)
    return out


def uniform(seed: int, n: int) -> np.ndarray:
    """n doubles in [0, 1): (x >> 11) * 2**-53."""
    return (u64(seed, n) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def fill(seed: int, ptr: int, n: int) -> None:
    """Write n seeded bytes at host address ptr (any host memory, e.g. pinned)."""
    if n:
        _L().gen_bytes(seed & MASK64, ctypes.c_void_p(ptr), n)


def random_bytes(seed: int, n: int) -> np.ndarray:
    out = np.empty(n, dtype=np.uint8)
    fill(seed, out.ctypes.data, n)
    return out


def fill_multi(seeds, offsets, lengths, ptr: int) -> None:
    seeds = np.ascontiguousarray(seeds, dtype=np.uint64)
    offsets = np.ascontiguousarray(offsets, dtype=np.uint64)
    lengths = np.ascontiguousarray(lengths, dtype=np.uint64)
    _L().gen_bytes_multi(seeds.ctypes.data, offsets.ctypes.data,
                         lengths.ctypes.data, len(seeds), ctypes.c_void_p(ptr))


def log_uniform_int(seed: int, n: int, lo: int, hi: int) -> np.ndarray:
    """floor(exp(U[ln lo, ln hi))) as int64, clipped into [lo, hi]."""
    u = uniform(seed, n)
    v = np.floor(np.exp(math.log(lo) + u * (math.log(hi) - math.log(lo))))
    return np.clip(v, lo, hi).astype(np.int64)


# ------------------------------------------------------------ workload recipes

def direct_one(n_bytes: int = 1 << 20, seed: int | None = None) -> np.ndarray:
    """One buffer of seeded uniform bytes (1 MiB by default)."""
    return random_bytes(config_seed(1) if seed is None else seed, n_bytes)


def direct_stream_seeds(n_jobs: int = 256) -> np.ndarray:
    """Per-job seeds of the streamed direct-hashing workload (8 MiB jobs)."""
    return u64(config_seed(2), n_jobs)


def cdc_base(seed: int | None = None) -> int:
    """Odd base of the rolling polynomial, drawn from the chunking seed."""
    s = config_seed(3) if seed is None else seed
    return sub_seed(s, 0) | 1


def cdc_layout(n_blocks: int = 4096, repeat_frac: float = 0.2,
               seed: int | None = None):
    """Which 64 KiB blocks are copies, and of which earlier block.

    Exactly round(repeat_frac * n_blocks) indices are drawn without replacement
    from {1..n_blocks-1} (seeded Fisher-Yates), processed in increasing order;
    each copies a uniformly chosen earlier block (possibly itself a copy).
    Returns src[b] = index of the fresh block whose bytes block b carries.
    """
    s = config_seed(3) if seed is None else seed
    n_rep = int(round(repeat_frac * n_blocks))
    idx = np.arange(1, n_blocks, dtype=np.int64)
    u = uniform(sub_seed(s, 1), max(len(idx) - 1, 0))
    for k, i in enumerate(range(len(idx) - 1, 0, -1)):
        j = int(u[k] * (i + 1))
        idx[i], idx[j] = idx[j], idx[i]
    reps = np.sort(idx[:n_rep])
    src = np.arange(n_blocks, dtype=np.int64)
    uc = uniform(sub_seed(s, 2), len(reps))
    for k, r in enumerate(reps):
        src[r] = src[int(uc[k] * r)]
    return src


def cdc_input(n_blocks: int = 4096, block: int = 65536,
              repeat_frac: float = 0.2, seed: int | None = None,
              out: np.ndarray | None = None) -> np.ndarray:
    """The chunking workload: seeded 64 KiB blocks, 20 % exact repeats."""
    s = config_seed(3) if seed is None else seed
    src = cdc_layout(n_blocks, repeat_frac, s)
    n = n_blocks * block
    if out is None:
        out = np.empty(n, dtype=np.uint8)
    content = sub_seed(s, 3)
    fresh = np.nonzero(src == np.arange(n_blocks))[0]
    seeds = np.array([splitmix64_at(content, int(b)) for b in fresh],
                     dtype=np.uint64)
    fill_multi(seeds, fresh.astype(np.uint64) * block,
               np.full(len(fresh), block, dtype=np.uint64), out.ctypes.data)
    for b in range(n_blocks):
        if src[b] != b:
            out[b * block:(b + 1) * block] = out[src[b] * block:(src[b] + 1) * block]
    return out


def serving_jobs(n_jobs: int = 20000, load_gbps: float = 20.0,
                 lo: int = 4096, hi: int = 1 << 26, direct_frac: float = 0.7,
                 arena_bytes: int = 4 << 30, seed: int | None = None):
    """Job list of the serving mix.

    Returns dict with int64 ``size``, int32 ``kind`` (0 direct, 1 chunking),
    float64 ``arrival_s`` (scheduled open-loop arrival times), int64
    ``offset`` (4 KiB-aligned slice start in the arena) and the arena seed.
    The arrival rate is load / mean(size) jobs per second.
    """
    s = config_seed(4) if seed is None else seed
    size = log_uniform_int(sub_seed(s, 1), n_jobs, lo, hi)
    size = np.minimum(size, arena_bytes)
    kind = (uniform(sub_seed(s, 2), n_jobs) >= direct_frac).astype(np.int32)
    lam = load_gbps * 1e9 / float(size.mean())
    gaps = -np.log1p(-uniform(sub_seed(s, 3), n_jobs)) / lam
    arrival = np.cumsum(gaps) - gaps[0]
    slots = (arena_bytes - size) // 4096 + 1
    offset = (np.floor(uniform(sub_seed(s, 4), n_jobs) * slots).astype(np.int64)
              * 4096)
    return {"size": size, "kind": kind, "arrival_s": arrival,
            "offset": offset, "arena_seed": sub_seed(s, 5),
            "arena_bytes": arena_bytes, "rate_per_s": lam}


def batch_small(n_buf: int = 1_000_000, lo: int = 512, hi: int = 16384,
                seed: int | None = None):
    """Offsets/lengths of the batched small-buffer workload.

    Lengths are log-uniform in [lo, hi]; each buffer starts on a 16-byte
    boundary right after the previous one.  Returns (offsets uint64,
    lengths uint32, arena_bytes, arena_seed).
    """
    s = config_seed(5) if seed is None else seed
    length = log_uniform_int(sub_seed(s, 1), n_buf, lo, hi)
    padded = (length + 15) // 16 * 16
    off = np.zeros(n_buf, dtype=np.int64)
    if n_buf > 1:
        off[1:] = np.cumsum(padded[:-1])
    arena = int(off[-1] + padded[-1]) if n_buf else 0
    return (off.astype(np.uint64), length.astype(np.uint32), arena,
            sub_seed(s, 2))
