"""MI355X hashing-offload library (CrystalGPU-style job layer + HIP kernels).

Python side of the C ABI in ``include/crystal.h``.  Functions named like the
C entry points marshal arguments to them; the helpers below them allocate
device memory and pick the current stream through PyTorch, which serves here
only as device-memory and stream plumbing.  Every hashing step runs in the HIP
kernels of ``libcrystal.so``; if that library is missing, calls raise.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib
from ._lib import (CALLBACK, CrystalError, K_CDC, K_MD5, K_MD5_DIRECT, K_NOP,
                   NONBLOCK, PENDING, check, crystal_batch_desc,
                   crystal_batch_tuning, crystal_cdc_params, crystal_config,
                   crystal_direct_params, crystal_drive_job,
                   crystal_drive_result, crystal_stage_times, crystal_stats,
                   crystal_task, last_error, load)

__all__ = [n for n in dir() if not n.startswith("_")]

DEFAULT_SEGMENT = 4096


def _ptr(x) -> int:
    if x is None:
        return 0
    if isinstance(x, int):
        return x
    if hasattr(x, "data_ptr"):
        return x.data_ptr()
    if isinstance(x, np.ndarray):
        return x.ctypes.data
    raise TypeError(f"cannot take the address of {type(x)}")


def _stream(s) -> int:
    if s is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(s, int):
        return s
    return s.cuda_stream


def cdc_params(base: int, min_len: int = 2048, max_len: int = 65536,
               mask_bits: int = 13) -> crystal_cdc_params:
    return crystal_cdc_params(base=base & ((1 << 64) - 1), min_len=min_len,
                              max_len=max_len, mask_bits=mask_bits, window=48)


# ----------------------------------------------------------- same-name calls

def crystal_md5_direct_device(d_in, d_job_off, d_job_len, d_seg_base, n_jobs,
                              n_segments, segment_bytes, d_seg_digests, d_roots,
                              stream=None):
    return check(load().crystal_md5_direct_device(
        _ptr(d_in), _ptr(d_job_off), _ptr(d_job_len), _ptr(d_seg_base), n_jobs,
        n_segments, segment_bytes, _ptr(d_seg_digests), _ptr(d_roots),
        _stream(stream)), "crystal_md5_direct_device")


def crystal_md5_batch_device(d_arena, d_off, d_len, d_order, n_buf, d_out,
                             block=0, grid=0, stream=None):
    return check(load().crystal_md5_batch_device(
        _ptr(d_arena), _ptr(d_off), _ptr(d_len), _ptr(d_order), n_buf, _ptr(d_out),
        block, grid, _stream(stream)), "crystal_md5_batch_device")


def crystal_cdc_workspace_bytes(n: int, params: crystal_cdc_params) -> int:
    return load().crystal_cdc_workspace_bytes(n, ctypes.byref(params))


def crystal_cdc_max_chunks(n: int, params: crystal_cdc_params) -> int:
    return load().crystal_cdc_max_chunks(n, ctypes.byref(params))


def crystal_cdc_device(d_in, n, params, d_ws, ws_bytes, d_n_chunks, d_ends,
                       d_digests, cap, stream=None):
    return check(load().crystal_cdc_device(
        _ptr(d_in), n, ctypes.byref(params), _ptr(d_ws), ws_bytes, _ptr(d_n_chunks),
        _ptr(d_ends), _ptr(d_digests), cap, _stream(stream)), "crystal_cdc_device")


def crystal_cdc_candidates_device(d_in, n, params, d_ws, ws_bytes, d_count,
                                  d_cand, cap, stream=None):
    return check(load().crystal_cdc_candidates_device(
        _ptr(d_in), n, ctypes.byref(params), _ptr(d_ws), ws_bytes, _ptr(d_count),
        _ptr(d_cand), cap, _stream(stream)), "crystal_cdc_candidates_device")


def crystal_cdc_select_device(n, params, d_ws, ws_bytes, d_n_chunks, d_ends, cap,
                              stream=None):
    return check(load().crystal_cdc_select_device(
        n, ctypes.byref(params), _ptr(d_ws), ws_bytes, _ptr(d_n_chunks), _ptr(d_ends),
        cap, _stream(stream)), "crystal_cdc_select_device")


def crystal_md5_chunks_device(d_in, d_ends, d_n_chunks, cap, d_digests,
                              stream=None):
    return check(load().crystal_md5_chunks_device(
        _ptr(d_in), _ptr(d_ends), _ptr(d_n_chunks), cap, _ptr(d_digests),
        _stream(stream)), "crystal_md5_chunks_device")


def crystal_window_hash_device(d_in, n, base, d_w, stream=None):
    return check(load().crystal_window_hash_device(
        _ptr(d_in), n, base & ((1 << 64) - 1), _ptr(d_w), _stream(stream)),
        "crystal_window_hash_device")


# ------------------------------------------------ tensor helpers (plumbing)

def to_device_bytes(data, device="cuda"):
    """Host bytes -> device uint8 tensor, padded to a 16-byte multiple."""
    import torch
    a = np.ascontiguousarray(np.asarray(data, dtype=np.uint8).reshape(-1))
    n = a.size
    t = torch.zeros(((n + 15) // 16) * 16 + 16, dtype=torch.uint8, device=device)
    if n:
        t[:n].copy_(torch.from_numpy(a))
    return t, n


def seg_table(job_lengths, segment: int = DEFAULT_SEGMENT):
    lens = np.asarray(job_lengths, dtype=np.uint64)
    nseg = (lens + np.uint64(segment - 1)) // np.uint64(segment)
    base = np.zeros(len(lens) + 1, dtype=np.uint64)
    base[1:] = np.cumsum(nseg)
    return base


def direct_device(d_in, job_offsets, job_lengths, segment: int = DEFAULT_SEGMENT,
                  stream=None):
    """Direct hashing of several jobs already resident in d_in.

    Returns (segment digests [S,16], roots [J,16], seg_base) as device tensors
    (seg_base as numpy)."""
    import torch
    dev = d_in.device
    off = np.asarray(job_offsets, dtype=np.uint64)
    ln = np.asarray(job_lengths, dtype=np.uint64)
    base = seg_table(ln, segment)
    S = int(base[-1])
    t_off = torch.from_numpy(off.view(np.int64)).to(dev)
    t_len = torch.from_numpy(ln.view(np.int64)).to(dev)
    t_base = torch.from_numpy(base.view(np.int64)).to(dev)
    seg = torch.empty((max(S, 1), 16), dtype=torch.uint8, device=dev)
    roots = torch.empty((max(len(off), 1), 16), dtype=torch.uint8, device=dev)
    crystal_md5_direct_device(d_in, t_off, t_len, t_base, len(off), S, segment,
                              seg, roots, stream)
    return seg[:S], roots[:len(off)], base, (t_off, t_len, t_base)


def cdc_device(d_in, n: int, params: crystal_cdc_params, stream=None):
    """Whole chunking pipeline on d_in[0, n). Returns (ends, digests) tensors."""
    import torch
    dev = d_in.device
    ws_bytes = crystal_cdc_workspace_bytes(n, params)
    cap = max(crystal_cdc_max_chunks(n, params), 1)
    ws = torch.empty(max(ws_bytes, 256), dtype=torch.uint8, device=dev)
    cnt = torch.zeros(1, dtype=torch.int64, device=dev)
    ends = torch.empty(cap, dtype=torch.int64, device=dev)
    dig = torch.empty((cap, 16), dtype=torch.uint8, device=dev)
    crystal_cdc_device(d_in, n, params, ws, ws_bytes, cnt, ends, dig, cap, stream)
    m = int(cnt.item())
    return ends[:m], dig[:m]


def batch_device(d_arena, offsets, lengths, order=None, block=256, grid=0,
                 stream=None):
    import torch
    dev = d_arena.device
    off = torch.from_numpy(np.asarray(offsets, dtype=np.uint64).view(np.int64)).to(dev)
    ln = torch.from_numpy(np.asarray(lengths, dtype=np.uint32).view(np.int32)).to(dev)
    o = None
    if order is not None:
        o = torch.from_numpy(np.asarray(order, dtype=np.uint32).view(np.int32)).to(dev)
    n = off.numel()
    out = torch.empty((max(n, 1), 16), dtype=torch.uint8, device=dev)
    crystal_md5_batch_device(d_arena, off, ln, o, n, out, block, grid, stream)
    return out[:n]
