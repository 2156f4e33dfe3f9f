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
from ._lib import (CALLBACK, CrystalError, K_CDC, K_MD5, K_MD5_DIRECT, K_NOP, K_SHA1_DIRECT,
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


def crystal_md5_segments_device(d_in, d_job_off, d_job_len, d_seg_base, n_jobs,
                                n_segments, segment_bytes, d_seg_digests, stream=None):
    return check(load().crystal_md5_segments_device(
        _ptr(d_in), _ptr(d_job_off), _ptr(d_job_len), _ptr(d_seg_base), n_jobs,
        n_segments, segment_bytes, _ptr(d_seg_digests), _stream(stream)),
        "crystal_md5_segments_device")


def crystal_md5_roots_device(d_seg_base, n_jobs, segment_bytes, d_seg_digests,
                             d_roots, stream=None):
    return check(load().crystal_md5_roots_device(
        _ptr(d_seg_base), n_jobs, segment_bytes, _ptr(d_seg_digests), _ptr(d_roots),
        _stream(stream)), "crystal_md5_roots_device")


def crystal_sha1_direct_device(d_in, d_job_off, d_job_len, d_seg_base, n_jobs,
                               n_segments, segment_bytes, d_seg_digests, d_roots,
                               stream=None):
    return check(load().crystal_sha1_direct_device(
        _ptr(d_in), _ptr(d_job_off), _ptr(d_job_len), _ptr(d_seg_base), n_jobs,
        n_segments, segment_bytes, _ptr(d_seg_digests), _ptr(d_roots),
        _stream(stream)), "crystal_sha1_direct_device")


def crystal_sha1_segments_device(d_in, d_job_off, d_job_len, d_seg_base, n_jobs,
                                 n_segments, segment_bytes, d_seg_digests, stream=None):
    return check(load().crystal_sha1_segments_device(
        _ptr(d_in), _ptr(d_job_off), _ptr(d_job_len), _ptr(d_seg_base), n_jobs,
        n_segments, segment_bytes, _ptr(d_seg_digests), _stream(stream)),
        "crystal_sha1_segments_device")


def crystal_sha1_roots_device(d_seg_base, n_jobs, segment_bytes, d_seg_digests,
                              d_roots, stream=None):
    return check(load().crystal_sha1_roots_device(
        _ptr(d_seg_base), n_jobs, segment_bytes, _ptr(d_seg_digests), _ptr(d_roots),
        _stream(stream)), "crystal_sha1_roots_device")


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
                  stream=None, hash: str = "md5"):
    """Direct hashing of several jobs already resident in d_in, with MD5
    (hash="md5", 16-byte digests) or SHA-1 (hash="sha1", 20-byte digests).

    Returns (segment digests [S,D], roots [J,D], seg_base) as device tensors
    (seg_base as numpy)."""
    import torch
    dev = d_in.device
    width, fn = ((16, crystal_md5_direct_device) if hash == "md5" else
                 (20, crystal_sha1_direct_device))
    off = np.asarray(job_offsets, dtype=np.uint64)
    ln = np.asarray(job_lengths, dtype=np.uint64)
    base = seg_table(ln, segment)
    S = int(base[-1])
    t_off = torch.from_numpy(off.view(np.int64)).to(dev)
    t_len = torch.from_numpy(ln.view(np.int64)).to(dev)
    t_base = torch.from_numpy(base.view(np.int64)).to(dev)
    # digest array padded to a multiple of 16 bytes (the root loader reads
    # whole 16-byte vectors)
    flat = torch.empty(((max(S, 1) * width + 15) // 16) * 16, dtype=torch.uint8, device=dev)
    seg = flat[:max(S, 1) * width].view(max(S, 1), width)
    roots = torch.empty((max(len(off), 1), width), dtype=torch.uint8, device=dev)
    fn(d_in, t_off, t_len, t_base, len(off), S, segment, seg, roots, stream)
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


# ------------------------------------------------------------------ job API

def crystal_init(max_input_bytes: int, max_output_bytes: int = 0,
                 host_pool_bytes: int = 0, device_pool_bytes: int = 0,
                 n_streams: int = 0, max_in_flight: int = 0, device: int = 0,
                 device_slab=None, streams=None, n_copy_streams: int = 0) -> None:
    cfg = crystal_config(max_input_bytes=max_input_bytes,
                         max_output_bytes=max_output_bytes,
                         host_pool_bytes=host_pool_bytes,
                         device_pool_bytes=device_pool_bytes,
                         n_streams=n_streams, max_in_flight=max_in_flight,
                         device=device, flags=0,
                         device_slab=_ptr(device_slab) or None,
                         n_copy_streams=n_copy_streams)
    keep = None
    if streams:  # [copy-in streams (n_copy_streams, default 1), compute streams...]
        keep = (ctypes.c_void_p * len(streams))(*[_stream(s) for s in streams])
        cfg.n_streams = len(streams) - (n_copy_streams or 1)
        cfg.streams = ctypes.cast(keep, ctypes.POINTER(ctypes.c_void_p))
    check(load().crystal_init(ctypes.byref(cfg)), "crystal_init")


def crystal_finalize() -> None:
    check(load().crystal_finalize(), "crystal_finalize")


def crystal_buffer_acquire(nbytes: int, flags: int = 0) -> int:
    h = ctypes.c_void_p()
    check(load().crystal_buffer_acquire(nbytes, flags, ctypes.byref(h)),
          "crystal_buffer_acquire")
    return h.value


def crystal_buffer_wrap(host_ptr, nbytes: int) -> int:
    h = ctypes.c_void_p()
    check(load().crystal_buffer_wrap(_ptr(host_ptr), nbytes, ctypes.byref(h)),
          "crystal_buffer_wrap")
    return h.value


def crystal_buffer_release(buf: int) -> None:
    check(load().crystal_buffer_release(buf), "crystal_buffer_release")


def crystal_buffer_host(buf: int) -> int:
    return load().crystal_buffer_host(buf)


def crystal_buffer_size(buf: int) -> int:
    return load().crystal_buffer_size(buf)


def buffer_view(buf: int) -> np.ndarray:
    """numpy uint8 view of a buffer's host memory (no copy)."""
    n = crystal_buffer_size(buf)
    if n == 0:
        return np.zeros(0, dtype=np.uint8)
    addr = crystal_buffer_host(buf)
    return np.ctypeslib.as_array((ctypes.c_uint8 * n).from_address(addr))


def crystal_output_bytes(kernel_id: int, in_bytes: int, params=None) -> int:
    return load().crystal_output_bytes(kernel_id, in_bytes,
                                       ctypes.byref(params) if params is not None else None)


def crystal_submit(task: crystal_task, kernel_id: int, inb: int, outb: int) -> None:
    check(load().crystal_submit(ctypes.byref(task), kernel_id, inb, outb),
          "crystal_submit")


def crystal_wait(task: crystal_task, timeout_ns: int = -1) -> int:
    return load().crystal_wait(ctypes.byref(task), timeout_ns)


def crystal_poll(task: crystal_task) -> int:
    return load().crystal_poll(ctypes.byref(task))


def crystal_get_stats() -> crystal_stats:
    s = crystal_stats()
    check(load().crystal_get_stats(ctypes.byref(s)), "crystal_get_stats")
    return s


def new_task(in_bytes: int, params=None, callback=None, user=None) -> crystal_task:
    t = crystal_task()
    t.in_bytes = in_bytes
    if params is not None:
        t.params = ctypes.cast(ctypes.byref(params), ctypes.c_void_p)
        t._params_ref = params
    if callback is not None:
        cb = CALLBACK(callback)
        t.callback = cb
        t._cb_ref = cb
    t.user = user
    return t


# ---------------------------------------------------------------- batching

def crystal_batch_plan(d_arena, d_off, d_len, n_buf: int, d_out, stream=None,
                       tune: int = 0, fixed: crystal_batch_tuning | None = None) -> int:
    desc = crystal_batch_desc(d_arena=_ptr(d_arena), d_off=_ptr(d_off),
                              d_len=_ptr(d_len), n_buf=n_buf, d_out=_ptr(d_out),
                              stream=_stream(stream))
    h = ctypes.c_void_p()
    check(load().crystal_batch_plan(ctypes.byref(desc), tune,
                                    ctypes.byref(fixed) if fixed is not None else None,
                                    ctypes.byref(h)), "crystal_batch_plan")
    return h.value


def crystal_batch_run(plan: int, iters: int = 1) -> None:
    check(load().crystal_batch_run(plan, iters), "crystal_batch_run")


def crystal_batch_get_tuning(plan: int) -> crystal_batch_tuning:
    t = crystal_batch_tuning()
    check(load().crystal_batch_get_tuning(plan, ctypes.byref(t)),
          "crystal_batch_get_tuning")
    return t


def crystal_batch_free(plan: int) -> None:
    load().crystal_batch_free(plan)


# -------------------------------------------------------------- naive path

def crystal_naive_run(kernel_id: int, params, h_in, n: int, h_out, out_cap: int):
    ob = ctypes.c_size_t()
    st = crystal_stage_times()
    check(load().crystal_naive_run(kernel_id,
                                   ctypes.byref(params) if params is not None else None,
                                   _ptr(h_in), n, _ptr(h_out), out_cap, ctypes.byref(ob),
                                   ctypes.byref(st)), "crystal_naive_run")
    return ob.value, st


# ------------------------------------------------------------------ driver

def crystal_drive(jobs, direct=None, cdc=None, window: int = 0) -> crystal_drive_result:
    """jobs: a ctypes array of crystal_drive_job (filled in place)."""
    res = crystal_drive_result()
    check(load().crystal_drive(jobs, len(jobs),
                               ctypes.byref(direct) if direct is not None else None,
                               ctypes.byref(cdc) if cdc is not None else None,
                               window, ctypes.byref(res)), "crystal_drive")
    return res


def parse_cdc_output(buf: np.ndarray):
    """Split a chunking job's output into (ends uint64[n], digests uint8[n,16])."""
    n = int(buf[:8].view(np.uint64)[0])
    ends = buf[8:8 + 8 * n].view(np.uint64)
    dig = buf[8 + 8 * n:8 + 24 * n].reshape(n, 16)
    return ends, dig
