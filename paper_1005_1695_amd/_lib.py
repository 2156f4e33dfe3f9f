"""ctypes prototypes of libcrystal.so (the C ABI in include/crystal.h).

Argument marshalling only: every hashing step runs in the library's HIP
kernels.  Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcrystal.so")

c_vp = ctypes.c_void_p
c_sz = ctypes.c_size_t
c_u64 = ctypes.c_uint64
c_u32 = ctypes.c_uint32
c_i32 = ctypes.c_int32
c_i64 = ctypes.c_int64
c_int = ctypes.c_int

OK = 0
EINVAL, EAGAIN, ENOMEM, EBUSY, ETIMEDOUT, EDEVICE, ESTATE, ECANCELED = range(-1, -9, -1)
PENDING = 1
K_NOP, K_MD5_DIRECT, K_CDC, K_MD5, K_SHA1_DIRECT = 0, 1, 2, 3, 4
NONBLOCK = 1
TUNE_NONE, TUNE_FULL = 0, 1


class crystal_direct_params(ctypes.Structure):
    _fields_ = [("segment_bytes", c_u32), ("reserved", c_u32)]


class crystal_cdc_params(ctypes.Structure):
    _fields_ = [("base", c_u64), ("min_len", c_u64), ("max_len", c_u64),
                ("mask_bits", c_u32), ("window", c_u32)]


class crystal_config(ctypes.Structure):
    _fields_ = [("max_input_bytes", c_sz), ("max_output_bytes", c_sz),
                ("host_pool_bytes", c_sz), ("device_pool_bytes", c_sz),
                ("n_streams", c_u32), ("max_in_flight", c_u32),
                ("device", c_i32), ("flags", c_u32),
                ("device_slab", c_vp), ("streams", ctypes.POINTER(c_vp)),
                ("n_copy_streams", c_u32)]


class crystal_task(ctypes.Structure):
    pass


CALLBACK = ctypes.CFUNCTYPE(None, ctypes.POINTER(crystal_task), c_vp)

crystal_task._fields_ = [
    ("in_bytes", c_sz), ("params", c_vp), ("callback", CALLBACK), ("user", c_vp),
    ("status", c_i32), ("stream_index", c_i32), ("out_bytes", c_sz),
    ("t_submit_ns", c_i64), ("t_admit_ns", c_i64), ("t_done_ns", c_i64),
    ("internal", c_vp * 4)]


class crystal_stats(ctypes.Structure):
    _fields_ = [("submitted", c_u64), ("completed", c_u64), ("failed", c_u64),
                ("bytes_in", c_u64), ("bytes_out", c_u64),
                ("device_pool_bytes", c_u64), ("device_pool_free", c_u64),
                ("device_pool_min_free", c_u64), ("host_pool_bytes", c_u64),
                ("host_pool_free", c_u64), ("outstanding", c_u32), ("running", c_u32)]


class crystal_batch_desc(ctypes.Structure):
    _fields_ = [("d_arena", c_vp), ("d_off", c_vp), ("d_len", c_vp),
                ("n_buf", c_u64), ("d_out", c_vp), ("stream", c_vp)]


class crystal_batch_tuning(ctypes.Structure):
    _fields_ = [("block", c_u32), ("waves_per_simd", c_u32), ("grab", c_u32),
                ("n_streams", c_u32), ("sorted", c_u32), ("depth", c_u32), ("tail", c_u32),
                ("replay_ms", ctypes.c_float)]


class crystal_stage_times(ctypes.Structure):
    _fields_ = [("alloc_ms", ctypes.c_double), ("copy_in_ms", ctypes.c_double),
                ("kernel_ms", ctypes.c_double), ("copy_out_ms", ctypes.c_double),
                ("free_ms", ctypes.c_double), ("total_ms", ctypes.c_double)]


class crystal_drive_job(ctypes.Structure):
    _fields_ = [("h_in", c_vp), ("bytes", c_u64), ("h_out", c_vp), ("out_cap", c_u64),
                ("arrival_s", ctypes.c_double), ("kernel_id", c_i32), ("status", c_i32),
                ("latency_s", ctypes.c_double), ("admit_wait_s", ctypes.c_double)]


class crystal_drive_result(ctypes.Structure):
    _fields_ = [("wall_s", ctypes.c_double), ("bytes", c_u64), ("ok", c_u64),
                ("failed", c_u64)]


P = ctypes.POINTER

# name -> (argtypes, restype); the exported symbols of include/crystal.h
SIGNATURES = {
    "crystal_init": ([P(crystal_config)], c_int),
    "crystal_finalize": ([], c_int),
    "crystal_buffer_acquire": ([c_sz, c_int, P(c_vp)], c_int),
    "crystal_buffer_wrap": ([c_vp, c_sz, P(c_vp)], c_int),
    "crystal_buffer_release": ([c_vp], c_int),
    "crystal_buffer_host": ([c_vp], c_vp),
    "crystal_buffer_size": ([c_vp], c_sz),
    "crystal_submit": ([P(crystal_task), c_int, c_vp, c_vp], c_int),
    "crystal_output_bytes": ([c_int, c_sz, c_vp], c_sz),
    "crystal_wait": ([P(crystal_task), c_i64], c_int),
    "crystal_poll": ([P(crystal_task)], c_int),
    "crystal_last_error": ([], ctypes.c_char_p),
    "crystal_get_stats": ([P(crystal_stats)], c_int),
    "crystal_md5_direct_device": ([c_vp, c_vp, c_vp, c_vp, c_u32, c_u64, c_u32, c_vp,
                                   c_vp, c_vp], c_int),
    "crystal_md5_segments_device": ([c_vp, c_vp, c_vp, c_vp, c_u32, c_u64, c_u32, c_vp,
                                     c_vp], c_int),
    "crystal_md5_roots_device": ([c_vp, c_u32, c_u32, c_vp, c_vp, c_vp], c_int),
    "crystal_sha1_direct_device": ([c_vp, c_vp, c_vp, c_vp, c_u32, c_u64, c_u32, c_vp,
                                    c_vp, c_vp], c_int),
    "crystal_sha1_segments_device": ([c_vp, c_vp, c_vp, c_vp, c_u32, c_u64, c_u32, c_vp,
                                      c_vp], c_int),
    "crystal_sha1_roots_device": ([c_vp, c_u32, c_u32, c_vp, c_vp, c_vp], c_int),
    "crystal_md5_batch_device": ([c_vp, c_vp, c_vp, c_vp, c_u64, c_vp, c_u32, c_u32,
                                  c_vp], c_int),
    "crystal_cdc_workspace_bytes": ([c_u64, P(crystal_cdc_params)], c_sz),
    "crystal_cdc_max_chunks": ([c_u64, P(crystal_cdc_params)], c_u64),
    "crystal_cdc_device": ([c_vp, c_u64, P(crystal_cdc_params), c_vp, c_sz, c_vp, c_vp,
                            c_vp, c_u64, c_vp], c_int),
    "crystal_cdc_candidates_device": ([c_vp, c_u64, P(crystal_cdc_params), c_vp, c_sz,
                                       c_vp, c_vp, c_u64, c_vp], c_int),
    "crystal_cdc_select_device": ([c_u64, P(crystal_cdc_params), c_vp, c_sz, c_vp, c_vp,
                                   c_u64, c_vp], c_int),
    "crystal_md5_chunks_device": ([c_vp, c_vp, c_vp, c_u64, c_vp, c_vp], c_int),
    "crystal_window_hash_device": ([c_vp, c_u64, c_u64, c_vp, c_vp], c_int),
    "crystal_batch_plan": ([P(crystal_batch_desc), c_int, P(crystal_batch_tuning),
                            P(c_vp)], c_int),
    "crystal_batch_run": ([c_vp, c_int], c_int),
    "crystal_batch_get_tuning": ([c_vp, P(crystal_batch_tuning)], c_int),
    "crystal_batch_free": ([c_vp], None),
    "crystal_naive_run": ([c_int, c_vp, c_vp, c_sz, c_vp, c_sz, P(c_sz),
                           P(crystal_stage_times)], c_int),
    "crystal_drive": ([P(crystal_drive_job), c_u64, P(crystal_direct_params),
                       P(crystal_cdc_params), c_u32, P(crystal_drive_result)], c_int),
}

_lib = None
MISSING: list[str] = []


def load():
    """Load libcrystal.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with "
                "`python -c 'import __graft_entry__ as g; g.build()'` "
                "(hipcc --offload-arch=gfx950); there is no fallback path")
        lib = ctypes.CDLL(LIB_PATH, mode=ctypes.RTLD_GLOBAL)
        MISSING.clear()
        for name, (args, res) in SIGNATURES.items():
            fn = getattr(lib, name, None)
            if fn is None:
                MISSING.append(name)
                continue
            fn.argtypes = args
            fn.restype = res
        _lib = lib
    return _lib


def last_error() -> str:
    msg = load().crystal_last_error()
    return msg.decode() if msg else ""


class CrystalError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what} failed with {code}: {last_error()}")
        self.code = code


def check(rc: int, what: str) -> int:
    if rc < 0:
        raise CrystalError(rc, what)
    return rc
