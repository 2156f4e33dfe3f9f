#!/usr/bin/env python3
"""Measurements of the other four workloads on one MI355X (bench.py covers
the streamed direct-hashing one).  Prints one JSON object per workload.

  direct_one   1 MiB direct hashing as one job: per-job latency (mean, 95 %
               CI, over >= 30 runs) through the job layer on one stream and
               through the naive per-job path; device-resident kernel times.
  chunking     256 MiB content-defined chunking (20 % repeated 64 KiB blocks):
               device-resident time per kernel, and host-fed GB/s as one job
               through the job layer vs the naive path.
  serving      Poisson arrivals of jobs of 4 KiB..64 MiB (70 % direct, 30 %
               chunking) from a 4 GiB pinned arena, device pool capped at
               16 GiB, swept over offered loads: achieved GB/s, p50/p99/p99.9
               latency from the scheduled arrival, admission wait.
  overhead     framework overhead per job with an empty kernel, by size
               (job layer vs naive path vs the copies alone).
  naive_stages stage breakdown of the naive direct-hashing path by size.
  stream_len   streams of 1..64 jobs of 1 MiB: job layer vs naive path.
  sha1_stream  256 jobs x 8 MiB of direct hashing with SHA-1: device-resident
               kernel times and ALU fraction; host-fed job layer vs naive.
  batch        1 000 000 buffers of 512 B..16 KiB resident on the device:
               tuned persistent plan (replay time, GB/s, integer-ALU and HBM
               fractions) vs one launch per buffer (timed on a sample).

Correctness is the test suite's job; this script only cross-checks GPU paths
against each other.  Usage: python bench_workloads.py [--only NAME] [--quick]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import statistics
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

OPS_PER_COMPRESSION = 64 * 5 + 4          # gfx950 VALU ops per MD5 block (see bench.py)
INT32_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
HBM_PEAK_GBPS = 8000.0
LINK_PEAK_GBPS = 63.0


def ci95(xs):
    xs = [float(x) for x in xs]
    m = statistics.mean(xs)
    if len(xs) < 2:
        return m, 0.0
    return m, 1.96 * statistics.stdev(xs) / math.sqrt(len(xs))


def pct(xs, q):
    return float(np.percentile(np.asarray(xs, dtype=np.float64), q))


def comp(length) -> int:
    return (int(length) + 8) // 64 + 1


def out(name, d):
    d = {"workload": name, **d}
    print(json.dumps(d), flush=True)
    return d


# ------------------------------------------------------------------ direct_one

def direct_one(P, torch, gen, reps=50):
    n = 1 << 20
    data = gen.direct_one(n)
    direct = P.crystal_direct_params(segment_bytes=4096)
    cap = P.crystal_output_bytes(P.K_MD5_DIRECT, n, direct)
    P.crystal_init(max_input_bytes=n, host_pool_bytes=16 << 20, device_pool_bytes=64 << 20,
                   n_streams=1)
    try:
        inb = P.crystal_buffer_acquire(n)
        P.buffer_view(inb)[:] = data
        outb = P.crystal_buffer_acquire(cap)
        lat, adm = [], []
        for r in range(reps + 5):
            t = P.new_task(n, direct)
            P.crystal_submit(t, P.K_MD5_DIRECT, inb, outb)
            assert P.crystal_wait(t) == 0
            if r >= 5:
                lat.append((t.t_done_ns - t.t_submit_ns) / 1e3)
                adm.append((t.t_admit_ns - t.t_submit_ns) / 1e3)
        job_root = bytes(P.buffer_view(outb)[cap - 16:cap])
        P.crystal_buffer_release(inb)
        P.crystal_buffer_release(outb)
    finally:
        P.crystal_finalize()
    host = torch.from_numpy(data).pin_memory()
    o = np.zeros(cap, np.uint8)
    nv = []
    for r in range(reps + 5):
        _, st = P.crystal_naive_run(P.K_MD5_DIRECT, direct, host.data_ptr(), n, o, cap)
        if r >= 5:
            nv.append(st.total_ms * 1e3)
    # device-resident kernel times
    d, _ = P.to_device_bytes(data)
    lens = np.array([n], np.uint64)
    base = P.seg_table(lens)
    tb = torch.from_numpy(base.view(np.int64)).cuda()
    toff = torch.zeros(1, dtype=torch.int64, device="cuda")
    tlen = torch.from_numpy(lens.view(np.int64)).cuda()
    seg = torch.empty((256, 16), dtype=torch.uint8, device="cuda")
    roots = torch.empty((1, 16), dtype=torch.uint8, device="cuda")
    s = torch.cuda.current_stream()
    ks, kr = [], []
    for r in range(reps + 5):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        e[0].record(s)
        P.crystal_md5_segments_device(d, toff, tlen, tb, 1, 256, 4096, seg, s.cuda_stream)
        e[1].record(s)
        P.crystal_md5_roots_device(tb, 1, 4096, seg, roots, s.cuda_stream)
        e[2].record(s)
        e[2].synchronize()
        if r >= 5:
            ks.append(e[0].elapsed_time(e[1]) * 1e3)
            kr.append(e[1].elapsed_time(e[2]) * 1e3)
    m, c = ci95(lat)
    nm, nc = ci95(nv)
    return out("direct_one", {
        "bytes": n, "runs": reps,
        "job_latency_us": {"mean": round(m, 1), "ci95": round(c, 1), "p50": round(pct(lat, 50), 1),
                           "p99": round(pct(lat, 99), 1)},
        "job_admit_us_mean": round(statistics.mean(adm), 1),
        "naive_latency_us": {"mean": round(nm, 1), "ci95": round(nc, 1),
                             "p50": round(pct(nv, 50), 1)},
        "speedup_vs_naive": round(nm / m, 2),
        "device_kernels_us": {"segments": round(statistics.mean(ks), 1),
                              "root": round(statistics.mean(kr), 1)},
        "chain_bound_note": "65 + 65 serial compressions per lane plus 1 MiB over the link",
        "job_root_matches_device": job_root == bytes(roots[0].cpu().numpy()),
    })


# -------------------------------------------------------------------- overhead

def overhead(P, torch, gen, reps=30, sizes=(4 << 10, 64 << 10, 1 << 20, 8 << 20, 64 << 20)):
    """Framework overhead per job (the paper's Sec. 5.1 dummy kernel, Fig. 5):
    one job at a time that copies n bytes in, runs an empty kernel and copies n
    bytes back, through the job layer and through the naive path; overhead =
    job latency minus the two pinned copies timed alone."""
    rows = []
    P.crystal_init(max_input_bytes=max(sizes), host_pool_bytes=2 * max(sizes) + (64 << 20),
                   device_pool_bytes=2 * max(sizes) + (64 << 20), n_streams=1)
    try:
        dev = torch.empty(max(sizes), dtype=torch.uint8, device="cuda")
        hbuf = torch.empty(max(sizes), dtype=torch.uint8).pin_memory()
        for n in sizes:
            inb = P.crystal_buffer_acquire(n)
            outb = P.crystal_buffer_acquire(n)
            P.buffer_view(inb)[:] = gen.random_bytes(n + 11, n)
            lat = []
            for r in range(reps + 3):
                t = P.new_task(n, None)
                P.crystal_submit(t, P.K_NOP, inb, outb)
                assert P.crystal_wait(t) == 0
                if r >= 3:
                    lat.append((t.t_done_ns - t.t_submit_ns) / 1e3)
            assert bytes(P.buffer_view(outb)[:64]) == bytes(P.buffer_view(inb)[:64])
            P.crystal_buffer_release(inb)
            P.crystal_buffer_release(outb)
            cp = []
            for r in range(reps + 3):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                dev[:n].copy_(hbuf[:n], non_blocking=True)
                hbuf[:n].copy_(dev[:n], non_blocking=True)
                torch.cuda.synchronize()
                if r >= 3:
                    cp.append((time.perf_counter() - t0) * 1e6)
            o = np.zeros(n, np.uint8)
            nv, alloc, free = [], [], []
            for r in range(min(reps, 10) + 2):
                _, st = P.crystal_naive_run(P.K_NOP, None, hbuf.data_ptr(), n, o, n)
                if r >= 2:
                    nv.append(st.total_ms * 1e3)
                    alloc.append(st.alloc_ms * 1e3)
                    free.append(st.free_ms * 1e3)
            m, c = ci95(lat)
            cm, _ = ci95(cp)
            nm, nc = ci95(nv)
            rows.append({"bytes": n, "job_us": round(m, 1), "job_ci95_us": round(c, 1),
                         "copies_alone_us": round(cm, 1),
                         "framework_overhead_us": round(m - cm, 1),
                         "naive_us": round(nm, 1), "naive_ci95_us": round(nc, 1),
                         "naive_alloc_us": round(statistics.mean(alloc), 1),
                         "naive_free_us": round(statistics.mean(free), 1)})
    finally:
        P.crystal_finalize()
    return out("overhead", {"rows": rows, "reps": reps,
                            "note": "job layer: pooled buffers, one compute stream, "
                                    "one job in flight"})


# --------------------------------------------------------------- naive stages

def naive_stages(P, torch, gen, sizes=(64 << 10, 1 << 20, 8 << 20, 64 << 20), reps=5):
    """Stage breakdown of the naive per-job direct-hashing path (the paper's
    Fig. 6): allocation, copy in, kernels, copy out, free."""
    rows = []
    direct = P.crystal_direct_params(segment_bytes=4096)
    for n in sizes:
        host = torch.from_numpy(gen.random_bytes(n + 5, n)).pin_memory()
        cap = P.crystal_output_bytes(P.K_MD5_DIRECT, n, direct)
        o = np.zeros(cap, np.uint8)
        acc = {k: [] for k in ("alloc_ms", "copy_in_ms", "kernel_ms", "copy_out_ms",
                               "free_ms", "total_ms")}
        for r in range(reps + 1):
            _, st = P.crystal_naive_run(P.K_MD5_DIRECT, direct, host.data_ptr(), n, o, cap)
            if r >= 1:
                for k in acc:
                    acc[k].append(getattr(st, k))
        row = {"bytes": n, **{k: round(statistics.mean(v), 4) for k, v in acc.items()}}
        row["alloc_share"] = round(row["alloc_ms"] / row["total_ms"], 3)
        rows.append(row)
    return out("naive_stages", {"rows": rows})


# ----------------------------------------------------------------- stream_len

def stream_len(P, torch, gen, lengths=(1, 2, 4, 8, 16, 32, 64)):
    """A stream of L jobs of 1 MiB direct hashing (the paper's Fig. 8): all L
    submitted at once through the job layer (pooled buffers, copy/compute
    overlap, batching) vs the naive path run L times; wall time per stream."""
    n = 1 << 20
    direct = P.crystal_direct_params(segment_bytes=4096)
    cap = P.crystal_output_bytes(P.K_MD5_DIRECT, n, direct)
    L_max = max(lengths)
    host = torch.empty(L_max * n, dtype=torch.uint8).pin_memory()
    gen.fill(gen.sub_seed(gen.config_seed(1), 9), host.data_ptr(), L_max * n)
    outs = torch.empty((L_max, cap), dtype=torch.uint8).pin_memory()
    rows = []
    P.crystal_init(max_input_bytes=n, host_pool_bytes=16 << 20, device_pool_bytes=1 << 30,
                   n_streams=3, max_in_flight=64)
    try:
        for L in lengths:
            jobs = (P.crystal_drive_job * L)()
            for k in range(L):
                jobs[k].h_in = host.data_ptr() + k * n
                jobs[k].bytes = n
                jobs[k].h_out = outs.data_ptr() + k * cap
                jobs[k].out_cap = cap
                jobs[k].kernel_id = P.K_MD5_DIRECT
            P.crystal_drive(jobs, direct, None, window=0)  # warm
            walls = []
            for r in range(10):
                res = P.crystal_drive(jobs, direct, None, window=0)
                assert res.ok == L
                walls.append(res.wall_s * 1e3)
            o = np.zeros(cap, np.uint8)
            t0 = time.perf_counter()
            for k in range(L):
                P.crystal_naive_run(P.K_MD5_DIRECT, direct, host.data_ptr() + k * n, n, o, cap)
            naive_ms = (time.perf_counter() - t0) * 1e3
            jm = statistics.median(walls)
            rows.append({"jobs": L, "pipelined_ms": round(jm, 3), "naive_ms": round(naive_ms, 3),
                         "speedup": round(naive_ms / jm, 2),
                         "pipelined_gbps": round(L * n / 1e9 / (jm / 1e3), 2)})
    finally:
        P.crystal_finalize()
    return out("stream_len", {"job_bytes": n, "rows": rows})


# ----------------------------------------------------------------- sha1_stream

OPS_PER_SHA1_COMPRESSION = 80 * 5 + 64 * 3 + 5 + 16  # steps, schedule, state adds, byte swaps


def sha1_stream(P, torch, gen, reps=10, n_streams=3, window=24):
    """The streamed direct-hashing workload with SHA-1 (the digest the paper's
    own measurements use): 256 jobs x 8 MiB.  Device-resident kernel times
    (segments, roots, a serial step) with the segment kernel's integer-ALU
    fraction; host-fed through the job layer (closed loop) vs the naive path."""
    n_jobs, job = 256, 8 << 20
    total = n_jobs * job
    seeds = gen.direct_stream_seeds(n_jobs)
    host = torch.empty(total, dtype=torch.uint8).pin_memory()
    gen.fill_multi(seeds, np.arange(n_jobs, dtype=np.uint64) * np.uint64(job),
                   np.full(n_jobs, job, dtype=np.uint64), host.data_ptr())
    d = host.to("cuda")
    lens = np.full(n_jobs, job, dtype=np.uint64)
    base = P.seg_table(lens)
    n_seg = int(base[-1])
    t_off = torch.from_numpy((np.arange(n_jobs, dtype=np.uint64) * np.uint64(job))
                             .view(np.int64)).cuda()
    t_len = torch.from_numpy(lens.view(np.int64)).cuda()
    t_base = torch.from_numpy(base.view(np.int64)).cuda()
    seg = torch.empty((n_seg, 20), dtype=torch.uint8, device="cuda")
    roots = torch.empty((n_jobs, 20), dtype=torch.uint8, device="cuda")
    s = torch.cuda.current_stream()
    ts, tr, tt = [], [], []
    for r in range(reps + 2):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        e[0].record(s)
        P.crystal_sha1_segments_device(d, t_off, t_len, t_base, n_jobs, n_seg, 4096, seg,
                                       s.cuda_stream)
        e[1].record(s)
        P.crystal_sha1_roots_device(t_base, n_jobs, 4096, seg, roots, s.cuda_stream)
        e[2].record(s)
        e[2].synchronize()
        if r >= 2:
            ts.append(e[0].elapsed_time(e[1]))
            tr.append(e[1].elapsed_time(e[2]))
            tt.append(e[0].elapsed_time(e[2]))
    seg_ms, root_ms, step_ms = (statistics.mean(x) for x in (ts, tr, tt))
    comps = n_seg * comp(4096)
    alu = comps * OPS_PER_SHA1_COMPRESSION / (seg_ms / 1e3) / 1e12
    dev_roots = roots.cpu().numpy()
    # host-fed: job layer (closed loop, 12 jobs in the system) vs naive path
    direct = P.crystal_direct_params(segment_bytes=4096)
    cap = P.crystal_output_bytes(P.K_SHA1_DIRECT, job, direct)
    outs = torch.empty((n_jobs, cap), dtype=torch.uint8).pin_memory()
    P.crystal_init(max_input_bytes=job, host_pool_bytes=64 << 20, device_pool_bytes=1 << 30,
                   n_streams=n_streams, max_in_flight=max(24, 2 * window))
    try:
        jobs = (P.crystal_drive_job * n_jobs)()
        for j in range(n_jobs):
            jobs[j].h_in = host.data_ptr() + j * job
            jobs[j].bytes = job
            jobs[j].h_out = outs.data_ptr() + j * cap
            jobs[j].out_cap = cap
            jobs[j].kernel_id = P.K_SHA1_DIRECT
        P.crystal_drive(jobs, direct, None, window=window)
        best = None
        for _ in range(3):
            res = P.crystal_drive(jobs, direct, None, window=window)
            lat = [jobs[j].latency_s * 1e3 for j in range(n_jobs)]
            g = res.bytes / 1e9 / res.wall_s
            if best is None or g > best[0]:
                best = (g, lat)
        same = all(bytes(outs[j, cap - 20:].numpy()) == dev_roots[j].tobytes()
                   for j in (0, 100, 255))
    finally:
        P.crystal_finalize()
    o = np.zeros(cap, np.uint8)
    t0 = time.perf_counter()
    nl = []
    for j in range(n_jobs):
        _, st = P.crystal_naive_run(P.K_SHA1_DIRECT, direct, host.data_ptr() + j * job, job,
                                    o, cap)
        nl.append(st.total_ms)
    naive = total / 1e9 / (time.perf_counter() - t0)
    return out("sha1_stream", {
        "jobs": n_jobs, "job_bytes": job,
        "device_ms": {"segments": round(seg_ms, 4), "roots": round(root_ms, 4),
                      "serial_step": round(step_ms, 4)},
        "device_gbps_serial_step": round(total / 1e9 / (step_ms / 1e3), 1),
        "segments_alu_tops": round(alu, 2), "segments_alu_frac": round(alu / INT32_PEAK_TOPS, 4),
        "ops_per_compression": OPS_PER_SHA1_COMPRESSION,
        "root_us_per_compression": round(root_ms * 1e3 / comp(20 * 2048), 3),
        "pipelined_streams": n_streams, "pipelined_window": window,
        "pipelined_gbps": round(best[0], 2), "pipelined_p50_ms": round(pct(best[1], 50), 3),
        "pipelined_p99_ms": round(pct(best[1], 99), 3),
        "naive_gbps": round(naive, 2), "naive_p50_ms": round(pct(nl, 50), 3),
        "speedup_vs_naive": round(best[0] / naive, 2),
        "link_frac": round(best[0] / LINK_PEAK_GBPS, 4),
        "job_roots_match_device": bool(same),
    })


# -------------------------------------------------------------------- chunking

def chunking(P, torch, gen, reps=10):
    n = 256 << 20
    base = gen.cdc_base()
    params = P.cdc_params(base)
    host = torch.empty(n, dtype=torch.uint8).pin_memory()
    gen.cdc_input(out=host.numpy())
    d = torch.empty(n + 256, dtype=torch.uint8, device="cuda")
    d[:n].copy_(host)
    ws_bytes = P.crystal_cdc_workspace_bytes(n, params)
    cap = P.crystal_cdc_max_chunks(n, params)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    ends = torch.empty(cap, dtype=torch.int64, device="cuda")
    dig = torch.empty((cap, 16), dtype=torch.uint8, device="cuda")
    s = torch.cuda.current_stream()
    tc, tsel, tch, tot = [], [], [], []
    for r in range(reps + 2):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(6)]
        # the steps one by one (chunk digests in index order) ...
        e[0].record(s)
        P.crystal_cdc_candidates_device(d, n, params, ws, ws_bytes, None, None, 0, s.cuda_stream)
        e[1].record(s)
        P.crystal_cdc_select_device(n, params, ws, ws_bytes, cnt, ends, cap, s.cuda_stream)
        e[2].record(s)
        P.crystal_md5_chunks_device(d, ends, cnt, cap, dig, s.cuda_stream)
        e[3].record(s)
        # ... and the whole pipeline (chunk digests longest first)
        e[4].record(s)
        P.crystal_cdc_device(d, n, params, ws, ws_bytes, cnt, ends, dig, cap, s.cuda_stream)
        e[5].record(s)
        e[5].synchronize()
        if r >= 2:
            tc.append(e[0].elapsed_time(e[1]))
            tsel.append(e[1].elapsed_time(e[2]))
            tch.append(e[2].elapsed_time(e[3]))
            tot.append(e[4].elapsed_time(e[5]))
    m = int(cnt.item())
    lens = np.diff(np.concatenate([[0], ends[:m].cpu().numpy()]))
    comps = int(sum(comp(x) for x in lens))
    dev_ms = statistics.mean(tot)
    # host-fed, one job through the job layer and through the naive path
    outcap = P.crystal_output_bytes(P.K_CDC, n, params)
    P.crystal_init(max_input_bytes=n, host_pool_bytes=64 << 20, device_pool_bytes=2 << 30,
                   n_streams=2)
    try:
        outb = P.crystal_buffer_acquire(outcap)
        inb = P.crystal_buffer_wrap(host.data_ptr(), n)
        jt = []
        for r in range(reps + 1):
            t = P.new_task(n, params)
            P.crystal_submit(t, P.K_CDC, inb, outb)
            assert P.crystal_wait(t) == 0
            if r >= 1:
                jt.append((t.t_done_ns - t.t_submit_ns) / 1e6)
        jends, jdig = P.parse_cdc_output(P.buffer_view(outb))
        same = (np.array_equal(jends, ends[:m].cpu().numpy().view(np.uint64)) and
                np.array_equal(jdig, dig[:m].cpu().numpy()))
        P.crystal_buffer_release(inb)
        P.crystal_buffer_release(outb)
    finally:
        P.crystal_finalize()
    o = np.zeros(outcap, np.uint8)
    nvt = []
    for r in range(3):
        _, st = P.crystal_naive_run(P.K_CDC, params, host.data_ptr(), n, o, outcap)
        nvt.append(st.total_ms)
    jm = statistics.mean(jt)
    return out("chunking", {
        "bytes": n, "chunks": m, "mean_chunk": round(n / m, 1), "candidates_per_MiB":
            None, "compressions": comps,
        "device_ms": {"candidates": round(statistics.mean(tc), 4),
                      "select": round(statistics.mean(tsel), 4),
                      "md5_chunks_index_order": round(statistics.mean(tch), 4),
                      "pipeline_total": round(dev_ms, 4),
                      "order_and_md5_chunks": round(dev_ms - statistics.mean(tc) -
                                                    statistics.mean(tsel), 4)},
        "device_gbps": round(n / 1e9 / (dev_ms / 1e3), 1),
        "candidates_hbm_gbps": round(n / 1e9 / (statistics.mean(tc) / 1e3), 1),
        "job_ms_mean": round(jm, 3), "job_gbps": round(n / 1e9 / (jm / 1e3), 2),
        "naive_ms_mean": round(statistics.mean(nvt), 3),
        "naive_gbps": round(n / 1e9 / (statistics.mean(nvt) / 1e3), 2),
        "link_frac_job": round(n / 1e9 / (jm / 1e3) / LINK_PEAK_GBPS, 4),
        "job_matches_device": bool(same),
    })


# --------------------------------------------------------------------- serving

def serving(P, torch, gen, loads, n_jobs, n_streams=3, direct_frac=0.7, n_copy_streams=0,
            in_flight=48):
    arena_bytes = 4 << 30
    arena = torch.empty(arena_bytes, dtype=torch.uint8).pin_memory()
    gen.fill(gen.sub_seed(gen.config_seed(4), 5), arena.data_ptr(), arena_bytes)
    base = gen.cdc_base()
    cdcp = P.cdc_params(base)
    direct = P.crystal_direct_params(segment_bytes=4096)
    spec0 = gen.serving_jobs(n_jobs=n_jobs, load_gbps=1.0, arena_bytes=arena_bytes,
                             direct_frac=direct_frac)
    caps = np.array([P.crystal_output_bytes(P.K_CDC if k else P.K_MD5_DIRECT, int(sz),
                                            cdcp if k else direct)
                     for sz, k in zip(spec0["size"], spec0["kind"])], dtype=np.int64)
    ooff = np.zeros(n_jobs, dtype=np.int64)
    ooff[1:] = np.cumsum((caps[:-1] + 255) // 256 * 256)
    outs = torch.empty(int(ooff[-1] + caps[-1]), dtype=torch.uint8).pin_memory()
    P.crystal_init(max_input_bytes=64 << 20, host_pool_bytes=16 << 20,
                   device_pool_bytes=16 << 30, n_streams=n_streams, max_in_flight=in_flight,
                   n_copy_streams=n_copy_streams)
    results = []
    try:
        for load in loads:
            spec = gen.serving_jobs(n_jobs=n_jobs, load_gbps=load, arena_bytes=arena_bytes,
                                    direct_frac=direct_frac)
            jobs = (P.crystal_drive_job * n_jobs)()
            for k in range(n_jobs):
                kid = P.K_CDC if spec["kind"][k] else P.K_MD5_DIRECT
                jobs[k].h_in = arena.data_ptr() + int(spec["offset"][k])
                jobs[k].bytes = int(spec["size"][k])
                jobs[k].h_out = outs.data_ptr() + int(ooff[k])
                jobs[k].out_cap = int(caps[k])
                jobs[k].arrival_s = float(spec["arrival_s"][k])
                jobs[k].kernel_id = kid
            stats0 = P.crystal_get_stats()
            res = P.crystal_drive(jobs, direct, cdcp, window=0)
            st = P.crystal_get_stats()
            lat = np.array([jobs[k].latency_s for k in range(n_jobs)]) * 1e3
            adm = np.array([jobs[k].admit_wait_s for k in range(n_jobs)]) * 1e3
            offered_s = float(spec["arrival_s"][-1])
            results.append({
                "offered_gbps": load, "jobs": n_jobs, "ok": int(res.ok), "failed": int(res.failed),
                "achieved_gbps": round(res.bytes / 1e9 / res.wall_s, 2),
                "offered_span_s": round(offered_s, 3), "wall_s": round(res.wall_s, 3),
                "p50_ms": round(pct(lat, 50), 3), "p99_ms": round(pct(lat, 99), 3),
                "p999_ms": round(pct(lat, 99.9), 3), "mean_ms": round(float(lat.mean()), 3),
                "admit_wait_p50_ms": round(pct(adm, 50), 3),
                "admit_wait_p99_ms": round(pct(adm, 99), 3),
                "pool_min_free_gib": round(st.device_pool_min_free / 2 ** 30, 2),
                "bytes": int(res.bytes), "completed_delta": int(st.completed - stats0.completed),
            })
            print(json.dumps({"serving_point": results[-1]}), flush=True)
    finally:
        P.crystal_finalize()
    # operating point: highest load whose achieved rate is >= 95 % of offered
    ok_pts = [r for r in results if r["achieved_gbps"] >= 0.95 * r["offered_gbps"]]
    op = max(ok_pts, key=lambda r: r["offered_gbps"]) if ok_pts else None
    return out("serving", {"points": results, "operating_point": op,
                           "mean_job_bytes": float(spec0["size"].mean()),
                           "direct_frac": direct_frac,
                           "device_pool_gib": 16, "compute_streams": n_streams,
                           "max_in_flight": in_flight})


# ----------------------------------------------------------------------- batch

def batch(P, torch, gen, n_buf, reps=20, sample_single=20000):
    off, ln, arena_bytes, seed = gen.batch_small(n_buf=n_buf)
    host = torch.empty(arena_bytes + 64, dtype=torch.uint8).pin_memory()
    gen.fill(seed, host.data_ptr(), arena_bytes + 64)
    d = host.to("cuda")
    t_off = torch.from_numpy(off.view(np.int64)).cuda()
    t_len = torch.from_numpy(ln.view(np.int32)).cuda()
    o = torch.zeros((n_buf, 16), dtype=torch.uint8, device="cuda")
    s = torch.cuda.Stream()
    t0 = time.perf_counter()
    plan = P.crystal_batch_plan(d, t_off, t_len, n_buf, o, stream=s, tune=P._lib.TUNE_FULL)
    plan_s = time.perf_counter() - t0
    try:
        tun = P.crystal_batch_get_tuning(plan)
        times = []
        for r in range(reps + 2):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(s)
            P.crystal_batch_run(plan, 1)
            b.record(s)
            b.synchronize()
            if r >= 2:
                times.append(a.elapsed_time(b))
    finally:
        P.crystal_batch_free(plan)
    ms = statistics.mean(times)
    total = int(ln.astype(np.int64).sum())
    comps = int(((ln.astype(np.int64) + 8) // 64 + 1).sum())
    ops = comps * OPS_PER_COMPRESSION
    # one launch per buffer, timed on a sample and scaled to the whole batch
    o2 = torch.zeros((n_buf, 16), dtype=torch.uint8, device="cuda")
    lib = P.load()
    ap, op_, lp, outp = d.data_ptr(), t_off.data_ptr(), t_len.data_ptr(), o2.data_ptr()
    k = min(sample_single, n_buf)
    torch.cuda.synchronize()
    ta = time.perf_counter()
    for i in range(k):
        lib.crystal_md5_batch_device(ap, op_ + 8 * i, lp + 4 * i, None, 1, outp + 16 * i, 64, 1,
                                     s.cuda_stream)
    s.synchronize()
    single_s = (time.perf_counter() - ta) * n_buf / k
    same = bool(torch.equal(o2[:k], o[:k]))
    return out("batch", {
        "buffers": n_buf, "bytes": total, "compressions": comps,
        "tuning": {"block": tun.block, "waves_per_simd": tun.waves_per_simd, "grab": tun.grab,
                   "streams": tun.n_streams, "sorted": tun.sorted, "depth": tun.depth,
                   "tail": tun.tail,
                   "tuned_replay_ms": round(tun.replay_ms, 4)},
        "plan_seconds": round(plan_s, 2),
        "replay_ms": round(ms, 4), "replay_ms_median": round(statistics.median(times), 4),
        "replay_ms_min": round(min(times), 4),
        "gbps": round(total / 1e9 / (ms / 1e3), 1),
        "alu_tops": round(ops / (ms / 1e3) / 1e12, 2),
        "alu_frac": round(ops / (ms / 1e3) / 1e12 / INT32_PEAK_TOPS, 4),
        "hbm_frac": round(total / 1e9 / (ms / 1e3) / HBM_PEAK_GBPS, 4),
        "one_launch_per_buffer_s_est": round(single_s, 3),
        "one_launch_sample": k,
        "speedup_vs_per_buffer": round(single_s / (ms / 1e3), 1),
        "per_buffer_matches_plan": same,
    })


def main() -> int:
    ap = argparse.ArgumentParser(description="per-workload measurements")
    ap.add_argument("--only", default="",
                    help="comma list: direct_one,overhead,naive_stages,stream_len,sha1_stream,"
                         "chunking,serving,batch")
    ap.add_argument("--quick", action="store_true", help="fewer jobs / buffers")
    ap.add_argument("--loads", default="5,10,20,30,40,45,50")
    ap.add_argument("--serving-jobs", type=int, default=0)
    ap.add_argument("--serving-streams", type=int, default=3)
    ap.add_argument("--serving-in-flight", type=int, default=48,
                    help="jobs dispatched but unfinished at once (the job layer's max_in_flight)")
    ap.add_argument("--serving-copy-streams", type=int, default=0,
                    help="copy-in streams of the job layer (0 = its default, 1)")
    ap.add_argument("--serving-direct-frac", type=float, default=0.7,
                    help="share of direct-hashing jobs in the serving mix (the rest chunk)")
    ap.add_argument("--batch-buffers", type=int, default=0)
    ap.add_argument("--sha1-streams", type=int, default=3)
    ap.add_argument("--sha1-window", type=int, default=24)
    ap.add_argument("--in-process", action="store_true",
                    help="run all selected workloads in this process (by default each "
                         "workload runs in a fresh child process)")
    args = ap.parse_args()
    names = ["direct_one", "overhead", "naive_stages", "stream_len", "sha1_stream",
             "chunking", "batch", "serving"]
    only = [x for x in args.only.split(",") if x]
    if len(only) != 1 and not args.in_process:
        # one process per workload: measured in the same process, the serving
        # mix ran well below its rate when it followed other large workloads
        rest = [a for a in sys.argv[1:] if not a.startswith("--only")]
        if "--only" in sys.argv:
            i = sys.argv.index("--only")
            rest = sys.argv[1:i] + sys.argv[i + 2:]
        rc = 0
        for n in names:
            if only and n not in only:
                continue
            r = subprocess.run([sys.executable, "-u", os.path.abspath(__file__), "--only", n,
                                *rest])
            rc = rc or r.returncode
        return rc
    import torch

    import gen
    import paper_1005_1695_amd as P
    P.load()
    torch.cuda.set_device(0)
    only = set(only)
    want = lambda n: not only or n in only
    if want("direct_one"):
        direct_one(P, torch, gen)
    if want("overhead"):
        overhead(P, torch, gen)
    if want("naive_stages"):
        naive_stages(P, torch, gen)
    if want("stream_len"):
        stream_len(P, torch, gen)
    if want("sha1_stream"):
        sha1_stream(P, torch, gen, n_streams=args.sha1_streams, window=args.sha1_window)
    if want("chunking"):
        chunking(P, torch, gen)
    if want("batch"):
        batch(P, torch, gen, args.batch_buffers or (100_000 if args.quick else 1_000_000))
    if want("serving"):
        loads = [float(x) for x in args.loads.split(",")]
        serving(P, torch, gen, loads, args.serving_jobs or (2000 if args.quick else 20000),
                args.serving_streams, args.serving_direct_frac, args.serving_copy_streams,
                args.serving_in_flight)
    return 0


if __name__ == "__main__":
    sys.exit(main())
