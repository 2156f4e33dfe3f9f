"""GPU tests of the job layer: paper API semantics (Fig. 3), pooled buffers,
overlapped streams, serving mix (alone == in the mix, bit for bit), the naive
per-job path, and tuned batch plans replayed several times."""
import ctypes
import hashlib

import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def P(torch_cuda):
    import paper_1005_1695_amd as P
    P.load()
    return P


@pytest.fixture()
def lib(P):
    P.crystal_init(max_input_bytes=64 << 20, host_pool_bytes=1 << 30,
                   device_pool_bytes=2 << 30, n_streams=4)
    yield P
    P.crystal_finalize()


def _submit(P, kernel, data, params=None, callback=None):
    n = len(data)
    inb = P.crystal_buffer_acquire(max(n, 1))
    P.buffer_view(inb)[:n] = data
    outb = P.crystal_buffer_acquire(max(P.crystal_output_bytes(kernel, n, params), 1))
    t = P.new_task(n, params, callback)
    P.crystal_submit(t, kernel, inb, outb)
    return t, inb, outb


def test_direct_job_1mib_with_callback(lib):
    P = lib
    seen = []
    data = gen.direct_one()
    t, inb, outb = _submit(P, P.K_MD5_DIRECT, data,
                           callback=lambda task, user: seen.append(task.contents.status))
    assert P.crystal_wait(t) == 0
    assert P.crystal_poll(t) == 1
    assert seen == [0]
    assert t.out_bytes == 16 * 257
    out = P.buffer_view(outb)[:t.out_bytes].reshape(257, 16)
    es, er = oracle.direct(data)
    assert np.array_equal(out[:256], es)
    assert out[256].tobytes() == er
    assert t.t_submit_ns <= t.t_admit_ns <= t.t_done_ns
    P.crystal_buffer_release(inb)
    P.crystal_buffer_release(outb)


@pytest.mark.parametrize("kind", ["nop", "md5", "direct64", "cdc_small", "cdc_default",
                                  "direct_ragged", "empty_cdc", "empty_direct", "sha1",
                                  "sha1_ragged", "empty_sha1"])
def test_each_kernel_as_a_job(lib, kind):
    P = lib
    base = gen.cdc_base()
    data = gen.random_bytes(len(kind), 3_000_001)
    params = None
    if kind == "nop":
        k = P.K_NOP
    elif kind == "md5":
        k = P.K_MD5
    elif kind.endswith("sha1") or kind.startswith("sha1"):
        k = P.K_SHA1_DIRECT
        params = P.crystal_direct_params(segment_bytes=4096)
        if kind == "sha1_ragged":
            data = data[:123457]
        if kind == "empty_sha1":
            data = data[:0]
    elif kind.startswith("direct"):
        k = P.K_MD5_DIRECT
        params = P.crystal_direct_params(segment_bytes=64 if kind == "direct64" else 4096)
        if kind == "direct_ragged":
            data = data[:123457]
        if kind == "empty_direct":
            data = data[:0]
    else:
        k = P.K_CDC
        params = (P.cdc_params(base, 64, 700, 6) if kind == "cdc_small"
                  else P.cdc_params(base))
        if kind == "empty_cdc":
            data = data[:0]
    t, inb, outb = _submit(P, k, data, params)
    assert P.crystal_wait(t) == 0
    out = P.buffer_view(outb)[:t.out_bytes]
    if k == P.K_NOP:
        assert np.array_equal(out, data)
    elif k == P.K_MD5:
        assert out.tobytes() == hashlib.md5(data.tobytes()).digest()
    elif k == P.K_MD5_DIRECT:
        seg = params.segment_bytes
        es, er = oracle.direct(data, seg)
        assert np.array_equal(out[:-16].reshape(-1, 16), es)
        assert out[-16:].tobytes() == er
    elif k == P.K_SHA1_DIRECT:
        es, er = oracle.sha1_direct(data, params.segment_bytes)
        assert np.array_equal(out[:-20].reshape(-1, 20), es)
        assert out[-20:].tobytes() == er
    else:
        ends, dig = P.parse_cdc_output(out)
        ee, ed = oracle.cdc(data, base, params.mask_bits, params.min_len, params.max_len)
        assert np.array_equal(ends, ee) and np.array_equal(dig, ed)
    P.crystal_buffer_release(inb)
    P.crystal_buffer_release(outb)


def test_concurrent_submitters(lib):
    """Four application threads acquire buffers, submit, wait for and release
    their own jobs at the same time (MD5 direct, SHA-1 direct, chunking, the
    empty kernel, at varied sizes), while the library's completion threads
    run their callbacks: every result equals the oracle's and every callback
    ran exactly once."""
    import threading
    P = lib
    base = gen.cdc_base()
    kinds = [(P.K_MD5_DIRECT, P.crystal_direct_params(segment_bytes=4096)),
             (P.K_SHA1_DIRECT, P.crystal_direct_params(segment_bytes=4096)),
             (P.K_CDC, P.cdc_params(base)),
             (P.K_NOP, None)]
    errors, seen = [], []
    lock = threading.Lock()

    def on_done(task, user):
        with lock:
            seen.append(int(task.contents.in_bytes))

    def worker(w):
        try:
            for r in range(12):
                k, params = kinds[(w + r) % 4]
                n = 1 + (w * 7919 + r * 104729) % 3_000_000
                data = gen.random_bytes(1000 * w + r, n)
                t, inb, outb = _submit(P, k, data, params, callback=on_done)
                assert P.crystal_wait(t) == 0, (w, r)
                out = P.buffer_view(outb)[:t.out_bytes]
                if k == P.K_NOP:
                    assert np.array_equal(out, data), (w, r)
                elif k == P.K_MD5_DIRECT:
                    es, er = oracle.direct(data)
                    assert np.array_equal(out[:-16].reshape(-1, 16), es), (w, r)
                    assert out[-16:].tobytes() == er, (w, r)
                elif k == P.K_SHA1_DIRECT:
                    es, er = oracle.sha1_direct(data)
                    assert np.array_equal(out[:-20].reshape(-1, 20), es), (w, r)
                    assert out[-20:].tobytes() == er, (w, r)
                else:
                    ends, dig = P.parse_cdc_output(out)
                    ee, ed = oracle.cdc(data, base)
                    assert np.array_equal(ends, ee) and np.array_equal(dig, ed), (w, r)
                P.crystal_buffer_release(inb)
                P.crystal_buffer_release(outb)
        except BaseException as e:  # reported by the main thread
            errors.append((w, e))

    threads = [threading.Thread(target=worker, args=(w,)) for w in range(4)]
    for th in threads:
        th.start()
    for th in threads:
        th.join(timeout=120)
    assert not any(th.is_alive() for th in threads)
    assert not errors, errors[:2]
    assert len(seen) == 48


def test_cdc_jobs_past_1024_tiles(P):
    """Chunking jobs of 65 MiB + 5 bytes (1041 tiles) through the job layer:
    past what one finishing workgroup takes, so selection and the chunk order
    run as separate kernels inside the batch; one job alone, then two
    submitted together."""
    P.crystal_init(max_input_bytes=66 << 20, host_pool_bytes=512 << 20,
                   device_pool_bytes=1 << 30, n_streams=2)
    try:
        base = gen.cdc_base()
        params = P.cdc_params(base)
        for batch in (1, 2):
            datas = [gen.random_bytes(900 + 7 * batch + k, (65 << 20) + 5) for k in range(batch)]
            subs = [_submit(P, P.K_CDC, d, params) for d in datas]
            for (t, inb, outb), d in zip(subs, datas):
                assert P.crystal_wait(t) == 0
                ends, dig = P.parse_cdc_output(P.buffer_view(outb)[:t.out_bytes])
                ee, ed = oracle.cdc(d, base)
                assert np.array_equal(ends, ee) and np.array_equal(dig, ed)
                P.crystal_buffer_release(inb)
                P.crystal_buffer_release(outb)
    finally:
        P.crystal_finalize()


@pytest.mark.parametrize("layout", ["one_copy_stream", "three_copy_streams",
                                    "default_with_2_compute",
                                    "caller_streams_2_copy_2_compute"])
def test_copy_stream_layouts(P, torch_cuda, layout):
    """Jobs submitted together under each copy-in stream layout: batches
    rotate over the copy-in streams, and every result equals the oracle's."""
    torch = torch_cuda
    keep = None
    if layout == "one_copy_stream":
        P.crystal_init(max_input_bytes=4 << 20, host_pool_bytes=128 << 20,
                       device_pool_bytes=256 << 20, n_streams=2, n_copy_streams=1)
    elif layout == "three_copy_streams":
        P.crystal_init(max_input_bytes=4 << 20, host_pool_bytes=128 << 20,
                       device_pool_bytes=256 << 20, n_streams=3, n_copy_streams=3)
    elif layout == "default_with_2_compute":  # two copy-in streams fit the queues
        P.crystal_init(max_input_bytes=4 << 20, host_pool_bytes=128 << 20,
                       device_pool_bytes=256 << 20, n_streams=2)
    else:
        keep = [torch.cuda.Stream() for _ in range(4)]
        P.crystal_init(max_input_bytes=4 << 20, host_pool_bytes=128 << 20,
                       device_pool_bytes=256 << 20, streams=keep, n_copy_streams=2)
    try:
        base = gen.cdc_base()
        subs = []
        for k in range(12):
            n = (1 << 20) + 4099 * k
            data = gen.random_bytes(700 + k, n)
            if k % 3 == 2:
                subs.append((data, P.K_CDC) + _submit(P, P.K_CDC, data, P.cdc_params(base)))
            else:
                subs.append((data, P.K_MD5_DIRECT) + _submit(P, P.K_MD5_DIRECT, data))
        streams_seen = set()
        for data, kid, t, inb, outb in subs:
            assert P.crystal_wait(t) == 0
            streams_seen.add(t.stream_index)
            out = P.buffer_view(outb)[:t.out_bytes]
            if kid == P.K_CDC:
                ends, dig = P.parse_cdc_output(out)
                ee, ed = oracle.cdc(data, base)
                assert np.array_equal(ends, ee) and np.array_equal(dig, ed)
            else:
                es, er = oracle.direct(data)
                assert np.array_equal(out[:-16].reshape(-1, 16), es)
                assert out[-16:].tobytes() == er
            P.crystal_buffer_release(inb)
            P.crystal_buffer_release(outb)
        assert streams_seen <= set(range(3))
    finally:
        P.crystal_finalize()


def test_poll_timeout_and_busy_release(lib):
    P = lib
    data = gen.random_bytes(1, 64 << 20)
    t, inb, outb = _submit(P, P.K_CDC, data, P.cdc_params(gen.cdc_base()))
    rc = P.crystal_wait(t, 0)
    if P.crystal_poll(t) == 0:
        assert rc == P._lib.ETIMEDOUT
    rc = P.load().crystal_buffer_release(inb)
    assert rc == P._lib.EBUSY or P.crystal_poll(t) == 1
    assert P.crystal_wait(t, -1) == 0
    assert P.crystal_poll(t) == 1
    if rc == P._lib.EBUSY:
        P.crystal_buffer_release(inb)
    P.crystal_buffer_release(outb)


def test_nonblocking_acquire_eagain(lib):
    P = lib
    held = []
    lib_ = P.load()
    h = ctypes.c_void_p()
    while True:
        rc = lib_.crystal_buffer_acquire(256 << 20, P.NONBLOCK, ctypes.byref(h))
        if rc != 0:
            break
        held.append(h.value)
    assert rc == P._lib.EAGAIN and len(held) == 4
    P.crystal_buffer_release(held.pop())
    held.append(P.crystal_buffer_acquire(256 << 20, P.NONBLOCK))
    for b in held:
        P.crystal_buffer_release(b)
    s = P.crystal_get_stats()
    assert s.host_pool_free == s.host_pool_bytes


def test_overlapped_stream_of_jobs(lib, torch_cuda):
    """16 jobs of 8 MiB submitted at once spread over the 4 streams and overlap
    in time; every output matches the oracle."""
    P = lib
    n_jobs, job = 16, 8 << 20
    seeds = gen.direct_stream_seeds(n_jobs)
    prepared, bufs = [], []
    cap = P.crystal_output_bytes(P.K_MD5_DIRECT, job, None)
    for j in range(n_jobs):
        data = gen.random_bytes(int(seeds[j]), job)
        inb = P.crystal_buffer_acquire(job)
        P.buffer_view(inb)[:] = data
        outb = P.crystal_buffer_acquire(cap)
        prepared.append((data, inb, outb))
        bufs += [inb, outb]
    tasks = []
    for data, inb, outb in prepared:  # submit back to back
        t = P.new_task(job)
        P.crystal_submit(t, P.K_MD5_DIRECT, inb, outb)
        tasks.append((t, data, outb))
    for t, data, outb in tasks:
        assert P.crystal_wait(t) == 0
        _, er = oracle.direct(data)
        assert bytes(P.buffer_view(outb)[-16:]) == er
    # jobs waiting together are dispatched together (one copy-in run, one
    # grouped kernel launch) or on different streams; either way their
    # admitted-to-done intervals overlap
    iv = sorted((t.t_admit_ns, t.t_done_ns) for t, _, _ in tasks)
    overlaps = sum(1 for a, b in zip(iv, iv[1:]) if b[0] < a[1])
    assert overlaps >= n_jobs // 2
    batches = len({(t.stream_index, t.t_admit_ns) for t, _, _ in tasks})
    assert batches < n_jobs
    for b in bufs:
        P.crystal_buffer_release(b)


def _drive_jobs(P, torch, sizes, kinds, arrivals, arena, offsets, base):
    n = len(sizes)
    jobs = (P.crystal_drive_job * n)()
    outs = []
    direct = P.crystal_direct_params(segment_bytes=4096)
    cdcp = P.cdc_params(base)
    for k in range(n):
        kid = P.K_CDC if kinds[k] else P.K_MD5_DIRECT
        cap = P.crystal_output_bytes(kid, int(sizes[k]), cdcp if kinds[k] else direct)
        o = torch.empty(cap, dtype=torch.uint8).pin_memory()
        outs.append(o)
        jobs[k].h_in = arena.data_ptr() + int(offsets[k])
        jobs[k].bytes = int(sizes[k])
        jobs[k].h_out = o.data_ptr()
        jobs[k].out_cap = cap
        jobs[k].arrival_s = float(arrivals[k])
        jobs[k].kernel_id = kid
    return jobs, outs, direct, cdcp


def test_serving_mix_alone_equals_mix(lib, torch_cuda):
    """Open-loop mixed arrivals overlap on the device; each job's output is
    identical to the same job run alone (naive path) and to the oracle."""
    P, torch = lib, torch_cuda
    spec = gen.serving_jobs(n_jobs=120, load_gbps=20.0, hi=8 << 20, arena_bytes=64 << 20,
                            seed=4242)
    arena = torch.empty(spec["arena_bytes"], dtype=torch.uint8).pin_memory()
    gen.fill(spec["arena_seed"], arena.data_ptr(), spec["arena_bytes"])
    base = gen.cdc_base()
    jobs, outs, direct, cdcp = _drive_jobs(P, torch, spec["size"], spec["kind"],
                                           spec["arrival_s"], arena, spec["offset"], base)
    res = P.crystal_drive(jobs, direct, cdcp, window=0)
    assert res.ok == 120 and res.failed == 0
    a = arena.numpy()
    for k in range(120):
        assert jobs[k].status == 0 and jobs[k].latency_s > 0
        sz, of = int(spec["size"][k]), int(spec["offset"][k])
        data = a[of:of + sz]
        kid = jobs[k].kernel_id
        mix = outs[k].numpy()
        alone = np.zeros(jobs[k].out_cap, dtype=np.uint8)
        ob, _ = P.crystal_naive_run(kid, cdcp if kid == P.K_CDC else direct, data, sz,
                                    alone, jobs[k].out_cap)
        assert np.array_equal(mix[:ob], alone[:ob]), k
        if kid == P.K_CDC:
            ends, dig = P.parse_cdc_output(mix)
            ee, ed = oracle.cdc(data, base)
            assert np.array_equal(ends, ee) and np.array_equal(dig, ed), k
        else:
            es, er = oracle.direct(data)
            assert mix[16 * len(es):16 * len(es) + 16].tobytes() == er, k


def test_batched_chains_mixed_jobs(P, torch_cuda):
    """Jobs submitted all at once are admitted together, so batches hold
    several chunking and direct jobs whose roots and chunk digests run in one
    chains launch; includes an empty and a 1-byte job of each kind, a ragged
    direct job and chunking jobs with min_len 1 KiB.  Every output equals the
    oracle's."""
    torch = torch_cuda
    P.crystal_init(max_input_bytes=4 << 20, host_pool_bytes=64 << 20,
                   device_pool_bytes=1 << 30, n_streams=1, max_in_flight=32)
    try:
        rng = np.random.default_rng(77)
        sizes = [0, 1, 0, 1, 4096 * 3 + 17] + [int(x) for x in
                                                np.exp(rng.uniform(np.log(4096),
                                                                   np.log(4 << 20), 43))]
        kinds = [1, 1, 0, 0, 0] + [int(k) for k in rng.random(43) < 0.5]
        n = len(sizes)
        offs = np.zeros(n, dtype=np.int64)
        offs[1:] = np.cumsum([(x + 4095) // 4096 * 4096 for x in sizes[:-1]])
        arena = torch.empty(int(offs[-1]) + sizes[-1] + 4096, dtype=torch.uint8).pin_memory()
        gen.fill(515, arena.data_ptr(), arena.numel())
        base = gen.cdc_base()
        jobs, outs, direct, _ = _drive_jobs(P, torch, sizes, kinds, [0.0] * n, arena, offs,
                                            base)
        cdcp = P.cdc_params(base, min_len=1024, max_len=16384, mask_bits=11)
        for k in range(n):
            if kinds[k]:
                jobs[k].out_cap = P.crystal_output_bytes(P.K_CDC, sizes[k], cdcp)
                outs[k] = torch.empty(jobs[k].out_cap, dtype=torch.uint8).pin_memory()
                jobs[k].h_out = outs[k].data_ptr()
        res = P.crystal_drive(jobs, direct, cdcp, window=0)
        assert res.ok == n and res.failed == 0
        a = arena.numpy()
        for k in range(n):
            data = a[int(offs[k]):int(offs[k]) + sizes[k]]
            mix = outs[k].numpy()
            if kinds[k]:
                ends, dig = P.parse_cdc_output(mix)
                ee, ed = oracle.cdc(data, base, min_len=1024, max_len=16384, mask_bits=11)
                assert np.array_equal(ends, ee) and np.array_equal(dig, ed), k
            else:
                es, er = oracle.direct(data)
                got = mix[:16 * len(es) + 16]
                assert got[:16 * len(es)].tobytes() == es.tobytes(), k
                assert got[16 * len(es):].tobytes() == er, k
    finally:
        P.crystal_finalize()


def test_batched_sha1_and_md5_direct_jobs(P, torch_cuda):
    """SHA-1 and MD5 direct jobs submitted at once share batches: each group
    runs one segment launch (and the SHA-1 group one root launch).  Includes
    empty, 1-byte and ragged jobs; every output equals the oracle's."""
    torch = torch_cuda
    P.crystal_init(max_input_bytes=4 << 20, host_pool_bytes=64 << 20,
                   device_pool_bytes=1 << 30, n_streams=1, max_in_flight=32)
    try:
        rng = np.random.default_rng(91)
        sizes = [0, 1, 0, 1, 4096 * 5 + 9] + [int(x) for x in
                                               np.exp(rng.uniform(np.log(4096),
                                                                  np.log(4 << 20), 35))]
        sha = [1, 1, 0, 0, 1] + [int(k) for k in rng.random(35) < 0.6]
        n = len(sizes)
        offs = np.zeros(n, dtype=np.int64)
        offs[1:] = np.cumsum([(x + 4095) // 4096 * 4096 for x in sizes[:-1]])
        arena = torch.empty(int(offs[-1]) + sizes[-1] + 4096, dtype=torch.uint8).pin_memory()
        gen.fill(616, arena.data_ptr(), arena.numel())
        jobs, outs, direct, cdcp = _drive_jobs(P, torch, sizes, [0] * n, [0.0] * n, arena,
                                               offs, gen.cdc_base())
        for k in range(n):
            if sha[k]:
                jobs[k].kernel_id = P.K_SHA1_DIRECT
                jobs[k].out_cap = P.crystal_output_bytes(P.K_SHA1_DIRECT, sizes[k], direct)
                outs[k] = torch.empty(jobs[k].out_cap, dtype=torch.uint8).pin_memory()
                jobs[k].h_out = outs[k].data_ptr()
        res = P.crystal_drive(jobs, direct, cdcp, window=0)
        assert res.ok == n and res.failed == 0
        a = arena.numpy()
        for k in range(n):
            data = a[int(offs[k]):int(offs[k]) + sizes[k]]
            mix = outs[k].numpy()
            w = 20 if sha[k] else 16
            es, er = (oracle.sha1_direct if sha[k] else oracle.direct)(data)
            assert mix[:w * len(es)].tobytes() == es.tobytes(), k
            assert mix[w * len(es):w * len(es) + w].tobytes() == er, k
    finally:
        P.crystal_finalize()


def test_closed_loop_window(lib, torch_cuda):
    P, torch = lib, torch_cuda
    n = 24
    arena = torch.empty(n * (4 << 20), dtype=torch.uint8).pin_memory()
    gen.fill(99, arena.data_ptr(), arena.numel())
    sizes = [4 << 20] * n
    offs = [k * (4 << 20) for k in range(n)]
    jobs, outs, direct, cdcp = _drive_jobs(P, torch, sizes, [0] * n, [0.0] * n, arena,
                                           offs, gen.cdc_base())
    res = P.crystal_drive(jobs, direct, cdcp, window=4)
    assert res.ok == n
    a = arena.numpy()
    for k in range(n):
        _, er = oracle.direct(a[offs[k]:offs[k] + sizes[k]])
        assert outs[k].numpy()[-16:].tobytes() == er


def test_naive_path_sha1(P, torch_cuda):
    data = gen.random_bytes(31, 5 << 20 | 77)
    out = np.zeros(P.crystal_output_bytes(P.K_SHA1_DIRECT, len(data), None), np.uint8)
    ob, st = P.crystal_naive_run(P.K_SHA1_DIRECT, None, data, len(data), out, len(out))
    es, er = oracle.sha1_direct(data)
    assert ob == len(out) == 20 * (len(es) + 1)
    assert np.array_equal(out[:-20].reshape(-1, 20), es) and out[-20:].tobytes() == er


def test_naive_path_stage_times(P, torch_cuda):
    data = gen.random_bytes(3, 8 << 20)
    out = np.zeros(P.crystal_output_bytes(P.K_MD5_DIRECT, len(data), None), np.uint8)
    ob, st = P.crystal_naive_run(P.K_MD5_DIRECT, None, data, len(data), out, len(out))
    es, er = oracle.direct(data)
    assert out[-16:].tobytes() == er and ob == len(out)
    assert st.alloc_ms > 0 and st.copy_in_ms > 0 and st.kernel_ms > 0
    assert st.total_ms >= st.alloc_ms + st.copy_in_ms + st.kernel_ms


def test_small_device_pool_admission(P, torch_cuda):
    """Jobs wait for room in a small device pool and all still complete."""
    P.crystal_init(max_input_bytes=16 << 20, device_pool_bytes=40 << 20,
                   host_pool_bytes=512 << 20, n_streams=2)
    try:
        tasks = []
        for j in range(12):
            data = gen.random_bytes(j, 16 << 20)
            tasks.append((_submit(P, P.K_MD5_DIRECT, data), data))
        for (t, inb, outb), data in tasks:
            assert P.crystal_wait(t) == 0
            assert P.buffer_view(outb)[-16:].tobytes() == oracle.direct(data)[1]
        s = P.crystal_get_stats()
        assert s.completed == 12 and s.device_pool_free == s.device_pool_bytes
        assert s.device_pool_min_free < 40 << 20
    finally:
        P.crystal_finalize()


def test_finalize_with_jobs_in_flight(P, torch_cuda):
    P.crystal_init(max_input_bytes=32 << 20, device_pool_bytes=64 << 20,
                   host_pool_bytes=1 << 30, n_streams=2)
    subs = []
    for j in range(24):
        data = gen.random_bytes(j + 500, 32 << 20)
        subs.append((_submit(P, P.K_MD5_DIRECT, data), data))
    P.crystal_finalize()
    ok = cancelled = 0
    for (t, _, outb), data in subs:
        st = t.status
        assert st in (0, P._lib.ECANCELED)
        if st == 0:
            ok += 1
        else:
            cancelled += 1
    assert ok + cancelled == 24


def test_batch_plan_replays(P, torch_cuda):
    torch = torch_cuda
    off, ln, arena, seed = gen.batch_small(n_buf=20000)
    data = gen.random_bytes(seed, arena + 64)
    d, _ = P.to_device_bytes(data)
    t_off = torch.from_numpy(off.view(np.int64)).cuda()
    t_len = torch.from_numpy(ln.view(np.int32)).cuda()
    out = torch.zeros((20000, 16), dtype=torch.uint8, device="cuda")
    exp = oracle.md5_batch(data, off, ln)
    s = torch.cuda.Stream()
    for tune in (P._lib.TUNE_NONE, P._lib.TUNE_FULL):
        with torch.cuda.stream(s):
            plan = P.crystal_batch_plan(d, t_off, t_len, 20000, out, stream=s, tune=tune)
        try:
            tun = P.crystal_batch_get_tuning(plan)
            assert tun.replay_ms > 0
            for rep in range(3):
                with torch.cuda.stream(s):
                    out.zero_()
                    P.crystal_batch_run(plan, 1)
                s.synchronize()
                assert np.array_equal(out.cpu().numpy(), exp), (tune, rep)
                junk = torch.randn(1 << 20, device="cuda").sum().item()  # eager work
                assert junk == junk
        finally:
            P.crystal_batch_free(plan)


# (sorted, depth, tail, waves_per_simd, n_streams): index order and global
# order, every loader depth, tails shorter than, equal to and longer than the
# batch, alone and split over branches
FIXED_PLANS = [(0, 1, 0, 2, 4), (1, 2, 0, 2, 4), (0, 3, 1000, 2, 1), (64, 2, 5000, 1, 2),
               (256, 1, 4096, 4, 1), (4096, 3, 100000, 1, 3), (64, 2, 1, 3, 1)]


@pytest.mark.parametrize("cfg", FIXED_PLANS, ids=lambda c: "s%d_d%d_t%d_w%d_b%d" % c)
def test_batch_plan_fixed_multi_stream(P, torch_cuda, cfg):
    torch = torch_cuda
    sorted_, depth, tail, wps, branches = cfg
    off, ln, arena, seed = gen.batch_small(n_buf=5000, seed=8)
    data = gen.random_bytes(seed, arena + 64)
    d, _ = P.to_device_bytes(data)
    t_off = torch.from_numpy(off.view(np.int64)).cuda()
    t_len = torch.from_numpy(ln.view(np.int32)).cuda()
    out = torch.zeros((5000, 16), dtype=torch.uint8, device="cuda")
    exp = oracle.md5_batch(data, off, ln)
    fixed = P.crystal_batch_tuning(block=128, waves_per_simd=wps, grab=4, n_streams=branches,
                                   sorted=sorted_, depth=depth, tail=tail)
    s = torch.cuda.Stream()
    plan = P.crystal_batch_plan(d, t_off, t_len, 5000, out, stream=s, fixed=fixed)
    try:
        for rep in range(2):
            with torch.cuda.stream(s):
                out.zero_()
                P.crystal_batch_run(plan, 1)
            s.synchronize()
            assert np.array_equal(out.cpu().numpy(), exp), rep
    finally:
        P.crystal_batch_free(plan)


def _edge_batch(aligned: bool):
    """Buffers whose lengths straddle every loader boundary: 64-byte blocks,
    128-byte groups and chunks of 1, 2 and 3 groups (plus the 55/56 padding
    edges), and empty buffers; 16-byte aligned starts, or starts at every
    byte offset."""
    base = [0, 1, 15, 16, 55, 56, 63, 64, 65, 119, 120, 127, 128, 129]
    for c in (256, 384, 512, 768, 1152):
        base += [c - 65, c - 64, c - 1, c, c + 1, c + 55, c + 56, c + 63, c + 64, c + 127]
    base += [4096, 5000, 16383]
    lens = np.array(base * 3, dtype=np.uint32)
    off = np.zeros(len(lens), dtype=np.uint64)
    pos = 0
    for i, L in enumerate(lens):
        if aligned:
            pos = (pos + 15) // 16 * 16
        else:
            pos += 1 + (i % 7)
        off[i] = pos
        pos += int(L)
    return off, lens, pos


@pytest.mark.parametrize("aligned", [True, False], ids=["a16", "any"])
@pytest.mark.parametrize("depth", [1, 2, 3])
def test_batch_plan_edges_every_depth(P, torch_cuda, depth, aligned):
    """The persistent kernel behind batch plans, at every loader depth, on
    buffers at the loader's block, group and chunk boundaries, empty
    buffers included, with and without a tail re-sort and over 1 or 2
    branches: every digest equals the oracle's."""
    torch = torch_cuda
    off, ln, end = _edge_batch(aligned)
    data = gen.random_bytes(777, end + 64)
    d, _ = P.to_device_bytes(data)
    t_off = torch.from_numpy(off.view(np.int64)).cuda()
    t_len = torch.from_numpy(ln.view(np.int32)).cuda()
    n = len(ln)
    exp = oracle.md5_batch(data, off, ln)
    out = torch.zeros((n, 16), dtype=torch.uint8, device="cuda")
    for sorted_, tail, branches in ((64, 0, 1), (0, n, 2), (1, 37, 1)):
        fixed = P.crystal_batch_tuning(block=64, waves_per_simd=1, grab=1, n_streams=branches,
                                       sorted=sorted_, depth=depth, tail=tail)
        s = torch.cuda.Stream()
        plan = P.crystal_batch_plan(d, t_off, t_len, n, out, stream=s, fixed=fixed)
        try:
            with torch.cuda.stream(s):
                out.zero_()
                P.crystal_batch_run(plan, 1)
            s.synchronize()
            got = out.cpu().numpy()
            bad = [i for i in range(n) if got[i].tobytes() != exp[i].tobytes()]
            assert not bad, (sorted_, tail, branches, [(int(off[i]), int(ln[i])) for i in bad[:5]])
        finally:
            P.crystal_batch_free(plan)


@pytest.mark.parametrize("bad", [dict(block=512), dict(block=96), dict(depth=4),
                                 dict(n_streams=9)])
def test_batch_plan_rejects_bad_tuning(P, torch_cuda, bad):
    torch = torch_cuda
    off, ln, arena, seed = gen.batch_small(n_buf=100, seed=3)
    data = gen.random_bytes(seed, arena + 64)
    d, _ = P.to_device_bytes(data)
    t_off = torch.from_numpy(off.view(np.int64)).cuda()
    t_len = torch.from_numpy(ln.view(np.int32)).cuda()
    out = torch.zeros((100, 16), dtype=torch.uint8, device="cuda")
    fixed = P.crystal_batch_tuning(**bad)
    with pytest.raises(P.CrystalError) as ei:
        P.crystal_batch_plan(d, t_off, t_len, 100, out, fixed=fixed)
    assert ei.value.code == P._lib.EINVAL


def test_batch_plan_full_size_sampled(P, torch_cuda):
    """The batched small-buffer workload at full size (10^6 buffers of
    log-uniform 512 B..16 KiB, 4.58 GB), with the tuned plan the workload
    benchmark times: 4000 sampled digests (and the longest and shortest
    buffers) equal the oracle's."""
    torch = torch_cuda
    off, ln, arena, seed = gen.batch_small()
    host = torch.empty(arena + 64, dtype=torch.uint8).pin_memory()
    gen.fill(seed, host.data_ptr(), arena + 64)
    d = host.to("cuda")
    t_off = torch.from_numpy(off.view(np.int64)).cuda()
    t_len = torch.from_numpy(ln.view(np.int32)).cuda()
    n = len(ln)
    out = torch.zeros((n, 16), dtype=torch.uint8, device="cuda")
    s = torch.cuda.Stream()
    plan = P.crystal_batch_plan(d, t_off, t_len, n, out, stream=s, tune=P._lib.TUNE_FULL)
    try:
        with torch.cuda.stream(s):
            out.zero_()
            P.crystal_batch_run(plan, 1)
        s.synchronize()
    finally:
        P.crystal_batch_free(plan)
    got = out.cpu().numpy()
    hv = host.numpy()
    rng = np.random.default_rng(5)
    pick = set(rng.choice(n, 4000, replace=False).tolist())
    pick |= {int(np.argmax(ln)), int(np.argmin(ln)), 0, n - 1}
    for m in sorted(pick):
        o, L = int(off[m]), int(ln[m])
        assert got[m].tobytes() == oracle.md5(hv[o:o + L]), m


def test_serving_mix_large_jobs_sampled(P, torch_cuda):
    """Open-loop mix with the full size range (4 KiB..64 MiB, 70 % direct /
    30 % chunking) through a 16 GiB pool at 40 GB/s offered: all jobs finish,
    and a sample that includes the largest jobs of each kind equals the
    oracle."""
    torch = torch_cuda
    n = 400
    spec = gen.serving_jobs(n_jobs=n, load_gbps=40.0, arena_bytes=1 << 30, seed=9090)
    arena = torch.empty(spec["arena_bytes"], dtype=torch.uint8).pin_memory()
    gen.fill(spec["arena_seed"], arena.data_ptr(), spec["arena_bytes"])
    base = gen.cdc_base()
    P.crystal_init(max_input_bytes=64 << 20, host_pool_bytes=16 << 20,
                   device_pool_bytes=16 << 30, n_streams=3, max_in_flight=64)
    try:
        jobs, outs, direct, cdcp = _drive_jobs(P, torch, spec["size"], spec["kind"],
                                               spec["arrival_s"], arena, spec["offset"], base)
        res = P.crystal_drive(jobs, direct, cdcp, window=0)
        assert res.ok == n and res.failed == 0
    finally:
        P.crystal_finalize()
    a = arena.numpy()
    sizes, kinds = np.asarray(spec["size"]), np.asarray(spec["kind"])
    pick = set(np.random.default_rng(3).choice(n, 24, replace=False).tolist())
    for kind in (0, 1):
        idx = np.flatnonzero(kinds == kind)
        pick |= set(idx[np.argsort(sizes[idx])[-3:]].tolist())
    for k in sorted(pick):
        sz, of = int(sizes[k]), int(spec["offset"][k])
        data = a[of:of + sz]
        mix = outs[k].numpy()
        if kinds[k]:
            ends, dig = P.parse_cdc_output(mix)
            ee, ed = oracle.cdc(data, base)
            assert np.array_equal(ends, ee) and np.array_equal(dig, ed), k
        else:
            es, er = oracle.direct(data)
            assert mix[:16 * len(es)].tobytes() == es.tobytes(), k
            assert mix[16 * len(es):16 * len(es) + 16].tobytes() == er, k
