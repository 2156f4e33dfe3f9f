"""GPU parity of the device-level hot path against the CPU oracle.

Every digest, candidate position and chunk boundary must match bit for bit
(the path is integer arithmetic; there is no tolerance).  Inputs come from
the seeded generators; expected values only from the oracle.
"""
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


def _np(t):
    return t.cpu().numpy()


# ------------------------------------------------------------- direct hashing

def test_direct_one_job_1mib(P, torch_cuda):
    data = gen.direct_one()
    d, n = P.to_device_bytes(data)
    seg, roots, base, _ = P.direct_device(d, [0], [n])
    exp_seg, exp_root = oracle.direct(data)
    assert np.array_equal(_np(seg), exp_seg)
    assert _np(roots)[0].tobytes() == exp_root


def test_direct_ragged_jobs(P, torch_cuda):
    lens = [0, 1, 15, 55, 56, 64, 4095, 4096, 4097, 8192 + 100, 100000, 3, 65536]
    # 16-byte aligned starts, plus two deliberately unaligned jobs
    offs, o = [], 0
    for i, ln in enumerate(lens):
        o = (o + 15) // 16 * 16 + (5 if i in (3, 10) else 0)
        offs.append(o)
        o += ln
    arena = gen.random_bytes(77, o + 64)
    d, _ = P.to_device_bytes(arena)
    seg, roots, base, _ = P.direct_device(d, offs, lens)
    seg, roots = _np(seg), _np(roots)
    for j, (of, ln) in enumerate(zip(offs, lens)):
        es, er = oracle.direct(arena[of:of + ln])
        assert np.array_equal(seg[int(base[j]):int(base[j + 1])], es), j
        assert roots[j].tobytes() == er, j


def test_golden_fixtures(P, torch_cuda):
    """The HIP path against the stored fixtures (tests/golden/): direct
    hashing of the seeded 1 MiB input and chunking of 1 MiB of the chunking
    recipe, compared with the stored digests and ends."""
    import os
    import sys
    sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
    import make_golden as mg
    data = mg.direct_input()
    d, n = P.to_device_bytes(data)
    seg, roots, _, _ = P.direct_device(d, [0], [n])
    es, er = mg.read_direct()
    assert [r.tobytes() for r in _np(seg)] == es
    assert _np(roots)[0].tobytes() == er
    cdata, base = mg.cdc_input()
    cd, cn = P.to_device_bytes(cdata)
    ends, dig = P.cdc_device(cd, cn, P.cdc_params(base))
    ee, ed = mg.read_cdc()
    assert _np(ends).astype(np.uint64).tolist() == ee
    assert [r.tobytes() for r in _np(dig)] == ed


def test_direct_root_loader_boundaries(P, torch_cuda):
    """Jobs whose digest arrays (16 bytes per segment) end on each side of
    the root loader's 64-byte block, 128-byte group and 384-byte chunk
    boundaries, with a ragged last segment in every other job, in one
    launch: segments and roots equal the oracle's."""
    nsegs = [1, 2, 3, 4, 5, 7, 8, 9, 15, 16, 17, 23, 24, 25, 31, 32, 33, 47, 48, 49, 71, 72,
             73, 95, 96, 97]
    lens = [k * 4096 - (1000 if i % 2 else 0) for i, k in enumerate(nsegs)]
    offs, o = [], 0
    for ln in lens:
        o = (o + 15) // 16 * 16
        offs.append(o)
        o += ln
    arena = gen.random_bytes(321, o + 64)
    d, _ = P.to_device_bytes(arena)
    seg, roots, base, _ = P.direct_device(d, offs, lens)
    seg, roots = _np(seg), _np(roots)
    for j, (of, ln) in enumerate(zip(offs, lens)):
        es, er = oracle.direct(arena[of:of + ln])
        assert np.array_equal(seg[int(base[j]):int(base[j + 1])], es), j
        assert roots[j].tobytes() == er, (j, nsegs[j])


@pytest.mark.parametrize("segment", [64, 128, 4096, 65536])
def test_direct_segment_sizes(P, torch_cuda, segment):
    data = gen.random_bytes(segment, 300001)
    d, n = P.to_device_bytes(data)
    seg, roots, base, _ = P.direct_device(d, [0], [n], segment=segment)
    es, er = oracle.direct(data, segment)
    assert np.array_equal(_np(seg), es)
    assert _np(roots)[0].tobytes() == er


def test_direct_stream_full_size_sampled(P, torch_cuda):
    """256 jobs x 8 MiB resident together (the streamed workload at full size,
    one launch); roots and segments of a sample of jobs checked."""
    torch = torch_cuda
    n_jobs, job = 256, 8 << 20
    seeds = gen.direct_stream_seeds(n_jobs)
    host = torch.empty(n_jobs * job, dtype=torch.uint8).pin_memory()
    gen.fill_multi(seeds, np.arange(n_jobs, dtype=np.uint64) * job,
                   np.full(n_jobs, job, dtype=np.uint64), host.data_ptr())
    d = host.to("cuda")
    seg, roots, base, _ = P.direct_device(d, np.arange(n_jobs) * job, [job] * n_jobs)
    torch.cuda.synchronize()
    roots = _np(roots)
    for j in (0, 1, 97, 128, 255):
        data = host[j * job:(j + 1) * job].numpy()
        es, er = oracle.direct(data)
        assert roots[j].tobytes() == er, j
        assert np.array_equal(_np(seg[int(base[j]):int(base[j + 1])]), es), j


# ------------------------------------------------------- SHA-1 direct hashing

def test_sha1_direct_one_job_1mib(P, torch_cuda):
    data = gen.direct_one()
    d, n = P.to_device_bytes(data)
    seg, roots, base, _ = P.direct_device(d, [0], [n], hash="sha1")
    exp_seg, exp_root = oracle.sha1_direct(data)
    assert np.array_equal(_np(seg), exp_seg)
    assert _np(roots)[0].tobytes() == exp_root


def test_sha1_direct_ragged_jobs(P, torch_cuda):
    """Ragged and empty jobs, two unaligned job starts, and (with 20-byte
    digests) roots whose digest runs start only 4-byte aligned."""
    lens = [0, 1, 15, 55, 56, 64, 4095, 4096, 4097, 8192 + 100, 100000, 3, 65536]
    offs, o = [], 0
    for i, ln in enumerate(lens):
        o = (o + 15) // 16 * 16 + (7 if i in (2, 9) else 0)
        offs.append(o)
        o += ln
    arena = gen.random_bytes(78, o + 64)
    d, _ = P.to_device_bytes(arena)
    seg, roots, base, _ = P.direct_device(d, offs, lens, hash="sha1")
    seg, roots = _np(seg), _np(roots)
    for j, (of, ln) in enumerate(zip(offs, lens)):
        es, er = oracle.sha1_direct(arena[of:of + ln])
        assert np.array_equal(seg[int(base[j]):int(base[j + 1])], es), j
        assert roots[j].tobytes() == er, j


@pytest.mark.parametrize("segment", [64, 192, 4096, 65536])
def test_sha1_direct_segment_sizes(P, torch_cuda, segment):
    data = gen.random_bytes(segment + 1, 300001)
    d, n = P.to_device_bytes(data)
    seg, roots, base, _ = P.direct_device(d, [0], [n], segment=segment, hash="sha1")
    es, er = oracle.sha1_direct(data, segment)
    assert np.array_equal(_np(seg), es)
    assert _np(roots)[0].tobytes() == er


def test_sha1_stream_full_size_sampled(P, torch_cuda):
    """256 jobs x 8 MiB in one SHA-1 launch pair; a sample checked."""
    torch = torch_cuda
    n_jobs, job = 256, 8 << 20
    seeds = gen.direct_stream_seeds(n_jobs)
    host = torch.empty(n_jobs * job, dtype=torch.uint8).pin_memory()
    gen.fill_multi(seeds, np.arange(n_jobs, dtype=np.uint64) * job,
                   np.full(n_jobs, job, dtype=np.uint64), host.data_ptr())
    d = host.to("cuda")
    seg, roots, base, _ = P.direct_device(d, np.arange(n_jobs) * job, [job] * n_jobs,
                                          hash="sha1")
    torch.cuda.synchronize()
    roots = _np(roots)
    for j in (0, 3, 128, 255):
        data = host[j * job:(j + 1) * job].numpy()
        es, er = oracle.sha1_direct(data)
        assert roots[j].tobytes() == er, j
        assert np.array_equal(_np(seg[int(base[j]):int(base[j + 1])]), es), j


# ------------------------------------------------------------------- batching

def test_batch_small_vs_oracle(P, torch_cuda):
    off, ln, arena, seed = gen.batch_small(n_buf=3000)
    data = gen.random_bytes(seed, arena + 64)
    d, _ = P.to_device_bytes(data)
    out = _np(P.batch_device(d, off, ln))
    assert np.array_equal(out, oracle.md5_batch(data, off, ln))
    # longest-first order and a small persistent-style grid: same digests
    order = np.argsort(-ln.astype(np.int64), kind="stable").astype(np.uint32)
    out2 = _np(P.batch_device(d, off, ln, order=order, block=128, grid=7))
    assert np.array_equal(out2, out)


def test_batch_unaligned_and_edges(P, torch_cuda):
    lens = np.array([0, 1, 3, 55, 56, 63, 64, 65, 119, 120, 127, 128, 129, 4096, 513],
                    dtype=np.uint32)
    off = np.cumsum(np.concatenate([[3], lens[:-1].astype(np.int64) + 1])).astype(np.uint64)
    data = gen.random_bytes(5, int(off[-1] + lens[-1]) + 64)
    d, _ = P.to_device_bytes(data)
    out = _np(P.batch_device(d, off, lens))
    assert np.array_equal(out, oracle.md5_batch(data, off, lens))


# ------------------------------------------------------------------ chunking

@pytest.mark.parametrize("base", [gen.cdc_base(), 3, 0xFFFFFFFFFFFFFFFF, 2])
def test_window_hash_vs_oracle(P, torch_cuda, base):
    torch = torch_cuda
    data = gen.random_bytes(base & 0xFF, 100003)
    d, n = P.to_device_bytes(data)
    w = torch.empty(n, dtype=torch.int64, device="cuda")
    P.crystal_window_hash_device(d, n, base, w)
    assert np.array_equal(_np(w).view(np.uint64), oracle.window_hash(data, base))


def _candidates(P, torch, data, params):
    d, n = P.to_device_bytes(data)
    ws_bytes = P.crystal_cdc_workspace_bytes(n, params)
    ws = torch.empty(max(ws_bytes, 256), dtype=torch.uint8, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    cap = n + 1
    cand = torch.empty(cap, dtype=torch.int64, device="cuda")
    P.crystal_cdc_candidates_device(d, n, params, ws, ws_bytes, cnt, cand, cap)
    k = int(cnt.item())
    return d, n, ws, ws_bytes, _np(cand[:k]).view(np.uint64)


# masks of up to 15 bits roll two parts per lane in 16-bit halves, 16..32
# bits in 32-bit registers, wider ones in 64-bit: the cases cover each side
# of both switches
@pytest.mark.parametrize("case", ["random13", "dense4", "none64", "zeros", "bits32",
                                  "bits40", "tiny", "bits1", "bits15", "bits16", "bits17"])
def test_candidates_vs_oracle(P, torch_cuda, case):
    base = gen.cdc_base()
    n, bits = 3 * (1 << 20) + 77, 13
    data = None
    if case.startswith("bits") and case not in ("bits32", "bits40"):
        bits = int(case[4:])
    if case == "dense4":
        bits = 4
    elif case == "none64":
        bits = 64
    elif case == "zeros":
        data = np.zeros(300000, np.uint8)
    elif case == "bits32":
        bits, n = 32, 1 << 20
    elif case == "bits40":
        bits, n = 40, 1 << 20
        base = 5
        data = np.zeros(n, np.uint8)
        data[::997] = 1  # sparse bytes so the wide mask still hits somewhere
    elif case == "tiny":
        n = 47
    if data is None:
        data = gen.random_bytes(n ^ bits, n)
    params = P.cdc_params(base, mask_bits=bits)
    *_, got = _candidates(P, torch_cuda, data, params)
    assert np.array_equal(got, oracle.candidates(data, base, bits))


# short inputs: the last lane's first part is cut short and its second part
# is short or empty (16 lanes per range, parts of 128 bytes)
@pytest.mark.parametrize("n", [48, 129, 200, 300, 4097, 6001])
def test_candidates_ragged_parts(P, torch_cuda, n):
    base = gen.cdc_base()
    data = gen.random_bytes(n + 7, n)
    params = P.cdc_params(base, mask_bits=4)
    *_, got = _candidates(P, torch_cuda, data, params)
    assert np.array_equal(got, oracle.candidates(data, base, 4))


# inputs whose range counts give the candidate launch 8, 4 and 2 lanes per
# 4 KiB range (the other tests cover 16 lanes, small inputs, and 1 lane,
# the 256 MiB input)
@pytest.mark.parametrize("n", [20 * (1 << 20) + 5, 50 * (1 << 20) + 1, 100 * (1 << 20) + 3],
                         ids=["8_lanes", "4_lanes", "2_lanes"])
def test_candidates_every_lane_split(P, torch_cuda, n):
    base = gen.cdc_base()
    data = gen.random_bytes(n & 0xFFFF, n)
    params = P.cdc_params(base, mask_bits=10)
    *_, got = _candidates(P, torch_cuda, data, params)
    assert np.array_equal(got, oracle.candidates(data, base, 10))


def test_window_hash_8_lanes_per_range(P, torch_cuda):
    """The full 64-bit window hash at every byte of a 20 MiB input, rolled
    by 8 lanes per 4 KiB range (512-byte parts, each after its own warm-up)."""
    torch = torch_cuda
    base = gen.cdc_base()
    data = gen.random_bytes(4321, 20 * (1 << 20) + 9)
    d, n = P.to_device_bytes(data)
    w = torch.empty(n, dtype=torch.int64, device="cuda")
    P.crystal_window_hash_device(d, n, base, w)
    assert np.array_equal(_np(w).view(np.uint64), oracle.window_hash(data, base))


SELECT_CASES = {
    # name: (data builder, base, min, max, mask_bits)
    "c3_like_16mib": (lambda: gen.cdc_input(n_blocks=256, seed=3), None, 2048, 65536, 13),
    "small_params": (lambda: gen.random_bytes(9, 2_000_003), None, 64, 700, 6),
    "zeros_min": (lambda: np.zeros(3_000_000, np.uint8), None, 2048, 65536, 13),
    "zeros_repair": (lambda: np.zeros(4_000_000, np.uint8), None, 3000, 65536, 13),
    "no_hit_max": (lambda: gen.random_bytes(10, 1_500_000), None, 2048, 65536, 64),
    "min_eq_max": (lambda: gen.random_bytes(11, 777_777), None, 5000, 5000, 13),
    "big_max": (lambda: gen.random_bytes(12, 3_000_000), None, 4096, 1 << 20, 16),
    "min_one": (lambda: gen.random_bytes(13, 200_000), None, 1, 64, 3),
    "short": (lambda: gen.random_bytes(14, 3000), None, 2048, 65536, 13),
    "exact_max": (lambda: gen.random_bytes(15, 65536), None, 2048, 65536, 64),
    # zero bytes make every position a candidate: tiles whose span reaches
    # them hold too many for LDS and walk through global memory, the others
    # walk from LDS
    "zeros_then_random": (lambda: np.concatenate([np.zeros(1 << 20, np.uint8),
                                                  gen.random_bytes(16, 3_000_001)]),
                          None, 2048, 65536, 13),
    # 272 tiles: past the short warm-up, each tile walks 2P before its start
    "tiles_272_long_warm": (lambda: gen.random_bytes(17, 17 * (1 << 20) + 5), None, 2048,
                            65536, 13),
}


@pytest.mark.parametrize("name", sorted(SELECT_CASES))
def test_select_and_pipeline_vs_oracle(P, torch_cuda, name):
    torch = torch_cuda
    build, base, mn, mx, bits = SELECT_CASES[name]
    base = gen.cdc_base() if base is None else base
    data = build()
    params = P.cdc_params(base, mn, mx, bits)
    d, n, ws, ws_bytes, cand = _candidates(P, torch, data, params)
    exp_cand = oracle.candidates(data, base, bits)
    assert np.array_equal(cand, exp_cand)
    exp_ends = oracle.select(exp_cand, n, mn, mx)
    cap = P.crystal_cdc_max_chunks(n, params)
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    ends = torch.empty(max(cap, 1), dtype=torch.int64, device="cuda")
    P.crystal_cdc_select_device(n, params, ws, ws_bytes, cnt, ends, cap)
    m = int(cnt.item())
    assert np.array_equal(_np(ends[:m]).view(np.uint64), exp_ends)
    # per-chunk digests from the selected ends
    dig = torch.empty((max(cap, 1), 16), dtype=torch.uint8, device="cuda")
    P.crystal_md5_chunks_device(d, ends, cnt, cap, dig)
    exp_e, exp_d = oracle.cdc(data, base, bits, mn, mx)
    assert np.array_equal(_np(dig[:m]), exp_d)
    # whole pipeline in one call
    e2, d2 = P.cdc_device(d, n, params)
    assert np.array_equal(_np(e2).view(np.uint64), exp_e)
    assert np.array_equal(_np(d2), exp_d)


def test_cdc_empty(P, torch_cuda):
    d, n = P.to_device_bytes(np.zeros(0, np.uint8))
    e, dg = P.cdc_device(d, 0, P.cdc_params(gen.cdc_base()))
    assert e.numel() == 0 and dg.shape[0] == 0


def test_select_over_1024_tiles_with_repairs(P, torch_cuda):
    """1041 tiles, past what one finishing workgroup takes: zero bytes with a
    3000-byte minimum put nearly every speculative tile chain out of phase,
    so the multi-kernel path verifies and repairs them (smaller inputs repair
    inside the one-workgroup finish: the zeros_repair case)."""
    base = gen.cdc_base()
    data = np.zeros(65 * (1 << 20) + 123, np.uint8)
    d, n = P.to_device_bytes(data)
    e, dg = P.cdc_device(d, n, P.cdc_params(base, 3000, 65536, 13))
    exp_e, exp_d = oracle.cdc(data, base, 13, 3000, 65536)
    assert np.array_equal(_np(e).view(np.uint64), exp_e)
    assert np.array_equal(_np(dg), exp_d)


def test_cdc_full_size_256mib(P, torch_cuda):
    """The chunking workload at full size (256 MiB, 20 % repeated blocks)."""
    torch = torch_cuda
    base = gen.cdc_base()
    host = torch.empty(256 << 20, dtype=torch.uint8).pin_memory()
    gen.cdc_input(out=host.numpy())
    d = torch.empty((256 << 20) + 64, dtype=torch.uint8, device="cuda")
    d[:256 << 20].copy_(host, non_blocking=False)
    e, dg = P.cdc_device(d, 256 << 20, P.cdc_params(base))
    exp_e, exp_d = oracle.cdc(host.numpy(), base)
    assert np.array_equal(_np(e).view(np.uint64), exp_e)
    assert np.array_equal(_np(dg), exp_d)
