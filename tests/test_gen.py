"""Seeded input generators: SplitMix64 stream and workload recipes."""
import numpy as np

import gen

M = (1 << 64) - 1


def _sm64_py(seed, k):
    # SplitMix64 written independently in Python integers (Steele et al. 2014).
    z = (seed + (k + 1) * 0x9E3779B97F4A7C15) & M
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M
    return z ^ (z >> 31)


def test_splitmix_matches_python():
    for seed in (0, 1, gen.SEED_BASE, M):
        got = gen.u64(seed, 20)
        assert [int(x) for x in got] == [_sm64_py(seed, k) for k in range(20)]
        assert gen.splitmix64_at(seed, 7) == _sm64_py(seed, 7)
    # offset start
    assert int(gen.u64(5, 3, first=10)[2]) == _sm64_py(5, 12)


def test_bytes_little_endian_and_truncation():
    seed = 1234
    full = gen.random_bytes(seed, 64)
    for k in range(8):
        w = _sm64_py(seed, k)
        assert bytes(full[8 * k:8 * k + 8]) == w.to_bytes(8, "little")
    for n in (0, 1, 7, 9, 63):
        assert bytes(gen.random_bytes(seed, n)) == bytes(full[:n])


def test_fill_multi():
    seeds = np.array([3, 4, 5], dtype=np.uint64)
    off = np.array([0, 100, 200], dtype=np.uint64)
    ln = np.array([10, 50, 33], dtype=np.uint64)
    out = np.zeros(300, dtype=np.uint8)
    gen.fill_multi(seeds, off, ln, out.ctypes.data)
    for s, o, l in zip(seeds, off, ln):
        assert bytes(out[int(o):int(o + l)]) == bytes(gen.random_bytes(int(s), int(l)))
    assert not out[10:100].any()


def test_uniform_range():
    u = gen.uniform(99, 10000)
    assert u.min() >= 0.0 and u.max() < 1.0
    assert abs(u.mean() - 0.5) < 0.02


def test_cdc_layout_full_size():
    src = gen.cdc_layout(4096, 0.2)
    reps = np.nonzero(src != np.arange(4096))[0]
    assert len(reps) == 819
    assert reps.min() >= 1 and reps.max() <= 4095
    # every copy points at an earlier fresh block
    assert np.all(src[reps] < reps)
    assert np.all(src[src] == src)


def test_cdc_input_small_repeats():
    data = gen.cdc_input(n_blocks=32, block=4096, repeat_frac=0.25, seed=77)
    src = gen.cdc_layout(32, 0.25, seed=77)
    blocks = data.reshape(32, 4096)
    for b in range(32):
        assert np.array_equal(blocks[b], blocks[src[b]])
    fresh = [b for b in range(32) if src[b] == b]
    assert len({bytes(blocks[b]) for b in fresh}) == len(fresh)


def test_serving_jobs_shape():
    j = gen.serving_jobs(n_jobs=5000, load_gbps=10.0, arena_bytes=1 << 28)
    s = j["size"]
    assert s.min() >= 4096 and s.max() <= (1 << 26)
    assert np.all(np.diff(j["arrival_s"]) >= 0) and j["arrival_s"][0] == 0.0
    assert np.all(j["offset"] % 4096 == 0)
    assert np.all(j["offset"] + s <= j["arena_bytes"])
    frac = j["kind"].mean()
    assert 0.27 < frac < 0.33
    # log-uniform: median near sqrt(lo*hi)
    med = np.median(s)
    assert 2 ** 18 < med < 2 ** 20


def test_batch_small_shape():
    off, ln, arena, seed = gen.batch_small(n_buf=20000)
    assert ln.min() >= 512 and ln.max() <= 16384
    assert np.all(off % 16 == 0)
    assert np.all(off[1:] >= off[:-1] + ln[:-1])
    assert arena >= int(off[-1]) + int(ln[-1])
    mean = ln.astype(np.float64).mean()
    assert 4300 < mean < 4900  # E = (16384-512)/ln(32) ~ 4580
