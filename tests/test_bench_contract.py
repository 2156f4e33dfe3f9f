"""CPU checks of bench.py's contract: the multi-GPU refusal, the MD5 block
count behind the roofline's operation count, and the rule that HBM traffic
is reported only from counters taken on the current kernel sources."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


@pytest.mark.parametrize("length,blocks", [(0, 1), (55, 1), (56, 2), (63, 2), (64, 2),
                                           (119, 2), (120, 3), (4096, 65), (32768, 513)])
def test_md5_block_count_at_the_padding_edges(length, blocks):
    # RFC 1321 Sec. 3.1-3.2: one 0x80 byte and the 8-byte length follow the
    # message, rounded up to whole 64-byte blocks
    assert bench.compressions(length) == blocks
    assert bench.compressions(length) == -(-(length + 9) // 64)


def test_traffic_comes_only_from_counters_on_the_same_sources():
    path = os.path.join(ROOT, "profiles", bench.COUNTERS_FILE)
    with open(path) as fh:
        d = json.load(fh)
    recorded = d["kernel_source_hash"]
    assert bench.load_traffic(recorded) == d["hbm_bytes_per_launch"] > 0
    assert bench.load_traffic("0" * 16) is None
