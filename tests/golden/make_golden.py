"""Writes the stored expected values under tests/golden/ from the oracle.

Each fixture is the oracle's output on a seeded synthetic input that the
input generators rebuild exactly; nothing here comes from the GPU path.
Run from the repository root:  python tests/golden/make_golden.py
"""
from __future__ import annotations

import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import gen  # noqa: E402
import oracle  # noqa: E402

DIRECT_FILE = os.path.join(HERE, "direct_1mib.txt")
CDC_FILE = os.path.join(HERE, "cdc_1mib.txt")
CDC_BLOCKS = 16  # 16 x 64 KiB = 1 MiB of the chunking recipe (20 % repeats)


def direct_input():
    return gen.direct_one(1 << 20)


def cdc_input():
    return gen.cdc_input(n_blocks=CDC_BLOCKS), gen.cdc_base()


def write_direct(path: str = DIRECT_FILE) -> None:
    seg, root = oracle.direct(direct_input())
    with open(path, "w") as f:
        f.write("# Direct hashing of gen.direct_one(1 MiB): MD5 of each 4 KiB segment,\n"
                "# then MD5 over the concatenated 16-byte segment digests (the reading of\n"
                "# the paper's direct hashing, Sec. 5.2).  Written by make_golden.py from\n"
                "# oracle.direct.  Lines: 'seg <index> <digest hex>', then 'root <hex>'.\n")
        for i, d in enumerate(seg):
            f.write(f"seg {i} {d.tobytes().hex()}\n")
        f.write(f"root {root.hex()}\n")


def write_cdc(path: str = CDC_FILE) -> None:
    data, base = cdc_input()
    ends, dig = oracle.cdc(data, base)
    with open(path, "w") as f:
        f.write("# Content-defined chunking of gen.cdc_input(16 blocks of 64 KiB, 20 % repeats)\n"
                "# with base gen.cdc_base(): 48-byte window, 13-bit mask, 2 KiB / 64 KiB\n"
                "# bounds, MD5 per chunk.  Written by make_golden.py from oracle.cdc.\n"
                f"# base {base:#018x}\n"
                "# Lines: 'chunk <exclusive end offset> <digest hex>'.\n")
        for e, d in zip(ends, dig):
            f.write(f"chunk {int(e)} {d.tobytes().hex()}\n")


def read_direct(path: str = DIRECT_FILE):
    seg, root = [], None
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        p = line.split()
        if p[0] == "seg":
            assert int(p[1]) == len(seg)
            seg.append(bytes.fromhex(p[2]))
        elif p[0] == "root":
            root = bytes.fromhex(p[1])
    return seg, root


def read_cdc(path: str = CDC_FILE):
    ends, dig = [], []
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        p = line.split()
        assert p[0] == "chunk"
        ends.append(int(p[1]))
        dig.append(bytes.fromhex(p[2]))
    return ends, dig


if __name__ == "__main__":
    write_direct()
    write_cdc()
    print("wrote", DIRECT_FILE, CDC_FILE)
