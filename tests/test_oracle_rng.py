"""Pins of the oracle's Philox4x32-10 (the counter-based generator behind
every uniform of the path, Sec. 4.1 RIS candidates and Sec. 4.2
continuations): published known-answer vectors and rocRAND's engine."""
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def _kat():
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append([int(x, 16) for x in line.split()])
    return rows


def test_known_answer_vectors(oracle_lib):
    for r in _kat():
        out = oracle_lib.philox(r[0:4], r[4:6])
        assert [int(x) for x in out] == r[6:10]


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not available")
def test_matches_rocrand_engine(oracle_lib, tmp_path):
    exe = tmp_path / "rr_ref"
    subprocess.run(["hipcc", "-O1", "-x", "hip", "--offload-arch=gfx950",
                    os.path.join(HERE, "helpers", "rocrand_philox_ref.cpp"), "-o", str(exe)],
                   check=True, cwd=str(tmp_path))
    rng = np.random.default_rng(7)
    cases = rng.integers(0, 2 ** 32, size=(200, 5), dtype=np.uint64)
    cases[:, 4] %= 1 << 20
    inp = "\n".join(" ".join("%x" % int(x) for x in row) for row in cases) + "\n"
    res = subprocess.run([str(exe)], input=inp, capture_output=True, text=True, check=True)
    lines = res.stdout.strip().split("\n")
    assert len(lines) == len(cases)
    for row, line in zip(cases, lines):
        klo, khi, slo, shi, blk = [int(x) for x in row]
        # rocRAND: counter = (block lo, block hi, subsequence lo, subsequence hi)
        ours = oracle_lib.philox([blk, 0, slo, shi], [klo, khi])
        assert [int(x) for x in ours] == [int(x, 16) for x in line.split()]


def test_uniform_mapping_exact_in_float32():
    # u = (x >> 8) * 2^-24 is exact in float32 and float64 and lies in [0, 1)
    x = np.array([0, 255, 256, 0xFFFFFFFF, 0x80000000], np.uint64)
    u64 = (x >> 8).astype(np.float64) * 2.0 ** -24
    u32 = (x >> 8).astype(np.float32) * np.float32(2.0 ** -24)
    assert np.array_equal(u64, u32.astype(np.float64))
    assert u64.max() < 1.0 and u64.min() == 0.0
