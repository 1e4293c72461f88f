"""The oracle's Philox4x32-10 block function against rocRAND's (a library
implementation of the same published generator, built here for the host from
its header): every output word equal on random counters and keys, carry
boundaries and all-zero / all-one words.  Pins the random-number stream the
sampler draws from to the generator's published definition."""
import os
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
HIPCC = os.path.join(ROCM, "bin", "hipcc")
HEADER = os.path.join(ROCM, "include", "rocrand", "rocrand_philox4x32_10.h")


@pytest.fixture(scope="module")
def rocrand_block(tmp_path_factory):
    if not (os.path.exists(HIPCC) and os.path.exists(HEADER)):
        pytest.skip("hipcc or the rocRAND header is not installed")
    exe = str(tmp_path_factory.mktemp("philox") / "rocrand_philox_block")
    subprocess.run([HIPCC, "-O1", "-std=c++17", "-x", "hip", "--cuda-host-only",
                    "-o", exe, os.path.join(HERE, "rocrand_philox_block.cpp")],
                   check=True, capture_output=True, timeout=300)

    def run(rows):
        text = "".join(" ".join(str(int(v)) for v in r) + "\n" for r in rows)
        out = subprocess.run([exe], input=text, capture_output=True, text=True,
                             check=True, timeout=60).stdout
        return np.array([[int(w) for w in line.split()] for line in out.splitlines()],
                        dtype=np.uint64)
    return run


def cases():
    rng = np.random.default_rng(2024)
    rows = [list(r) for r in rng.integers(0, 1 << 32, size=(3000, 6), dtype=np.uint64)]
    top = (1 << 32) - 1
    edge = [0, 1, top, top - 1, 1 << 31, (1 << 31) - 1]
    for a in edge:
        for b in edge:
            rows.append([a, b, a, b, b, a])
            rows.append([a, 0, 0, 0, b, 0])
            rows.append([0, 0, 0, a, 0, b])
    # the counters the sampler uses: (trajectory index lo, hi, 0, 0 or 1)
    for j in (0, 1, 63, 64, 1 << 20, (1 << 32) + 5):
        for blk in (0, 1):
            rows.append([j & top, j >> 32, 0, blk, 1001, 0])
    return rows


def test_philox_equals_rocrand(orc, rocrand_block):
    rows = cases()
    ref = rocrand_block(rows)
    assert ref.shape == (len(rows), 4)
    got = np.array([orc.philox(r[:4], r[4:]) for r in rows], dtype=np.uint64)
    bad = np.nonzero(np.any(got != ref, axis=1))[0]
    assert bad.size == 0, [rows[i] for i in bad[:5]]

