"""Pins of the oracle's counter-based generator (Philox4x32-10, Salmon et
al. SC'11) and of its uniform mapping, which drives the inverse-transform
sampling of Sec. 2.1.1."""
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import stats

HERE = os.path.dirname(os.path.abspath(__file__))


def _rocrand_ref(tmp_path, rows):
    hdr = "/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"
    if not os.path.exists(hdr) or shutil.which("g++") is None:
        pytest.skip("rocRAND headers or g++ not available")
    exe = str(tmp_path / "philox_ref")
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                           os.path.join(HERE, "rocrand_philox_ref.cpp"), "-o", exe])
    inp = "\n".join(" ".join(str(v) for v in r) for r in rows) + "\n"
    out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout
    return [list(map(int, line.split())) for line in out.strip().splitlines()]


def test_philox_matches_rocrand_library(oracle, tmp_path):
    rng = np.random.default_rng(123)
    rows = [[0, 0, 0, 0, 0, 0], [0xFFFFFFFF] * 6, [1, 2, 3, 4, 5, 6]]
    rows += rng.integers(0, 2**32, size=(500, 6), dtype=np.uint64).tolist()
    ref = _rocrand_ref(tmp_path, rows)
    assert len(ref) == len(rows)
    for r, expect in zip(rows, ref):
        assert oracle.philox(r[:4], r[4:]) == expect


def test_philox_output_is_uniform_and_uncorrelated(oracle):
    # 2^14 counters x 4 words: chi^2 of the top byte and serial correlation.
    words = []
    for pid in range(4096):
        words += oracle.philox([pid, 0, 1, 0], [7, 0])
    w = np.array(words, dtype=np.uint64)
    top = (w >> 24).astype(np.int64)
    hist = np.bincount(top, minlength=256)
    chi2 = stats.chisquare(hist)
    assert chi2.pvalue > 1e-4
    u = (w.astype(np.float64) + 0.5) / 2**32
    r = np.corrcoef(u[:-1], u[1:])[0, 1]
    assert abs(r) < 4.0 / np.sqrt(u.size)


def test_philox_counter_and_key_sensitivity(oracle):
    base = oracle.philox([5, 6, 7, 8], [9, 10])
    for i in range(4):
        c = [5, 6, 7, 8]
        c[i] ^= 1
        assert oracle.philox(c, [9, 10]) != base
    assert oracle.philox([5, 6, 7, 8], [9, 11]) != base


def test_uniform_mapping_open_interval_and_fp32_exact(oracle):
    xs = [0, 1, 511, 512, 0x7FFFFFFF, 0x80000000, 0xFFFFFE00, 0xFFFFFFFF]
    xs += list(np.random.default_rng(1).integers(0, 2**32, size=2000))
    for x in xs:
        u = oracle.uniform(int(x))
        assert 0.0 < u < 1.0
        assert float(np.float32(u)) == u           # same value on an FP32 path
        assert float(np.float32(1.0 - u)) == 1.0 - u  # 1-u (free path) exact too
        # complementary words map to complementary uniforms
        assert oracle.uniform(int(x) ^ 0xFFFFFFFF) + u == 1.0
    assert oracle.uniform(0) == 2.0**-24
    assert oracle.uniform(0xFFFFFFFF) == 1.0 - 2.0**-24
