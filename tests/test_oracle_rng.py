"""Pins of the oracle's random streams.

* Philox4x32-10 against rocRAND's independently written host-callable engine
  (compiled from the installed header) on random (counter, key) pairs.
* The uniform map u = (2*(x >> 9) + 1) * 2^-24, exhaustively over all 2^23
  values of the top bits: exact, strictly inside (0, 1), symmetric.
"""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def kat_exe():
    if shutil.which("g++") is None or not os.path.exists("/opt/rocm/include/rocrand"):
        pytest.skip("needs g++ and the rocRAND headers")
    d = tempfile.mkdtemp(prefix="philox_kat_")
    exe = os.path.join(d, "kat")
    subprocess.run(["g++", "-O1", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                    os.path.join(HERE, "philox_rocrand_kat.cpp"), "-o", exe], check=True)
    yield exe
    shutil.rmtree(d, ignore_errors=True)


def test_philox_matches_rocrand(oracle_lib, kat_exe):
    rng = np.random.default_rng(12345)
    n = 2000
    ctr = rng.integers(0, 2**32, size=(n, 4), dtype=np.uint64)
    ctr[:, 1] &= (1 << 30) - 1          # keep 4*(c0 | c1<<32) inside 64 bits
    key = rng.integers(0, 2**32, size=(n, 2), dtype=np.uint64)
    # edge counters and keys
    ctr[0] = 0; key[0] = 0
    ctr[1] = [0xFFFFFFFF, (1 << 30) - 1, 0xFFFFFFFF, 0xFFFFFFFF]; key[1] = [0xFFFFFFFF] * 2
    lines = "\n".join(" ".join(str(int(v)) for v in (*c, *k)) for c, k in zip(ctr, key))
    out = subprocess.run([kat_exe], input=lines, capture_output=True, text=True, check=True)
    ref = np.array([[int(v) for v in l.split()] for l in out.stdout.strip().splitlines()],
                   dtype=np.uint64)
    assert ref.shape == (n, 4)
    got = np.array([oracle.philox(c.astype(np.uint32), k.astype(np.uint32))
                    for c, k in zip(ctr, key)], dtype=np.uint64)
    assert np.array_equal(got, ref)


def test_philox_words_uniform(oracle_lib):
    # chi-square of the top byte of 4*20000 words from consecutive counters
    words = np.concatenate([oracle.philox([i, 7, 0, 0], [0xDEADBEEF, 0x12345678])
                            for i in range(20000)])
    hist = np.bincount(words >> 24, minlength=256)
    exp = words.size / 256
    chi2 = ((hist - exp) ** 2 / exp).sum()
    z = (chi2 - 255) / np.sqrt(2 * 255)
    assert abs(z) < 5, z


def test_uniform_map_exhaustive(oracle_lib):
    top = np.arange(1 << 23, dtype=np.uint32)
    x = (top << 9) | np.uint32(0x1FF)          # low bits must not matter
    u = oracle.uniform(x)
    u0 = oracle.uniform(top << 9)
    assert np.array_equal(u, u0)
    exact = (2.0 * top.astype(np.float64) + 1.0) * 2.0 ** -24
    assert np.array_equal(u.astype(np.float64), exact)
    assert u.min() == np.float32(2.0 ** -24) and u.max() == np.float32(1 - 2.0 ** -24)
    assert np.all(u > 0) and np.all(u < 1)
    # symmetric: u(x) + u(~x) == 1 exactly
    assert np.all(u.astype(np.float64) + u[::-1].astype(np.float64) == 1.0)
    # -ln(u) is finite and bounded by 24 ln 2
    assert -np.log(u.min().astype(np.float64)) < 16.64
