"""Pins for the oracle's Philox4x32-10 (``oracle.philox``).

The oracle's generator is written from the SC'11 definition.  It is pinned
against a second, independent implementation (rocRAND's open-source header
engine, compiled here on the host) and by statistical properties.
"""

import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

from oracle import philox

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_exe():
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to build the rocRAND helper")
    d = tempfile.mkdtemp(prefix="philox_pin_")
    exe = os.path.join(d, "words")
    src = os.path.join(HERE, "golden", "rocrand_philox_words.cpp")
    subprocess.run([hipcc, "-O1", src, "-o", exe], check=True,
                   capture_output=True)
    yield exe
    shutil.rmtree(d, ignore_errors=True)


def _rocrand(exe, seed, stream, real, e0, count):
    out = subprocess.run([exe, str(seed), str(stream), str(real), str(e0),
                          str(count)], check=True, capture_output=True,
                         text=True).stdout.split()
    return np.array([int(t) for t in out], dtype=np.uint64)


CASES = [
    (0, 0, 0, 0, 64),
    (0, 1, 0, 0, 64),
    (0, 0, 1, 0, 64),
    (12345, 0, 1, 3, 61),                    # unaligned start
    (0xDEADBEEFCAFEF00D, 1, 0, 1 << 20, 33),  # high key word in use
    (7, 0, 1, (1 << 34) + 5, 40),            # counter high word in use
    (2**64 - 1, 0, 0, 2**35 - 7, 16),        # carry across words
]


@pytest.mark.parametrize("seed,stream,real,e0,count", CASES)
def test_matches_rocrand(rocrand_exe, seed, stream, real, e0, count):
    want = _rocrand(rocrand_exe, seed, stream, real, e0, count)
    got = philox.words(seed, stream, real, e0, count).astype(np.uint64)
    np.testing.assert_array_equal(got, want)


def test_words_are_slices_of_one_sequence():
    full = philox.words(3, 0, 1, 0, 1000)
    for a in (0, 1, 2, 3, 17, 998):
        part = philox.words(3, 0, 1, a, 1000 - a)
        np.testing.assert_array_equal(part, full[a:])


def test_bit_balance_and_uniformity():
    w = philox.words(99, 0, 0, 0, 1 << 18)
    bits = np.unpackbits(w.view(np.uint8))
    # each bit position is a fair coin: |mean - 1/2| within 6 sigma
    per_pos = np.unpackbits(w.view(np.uint8)).reshape(-1, 32).mean(axis=0)
    sig = 0.5 / np.sqrt(w.size)
    assert np.all(np.abs(per_pos - 0.5) < 6 * sig)
    assert abs(bits.mean() - 0.5) < 6 * 0.5 / np.sqrt(bits.size)
    # byte histogram chi-square (255 dof): mean 255, sd ~22.6
    hist = np.bincount(w.view(np.uint8), minlength=256)
    exp = w.size * 4 / 256
    chi2 = float(((hist - exp) ** 2 / exp).sum())
    assert chi2 < 255 + 6 * 22.6


def test_streams_and_realizations_differ():
    a = philox.words(5, 0, 0, 0, 4096)
    b = philox.words(5, 0, 1, 0, 4096)
    c = philox.words(5, 1, 0, 0, 4096)
    d = philox.words(6, 0, 0, 0, 4096)
    for u, v in ((a, b), (a, c), (b, c), (a, d)):
        # independent 32-bit words agree with probability 2^-32 each
        assert np.count_nonzero(u == v) <= 1
