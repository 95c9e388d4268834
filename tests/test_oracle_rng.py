"""Pins of the oracle's random numbers (CPU only).

Philox4x32-10 (Salmon et al., SC'11) is checked against rocRAND's independent
engine compiled for the host from its public header; the bounded-integer and
Bernoulli maps against exact rational arithmetic.
"""
import os
import shutil
import subprocess
from fractions import Fraction

import numpy as np
import pytest

from oracle import cnd_oracle as O
from oracle import miniref

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_ref(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists("/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"):
        pytest.skip("hipcc/rocRAND headers not available: Philox pin cannot run")
    exe = tmp_path_factory.mktemp("rr") / "rocrand_philox_ref"
    subprocess.run([hipcc, "-O1", "--offload-arch=gfx950", os.path.join(HERE, "rocrand_philox_ref.cpp"),
                    "-o", str(exe)], check=True, cwd="/tmp")
    return str(exe)


def _cases():
    rng = np.random.default_rng(11)
    cases = [
        (0, 0, 0, 0, 0, 0),
        (0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF, (1 << 30) - 1, 0xFFFFFFFF, 0xFFFFFFFF),
        (1, 0, 0, 0, 0, 0),
        (0, 1, 0, 0, 0, 0),
        (0, 0, 1, 0, 0, 0),
        (0, 0, 0, 1, 0, 0),
        (0, 0, 0, 0, 1, 0),
        (0, 0, 0, 0, 0, 1),
    ]
    for _ in range(200):
        k0, k1, c0, c2, c3 = (int(x) for x in rng.integers(0, 2**32, size=5, dtype=np.uint64))
        c1 = int(rng.integers(0, 2**30))
        cases.append((k0, k1, c0, c1, c2, c3))
    # the counter layout the method uses: (slot, individual, generation, stream<<24 | attempt)
    for stream in range(6):
        for attempt in (0, 1, 7, (1 << 24) - 1):
            cases.append((123456789, 0, 17, 5, 3, (stream << 24) | attempt))
    return cases


def test_philox_matches_rocrand(rocrand_ref):
    cases = _cases()
    inp = "\n".join(" ".join(str(x) for x in c) for c in cases) + "\n"
    out = subprocess.run([rocrand_ref], input=inp, capture_output=True, text=True, check=True).stdout.split("\n")
    for c, line in zip(cases, out):
        k0, k1, c0, c1, c2, c3 = c
        ref = [int(x) for x in line.split()]
        got = O.philox([c0, c1, c2, c3], [k0, k1]).tolist()
        assert got == ref, (c, got, ref)


def test_philox_two_transcriptions_agree():
    rng = np.random.default_rng(5)
    for _ in range(300):
        ctr = [int(x) for x in rng.integers(0, 2**32, size=4, dtype=np.uint64)]
        key = [int(x) for x in rng.integers(0, 2**32, size=2, dtype=np.uint64)]
        assert O.philox(ctr, key).tolist() == list(miniref.philox4x32_10(ctr, key))


def test_draw_layout():
    # counter = (slot, individual, generation, stream<<24 | attempt), key = seed split in words
    seed = (7 << 32) | 99
    got = O.draw(seed, 3, 4, 5, O.ST_MUTATE, 6).tolist()
    assert got == O.philox([3, 4, 5, (4 << 24) | 6], [99, 7]).tolist()


def test_bounded_exact():
    for m in (1, 2, 3, 10, 200, 10_000, 200_000, 2**31 - 1, 2**32 - 1):
        assert O.bounded(0, m) == 0
        assert O.bounded(2**32 - 1, m) == m - 1
        assert O.bounded(2**31, m) == m // 2
        for w in (1, 12345, 2**31 + 5, 4_000_000_000):
            assert O.bounded(w, m) == (w * m) // 2**32
            assert O.bounded(w, m) == int(Fraction(w, 2**32) * m)


def test_bounded_is_uniform_enough():
    # the map w -> floor(w m / 2^32) hits each of m values either floor(2^32/m)
    # or ceil(2^32/m) times; sampled over Philox words it looks uniform.
    m = 7
    words = [int(O.draw(1, j, 0, 0, 0)[0]) for j in range(7000)]
    counts = np.bincount([O.bounded(w, m) for w in words], minlength=m)
    expected = len(words) / m
    chi2 = ((counts - expected) ** 2 / expected).sum()
    assert chi2 < 22.46  # 0.999 quantile of chi-square with 6 dof


def test_threshold_exact():
    for p in (0.0, 1e-9, 0.05, 0.3, 0.5, 0.6, 0.7, 0.999999, 1.0):
        want = 0 if p <= 0 else (2**32 if p >= 1 else int(Fraction(p) * 2**32))
        assert O.threshold(p) == want
    assert O.threshold(0.7) == 3006477107
    assert O.threshold(0.05) == 214748364
    assert O.threshold(-1) == 0 and O.threshold(2.0) == 2**32
