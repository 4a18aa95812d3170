"""Pins for the oracle's randomness: Philox4x32-10 and Lemire's bounded draw.

The paper leaves the random source open; the method fixes Philox4x32-10
keyed by (seed, sample id) and an exact bounded integer per sample.  The
block function is checked against rocRAND's open-source engine (compiled
here for the host); the bounded draw against the exact uniformity it must
have, exhaustively on narrow words.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import stats

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_xcheck(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("xcheck") / "philox_xcheck")
    subprocess.run([hipcc, "--offload-arch=gfx950", "-O1", os.path.join(HERE, "philox_xcheck.cpp"), "-o", exe],
                   check=True, capture_output=True)
    return exe


def test_philox_block_matches_rocrand(rocrand_xcheck):
    rng = np.random.default_rng(12345)
    cases = [(0, 0, 0, 0, 0, 0), (1, 2, 3, 4, 5, 6), (0xFFFFFFFF, 0, 0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF)]
    for _ in range(300):
        c = rng.integers(0, 2 ** 32, size=6, dtype=np.uint64)
        c[1] %= 2 ** 30
        cases.append(tuple(int(x) for x in c))
    inp = "\n".join(" ".join(str(x) for x in c) for c in cases) + "\n"
    out = subprocess.run([rocrand_xcheck], input=inp, capture_output=True, text=True, check=True).stdout
    lines = out.strip().split("\n")
    assert len(lines) == len(cases)
    for c, line in zip(cases, lines):
        want = [int(x) for x in line.split()]
        got = oracle.philox4x32_10(c[:4], c[4:]).tolist()
        assert got == want, c


@pytest.mark.parametrize("bits", [6, 8])
def test_lemire_is_exactly_uniform_on_narrow_words(bits):
    """Every r in [0,R) has exactly floor(2^b/R) accepted preimages and
    exactly 2^b mod R words are rejected."""
    size = 1 << bits
    for R in range(1, size + 1):
        hits = np.zeros(R, np.int64)
        rejected = 0
        for x in range(size):
            ok, r = oracle.lemire(x, R, bits)
            if ok:
                assert 0 <= r < R
                hits[r] += 1
            else:
                rejected += 1
        assert np.all(hits == size // R), R
        assert rejected == size % R, R


def test_lemire_64bit_edges():
    assert oracle.lemire(0, 1, 64) == (True, 0)
    assert oracle.lemire(2 ** 64 - 1, 1, 64) == (True, 0)
    # R = 2^64 - 1: every word is accepted and r = floor(x R / 2^64) <= x
    for x in (0, 1, 12345, 2 ** 63, 2 ** 64 - 1):
        assert oracle.lemire(x, 2 ** 64 - 1, 64)[1] <= x
    # R = 2^63 + 1: (2^64 - R) mod R = 2^63 - 1, the low half must be >= that
    R = 2 ** 63 + 1
    ok, r = oracle.lemire(1, R, 64)  # x R mod 2^64 = R >= t: accepted, r = 0
    assert ok and r == 0
    ok, _ = oracle.lemire(2, R, 64)  # 2R mod 2^64 = 2 < t: rejected
    assert not ok


def test_draw_consumes_candidates_in_order():
    """r is the first accepted 64-bit word among (w0|w1, w2|w3) of attempt
    0, then attempt 1, ...; a large R forces rejections."""
    R = 2 ** 63 + 12345  # about half of all words are rejected
    seed = 0x0123456789ABCDEF
    saw_retry = False
    for sid in range(200):
        got = oracle.draw(seed, 1, sid, R)
        want = None
        attempt = 0
        while want is None:
            w = oracle.philox4x32_10([sid & 0xFFFFFFFF, sid >> 32, 1, attempt],
                                     [seed & 0xFFFFFFFF, seed >> 32]).tolist()
            for x in (w[0] | (w[1] << 32), w[2] | (w[3] << 32)):
                ok, r = oracle.lemire(x, R, 64)
                if ok:
                    want = r
                    break
            saw_retry |= attempt > 0
            attempt += 1
        assert got == want
    assert saw_retry


def test_draws_are_uniform_and_in_range():
    for R in (1, 2, 7, 1000):
        vals = np.array([oracle.draw(42, 0, i, R) for i in range(20000)])
        assert vals.min() >= 0 and vals.max() < R
        if R > 1:
            counts = np.bincount(vals, minlength=R)
            assert stats.chisquare(counts).pvalue > 1e-4
    big = 2 ** 62 + 3
    vals = [oracle.draw(7, 1, i, big) for i in range(5000)]
    assert max(vals) < big
    # top two bits of r / big: quartiles uniform
    q = np.bincount([int(v * 4 // big) for v in vals], minlength=4)
    assert stats.chisquare(q).pvalue > 1e-4


def test_tags_and_seeds_give_distinct_streams():
    a = [oracle.draw(1, 0, i, 2 ** 40) for i in range(64)]
    b = [oracle.draw(1, 1, i, 2 ** 40) for i in range(64)]
    c = [oracle.draw(2, 0, i, 2 ** 40) for i in range(64)]
    assert a != b and a != c
    assert len(set(a)) == 64


def test_batch_draws_equal_single_draws():
    """oracle.draws (one C loop) is draw() id by id, from any first id."""
    for first, R in ((0, 1000), (2 ** 33 - 5, 2 ** 63 + 12345), (77, 4098)):
        got = oracle.draws(3, 1, first, 300, R)
        assert got.dtype == np.uint64
        assert got.tolist() == [oracle.draw(3, 1, first + i, R) for i in range(300)]
