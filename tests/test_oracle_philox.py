"""Pins of the oracle's Philox4x32-10 and of the maps from words to numbers."""
import os
import shutil
import subprocess
from fractions import Fraction

import numpy as np
import pytest

from oracle import philox

HERE = os.path.dirname(os.path.abspath(__file__))


def _kat():
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            v = [int(t, 16) for t in line.split()]
            rows.append((v[:4], v[4:6], v[6:10]))
    return rows


def test_known_answer_vectors():
    rows = _kat()
    assert len(rows) == 3
    for ctr, key, out in rows:
        got = philox.philox4x32_10(np.array(ctr), np.array(key))
        assert [int(x) for x in got] == out


def test_batched_equals_single():
    rng = np.random.default_rng(5)
    ctr = rng.integers(0, 2**32, size=(64, 4), dtype=np.uint64)
    key = rng.integers(0, 2**32, size=2, dtype=np.uint64)
    batch = philox.philox4x32_10(ctr, key)
    for k in range(64):
        assert np.array_equal(batch[k], philox.philox4x32_10(ctr[k], key))


def test_against_rocrand_host_build(tmp_path):
    """Run rocRAND's own Philox4x32-10 (header compiled for the host) on random
    counters/keys and compare every word."""
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "rr")
    r = subprocess.run([hipcc, "-x", "hip", "--offload-arch=gfx950", "-O1",
                        os.path.join(HERE, "rocrand_philox_ref.cpp"), "-o", exe],
                       capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip("could not build rocRAND probe: " + r.stderr[-400:])
    rng = np.random.default_rng(11)
    ctr = rng.integers(0, 2**32, size=(500, 4), dtype=np.uint64)
    key = rng.integers(0, 2**32, size=(500, 2), dtype=np.uint64)
    ctr[:10] = [[b, i, 0xFFFFFFFF, 0] for b, i in zip(range(10), range(10))]
    inp = "\n".join(" ".join(str(int(x)) for x in list(c) + list(k)) for c, k in zip(ctr, key))
    out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout
    ref = np.array([[int(t) for t in line.split()] for line in out.strip().splitlines()])
    got = philox.philox4x32_10(ctr, key)
    assert np.array_equal(got.astype(np.int64), ref)


def test_counter_layout_words():
    """Word w of an individual is output word w % 4 of counter block w // 4."""
    seed = (7 << 32) | 123
    w = philox.words(seed, [3, 9], 17, 5, 10)
    key = np.array([123, 7])
    for row, ind in enumerate([3, 9]):
        for k in range(10):
            blk = philox.philox4x32_10(np.array([k // 4, ind, 17, 5]), key)
            assert w[row, k] == blk[k % 4]
            assert philox.word_at(seed, ind, 17, 5, k) == blk[k % 4]


def test_lemire_partition():
    """floor(w m / 2^32) takes every value in [0, m); the words mapping to t
    form the interval [ceil(t 2^32/m), ceil((t+1) 2^32/m)), of size
    floor(2^32/m) or that plus one, checked at its two ends."""
    for m in [1, 2, 3, 7, 10, 99, 100, 199, 255, 256, 5702, 6000]:
        t = np.arange(m, dtype=np.int64)
        lo = np.array([-(-(int(tt) << 32) // m) for tt in t], dtype=np.uint64)
        hi = np.array([-(-((int(tt) + 1) << 32) // m) for tt in t], dtype=np.uint64)
        assert np.all(philox.lemire(lo, m) == t)
        assert np.all(philox.lemire(hi - np.uint64(1), m) == t)
        sizes = (hi - lo).astype(np.int64)
        q = (1 << 32) // m
        assert np.all((sizes == q) | (sizes == q + 1))
        assert int(sizes.sum()) == 1 << 32


def test_uniform_maps_exact_and_ranges():
    w = np.array([0, 1, 255, 256, 0x7FFFFFFF, 0xFFFFFF00, 0xFFFFFFFF], dtype=np.uint64)
    r = philox.unit_open_closed(w)
    assert r.dtype == np.float32
    for wi, ri in zip(w, r):
        assert Fraction(float(ri)) == Fraction((int(wi) >> 8) + 1, 1 << 24)
    assert r[0] > 0 and r[-1] == 1.0
    u0 = philox.unit_closed_open64(w)
    assert u0[0] == 0.0 and u0[-1] < 1.0
    for wi, ui in zip(w, u0):
        assert Fraction(float(ui)) == Fraction(int(wi) >> 8, 1 << 24)


def test_words_uniform_chi2():
    from scipy.stats import chisquare
    w = philox.words(3, np.arange(4000), 0, 0, 16).ravel()
    counts = np.bincount(philox.lemire(w, 16), minlength=16)
    assert chisquare(counts).pvalue > 1e-4


def test_integer_crossover_test_is_the_float_rule():
    """The matrix-core kernel draws its crossover tests as (w >> 8) <
    floor(CR 2^24) in integers; that must be exactly the rule r <= CR (Eqs. (8),
    (9)) for the oracle's uniform r = ((w >> 8) + 1) 2^-24 and every float32 CR in
    [0, 1], the end points and the values next to every threshold included."""
    rng = np.random.default_rng(17)
    crs = np.concatenate([rng.random(3000).astype(np.float32),
                          np.array([0.0, 1.0, 0.5, 2.0 ** -24, 2.0 ** -25, 1.0 - 2.0 ** -24,
                                    np.nextafter(np.float32(1), np.float32(0))], np.float32)])
    for cr in crs:
        thr = np.uint64(np.float32(cr) * np.float32(16777216.0))   # floor: CR 2^24 is exact
        # words on both sides of the threshold, plus random ones
        edge = np.array([min(max(int(thr) + d, 0), 2 ** 24 - 1) for d in (-1, 0, 1)],
                        np.uint64) << np.uint64(8)   # 32-bit words only
        w = np.concatenate([edge, edge + np.uint64(255), rng.integers(0, 2 ** 32, 256, dtype=np.uint64)])
        want = philox.unit_open_closed(w) <= np.float32(cr)
        got = (w >> np.uint64(8)) < thr
        assert np.array_equal(got, want), float(cr)
