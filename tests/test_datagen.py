"""Seeded input generators: C fast path equals the numpy twin; determinism; shapes."""
import hashlib

import numpy as np

import datagen as dg


def test_u64_c_equals_numpy():
    for seed, stream, start in ((1, 1, 0), (2, 7, 12345), (2**63 + 5, 3, 2**40)):
        assert np.array_equal(dg.u64(5000, seed, stream, start), dg.u64_np(5000, seed, stream, start))


def test_splitmix_reference_values():
    # SplitMix64 finaliser of a known input, computed by hand from the published constants
    z = 0x9E3779B97F4A7C15
    x = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9 % 2**64
    x = (x ^ (x >> 27)) * 0x94D049BB133111EB % 2**64
    x ^= x >> 31
    assert int(dg._mix64_np(np.array([z], dtype=np.uint64))[0]) == x


def test_uniform_c_equals_numpy():
    for sigma in (1, 2, 4, 16, 20, 64, 256):
        a = dg.uniform_text(100003, sigma, seed=1)
        b = dg.uniform_np(100003, sigma, seed=1)
        assert np.array_equal(a, b)
        assert a.max() < sigma


def test_uniform_large_is_parallel_and_deterministic():
    a = dg.uniform_text(1 << 22, 4, seed=1)
    b = dg.uniform_text(1 << 22, 4, seed=1)
    assert np.array_equal(a, b)
    # slices equal the numpy twin at an arbitrary start
    assert np.array_equal(a[3_000_000:3_000_100], dg.uniform_np(100, 4, 1, start=3_000_000))
    h = np.bincount(a, minlength=4) / a.size
    assert np.all(np.abs(h - 0.25) < 0.002)


def test_zipf_c_equals_numpy_and_law():
    cdf = dg.zipf_cdf(64, 1.0)
    a = dg.zipf_text(200000, 64, 1.0, seed=5)
    b = dg.zipf_np(200000, cdf, seed=5)
    assert np.array_equal(a, b)
    p = np.bincount(a, minlength=64) / a.size
    w = 1.0 / np.arange(1, 65)
    assert abs(p[0] - w[0] / w.sum()) < 0.005
    assert p[0] > p[1] > p[3] > p[15]


def test_periodic():
    t = dg.periodic_text(4096 * 3, ord("a"), ord("b"), 4096)
    assert t[4095] == ord("b") and t[8191] == ord("b") and t[4094] == ord("a")
    assert int((t == ord("b")).sum()) == 3


def test_patterns_and_traces():
    t = dg.uniform_text(1 << 20, 4, seed=1)
    p, off = dg.substring_pattern(t, 8, seed=1, idx=0)
    assert bytes(t[off:off + 8]) == p
    q = dg.random_pattern(16, 4, seed=2, idx=3)
    assert len(q) == 16 and max(q) < 4
    ms = dg.log_uniform_lengths(4096, 2, 1024, seed=3)
    assert ms.min() >= 2 and ms.max() <= 1024
    assert 0.2 < np.mean(ms <= 45) < 0.8
    arr = dg.poisson_arrivals(20000, 1000.0, seed=14)
    assert np.all(np.diff(arr) > 0) and abs(arr[-1] - 20.0) < 1.0


def test_recorded_digests():
    """SHA-256 of fixed generator outputs (tests/golden/datagen_sha256.txt)."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "datagen_sha256.txt")
    from tests.golden.make_datagen_digests import digests
    want = dict(l.split() for l in open(path) if l.strip() and not l.startswith("#"))
    assert digests() == want
