"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Each ``pin_*`` function takes an ``oracle.Oracle`` and raises AssertionError on a
violation. The pins are run against the real oracle (they must all pass) and
against builds with a planted mistake (at least one must fail), so a plausible
slip anywhere in the oracle is caught.

Sources of truth used here:
  * hand-checked lists (tests/golden/hand_cases.txt), from the problem statement
    in the paper's Section 1;
  * Python's ``re`` engine with a zero-width lookahead, an independent library
    search that reports overlapping occurrences;
  * iterated ``bytes.find`` restarted one byte after each hit;
  * closed forms: a^m in a^n, a^(m-1)b in a periodic text, (ab)^k in (ab)^N, and
    the exact total over all binary texts of length n, which is
    (n - m + 1) * 2^(n - m) for any binary pattern of length m <= n (each of the
    n - m + 1 windows equals p in exactly 2^(n-m) texts);
  * planted occurrences and boundary cases.
"""
from __future__ import annotations

import itertools
import os
import re

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "hand_cases.txt")


def load_hand_cases():
    cases = []
    with open(GOLDEN) as f:
        for line in f:
            if not line.strip() or line.startswith("#"):
                continue
            t, p, pos = line.rstrip("\n").split("\t")
            want = [] if pos == "-" else [int(x) for x in pos.split()]
            cases.append((t.encode(), p.encode(), want))
    return cases


def re_find_all(t: bytes, p: bytes) -> list[int]:
    return [mo.start() for mo in re.finditer(b"(?=" + re.escape(p) + b")", t)]


def find_iter(t: bytes, p: bytes) -> list[int]:
    out, i = [], t.find(p)
    while i >= 0:
        out.append(i)
        i = t.find(p, i + 1)
    return out


def pin_hand_cases(orc):
    for t, p, want in load_hand_cases():
        got = orc.find_all(t, p).tolist()
        assert got == want, (t, p, got, want)
        assert orc.count(t, p) == len(want), (t, p)


def pin_exhaustive_binary(orc, nmax: int = 9):
    """Every binary text with n <= nmax against every pattern with m <= 4."""
    for n in range(0, nmax + 1):
        texts = [bytes(x) for x in itertools.product((0, 1), repeat=n)]
        for m in range(1, 5):
            for p in itertools.product((0, 1), repeat=m):
                p = bytes(p)
                total = 0
                for t in texts:
                    got = orc.find_all(t, p).tolist() if n else []
                    assert got == re_find_all(t, p), (t, p, got)
                    total += len(got)
                want = (n - m + 1) * 2 ** (n - m) if m <= n else 0
                assert total == want, (n, p, total, want)


def pin_binary_total_closed_form(orc, n: int = 12):
    """Sum over all 2^n binary texts of |occ| equals (n-m+1) 2^(n-m) (counts only)."""
    texts = [bytes(x) for x in itertools.product((0, 1), repeat=n)]
    for m in (1, 3, 5):
        for p in (bytes([0] * m), bytes([i & 1 for i in range(m)]), bytes([1] + [0] * (m - 1))):
            total = sum(orc.count(t, p) for t in texts)
            assert total == (n - m + 1) * 2 ** (n - m), (p, total)


def pin_random_vs_library(orc, cases: int = 20000, seed: int = 7):
    rng = np.random.default_rng(seed)
    for _ in range(cases):
        sigma = int(rng.choice([1, 2, 3, 4, 256]))
        n = int(rng.integers(0, 300))
        m = int(rng.integers(1, 13))
        t = rng.integers(0, sigma, n, dtype=np.uint8).tobytes()
        if n >= m and rng.random() < 0.5:
            r = int(rng.integers(0, n - m + 1))
            p = t[r:r + m]
        else:
            p = rng.integers(0, sigma, m, dtype=np.uint8).tobytes()
        got = orc.find_all(t, p).tolist() if n else []
        want = find_iter(t, p)
        assert got == want, (t, p, got, want)
        if n:
            assert orc.kmp_find_all(t, p).tolist() == want, (t, p)


def pin_closed_forms(orc):
    # p = a^m in t = a^n: every start 0..n-m
    for n, m in ((1, 1), (7, 3), (100, 100), (1000, 17), (4096, 64)):
        got = orc.find_all(b"a" * n, b"a" * m)
        assert np.array_equal(got, np.arange(n - m + 1)), (n, m)
    # t = a^n with b at i % P == P-1, p = a^(m-1) b: hits exactly at P k + P - m
    for P, n, m in ((64, 64 * 40, 4), (64, 64 * 40 + 5, 64), (4096, 4096 * 9, 256), (16, 160, 1)):
        t = bytearray(b"a" * n)
        for i in range(P - 1, n, P):
            t[i] = ord("b")
        p = b"a" * (m - 1) + b"b"
        want = [P * k + P - m for k in range(n // P) if P * k + P - m >= 0]
        assert orc.find_all(bytes(t), p).tolist() == want, (P, n, m)
    # p = (ab)^k in t = (ab)^N: every even offset <= n - m
    for N, k in ((10, 1), (50, 7), (300, 64)):
        t, p = b"ab" * N, b"ab" * k
        assert orc.find_all(t, p).tolist() == list(range(0, 2 * N - 2 * k + 1, 2)), (N, k)


def pin_planted_and_edges(orc, seed: int = 11):
    rng = np.random.default_rng(seed)
    for _ in range(200):
        n = int(rng.integers(1, 2000))
        m = int(rng.integers(1, min(n, 70) + 1))
        t = rng.integers(0, 256, n, dtype=np.uint8)
        r = int(rng.integers(0, n - m + 1))
        p = t[r:r + m].copy()
        got = orc.find_all(t, p)
        assert r in got.tolist()
        assert np.all(np.diff(got) > 0)
        for i in got.tolist():
            assert np.array_equal(t[i:i + m], p)
        # hits at both ends (when the two copies do not overlap)
        if n < 2 * m:
            continue
        t2 = t.copy()
        t2[:m] = p
        t2[n - m:] = p
        g2 = orc.find_all(t2, p).tolist()
        assert g2[0] == 0 and g2[-1] == n - m
    # m > n, m == n
    assert orc.find_all(b"abc", b"abcd").size == 0
    assert orc.find_all(b"abc", b"abc").tolist() == [0]
    assert orc.find_all(b"abc", b"abd").size == 0
    assert orc.count(b"", b"a") == 0
    # threaded split equals the single range
    t = np.frombuffer(b"ab" * 70000, dtype=np.uint8)
    a = orc.find_all(t, b"bab", threads=1)
    b = orc.find_all(t, b"bab", threads=5)
    assert np.array_equal(a, b) and a.size == 69999
    assert orc.count(t, b"bab", threads=3) == 69999


def pin_statistics(orc):
    """E|occ| = (n-m+1) sigma^-m on i.i.d. uniform text (not exact: 6-sigma band)."""
    rng = np.random.default_rng(3)
    n = 1 << 18
    t = rng.integers(0, 4, n, dtype=np.uint8)
    p = bytes([0, 1, 2, 3, 0, 1])
    mean = (n - 6 + 1) / 4 ** 6
    c = orc.count(t, p)
    assert abs(c - mean) < 6 * np.sqrt(mean) + 1, (c, mean)


ALL_PINS = [pin_hand_cases, pin_exhaustive_binary, pin_binary_total_closed_form,
            pin_random_vs_library, pin_closed_forms, pin_planted_and_edges, pin_statistics]


def failing_pins(orc) -> list[str]:
    bad = []
    for f in ALL_PINS:
        try:
            if f is pin_random_vs_library:
                f(orc, cases=3000)
            elif f is pin_exhaustive_binary:
                f(orc, nmax=7)
            else:
                f(orc)
        except AssertionError:
            bad.append(f.__name__)
    return bad
