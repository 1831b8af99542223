"""Seeded synthetic inputs for exact string matching (texts, patterns, traces).

This package only generates inputs. It holds none of the matching arithmetic and
is the one module shared by the CPU oracle's tests and the GPU library's tests
and benchmark.

Random numbers: a counter-based SplitMix64 stream. For a (seed, stream) pair,
``key = mix64(seed * GAMMA ^ stream)`` and draw ``i`` is
``mix64(key + (i + 1) * GAMMA)``. The C file ``datagen.c`` is the fast path
(multi-threaded, used for 2^30-byte texts); the numpy functions suffixed
``_np`` are its twin and are checked equal to it in the tests.

Workload shapes follow the paper's experimental set-up (Section 2): i.i.d.
uniform "Rand sigma" texts, patterns drawn as random substrings of the text, and
pattern lengths m in {2, 4, ..., 1024}. The natural-language and biological
files the paper uses are not available; order-0 Zipf texts and uniform texts
with the same alphabet size stand in for them.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

GAMMA = 0x9E3779B97F4A7C15
MASK64 = (1 << 64) - 1

# stream identifiers (fixed; changing them changes every generated input)
STREAM_TEXT = 1
STREAM_PAT_OFFSET = 2
STREAM_PAT_BYTES = 3
STREAM_LENGTHS = 4
STREAM_ARRIVALS = 5
STREAM_CHOICE = 6
STREAM_KIND = 7

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libdatagen.so")
_SRC = os.path.join(_HERE, "datagen.c")
_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile datagen.c into libdatagen.so with gcc (OpenMP)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp, _SRC])
        os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    with _lock:
        if _lib is None:
            build()
            L = ctypes.CDLL(_SO)
            u8p = ctypes.POINTER(ctypes.c_uint8)
            u64 = ctypes.c_uint64
            L.dg_u64.argtypes = [ctypes.POINTER(ctypes.c_uint64), u64, u64, u64, u64]
            L.dg_uniform.argtypes = [u8p, u64, ctypes.c_uint32, u64, u64, u64]
            L.dg_zipf.argtypes = [u8p, u64, ctypes.POINTER(ctypes.c_double), ctypes.c_uint32,
                                  u64, u64, u64]
            L.dg_periodic.argtypes = [u8p, u64, ctypes.c_uint8, ctypes.c_uint8, u64, u64]
            for f in (L.dg_u64, L.dg_uniform, L.dg_zipf, L.dg_periodic):
                f.restype = None
            _lib = L
    return _lib


def _u8ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


# ----------------------------------------------------------------------------
# numpy twins (reference; used for small sizes and to pin the C fast path)
# ----------------------------------------------------------------------------

def _mix64_np(z: np.ndarray) -> np.ndarray:
    z = z.astype(np.uint64, copy=True)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def _key(seed: int, stream: int) -> int:
    z = ((seed * GAMMA) & MASK64) ^ stream
    return int(_mix64_np(np.array([z], dtype=np.uint64))[0])


def u64_np(count: int, seed: int, stream: int, start: int = 0) -> np.ndarray:
    key = _key(seed, stream)
    i = np.arange(start + 1, start + count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(key) + i * np.uint64(GAMMA)
    return _mix64_np(z)


def uniform_np(count: int, sigma: int, seed: int, stream: int = STREAM_TEXT,
               start: int = 0) -> np.ndarray:
    x = u64_np(count, seed, stream, start)
    return ((x >> np.uint64(32)) % np.uint64(sigma)).astype(np.uint8)


def zipf_np(count: int, cdf: np.ndarray, seed: int, stream: int = STREAM_TEXT,
            start: int = 0) -> np.ndarray:
    x = u64_np(count, seed, stream, start)
    u = (x >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
    return np.searchsorted(cdf, u, side="right").astype(np.uint8)


# ----------------------------------------------------------------------------
# fast generators (C)
# ----------------------------------------------------------------------------

def u64(count: int, seed: int, stream: int, start: int = 0) -> np.ndarray:
    out = np.empty(count, dtype=np.uint64)
    if count:
        lib().dg_u64(out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), count, seed & MASK64,
                     stream, start)
    return out


def unit_floats(count: int, seed: int, stream: int, start: int = 0) -> np.ndarray:
    """53-bit uniforms in [0, 1) from the stream."""
    return (u64(count, seed, stream, start) >> np.uint64(11)).astype(np.float64) * (
        1.0 / 9007199254740992.0)


def uniform_text(n: int, sigma: int, seed: int, stream: int = STREAM_TEXT,
                 out: np.ndarray | None = None) -> np.ndarray:
    """i.i.d. uniform bytes over {0, ..., sigma-1} (the paper's Rand sigma texts)."""
    if not 1 <= sigma <= 256:
        raise ValueError("sigma must be in [1, 256]")
    if out is None:
        out = np.empty(n, dtype=np.uint8)
    if n:
        lib().dg_uniform(_u8ptr(out), n, sigma, seed & MASK64, stream, 0)
    return out


def zipf_cdf(K: int, s: float) -> np.ndarray:
    """CDF of the order-0 Zipf law P(rank k) = k^-s / sum_{j<=K} j^-s, k = 1..K."""
    w = np.arange(1, K + 1, dtype=np.float64) ** (-float(s))
    c = np.cumsum(w) / w.sum()
    c[-1] = 1.0
    return c


def zipf_text(n: int, K: int, s: float, seed: int, stream: int = STREAM_TEXT,
              out: np.ndarray | None = None) -> np.ndarray:
    """Order-0 Zipf(s) bytes over {0, ..., K-1}; byte k-1 has rank k."""
    cdf = np.ascontiguousarray(zipf_cdf(K, s))
    if out is None:
        out = np.empty(n, dtype=np.uint8)
    if n:
        lib().dg_zipf(_u8ptr(out), n, cdf.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), K,
                      seed & MASK64, stream, 0)
    return out


def periodic_text(n: int, a: int, b: int, period: int, out: np.ndarray | None = None) -> np.ndarray:
    """Byte a everywhere except byte b at every index i with i % period == period-1."""
    if out is None:
        out = np.empty(n, dtype=np.uint8)
    if n:
        lib().dg_periodic(_u8ptr(out), n, a, b, period, 0)
    return out


# ----------------------------------------------------------------------------
# patterns and traces
# ----------------------------------------------------------------------------

def substring_offset(n: int, m: int, seed: int, idx: int) -> int:
    """Offset of the idx-th substring pattern: draw(idx) mod (n - m + 1)."""
    if m > n:
        raise ValueError("m > n")
    x = int(u64_np(1, seed, STREAM_PAT_OFFSET, idx)[0])
    return x % (n - m + 1)


def substring_pattern(text: np.ndarray, m: int, seed: int, idx: int) -> tuple[bytes, int]:
    """A pattern copied from the text (the paper draws its patterns this way)."""
    off = substring_offset(len(text), m, seed, idx)
    return bytes(text[off:off + m]), off


def random_pattern(m: int, sigma: int, seed: int, idx: int) -> bytes:
    """An i.i.d. uniform pattern over {0..sigma-1}; idx selects a disjoint slice."""
    return uniform_np(m, sigma, seed, STREAM_PAT_BYTES, start=idx * 4096).tobytes()


def log_uniform_lengths(count: int, lo: int, hi: int, seed: int) -> np.ndarray:
    """m = clamp(round(2^(log2 lo + u (log2 hi - log2 lo))), lo, hi)."""
    u = (u64_np(count, seed, STREAM_LENGTHS) >> np.uint64(11)).astype(np.float64) * (
        1.0 / 9007199254740992.0)
    e = np.log2(lo) + u * (np.log2(hi) - np.log2(lo))
    return np.clip(np.rint(np.exp2(e)), lo, hi).astype(np.int64)


def poisson_arrivals(count: int, qps: float, seed: int) -> np.ndarray:
    """Arrival times (seconds) of an open-loop Poisson process with rate qps."""
    u = (u64_np(count, seed, STREAM_ARRIVALS) >> np.uint64(11)).astype(np.float64) * (
        1.0 / 9007199254740992.0)
    return np.cumsum(-np.log1p(-u) / qps)


def choices(count: int, k: int, seed: int, stream: int = STREAM_CHOICE) -> np.ndarray:
    """count draws uniform over {0..k-1}."""
    return ((u64_np(count, seed, stream) >> np.uint64(32)) % np.uint64(k)).astype(np.int64)
