"""CPU oracle for exact string matching -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline leg
may import this package. The GPU library never imports it, and the two share no
code (only the seeded input generators in ``datagen`` feed both).

It computes the paper's problem statement (Section 1): all occurrences of a
pattern p of length m in a text t of length n, as ascending 0-based offsets,
overlapping occurrences included. ``find_all`` is the naive O(nm) definition
(Brute-Force, Fig. 1) in plain C; ``kmp_find_all`` is an independent
Knuth-Morris-Pratt cross-check (Fig. 1). ``find_all`` may split the range of
candidate starts over threads; each thread runs the same definition over its own
contiguous range and the lists are concatenated in range order.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading
from concurrent.futures import ThreadPoolExecutor

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "sm_oracle.c")
SO = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_default = None


def build(out_path: str = SO, mutant: int | None = None, force: bool = False) -> str:
    """Compile the oracle with gcc. ``mutant`` plants a numbered mistake (tests only)."""
    if force or mutant is not None or not os.path.exists(out_path) or \
            os.path.getmtime(out_path) < os.path.getmtime(SRC):
        cmd = ["gcc", "-O2", "-shared", "-fPIC", "-o", out_path + ".tmp%d" % os.getpid(), SRC]
        if mutant is not None:
            cmd.insert(1, "-DORACLE_MUTANT=%d" % mutant)
        subprocess.check_call(cmd)
        os.replace(out_path + ".tmp%d" % os.getpid(), out_path)
    return out_path


def _as_np(x) -> np.ndarray:
    if isinstance(x, np.ndarray):
        return np.ascontiguousarray(x, dtype=np.uint8)
    return np.frombuffer(bytes(x), dtype=np.uint8)


class Oracle:
    """Bindings to one build of the oracle library."""

    def __init__(self, so_path: str):
        L = ctypes.CDLL(so_path)
        u8p = ctypes.c_void_p
        u64 = ctypes.c_uint64
        L.oracle_naive.argtypes = [u8p, u64, u8p, u64, u64, u64, ctypes.c_void_p, u64]
        L.oracle_naive.restype = u64
        L.oracle_kmp.argtypes = [u8p, u64, u8p, u64, ctypes.c_void_p, u64, ctypes.c_void_p]
        L.oracle_kmp.restype = u64
        self._L = L

    # ---- naive definition -------------------------------------------------
    def _range(self, t: np.ndarray, p: np.ndarray, lo: int, hi: int) -> np.ndarray:
        n, m = len(t), len(p)
        cap = max(1, min(hi - lo, 1 << 16))
        while True:
            out = np.empty(cap, dtype=np.int64)
            c = self._L.oracle_naive(t.ctypes.data, n, p.ctypes.data, m, lo, hi, out.ctypes.data,
                                     cap)
            if c <= cap:
                return out[:c]
            cap = int(c)

    def find_all(self, text, pat, lo: int = 0, hi: int | None = None,
                 threads: int = 1) -> np.ndarray:
        t, p = _as_np(text), _as_np(pat)
        n, m = len(t), len(p)
        if m == 0:
            raise ValueError("empty pattern")
        if m > n:
            return np.empty(0, dtype=np.int64)
        end = n - m + 1
        hi = end if hi is None else min(hi, end)
        if hi <= lo:
            return np.empty(0, dtype=np.int64)
        if threads <= 1 or hi - lo < (1 << 16):
            return self._range(t, p, lo, hi)
        step = -(-(hi - lo) // threads)
        bounds = [(a, min(a + step, hi)) for a in range(lo, hi, step)]
        with ThreadPoolExecutor(len(bounds)) as ex:
            parts = list(ex.map(lambda b: self._range(t, p, b[0], b[1]), bounds))
        return np.concatenate(parts)

    def count(self, text, pat, threads: int = 1) -> int:
        t, p = _as_np(text), _as_np(pat)
        n, m = len(t), len(p)
        if m == 0:
            raise ValueError("empty pattern")
        if m > n:
            return 0
        end = n - m + 1
        dummy = np.empty(1, dtype=np.int64)
        if threads <= 1 or end < (1 << 16):
            return int(self._L.oracle_naive(t.ctypes.data, n, p.ctypes.data, m, 0, end,
                                            dummy.ctypes.data, 0))
        step = -(-end // threads)
        bounds = [(a, min(a + step, end)) for a in range(0, end, step)]

        def one(b):
            return int(self._L.oracle_naive(t.ctypes.data, n, p.ctypes.data, m, b[0], b[1],
                                             dummy.ctypes.data, 0))
        with ThreadPoolExecutor(len(bounds)) as ex:
            return sum(ex.map(one, bounds))

    # ---- KMP cross-check ----------------------------------------------------
    def kmp_find_all(self, text, pat) -> np.ndarray:
        t, p = _as_np(text), _as_np(pat)
        n, m = len(t), len(p)
        if m == 0:
            raise ValueError("empty pattern")
        if m > n:
            return np.empty(0, dtype=np.int64)
        fail = np.empty(m + 1, dtype=np.int64)
        cap = max(1, min(n - m + 1, 1 << 16))
        while True:
            out = np.empty(cap, dtype=np.int64)
            c = self._L.oracle_kmp(t.ctypes.data, n, p.ctypes.data, m, out.ctypes.data, cap,
                                   fail.ctypes.data)
            if c <= cap:
                return out[:c]
            cap = int(c)


def default() -> Oracle:
    global _default
    with _lock:
        if _default is None:
            _default = Oracle(build())
    return _default


def find_all(text, pat, lo: int = 0, hi: int | None = None, threads: int = 1) -> np.ndarray:
    return default().find_all(text, pat, lo, hi, threads)


def count(text, pat, threads: int = 1) -> int:
    return default().count(text, pat, threads)


def kmp_find_all(text, pat) -> np.ndarray:
    return default().kmp_find_all(text, pat)
