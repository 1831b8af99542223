"""MI355X-native online exact string matching (Python binding of include/sm.h).

Every step of the search runs in the HIP kernels of ``libsm.so``; this module only
marshals arguments. PyTorch tensors provide device memory and streams.

    import torch, paper_1012_2547_amd as sm
    text = torch.randint(0, 4, (1 << 30,), dtype=torch.uint8, device="cuda")
    pos = sm.find_all(text, b"\\x00\\x01\\x02\\x03")     # int64 tensor on the GPU
    n = sm.count(text, b"\\x00\\x01")
"""
from __future__ import annotations

import ctypes

import numpy as np

from ._native import (ALGO_AUTO, ALGO_BLOCK, ALGO_BNDM, ALGO_BRUTE, ALGO_FSBNDM, ALGO_HASHQ, ALGO_NAMES, ALGO_SBNDM,
                      ALGO_SHIFT_AND, SM_OK, SM_TRUNCATED, Opts, PlanInfo, Prof, SmError,
                      TuneEntry, check, last_error, load)

__all__ = ["pack_patterns", "find_all", "count", "find_all_async", "find_all_noalloc", "count_async", "workspace_size", "plan_query",
           "Corpus", "opts", "prof_enable", "prof_collect", "tune_get", "tune_set", "SmError", "ALGO_AUTO",
           "ALGO_SHIFT_AND", "ALGO_BNDM", "ALGO_SBNDM", "ALGO_HASHQ", "ALGO_BLOCK", "ALGO_BRUTE", "ALGO_FSBNDM", "ALGO_NAMES", "version",
           "Batch", "Server", "batch_set_wave_bytes", "batch_set_write_policy", "now_ns", "workspace_size_upto"]


def version() -> str:
    return load().sm_version().decode()


def opts(algo: int = 0, lane_bytes: int = 0, q: int = 0, sigma_hint: int = 0,
         tiles_per_wg: int = 0, hbits: int = 0) -> Opts:
    o = Opts()
    o.algo, o.lane_bytes, o.q = algo, lane_bytes, q
    o.sigma_hint, o.tiles_per_wg, o.hbits = sigma_hint, tiles_per_wg, hbits
    return o


def _pat(pat) -> tuple[bytes, int]:
    if isinstance(pat, np.ndarray):
        pat = pat.astype(np.uint8, copy=False).tobytes()
    b = bytes(pat)
    return b, len(b)


def _pat_ptr(b: bytes):
    # a non-NULL pointer even for an empty pattern (m == 0 is rejected by the library)
    return ctypes.cast(ctypes.c_char_p(b if b else b"\0"), ctypes.c_void_p)


def _is_dev(t) -> bool:
    return hasattr(t, "is_cuda") and t.is_cuda


def _stream_ptr(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else stream)


def workspace_size(n: int, m: int, o: Opts | None = None) -> int:
    return int(load().sm_workspace_size(n, m, ctypes.byref(o) if o is not None else None))


def workspace_size_upto(n: int, m_max: int, o: Opts | None = None) -> int:
    """Bytes of a workspace that serves every pattern length 1..m_max under o."""
    return int(load().sm_workspace_size_upto(n, m_max, ctypes.byref(o) if o is not None else None))


def plan_query(pat, o: Opts | None = None) -> dict:
    b, m = _pat(pat)
    info = PlanInfo()
    check(load().sm_plan_query(_pat_ptr(b), m, ctypes.byref(o) if o is not None else None,
                               ctypes.byref(info)))
    return {"algo": ALGO_NAMES[info.algo], "lane_bytes": info.lane_bytes, "q": info.q,
            "hbits": info.hbits, "tiles_per_wg": info.tiles_per_wg, "suffix": info.suffix}


def find_all_async(text, pat, out, d_count, work, o: Opts | None = None, stream=None) -> int:
    """Enqueue a search; total -> d_count[0], first len(out) positions -> out. No sync."""
    b, m = _pat(pat)
    return check(load().sm_find_all_async(
        ctypes.c_void_p(text.data_ptr()), text.numel(), _pat_ptr(b), m,
        ctypes.c_void_p(out.data_ptr() if out is not None and out.numel() else 0),
        out.numel() if out is not None else 0, ctypes.c_void_p(d_count.data_ptr()),
        ctypes.c_void_p(work.data_ptr()), work.numel(),
        ctypes.byref(o) if o is not None else None, _stream_ptr(stream)))


def find_all_noalloc(text, pat, out, d_count, o: Opts | None = None, stream=None) -> int:
    """As find_all_async, with the library's static device scratch as workspace (no
    allocation; calls on one device must not overlap in time)."""
    b, m = _pat(pat)
    return check(load().sm_find_all_noalloc(
        ctypes.c_void_p(text.data_ptr()), text.numel(), _pat_ptr(b), m,
        ctypes.c_void_p(out.data_ptr() if out is not None and out.numel() else 0),
        out.numel() if out is not None else 0, ctypes.c_void_p(d_count.data_ptr()),
        ctypes.byref(o) if o is not None else None, _stream_ptr(stream)))


def count_async(text, pat, d_count, work, o: Opts | None = None, stream=None) -> int:
    b, m = _pat(pat)
    return check(load().sm_count_async(
        ctypes.c_void_p(text.data_ptr()), text.numel(), _pat_ptr(b), m,
        ctypes.c_void_p(d_count.data_ptr()), ctypes.c_void_p(work.data_ptr()), work.numel(),
        ctypes.byref(o) if o is not None else None, _stream_ptr(stream)))


def count(text, pat, o: Opts | None = None, stream=None) -> int:
    """Number of occurrences of pat in text (a uint8 device tensor, or host bytes/ndarray)."""
    L = load()
    b, m = _pat(pat)
    c = ctypes.c_uint64(0)
    if _is_dev(text):
        if o is not None:
            import torch
            work = torch.empty(workspace_size(text.numel(), m, o), dtype=torch.uint8,
                               device=text.device)
            dc = torch.zeros(1, dtype=torch.int64, device=text.device)
            count_async(text, pat, dc, work, o, stream)
            return int(dc.item())
        check(L.sm_count_dev(ctypes.c_void_p(text.data_ptr()), text.numel(), _pat_ptr(b), m,
                             ctypes.byref(c), _stream_ptr(stream)))
        return int(c.value)
    t = np.ascontiguousarray(np.frombuffer(bytes(text), np.uint8) if not isinstance(
        text, np.ndarray) else text, dtype=np.uint8)
    check(L.sm_count(ctypes.c_void_p(t.ctypes.data if t.size else 0), t.size, _pat_ptr(b), m,
                     ctypes.byref(c)))
    return int(c.value)


def find_all(text, pat, cap: int | None = None, o: Opts | None = None, stream=None):
    """Sorted int64 occurrence positions.

    Device tensor in -> device tensor out (counted first, then written, unless cap
    is given). Host bytes/ndarray in -> numpy array out.
    """
    L = load()
    b, m = _pat(pat)
    if _is_dev(text):
        import torch
        n = text.numel()
        if o is not None:
            work = torch.empty(workspace_size(n, m, o), dtype=torch.uint8, device=text.device)
            dc = torch.zeros(1, dtype=torch.int64, device=text.device)
            if cap is None:
                count_async(text, pat, dc, work, o, stream)
                cap = int(dc.item())
            out = torch.empty(max(cap, 0), dtype=torch.int64, device=text.device)
            find_all_async(text, pat, out, dc, work, o, stream)
            total = int(dc.item())
            return out[:min(total, cap)]
        if cap is None:
            cap = count(text, pat, None, stream)
        out = torch.empty(max(cap, 0), dtype=torch.int64, device=text.device)
        c = ctypes.c_uint64(0)
        check(L.sm_find_all_dev(ctypes.c_void_p(text.data_ptr()), n, _pat_ptr(b), m,
                                ctypes.c_void_p(out.data_ptr() if cap else 0), cap, ctypes.byref(c),
                                _stream_ptr(stream)))
        return out[:min(int(c.value), cap)]
    t = np.ascontiguousarray(np.frombuffer(bytes(text), np.uint8) if not isinstance(
        text, np.ndarray) else text, dtype=np.uint8)
    if cap is None:
        cap = count(t, pat)
    out = np.empty(max(cap, 1), dtype=np.int64)
    c = ctypes.c_uint64(0)
    check(L.sm_find_all(ctypes.c_void_p(t.ctypes.data if t.size else 0), t.size, _pat_ptr(b), m,
                        ctypes.c_void_p(out.ctypes.data), cap, ctypes.byref(c)))
    return out[:min(int(c.value), cap)]


def pack_patterns(patterns) -> tuple[np.ndarray, np.ndarray]:
    """Concatenate patterns: (bytes as uint8 array, offsets as uint64 array of P + 1)."""
    bs = [bytes(p) if not isinstance(p, np.ndarray) else p.astype(np.uint8).tobytes()
          for p in patterns]
    off = np.zeros(len(bs) + 1, dtype=np.uint64)
    off[1:] = np.cumsum([len(b) for b in bs])
    buf = np.frombuffer(b"".join(bs) + b"\0", dtype=np.uint8)
    return buf, off


def _vp(a):
    return ctypes.c_void_p(a.ctypes.data if isinstance(a, np.ndarray) else a.data_ptr())


class Corpus:
    """A device-resident text reused across queries (sm_corpus_*)."""

    def __init__(self, text):
        L = load()
        self._h = ctypes.c_void_p(0)
        self._keep = None
        if _is_dev(text):
            self._keep = text  # borrowed: keep the tensor alive
            check(L.sm_corpus_open(ctypes.c_void_p(text.data_ptr()), text.numel(), 1,
                                   ctypes.byref(self._h)))
        else:
            t = np.ascontiguousarray(np.frombuffer(bytes(text), np.uint8) if not isinstance(
                text, np.ndarray) else text, dtype=np.uint8)
            check(L.sm_corpus_open(ctypes.c_void_p(t.ctypes.data if t.size else 0), t.size, 0,
                                   ctypes.byref(self._h)))

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h:
            check(load().sm_corpus_close(self._h))
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def stats(self) -> tuple[np.ndarray, int, float]:
        """(byte histogram, distinct bytes, effective alphabet size 1/sum p^2)"""
        h = np.zeros(256, dtype=np.uint64)
        s = ctypes.c_int32(0)
        se = ctypes.c_double(0)
        check(load().sm_corpus_stats(self._h, ctypes.c_void_p(h.ctypes.data), ctypes.byref(s),
                                     ctypes.byref(se)))
        return h, int(s.value), float(se.value)

    def find_all_async(self, pat, out, d_count, work, o: Opts | None = None, stream=None) -> int:
        b, m = _pat(pat)
        return check(load().sm_corpus_find_all_async(
            self._h, _pat_ptr(b), m,
            ctypes.c_void_p(out.data_ptr() if out is not None and out.numel() else 0),
            out.numel() if out is not None else 0, ctypes.c_void_p(d_count.data_ptr()),
            ctypes.c_void_p(work.data_ptr()), work.numel(),
            ctypes.byref(o) if o is not None else None, _stream_ptr(stream)))

    def count_async(self, pat, d_count, work, o: Opts | None = None, stream=None) -> int:
        b, m = _pat(pat)
        return check(load().sm_corpus_count_async(
            self._h, _pat_ptr(b), m, ctypes.c_void_p(d_count.data_ptr()),
            ctypes.c_void_p(work.data_ptr()), work.numel(),
            ctypes.byref(o) if o is not None else None, _stream_ptr(stream)))

    # ---- batched search (sm_batch_*) --------------------------------------
    def batch_workspace_size(self, patterns) -> int:
        buf, off = pack_patterns(patterns)
        return int(load().sm_batch_workspace_size(self._h, _vp(buf), _vp(off), len(off) - 1))

    def batch_count(self, patterns) -> np.ndarray:
        """Occurrence counts of every pattern (uint64 array, host)."""
        buf, off = pack_patterns(patterns)
        out = np.zeros(max(len(off) - 1, 1), dtype=np.uint64)
        check(load().sm_batch_count(self._h, _vp(buf), _vp(off), len(off) - 1, _vp(out)))
        return out[:len(off) - 1]

    def batch_find_all(self, patterns, cap: int | None = None):
        """(positions int64, offsets uint64 of P + 1): pattern i's occurrences are
        positions[offsets[i]:offsets[i+1]] (entries past cap are not written)."""
        buf, off = pack_patterns(patterns)
        P = len(off) - 1
        if cap is None:
            cap = int(self.batch_count(patterns).sum())
        out = np.empty(max(cap, 1), dtype=np.int64)
        oo = np.zeros(P + 1, dtype=np.uint64)
        check(load().sm_batch_find_all(self._h, _vp(buf), _vp(off), P, _vp(out), cap, _vp(oo)))
        return out[:min(cap, int(oo[P]))], oo

    def batch_count_async(self, patterns, d_counts, work, stream=None) -> int:
        buf, off = pack_patterns(patterns)
        return check(load().sm_batch_count_async(self._h, _vp(buf), _vp(off), len(off) - 1,
                                                 _vp(d_counts), _vp(work), work.numel(),
                                                 _stream_ptr(stream)))

    def batch_find_all_async(self, patterns, d_out, d_out_off, work, stream=None) -> int:
        buf, off = pack_patterns(patterns)
        return check(load().sm_batch_find_all_async(
            self._h, _vp(buf), _vp(off), len(off) - 1,
            ctypes.c_void_p(d_out.data_ptr() if d_out is not None and d_out.numel() else 0),
            d_out.numel() if d_out is not None else 0, _vp(d_out_off), _vp(work), work.numel(),
            _stream_ptr(stream)))

    def batch_open(self, patterns) -> "Batch":
        """Count step of a batched find_all, kept for windowed writes (sm_batch_open)."""
        return Batch(self, patterns)

    def count(self, pat) -> int:
        b, m = _pat(pat)
        c = ctypes.c_uint64(0)
        check(load().sm_corpus_count(self._h, _pat_ptr(b), m, ctypes.byref(c)))
        return int(c.value)

    def find_all(self, pat, cap: int | None = None) -> np.ndarray:
        b, m = _pat(pat)
        if cap is None:
            cap = self.count(pat)
        out = np.empty(max(cap, 1), dtype=np.int64)
        c = ctypes.c_uint64(0)
        check(load().sm_corpus_find_all(self._h, _pat_ptr(b), m, ctypes.c_void_p(out.ctypes.data),
                                        cap, ctypes.byref(c)))
        return out[:min(int(c.value), cap)]


class Batch:
    """Counted batch whose CSR output is written in windows (sm_batch_*)."""

    def __init__(self, corpus: Corpus, patterns):
        buf, off = pack_patterns(patterns)
        self.P = len(off) - 1
        self._corpus = corpus  # the corpus must outlive the batch
        self._h = ctypes.c_void_p(0)
        check(load().sm_batch_open(corpus.handle, _vp(buf), _vp(off), self.P, ctypes.byref(self._h)))
        self.offsets = np.zeros(self.P + 1, dtype=np.uint64)
        check(load().sm_batch_offsets(self._h, _vp(self.offsets)))
        self.total = int(self.offsets[-1])

    def write_async(self, lo: int, hi: int, d_out, stream=None) -> int:
        """CSR entries [lo, hi) -> d_out[0:hi-lo] (device tensor), enqueued on stream."""
        return check(load().sm_batch_write_async(
            self._h, lo, hi, ctypes.c_void_p(d_out.data_ptr() if hi > lo else 0), _stream_ptr(stream)))

    def close(self):
        if self._h:
            check(load().sm_batch_close(self._h))
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch_set_wave_bytes(nbytes: int) -> None:
    """Output-wave budget of the synchronous batched find_all (0 = default 16 GiB)."""
    check(load().sm_batch_set_wave_bytes(nbytes))


def batch_set_write_policy(policy: int) -> None:
    """Batched write pass: 0 automatic, 1 each pattern's own scanner, 2 shared filter
    whenever the pattern is sparse enough, 3 the single-pattern pipeline for every
    pattern of at most 64 bytes (speed only; results are identical)."""
    check(load().sm_batch_set_write_policy(policy))


def now_ns() -> int:
    """The server's clock (CLOCK_MONOTONIC, ns)."""
    return int(load().sm_now_ns())


class Server:
    """Continuous-batching query server over resident corpora (sm_server_*).

    submit() queues a query and returns a ticket; wait(ticket) returns
    (count, positions as a numpy view of library memory, result fields); the view
    is valid until free(ticket) (result() copies and frees in one call)."""

    def __init__(self, pool_bytes: int = 0, host_bytes: int = 0, max_batch: int = 0, slots: int = 0,
                 max_pending: int = 0, graphs: bool = True):
        from ._native import ServerConfig
        cfg = ServerConfig()
        cfg.pool_bytes, cfg.host_bytes, cfg.max_batch = pool_bytes, host_bytes, max_batch
        cfg.slots, cfg.max_pending = slots, max_pending
        cfg.graphs_off = 0 if graphs else 1
        self._h = ctypes.c_void_p(0)
        self._corpora = []
        check(load().sm_server_create(ctypes.byref(cfg), ctypes.byref(self._h)))

    def add_corpus(self, corpus: Corpus) -> int:
        cid = ctypes.c_uint32(0)
        check(load().sm_server_add_corpus(self._h, corpus.handle, ctypes.byref(cid)))
        self._corpora.append(corpus)  # kept open while the server runs
        return int(cid.value)

    def submit(self, corpus_id: int, pat, arrival_ns: int = 0) -> int:
        b, m = _pat(pat)
        t = ctypes.c_uint64(0)
        check(load().sm_server_submit(self._h, corpus_id, _pat_ptr(b), m, arrival_ns, ctypes.byref(t)))
        return int(t.value)

    def wait(self, ticket: int, timeout_us: int = -1):
        """(count, positions view or None if still running, fields dict)."""
        from ._native import Result
        r = Result()
        st = load().sm_server_wait(self._h, ticket, timeout_us, ctypes.byref(r))
        if st == -4 and r.done_ns == 0:  # SM_EBUSY: still running
            return None
        check(st)
        pos = (np.ctypeslib.as_array(r.positions, shape=(r.count,)) if r.count
               else np.empty(0, dtype=np.int64))
        return int(r.count), pos, {"arrival_ns": r.arrival_ns, "start_ns": r.start_ns,
                                   "done_ns": r.done_ns, "batch_size": r.batch_size,
                                   "corpus": r.corpus}

    def free(self, ticket: int) -> None:
        check(load().sm_result_free(self._h, ticket))

    def result(self, ticket: int) -> np.ndarray:
        """Wait, copy the positions out and free the result."""
        _, pos, _ = self.wait(ticket)
        out = pos.copy()
        self.free(ticket)
        return out

    def stats(self) -> dict:
        from ._native import ServerMetrics
        s = ServerMetrics()
        check(load().sm_server_stats(self._h, ctypes.byref(s)))
        return {k: getattr(s, k) for k, _ in ServerMetrics._fields_}

    def reset_stats(self) -> None:
        check(load().sm_server_reset_stats(self._h))

    def close(self):
        if self._h:
            check(load().sm_server_destroy(self._h))
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def tune_get() -> list[dict]:
    L = load()
    n = ctypes.c_uint32(0)
    check(L.sm_tune_get(None, 0, ctypes.byref(n)))
    arr = (TuneEntry * max(n.value, 1))()
    check(L.sm_tune_get(arr, n.value, ctypes.byref(n)))
    keys = [f[0] for f in TuneEntry._fields_ if f[0] != "reserved"]
    return [{k: getattr(arr[i], k) for k in keys} for i in range(n.value)]


def tune_set(entries: list[dict]) -> None:
    """Replace the planner's tuning table ([] restores the built-in table)."""
    arr = (TuneEntry * max(len(entries), 1))()
    for i, e in enumerate(entries):
        for k, v in e.items():
            if k in dict(TuneEntry._fields_):
                setattr(arr[i], k, int(v))
    check(load().sm_tune_set(arr, len(entries)))


def prof_enable(on: bool = True, every: int = 1) -> None:
    """Record kernel times of every `every`-th call from now on (off when on is False)."""
    check(load().sm_prof_enable(every if on else 0))


def prof_collect() -> dict:
    p = Prof()
    check(load().sm_prof_collect(ctypes.byref(p)))
    return {"calls": p.calls, "count_ms": p.count_ms, "emit_ms": p.emit_ms,
            "total_ms": p.total_ms, "text_bytes": p.text_bytes,
            "sampled_calls": p.sampled_calls, "sampled_count_ms": p.sampled_count_ms,
            "batch_calls": p.batch_calls, "batch_ms": p.batch_ms,
            "filter_launches": p.filter_launches, "filter_ms": p.filter_ms,
            "filter_pattern_bytes": p.filter_pattern_bytes}
