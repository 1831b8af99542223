"""C ABI contract checks that need no GPU: exports, validation, planner.

Every call here returns before any device work (argument errors, m > n, n == 0,
planner introspection), so these run on a machine without a GPU.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    from paper_1012_2547_amd import _native
    if not os.path.exists(_native.LIB_PATH):
        from paper_1012_2547_amd import build
        build.build()
    return _native.load()


def header_functions():
    names = set()
    for h in os.listdir(os.path.join(ROOT, "include")):
        if h.endswith(".h"):
            src = open(os.path.join(ROOT, "include", h)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"\b(sm_[a-z0-9_]+)\s*\(", src))
    return sorted(names)


def test_every_declared_symbol_is_exported(L):
    names = header_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L, n), n


def test_binding_declares_every_header_function():
    from paper_1012_2547_amd import _native
    assert set(header_functions()) <= set(_native.PROTOTYPES)


def test_version(L):
    assert b"gfx950" in L.sm_version()


def _u64():
    return ctypes.c_uint64(12345)


def test_validation_errors(L):
    from paper_1012_2547_amd._native import SM_EINVAL, SM_OK
    t = ctypes.create_string_buffer(b"abcabc")
    p = ctypes.create_string_buffer(b"bc")
    c = _u64()
    # m == 0
    assert L.sm_count(t, 6, p, 0, ctypes.byref(c)) == SM_EINVAL
    assert b"m = 0" in L.sm_last_error()
    # NULL pattern
    assert L.sm_count(t, 6, None, 2, ctypes.byref(c)) == SM_EINVAL
    # NULL text with n > 0
    assert L.sm_count(None, 6, p, 2, ctypes.byref(c)) == SM_EINVAL
    # NULL count
    assert L.sm_count(t, 6, p, 2, None) == SM_EINVAL
    # NULL output with cap > 0
    assert L.sm_find_all(t, 6, p, 2, None, 5, ctypes.byref(c)) == SM_EINVAL
    assert L.sm_find_all_dev(t, 6, p, 2, None, 5, ctypes.byref(c), None) == SM_EINVAL
    # m too large for the ABI
    assert L.sm_count(t, 6, p, 1 << 33, ctypes.byref(c)) == SM_EINVAL


def test_degenerate_sizes_return_zero_without_device(L):
    from paper_1012_2547_amd._native import SM_OK
    t = ctypes.create_string_buffer(b"abc")
    p = ctypes.create_string_buffer(b"abcd")
    c = _u64()
    assert L.sm_count(t, 3, p, 4, ctypes.byref(c)) == SM_OK and c.value == 0      # m > n
    c = _u64()
    assert L.sm_count(None, 0, p, 1, ctypes.byref(c)) == SM_OK and c.value == 0   # n == 0
    c = _u64()
    assert L.sm_find_all(t, 3, p, 4, None, 0, ctypes.byref(c)) == SM_OK and c.value == 0
    c = _u64()
    assert L.sm_count_dev(t, 3, p, 4, ctypes.byref(c), None) == SM_OK and c.value == 0


def test_prof_enable_stride(L):
    from paper_1012_2547_amd._native import SM_EINVAL, SM_OK
    assert L.sm_prof_enable(-1) == SM_EINVAL
    for k in (0, 1, 8, 0):
        assert L.sm_prof_enable(k) == SM_OK


def test_batch_write_policy_range(L):
    from paper_1012_2547_amd._native import SM_EINVAL, SM_OK
    for v in (0, 1, 2, 3):
        assert L.sm_batch_set_write_policy(v) == SM_OK
    assert L.sm_batch_set_write_policy(4) == SM_EINVAL
    assert L.sm_batch_set_write_policy(-1) == SM_EINVAL
    assert L.sm_batch_set_write_policy(0) == SM_OK


def test_invalid_options(L):
    import paper_1012_2547_amd as sm
    with pytest.raises(sm.SmError):
        sm.plan_query(b"a" * 65, sm.opts(algo=sm.ALGO_BNDM))        # BNDM needs m <= 64
    with pytest.raises(sm.SmError):
        sm.plan_query(b"abc", sm.opts(algo=sm.ALGO_HASHQ, q=4))       # q > m
    with pytest.raises(sm.SmError):
        sm.plan_query(b"abc", sm.opts(lane_bytes=48))
    with pytest.raises(sm.SmError):
        sm.plan_query(b"abc", sm.opts(algo=9))
    with pytest.raises(sm.SmError):
        sm.plan_query(b"a" * 100, sm.opts(algo=sm.ALGO_HASHQ, hbits=20))
    with pytest.raises(sm.SmError):
        sm.plan_query(b"a" * 64, sm.opts(algo=sm.ALGO_FSBNDM))      # FSBNDM needs m <= 63
    with pytest.raises(sm.SmError):
        sm.plan_query(b"a" * 30, sm.opts(algo=sm.ALGO_BNDM, q=8))   # BNDMq: q in {1, 2, 4}
    with pytest.raises(sm.SmError):
        sm.plan_query(b"a" * 143, sm.opts(algo=sm.ALGO_BLOCK))      # block filter: 144 <= m


def test_long_pattern_scanner_plans(L):
    """SBNDM takes any m (its factor form beyond 64 bytes), with every q; FSBNDM up to 63;
    BNDM up to 64 with q = 2 or 4."""
    import paper_1012_2547_amd as sm
    for m in (65, 100, 1000, 5000):
        for q in (0, 2, 4, 8):
            p = sm.plan_query(bytes(range(4)) * (m // 4) + bytes(m % 4), sm.opts(algo=sm.ALGO_SBNDM, q=q))
            assert p["algo"] == "sbndm" and (p["q"] == q if q > 1 else p["q"] in (0, 2, 4, 8)), (m, q)
    assert sm.plan_query(b"x" * 63, sm.opts(algo=sm.ALGO_FSBNDM))["algo"] == "fsbndm"
    for q in (2, 4):
        assert sm.plan_query(b"x" * 64, sm.opts(algo=sm.ALGO_BNDM, q=q))["q"] == q


def test_block_filter_workspace(L):
    """The block filter's tiles of 256 sampled blocks (a 16-byte multiple of starts each)
    may begin up to 15 starts before the text: the planner's workspace (auto) covers the
    forced block filter's at every length of its range, and both grow with n."""
    import paper_1012_2547_amd as sm
    blk = sm.opts(algo=sm.ALGO_BLOCK)
    for n in (144, 145, 4096, 32768 + 15, 1 << 20, (1 << 20) + 7):
        for m in (144, 145, 159, 160, 175, 176, 1000, 4096):
            if m > n:
                continue
            fb = sm.workspace_size(n, m, blk)
            assert fb > 0 and sm.workspace_size(n, m) >= fb, (n, m)
            assert sm.workspace_size(n + (1 << 20), m, blk) >= fb, (n, m)


def test_workspace_covers_table_shift_and_beyond_64(L):
    """Shift-And keeps hit bitmaps at any m (its suffix form beyond 49): where the tuning
    table picks it for m > 64, the planner's workspace under that alphabet hint covers the
    forced configuration's, at both ends of the entry's length range."""
    import paper_1012_2547_amd as sm
    n = (1 << 20) + 7
    seen = 0
    for e in sm.tune_get():
        if e["algo"] != sm.ALGO_SHIFT_AND or e["m_hi"] <= 64:
            continue
        sigma = min(e["sigma_hi"], 256)
        for m in {max(e["m_lo"], 65), min(e["m_hi"], 4000)}:
            forced = sm.opts(algo=sm.ALGO_SHIFT_AND, lane_bytes=e["lane_bytes"],
                             tiles_per_wg=e["tiles_per_wg"], sigma_hint=sigma)
            assert sm.workspace_size(n, m, sm.opts(sigma_hint=sigma)) >= sm.workspace_size(n, m, forced), (e, m)
            seen += 1
    # the same with a table that puts Shift-And at every length of one alphabet bucket
    try:
        sm.tune_set([dict(sigma_lo=3, sigma_hi=7, m_lo=1, m_hi=0xFFFFFFFF, algo=sm.ALGO_SHIFT_AND,
                          lane_bytes=32, q=0, tiles_per_wg=1, hbits=0)])
        forced = sm.opts(algo=sm.ALGO_SHIFT_AND, lane_bytes=32, tiles_per_wg=1, sigma_hint=4)
        for m in (65, 100, 1000, 5000):
            assert sm.workspace_size(n, m, sm.opts(sigma_hint=4)) >= sm.workspace_size(n, m, forced), m
            assert sm.plan_query(bytes(range(4)) * (m // 4 + 1), sm.opts(sigma_hint=4))["algo"] == "shift_and"
    finally:
        sm.tune_set([])  # the built-in table again


def test_shift_and_suffix_by_period(L):
    """Shift-And beyond m = 49 scans the pattern's last 17 bytes, or its last 49 when the
    pattern's smallest period lies in 18..49 (a start one period after an occurrence is
    then still taken without reading); shorter patterns have no suffix form; beyond
    2^24 bytes the pattern is not searched for a period and keeps 49."""
    import numpy as np
    import paper_1012_2547_amd as sm
    sa = sm.opts(algo=sm.ALGO_SHIFT_AND)
    rng = np.random.default_rng(5)
    for P, want in ((1, 17), (5, 17), (17, 17), (18, 49), (30, 49), (49, 49), (50, 17), (64, 17)):
        unit = rng.integers(0, 4, P, dtype=np.uint8)
        unit[0] = 7  # no smaller period
        for m in (50, 64, 300):
            p = bytes(np.tile(unit, m // P + 1)[:m])
            assert sm.plan_query(p, sa)["suffix"] == want, (P, m)
    assert sm.plan_query(bytes(range(200)), sa)["suffix"] == 17   # aperiodic
    assert sm.plan_query(b"ab" * 24, sa)["suffix"] == 0            # m = 48: no suffix form
    assert sm.plan_query(bytes(40), sm.opts(algo=sm.ALGO_SBNDM))["suffix"] == 0
    assert sm.plan_query(bytes((1 << 24) + 1), sa)["suffix"] == 49  # too long to look


def test_planner_choices(L):
    import paper_1012_2547_amd as sm
    assert sm.plan_query(b"ab")["algo"] in ("shift_and", "bndm", "sbndm")
    hq = sm.opts(algo=sm.ALGO_HASHQ)
    p = sm.plan_query(bytes(range(4)) * 64, hq)   # m = 256 over 4 symbols
    assert p["algo"] == "hashq" and 2 <= p["q"] <= 16 and 8 <= p["hbits"] <= 13
    p2 = sm.plan_query(bytes(range(256)) * 2, hq)  # m = 512 over 256 symbols: short grams suffice
    assert p2["q"] < p["q"]
    # long patterns: the block filter, one block per m - 15 starts; not on one symbol
    b = sm.plan_query(bytes(range(4)) * 64)
    assert b["algo"] == "block" and b["lane_bytes"] == 240  # 16-byte multiple <= m - 15
    assert sm.plan_query(b"a" * 300)["algo"] != "block"
    assert sm.plan_query(bytes(range(4)) * 25)["algo"] != "block"  # m = 100 < 144
    f = sm.plan_query(b"x" * 30, sm.opts(algo=sm.ALGO_BNDM, lane_bytes=32))
    assert f["algo"] == "bndm" and f["lane_bytes"] == 32


def test_one_symbol_texts_plan_shift_and(L):
    """On a text of (nearly) one symbol (sigma 1) the planner takes Shift-And (for m > 64 its
    suffix form), whatever the table says for sigma <= 2: skip algorithms degrade to O(nm)
    there."""
    import paper_1012_2547_amd as sm
    for p in (b"a" * 63 + b"b", b"a" * 40, b"ab" * 16):
        assert sm.plan_query(p, sm.opts(sigma_hint=1))["algo"] == "shift_and", p[:4]
        assert sm.plan_query(p, sm.opts(sigma_hint=2))["algo"] != "shift_and" or len(p) < 32
    assert sm.plan_query(b"a" * 64)["algo"] == "shift_and"      # sigma estimated from the pattern: 1
    assert sm.plan_query(b"a" * 200, sm.opts(sigma_hint=1))["algo"] == "shift_and"  # suffix form
    assert sm.plan_query(b"ab" * 100, sm.opts(sigma_hint=2))["algo"] != "shift_and"
    f = sm.plan_query(b"a" * 50, sm.opts(algo=sm.ALGO_BNDM, sigma_hint=1))
    assert f["algo"] == "bndm"                                   # explicit choices are kept


def test_workspace_size_monotone(L):
    import paper_1012_2547_amd as sm
    a = sm.workspace_size(1 << 20, 8)
    b = sm.workspace_size(1 << 30, 8)
    assert 0 < a < b
    assert sm.workspace_size(10, 20) > 0


def test_workspace_size_upto_covers_every_length(L):
    """A shared workspace: at least the size of every length up to M, with the planner's
    lanes from the built-in table and from a table whose narrowest lane sits at an
    interior length (and, past the block filter's range, at long lengths)."""
    import paper_1012_2547_amd as sm
    tables = [None,
              [dict(sigma_lo=1, sigma_hi=256, m_lo=1, m_hi=8, algo=1, lane_bytes=128),
               dict(sigma_lo=1, sigma_hi=256, m_lo=9, m_hi=11, algo=3, lane_bytes=16),
               dict(sigma_lo=1, sigma_hi=256, m_lo=12, m_hi=6000, algo=4, lane_bytes=128),
               dict(sigma_lo=1, sigma_hi=256, m_lo=6001, m_hi=7000, algo=4, lane_bytes=32),
               dict(sigma_lo=1, sigma_hi=256, m_lo=7001, m_hi=0xFFFFFFFF, algo=4, lane_bytes=128)]]
    try:
        for tab in tables:
            if tab is not None:
                sm.tune_set(tab)
            for n in (5000, 1 << 20):
                for M in (1, 9, 64, 300, 4097, 9000):
                    got = sm.workspace_size_upto(n, M)
                    each = max(sm.workspace_size(n, m) for m in range(1, M + 1))
                    assert got >= each, (n, M)
                    if M <= 4097:
                        assert got == each, (n, M)
            o = sm.opts(lane_bytes=64)
            assert sm.workspace_size_upto(1 << 20, 100, o) == max(
                sm.workspace_size(1 << 20, m, o) for m in range(1, 101))
    finally:
        sm.tune_set([])
    assert sm.workspace_size_upto(1 << 20, 0) == 0


def test_tuning_table_roundtrip(L):
    import paper_1012_2547_amd as sm
    base = sm.tune_get()
    assert len(base) > 50
    assert all(1 <= e["algo"] <= 7 and e["m_lo"] <= e["m_hi"] for e in base)
    # every (sigma, m) of the sweep grid is covered by some entry
    for s in (2, 4, 16, 64, 256):
        for m in (1, 2, 3, 5, 8, 63, 64, 65, 100, 1000, 5000):
            assert any(e["sigma_lo"] <= s <= e["sigma_hi"] and e["m_lo"] <= m <= e["m_hi"]
                       for e in base), (s, m)
    custom = [dict(sigma_lo=1, sigma_hi=256, m_lo=1, m_hi=64, algo=3, lane_bytes=32)]
    sm.tune_set(custom)
    try:
        assert sm.plan_query(b"abcdefgh")["algo"] == "sbndm"
        assert sm.plan_query(b"abcdefgh")["lane_bytes"] == 32
        assert sm.plan_query(bytes(range(100)))["algo"] == "hashq"  # no entry: heuristic
    finally:
        sm.tune_set([])
    assert sm.tune_get() == base
    with pytest.raises(sm.SmError):
        sm.tune_set([dict(sigma_lo=1, sigma_hi=2, m_lo=5, m_hi=1, algo=1)])
    with pytest.raises(sm.SmError):
        sm.tune_set([dict(sigma_lo=1, sigma_hi=2, m_lo=1, m_hi=5, algo=8)])


def test_sigma_estimate_from_pattern_steers_plan(L):
    import paper_1012_2547_amd as sm
    # a 150-byte pattern over 2 symbols plans long q-grams; over 150 symbols the table
    # entry of the largest alphabet bucket applies instead
    lo = sm.plan_query(bytes([0, 1]) * 75)
    hi = sm.plan_query(bytes(range(150)))
    assert lo["algo"] == "hashq" and lo["q"] >= 8
    assert (hi["algo"], hi["q"]) != (lo["algo"], lo["q"])
    assert sm.plan_query(bytes(range(150)), sm.opts(sigma_hint=2)) == lo
