"""GPU parity: every scan kernel, forced in turn, against the CPU oracle (bit-exact).

Occurrence lists are integer data, so the bar is exact equality of the sorted
int64 position lists (and of the totals).
"""
import numpy as np
import pytest

import datagen as dg
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def sm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1012_2547_amd as sm
    sm.version()  # fails loudly when libsm.so is missing
    return sm


DEV = "cuda:0"
BP_ALGOS = (1, 2, 3)          # Shift-And, BNDM, SBNDM (beyond m = 64: suffix / factor forms)
ALL_ALGOS = (1, 2, 3, 4, 5, 6, 7)  # + Hash-q, block filter (144 <= m <= 4096), brute force (m <= 8),
                                   # FSBNDM (m <= 63)


def gpu_find(sm, text_t, pat, algo=0, lane=0, q=0, cap=None, tpw=0, sigma_hint=0):
    o = sm.opts(algo=algo, lane_bytes=lane, q=q, tiles_per_wg=tpw, sigma_hint=sigma_hint)
    n, m = text_t.numel(), len(pat)
    work = torch.empty(max(sm.workspace_size(n, m, o), 256), dtype=torch.uint8, device=DEV)
    dc = torch.zeros(1, dtype=torch.int64, device=DEV)
    sm.count_async(text_t, pat, dc, work, o)
    total_c = int(dc.item())
    if cap is None:
        cap = total_c
    out = torch.full((max(cap, 1),), -7, dtype=torch.int64, device=DEV)
    sm.find_all_async(text_t, pat, out[:cap], dc, work, o)
    total = int(dc.item())
    assert total == total_c
    res = out[:min(total, cap)].cpu().numpy()
    # nothing written past min(total, cap)
    assert np.all(out[min(total, cap):].cpu().numpy() == -7)
    return res, total


def applicable(algo, m, q=0):
    if algo == 2:
        return m <= 64
    if algo in BP_ALGOS:  # Shift-And and SBNDM take any m
        return True
    if algo == 5:
        return 144 <= m <= 4096
    if algo == 6:
        return m <= 8
    if algo == 7:
        return m <= 63
    return m >= max(q, 1)


def check_case(sm, t_np, t_dev, pat, algos=ALL_ALGOS, lanes=(64,)):
    want = oracle.find_all(t_np, pat)
    for a in algos:
        if not applicable(a, len(pat)):
            continue
        for L in lanes:
            got, tot = gpu_find(sm, t_dev, pat, algo=a, lane=L)
            assert tot == want.size, (a, L, len(pat), tot, want.size)
            assert np.array_equal(got, want), (a, L, len(pat))


M_SET = (1, 2, 3, 4, 5, 7, 8, 9, 15, 16, 17, 18, 31, 32, 33, 48, 49, 50, 61, 62, 63, 64)
M_LONG = (65, 100, 128, 255, 256, 513, 1024)


@pytest.mark.parametrize("sigma", [2, 4, 16, 256])
def test_grid_all_algorithms(sm, sigma):
    n = 50_000 + 37  # several tiles at L=16, ragged tail
    t_np = dg.uniform_text(n, sigma, seed=100 + sigma)
    t_dev = torch.from_numpy(t_np).to(DEV)
    for i, m in enumerate(M_SET + M_LONG):
        p_sub, _ = dg.substring_pattern(t_np, m, seed=5, idx=i)
        check_case(sm, t_np, t_dev, p_sub, lanes=(16, 64))
        if m <= 8:
            check_case(sm, t_np, t_dev, dg.random_pattern(m, sigma, seed=6, idx=i), lanes=(32,))


def test_hashq_every_q(sm):
    n = 40_000
    for sigma in (2, 4, 64):
        t_np = dg.uniform_text(n, sigma, seed=3)
        t_dev = torch.from_numpy(t_np).to(DEV)
        for m in (16, 17, 70, 300):
            p, _ = dg.substring_pattern(t_np, m, seed=9, idx=m)
            want = oracle.find_all(t_np, p)
            for q in range(1, 17):
                if q > m:
                    continue
                for L in (16, 128):
                    got, tot = gpu_find(sm, t_dev, p, algo=4, lane=L, q=q)
                    assert np.array_equal(got, want) and tot == want.size, (sigma, m, q, L)


def test_sbndm_every_q(sm):
    """The q-gram form of SBNDM (q = 2, 4, 8) on small and large alphabets, with
    periodic patterns and q = m."""
    n = 40_000
    for sigma in (2, 4, 64):
        t_np = dg.uniform_text(n, sigma, seed=13)
        t_dev = torch.from_numpy(t_np).to(DEV)
        pats = [dg.substring_pattern(t_np, m, seed=19, idx=m)[0] for m in (2, 4, 5, 8, 9, 31, 64)]
        pats += [b"\x01\x00" * 16, bytes(t_np[:8])]
        for p in pats:
            want = oracle.find_all(t_np, p)
            for q in (2, 4, 8):
                if q > len(p):
                    continue
                for L, tpw in ((16, 1), (64, 2)):
                    got, tot = gpu_find(sm, t_dev, p, algo=3, lane=L, q=q, tpw=tpw)
                    assert np.array_equal(got, want) and tot == want.size, (sigma, len(p), q, L)
    with pytest.raises(sm.SmError):
        gpu_find(sm, t_dev, b"abcdefgh", algo=3, lane=64, q=3)


def test_sbndm_factor_form(sm):
    """SBNDM for m > 64, its factor form: the pattern's last 64 bytes searched over the
    text shifted by m - 64, the first m - 64 bytes of each start found verified. Every q,
    lanes of 16, 64 and 128 starts, lengths 65 .. 3100 (beyond 3072 the pattern reaches
    the preparation kernel through the workspace), occurrences at both text ends,
    patterns whose last 64 bytes occur without the rest, and periodic patterns with
    many overlapping occurrences (dense tiles, written by the emit pass's rescan)."""
    n = 60_000 + 11
    rng = np.random.default_rng(37)
    for sigma in (2, 4, 64):
        t_np = dg.uniform_text(n, sigma, seed=31 + sigma)
        t_dev = torch.from_numpy(t_np).to(DEV)
        pats = [dg.substring_pattern(t_np, m, seed=41, idx=m)[0]
                for m in (65, 66, 97, 128, 143, 200, 1100, 3100)]
        pats += [bytes(t_np[:70]), bytes(t_np[-129:])]
        for m in (80, 300):  # the factor occurs, the prefix does not
            sub = dg.substring_pattern(t_np, m, seed=43, idx=m)[0]
            pre = bytes((rng.integers(0, sigma, m - 64) + 1) % 256)
            pats.append(pre + sub[-64:])
        for p in pats:
            want = oracle.find_all(t_np, p)
            for q in (1, 2, 4, 8):
                for L, tpw in ((16, 1), (64, 2), (128, 1)):
                    got, tot = gpu_find(sm, t_dev, p, algo=3, lane=L, q=q, tpw=tpw)
                    assert np.array_equal(got, want) and tot == want.size, (sigma, len(p), q, L)
    # periodic text and patterns: every second (third) start an occurrence
    for unit, reps, tail in ((b"ab", 40, b""), (b"ab", 60, b"a"), (b"abc", 43, b"ab")):
        t_np = np.frombuffer(unit * (n // len(unit)), dtype=np.uint8).copy()
        t_np[5000:5003] = ord("z")  # one break in the period
        t_dev = torch.from_numpy(t_np).to(DEV)
        p = unit * reps + tail
        want = oracle.find_all(t_np, p)
        assert want.size > 10_000
        for q in (1, 8):
            for L in (16, 128):
                got, tot = gpu_find(sm, t_dev, p, algo=3, lane=L, q=q)
                assert np.array_equal(got, want) and tot == want.size, (len(p), q, L)


def test_bndm_q_and_fsbndm(sm):
    """BNDMq (the window's last q = 2 or 4 bytes read at once; shifts capped at m - q + 1)
    and FSBNDM (the byte after the window read first as a look-ahead) on small and large
    alphabets, with periodic patterns, q = m, occurrences at both text ends (the last
    windows have no look-ahead byte) and lanes of 16 and 64 starts."""
    n = 40_000 + 13
    for sigma in (2, 4, 64):
        t_np = dg.uniform_text(n, sigma, seed=23)
        t_dev = torch.from_numpy(t_np).to(DEV)
        pats = [dg.substring_pattern(t_np, m, seed=29, idx=m)[0] for m in (2, 3, 4, 5, 8, 9, 17, 31, 50, 63, 64)]
        pats += [b"\x01\x00" * 16, bytes(t_np[:8]), bytes(t_np[-12:]), bytes(t_np[-63:]), bytes(t_np[:2])]
        for p in pats:
            want = oracle.find_all(t_np, p)
            for L, tpw in ((16, 1), (64, 2)):
                for q in (2, 4):
                    if q > len(p):
                        continue
                    got, tot = gpu_find(sm, t_dev, p, algo=2, lane=L, q=q, tpw=tpw)
                    assert np.array_equal(got, want) and tot == want.size, ("bndm", sigma, len(p), q, L)
                if len(p) <= 63:
                    got, tot = gpu_find(sm, t_dev, p, algo=7, lane=L, tpw=tpw)
                    assert np.array_equal(got, want) and tot == want.size, ("fsbndm", sigma, len(p), L)
    # texts of one symbol: every window matches up to its end
    a_n = np.full(5000, 7, dtype=np.uint8)
    a_dev = torch.from_numpy(a_n).to(DEV)
    for m in (2, 5, 33, 63):
        want = oracle.find_all(a_n, bytes([7]) * m)
        for a, q in ((2, 2), (2, 4), (7, 0)):
            if q > m:
                continue
            got, tot = gpu_find(sm, a_dev, bytes([7]) * m, algo=a, lane=64, q=q)
            assert np.array_equal(got, want), (a, q, m)
    with pytest.raises(sm.SmError):
        gpu_find(sm, t_dev, b"abcdefgh", algo=2, lane=64, q=8)
    with pytest.raises(sm.SmError):
        gpu_find(sm, t_dev, bytes(64), algo=7, lane=64)


def test_block_filter(sm):
    """The block filter reads one aligned 16-byte block per S text bytes (S the largest
    multiple of 16 <= m - 15): every length from its smallest (144: a block per 128
    starts) to its largest (4096), lengths where S = m - 15 and where S = m - 30 (a
    block's bucket then holds alignments of the previous block's starts), every text
    alignment (the sampled blocks move with it), small and large alphabets, planted
    occurrences at both text ends, periodic patterns (the period rule), patterns
    whose blocks recur in the text without an occurrence, tiles per workgroup, and
    truncation. Out-of-range lengths are rejected."""
    rng = np.random.default_rng(21)
    for sigma in (2, 4, 256):
        n = 300_001
        t_np = dg.uniform_text(n, sigma, seed=40 + sigma)
        t_dev = torch.from_numpy(t_np).to(DEV)
        for i, m in enumerate((144, 145, 159, 160, 174, 175, 200, 255, 256, 257, 1000, 1024, 4096)):
            pats = [dg.substring_pattern(t_np, m, seed=41, idx=i)[0], bytes(t_np[:m]),
                    bytes(t_np[n - m:]), bytes(rng.integers(0, sigma, m, dtype=np.uint8))]
            for p in pats:
                want = oracle.find_all(t_np, p)
                for tpw in (1, 2, 3):
                    got, tot = gpu_find(sm, t_dev, p, algo=5, tpw=tpw)
                    assert tot == want.size and np.array_equal(got, want), (sigma, m, tpw)
    # every alignment of the text in memory: the blocks sampled differ with it
    base_np = dg.uniform_text(200_000 + 16, 4, seed=47)
    base = torch.from_numpy(base_np).to(DEV)
    for off in range(16):
        t_np = base_np[off:off + 200_000]
        t_dev = base[off:off + 200_000]
        for m in (144, 174, 175, 600):
            for p in (bytes(t_np[:m]), bytes(t_np[-m:]), bytes(t_np[777:777 + m])):
                want = oracle.find_all(t_np, p)
                got, tot = gpu_find(sm, t_dev, p, algo=5, tpw=1 + off % 3)
                assert tot == want.size and np.array_equal(got, want), (off, m)
    # periodic texts and patterns: many candidates per block, dense occurrences
    for per in (1, 2, 3, 7, 16, 17, 40, 64, 65):
        base = bytes(rng.integers(0, 4, per, dtype=np.uint8))
        t_np = np.frombuffer((base * (200_000 // per + 2))[:200_003], np.uint8).copy()
        t_dev = torch.from_numpy(t_np).to(DEV)
        for m in (144, 145, 300, 513):
            p = bytes(t_np[5:5 + m])
            want = oracle.find_all(t_np, p)
            got, tot = gpu_find(sm, t_dev, p, algo=5, tpw=2)
            assert tot == want.size and np.array_equal(got, want), (per, m)
            for cap in (1, want.size // 2):
                got, tot = gpu_find(sm, t_dev, p, algo=5, cap=cap)
                assert np.array_equal(got, want[:cap]), (per, m, cap)
    # a run of one byte with a different last byte: every block matches, no occurrence
    t_np = np.full(100_000, 7, np.uint8)
    t_np[77_777] = 9
    t_dev = torch.from_numpy(t_np).to(DEV)
    for m in (144, 200, 3000):
        p = bytes([7] * (m - 1) + [9])
        got, tot = gpu_find(sm, t_dev, p, algo=5)
        assert tot == 1 and got.tolist() == [77_777 - m + 1], m
    for m in (143, 4097):
        with pytest.raises(sm.SmError):
            gpu_find(sm, t_dev, bytes(m), algo=5)


def test_brute_force_packed(sm):
    """Brute force over packed bytes (m <= 8): every m, every lane width (the bitmap
    form from 32 starts per lane, rescans at 16), every text offset modulo 16,
    sparse and dense outputs, bytes 0x00, 0x7F, 0x80, 0xFF (edge cases of the
    zero-byte test), truncation."""
    rng = np.random.default_rng(31)
    base_np = rng.choice(np.array([0, 0x7F, 0x80, 0xFF], np.uint8), 70_000)
    base = torch.from_numpy(base_np).to(DEV)
    for off in (0, 1, 3, 7, 13):
        t_np = base_np[off:off + 60_001]
        t_dev = base[off:off + 60_001]
        for m in range(1, 9):
            for p in (bytes(t_np[101:101 + m]), bytes(t_np[-m:]), bytes([0x80] * m)):
                want = oracle.find_all(t_np, p)
                for L, tpw in ((16, 1), (32, 2), (64, 1), (128, 3)):
                    got, tot = gpu_find(sm, t_dev, p, algo=6, lane=L, tpw=tpw)
                    assert tot == want.size and np.array_equal(got, want), (off, m, L, tpw)
    for sigma in (2, 256):
        t_np = dg.uniform_text(200_003, sigma, seed=50 + sigma)
        t_dev = torch.from_numpy(t_np).to(DEV)
        for m in (1, 2, 5, 8):
            p, _ = dg.substring_pattern(t_np, m, seed=51, idx=m)
            want = oracle.find_all(t_np, p)
            got, tot = gpu_find(sm, t_dev, p, algo=6, lane=64)
            assert tot == want.size and np.array_equal(got, want), (sigma, m)
            for cap in (1, want.size // 2):
                got, tot = gpu_find(sm, t_dev, p, algo=6, lane=64, cap=cap)
                assert np.array_equal(got, want[:cap]), (sigma, m, cap)
    with pytest.raises(sm.SmError):
        gpu_find(sm, t_dev, bytes(9), algo=6)


def test_tiles_per_workgroup_and_lanes_deterministic(sm):
    t_np = dg.uniform_text(300_001, 4, seed=8)
    t_dev = torch.from_numpy(t_np).to(DEV)
    for m in (6, 20, 200):
        p, _ = dg.substring_pattern(t_np, m, seed=1, idx=m)
        want = oracle.find_all(t_np, p)
        for a in ALL_ALGOS:
            if not applicable(a, m):
                continue
            for L in (16, 32, 64, 128):
                for tpw in (1, 3, 8):
                    got, _ = gpu_find(sm, t_dev, p, algo=a, lane=L, tpw=tpw)
                    assert np.array_equal(got, want), (m, a, L, tpw)


def test_closed_form_dense_output(sm):
    n = (1 << 20) + 3
    t_dev = torch.full((n,), ord("a"), dtype=torch.uint8, device=DEV)
    for m in (1, 4, 16, 64, 256):
        for a in ALL_ALGOS:
            if not applicable(a, m):
                continue
            got, tot = gpu_find(sm, t_dev, b"a" * m, algo=a)
            assert tot == n - m + 1
            assert np.array_equal(got, np.arange(n - m + 1)), (m, a)


def test_closed_form_periodic(sm):
    P = 4096
    n = P * 300 + 17
    t_np = dg.periodic_text(n, ord("a"), ord("b"), P)
    t_dev = torch.from_numpy(t_np).to(DEV)
    for m in (4, 16, 64, 256, 1024):
        p = b"a" * (m - 1) + b"b"
        want = np.array([P * k + P - m for k in range(n // P)], dtype=np.int64)
        for a in ALL_ALGOS:
            if not applicable(a, m):
                continue
            got, tot = gpu_find(sm, t_dev, p, algo=a)
            assert np.array_equal(got, want), (m, a)


def test_truncation(sm):
    t_np = dg.uniform_text(100_000, 2, seed=4)
    t_dev = torch.from_numpy(t_np).to(DEV)
    p = bytes([0, 1, 0])
    want = oracle.find_all(t_np, p)
    assert want.size > 1000
    for a in ALL_ALGOS:
        if not applicable(a, len(p)):
            continue
        for cap in (0, 1, 77, want.size - 1, want.size, want.size + 5):
            got, tot = gpu_find(sm, t_dev, p, algo=a, cap=cap)
            assert tot == want.size
            assert np.array_equal(got, want[:cap]), (a, cap)


def test_dense_bitmap_form_mixed_tiles(sm):
    """Shift-And scans with lanes of >= 32 starts keep each lane's hits as a
    bitmap in the count pass; tiles with more hits than the stash holds leave it
    to the emit pass, which expands it, and the others fill their stash from it.
    A text of dense, sparse and empty regions of ragged lengths, every lane
    width, with truncation; at L = 16 the same searches take the rescanning
    paths (first-hit slots when planned sparse, sigma hint 256) and must agree."""
    parts = [np.zeros(9001, np.uint8), dg.uniform_text(70_003, 4, seed=31),
             np.zeros(5003, np.uint8), dg.uniform_text(40_009, 2, seed=32),
             np.full(33_331, 200, np.uint8), np.zeros(20_011, np.uint8),
             dg.uniform_text(31_999, 2, seed=33)]
    t_np = np.concatenate(parts)
    t_dev = torch.from_numpy(t_np).to(DEV)
    pats = [b"\0", b"\0\0", b"\0\0\0\0", b"\0\1", bytes([1, 0, 1, 1, 0]), b"\0" * 7]
    for p in pats:
        want = oracle.find_all(t_np, p)
        for L, tpw, hint in ((32, 1, 2), (64, 1, 2), (64, 3, 2), (128, 2, 2), (128, 1, 256),
                             (16, 1, 2), (16, 2, 256), (64, 2, 256)):
            got, tot = gpu_find(sm, t_dev, p, algo=1, lane=L, tpw=tpw, sigma_hint=hint)
            assert tot == want.size, (p, L, tpw, hint, tot, want.size)
            assert np.array_equal(got, want), (p, L, tpw, hint)
        for cap in (0, 3, want.size // 3, want.size - 1):
            got, tot = gpu_find(sm, t_dev, p, algo=1, lane=64, cap=cap, sigma_hint=2)
            assert tot == want.size and np.array_equal(got, want[:cap]), (p, cap)


def test_shift_and_whole_tiles_at_every_alignment(sm):
    """In whole tiles the Shift-And lanes run with wave-uniform unit bounds: the units
    whose 16 window ends all belong to the lane take every hit unmasked, the first and
    last ones mask their neighbours' ends. Where a lane's first start falls inside its
    16-byte unit follows from the text's device address, so every offset 0..15 is run,
    with dense and sparse hits, every state width (byte, 32-bit and 64-bit masks, checks
    every 16, 4 and 1 bytes) and lane width, in count and find mode, against the oracle."""
    base_np = np.concatenate([dg.uniform_text(60_000, 2, seed=41), np.zeros(7_001, np.uint8),
                              dg.uniform_text(60_000, 4, seed=42)])
    base = torch.from_numpy(base_np).to(DEV)
    for off in range(16):
        t_np = base_np[off:]
        t_dev = base[off:]  # device pointer offset by `off` bytes
        pats = [bytes(t_np[1000:1000 + m]) for m in (1, 3, 8, 9, 16, 17, 30, 49, 50, 57, 64)]
        pats += [bytes(m) for m in (1, 8, 17)]  # every start of the zero run
        for p in pats:
            want = oracle.find_all(t_np, p)
            for L, tpw in ((32, 1), (64, 1), (64, 2), (128, 1)):
                got, tot = gpu_find(sm, t_dev, p, algo=1, lane=L, tpw=tpw)
                assert tot == want.size and np.array_equal(got, want), (off, len(p), L, tpw)


def test_edges_and_alignment(sm):
    rng = np.random.default_rng(0)
    base_np = rng.integers(0, 3, 20_000, dtype=np.uint8)
    base = torch.from_numpy(base_np).to(DEV)
    for off in range(0, 16):
        for n in (1, 2, 15, 16, 17, 255, 4097, 19_000 - off):
            t_np = base_np[off:off + n]
            t_dev = base[off:off + n]  # device pointer offset by `off` bytes
            for m in (1, 2, 5, 16, 40, 64, 70):
                if m > n:
                    continue
                for p in (bytes(t_np[:m]), bytes(t_np[n - m:])):
                    want = oracle.find_all(t_np, p)
                    assert want[0] == 0 or p != bytes(t_np[:m])
                    for a in ALL_ALGOS:
                        if not applicable(a, m):
                            continue
                        got, _ = gpu_find(sm, t_dev, p, algo=a, lane=16)
                        assert np.array_equal(got, want), (off, n, m, a)


def test_zero_bytes_at_text_end(sm):
    """A pattern of 0x00 bytes must not match past the end of the text."""
    for n in (1000, 1024, 4096 * 4 + 5):
        t_np = np.ones(n, dtype=np.uint8)
        t_np[-3:] = 0
        t_dev = torch.from_numpy(t_np).to(DEV)
        for m in (1, 2, 3, 4, 8, 64, 100):
            want = oracle.find_all(t_np, bytes(m))
            for a in ALL_ALGOS:
                if not applicable(a, m):
                    continue
                got, tot = gpu_find(sm, t_dev, bytes(m), algo=a)
                assert np.array_equal(got, want), (n, m, a)


def test_m_equals_n_and_m_greater_than_n(sm):
    t_np = dg.uniform_text(64, 4, seed=2)
    t_dev = torch.from_numpy(t_np).to(DEV)
    for a in ALL_ALGOS:  # m = n = 64
        if not applicable(a, 64):
            continue
        got, tot = gpu_find(sm, t_dev, bytes(t_np), algo=a)
        assert got.tolist() == [0]
        got, tot = gpu_find(sm, t_dev, bytes(t_np[:63]) + b"\xff", algo=a)
        assert tot == 0
    got, tot = gpu_find(sm, t_dev, bytes(65))
    assert tot == 0
    t_np = dg.uniform_text(300, 4, seed=3)  # the block filter at m = n and m = n + 1
    t_dev = torch.from_numpy(t_np).to(DEV)
    got, tot = gpu_find(sm, t_dev, bytes(t_np), algo=5)
    assert got.tolist() == [0]
    got, tot = gpu_find(sm, t_dev, bytes(t_np[:299]) + b"\xff", algo=5)
    assert tot == 0
    o = sm.opts(algo=5)
    work = torch.empty(1 << 16, dtype=torch.uint8, device=DEV)
    dc = torch.zeros(1, dtype=torch.int64, device=DEV)
    sm.count_async(t_dev, bytes(t_np) + b"\x00", dc, work, o)
    assert int(dc.item()) == 0


def test_config1_exact(sm):
    """n = 2^20 uniform over 4 symbols (seed 1), m = 8 substring: full list."""
    t_np = dg.uniform_text(1 << 20, 4, seed=1)
    p, off = dg.substring_pattern(t_np, 8, seed=1, idx=0)
    t_dev = torch.from_numpy(t_np).to(DEV)
    want = oracle.find_all(t_np, p)
    assert off in want.tolist()
    got = sm.find_all(t_dev, p).cpu().numpy()
    assert np.array_equal(got, want)
    for a in ALL_ALGOS:
        if not applicable(a, len(p)):
            continue
        g2, _ = gpu_find(sm, t_dev, p, algo=a)
        assert np.array_equal(g2, want), a


def test_host_and_corpus_paths(sm):
    t_np = dg.zipf_text(200_000, 64, 1.0, seed=1)
    c = sm.Corpus(t_np)
    hist, sigma, sigma_eff = c.stats()
    bc = np.bincount(t_np, minlength=256)
    assert np.array_equal(hist, bc.astype(np.uint64))
    assert sigma == int((bc > 0).sum())
    assert abs(sigma_eff - 1.0 / np.sum((bc / bc.sum()) ** 2)) < 1e-6 * sigma_eff
    for m in (4, 16, 64, 256):
        p, _ = dg.substring_pattern(t_np, m, seed=2, idx=m)
        want = oracle.find_all(t_np, p)
        assert np.array_equal(c.find_all(p), want)
        assert c.count(p) == want.size
        assert np.array_equal(sm.find_all(t_np, p), want)       # host buffers
        assert sm.count(t_np, p) == want.size
    c.close()


def test_device_sync_paths(sm):
    t_np = dg.uniform_text(123_457, 16, seed=9)
    t_dev = torch.from_numpy(t_np).to(DEV)
    for m in (2, 9, 33, 64, 65, 500):
        p, _ = dg.substring_pattern(t_np, m, seed=3, idx=m)
        want = oracle.find_all(t_np, p)
        got = sm.find_all(t_dev, p).cpu().numpy()
        assert np.array_equal(got, want), m
        assert sm.count(t_dev, p) == want.size


def test_workspace_reuse_across_calls(sm):
    """One workspace, many calls with varying n, m, algorithm and workspace size:
    nothing left in the workspace by earlier calls may leak into later ones."""
    rng = np.random.default_rng(5)
    # the largest need: the most tiles (16-byte lanes) with the bitmap region (m <= 64)
    most = max(sm.workspace_size(1 << 19, m, sm.opts(lane_bytes=16)) for m in (1, 4096))
    big = torch.empty(most + (1 << 16), dtype=torch.uint8, device=DEV)
    base_np = dg.uniform_text(1 << 19, 4, seed=77)
    base = torch.from_numpy(base_np).to(DEV)
    for i in range(400):
        n = int(rng.integers(1, 1 << 19))
        m = int(rng.integers(1, 1200)) if i % 3 else int(rng.integers(1, 20))
        if m > n:
            m = n
        algo = int(rng.choice([1, 2, 3, 4] + ([6] if m <= 8 else []))) if m <= 64 else \
            int(rng.choice([4, 5])) if 144 <= m <= 4096 else 4
        o = sm.opts(algo=algo, lane_bytes=int(rng.choice([16, 64])))
        need = sm.workspace_size(n, m, o)
        work = big[:need + int(rng.integers(0, 1 << 16)) // 256 * 256]
        t_np = base_np[:n]
        if rng.random() < 0.7:
            r = int(rng.integers(0, n - m + 1))
            p = bytes(t_np[r:r + m])
        else:
            p = bytes(rng.integers(0, 4, m, dtype=np.uint8))
        want = oracle.find_all(t_np, p)
        out = torch.empty(max(want.size, 1), dtype=torch.int64, device=DEV)
        dc = torch.zeros(1, dtype=torch.int64, device=DEV)
        sm.find_all_async(base[:n], p, out[:want.size], dc, work, o)
        assert int(dc.item()) == want.size, (i, n, m, algo)
        assert np.array_equal(out[:want.size].cpu().numpy(), want), (i, n, m, algo)


def _suffix_check(sm, t_np, pats, lanes=(16, 64, 128), tpws=(1, 2)):
    t_dev = torch.from_numpy(t_np).to(DEV)
    for p in pats:
        want = oracle.find_all(t_np, p)
        for lane in lanes:
            for tpw in tpws:
                got, total = gpu_find(sm, t_dev, p, algo=1, lane=lane, tpw=tpw)
                assert total == want.size, (len(p), lane, tpw)
                assert np.array_equal(got, want), (len(p), lane, tpw)
        # truncated output: the sorted prefix
        if want.size > 3:
            got, total = gpu_find(sm, t_dev, p, algo=1, cap=want.size // 2)
            assert total == want.size and np.array_equal(got, want[:want.size // 2])


def test_shift_and_suffix_form_by_period(sm):
    """The suffix form scans the pattern's last 17 bytes (32-bit state) unless the
    pattern's smallest period lies in (17, 49], when it scans the last 49: a start one
    period after an occurrence is then taken without reading. Patterns of smallest period
    1..64 on texts repeating them (every period a candidate, most of them occurrences),
    with the repetition broken here and there, against the oracle."""
    rng = np.random.default_rng(77)
    for P in (1, 5, 17, 18, 30, 49, 50, 64):
        unit = rng.integers(0, 4, P, dtype=np.uint8)
        unit[0] = 7  # no smaller period
        t_np = np.tile(unit, 70_000 // P + 2)[:70_000 + P % 7].copy()
        for k in range(0, t_np.size, 9_973):  # broken repeats
            t_np[k] = 9
        pats = [bytes(t_np[20:20 + m]) for m in (50, 64, 65, 130, 1000)]
        _suffix_check(sm, t_np, pats, lanes=(16, 64, 128), tpws=(1,))


@pytest.mark.parametrize("sigma", [2, 4, 256])
def test_shift_and_suffix_form_random(sm, sigma):
    """Shift-And with m > 64 (the last 49 bytes scanned, the first m - 49 verified), forced,
    on i.i.d. texts: substring and random patterns, ragged tails."""
    t_np = dg.uniform_text(300_007, sigma, seed=41 + sigma)
    pats = [dg.substring_pattern(t_np, m, seed=6, idx=m)[0] for m in (65, 66, 80, 127, 128, 200, 1000, 3000)]
    pats += [dg.random_pattern(m, sigma, seed=6, idx=m) for m in (65, 300)]
    pats.append(bytes(t_np[-150:]))                               # occurrence ending at the text end
    pats.append(bytes(t_np[:70]))                                 # occurrence at 0
    _suffix_check(sm, t_np, pats)


def test_shift_and_suffix_form_periodic(sm):
    """The period rule (a start one period <= 49 after an occurrence is accepted without
    reading) on periodic texts and patterns, and its absence for longer periods."""
    n = 200_003
    a_n = np.full(n, ord("a"), dtype=np.uint8)
    _suffix_check(sm, a_n, [b"a" * m for m in (65, 100, 500)] + [b"a" * 99 + b"b", b"b" + b"a" * 99])
    gaps = a_n.copy()
    gaps[96::97] = ord("b")                                        # b every 97 bytes
    _suffix_check(sm, gaps, [b"a" * 96 + b"b" + b"a" * 40, b"a" * 96 + b"b" + b"a" * 96 + b"b",
                             b"a" * 70, b"a" * 5 + b"b" + b"a" * 96 + b"b" + b"a" * 3,
                             b"a" * 30 + b"b" + b"a" * 60], lanes=(16, 64), tpws=(1,))
    ab = np.frombuffer(b"ab" * (n // 2), dtype=np.uint8).copy()
    _suffix_check(sm, ab, [b"ab" * 50, b"ab" * 50 + b"a", b"ba" * 60, b"ab" * 40 + b"b"], lanes=(64,), tpws=(1, 2))
    for u in (49, 60, 70):                                         # the shortcut up to 49 only
        unit = dg.random_pattern(u, 4, seed=8, idx=u)
        per = np.frombuffer(unit * (n // u + 1), dtype=np.uint8)[:n].copy()
        _suffix_check(sm, per, [unit * 3, unit * 2 + unit[:10], unit[5:] + unit * 2], lanes=(64,), tpws=(1,))
    # m = n, and a pattern longer than the text
    _suffix_check(sm, ab[:300], [bytes(ab[:300]), bytes(ab[:299]) + b"b"], lanes=(16,), tpws=(1,))
    t_dev = torch.from_numpy(ab[:100]).to(DEV)
    assert gpu_find(sm, t_dev, b"ab" * 60, algo=1)[1] == 0


def test_shift_and_suffix_form_bitmap(sm):
    """The suffix form (m > 49) keeps its candidates as lane bitmaps and settles them after
    the scan; dense tiles leave their occurrence bitmaps to the emit pass. m = 50..64 and
    longer, every lane width (BitAcc of one and of two words), on a^n, (ab)^n and a text of
    dense, sparse and empty regions, with truncation."""
    n = 150_001
    a_n = np.full(n, ord("a"), dtype=np.uint8)
    ab = np.frombuffer(b"ab" * (n // 2 + 1), dtype=np.uint8)[:n].copy()
    parts = [np.zeros(9001, np.uint8), dg.uniform_text(30_003, 2, seed=35),
             np.zeros(15_013, np.uint8), np.full(7_777, 200, np.uint8), np.zeros(21_011, np.uint8),
             dg.uniform_text(11_999, 2, seed=36)]
    mixed = np.concatenate(parts)
    for t_np, pats in ((a_n, [b"a" * m for m in (50, 57, 64, 65, 130)]),
                       (ab, [b"ab" * 25, b"ba" * 28 + b"b", b"ab" * 32, b"ab" * 40 + b"a"]),
                       (mixed, [bytes(m) for m in (50, 57, 64, 90, 300)])):
        _suffix_check(sm, t_np, pats, lanes=(32, 64, 128, 16), tpws=(1, 2))
        t_dev = torch.from_numpy(t_np).to(DEV)
        for p in pats:
            want = oracle.find_all(t_np, p)
            for cap in (1, want.size // 3, want.size - 1):
                if 0 < cap < want.size:
                    got, tot = gpu_find(sm, t_dev, p, algo=1, lane=128, cap=cap)
                    assert tot == want.size and np.array_equal(got, want[:cap]), (len(p), cap)


def test_one_symbol_texts_planned(sm):
    """The planner's own choice on corpora of one symbol (sigma_eff 1): every m, closed forms."""
    n = 1 << 20
    t_np = np.full(n, ord("a"), dtype=np.uint8)
    t_np[4095::4096] = ord("b")
    c = sm.Corpus(t_np)
    for m in (4, 16, 64, 65, 256, 1000):
        p = b"a" * (m - 1) + b"b"
        pos = c.find_all(p)
        assert np.array_equal(pos, np.arange(n // 4096, dtype=np.int64) * 4096 + 4096 - m), m
    c.close()
    c = sm.Corpus(np.full(n, ord("a"), dtype=np.uint8))
    for m in (64, 65, 256, 1000):
        assert c.count(b"a" * m) == n - m + 1
        pos = c.find_all(b"a" * m)
        assert pos.size == n - m + 1 and pos[0] == 0 and pos[-1] == n - m and np.all(np.diff(pos) == 1)
    c.close()


@pytest.mark.parametrize("sigma", [4, 256])
def test_shared_workspace_upto(sm, sigma):
    """One workspace of exactly workspace_size_upto(n, M) bytes serves every length 1..M
    with the planner's own choices (which differ in lane width from length to length),
    as a corpus (measured sigma) and as a plain text (sigma estimated from the pattern)."""
    t_np = dg.uniform_text(200_003, sigma, seed=31)
    t_dev = torch.from_numpy(t_np).to(DEV)
    M = 160
    need = sm.workspace_size_upto(t_np.size, M)
    assert need >= max(sm.workspace_size(t_np.size, m) for m in range(1, M + 1))
    work = torch.empty(need, dtype=torch.uint8, device=DEV)
    c = sm.Corpus(t_dev)
    dc = torch.zeros(1, dtype=torch.int64, device=DEV)
    for m in range(1, M + 1):
        p, _ = dg.substring_pattern(t_np, m, seed=5, idx=m)
        want = oracle.find_all(t_np, p)
        out = torch.empty(max(want.size, 1), dtype=torch.int64, device=DEV)
        c.find_all_async(p, out[:want.size], dc, work)
        assert int(dc.item()) == want.size, m
        assert np.array_equal(out[:want.size].cpu().numpy(), want), m
        sm.find_all_async(t_dev, p, out[:want.size], dc, work)
        assert int(dc.item()) == want.size, m
        assert np.array_equal(out[:want.size].cpu().numpy(), want), m
    c.close()


def test_corpus_async_paths(sm):
    """Corpus queries planned with the measured sigma_eff (zipf and uniform texts)."""
    for t_np in (dg.zipf_text(300_000, 64, 1.0, seed=3), dg.uniform_text(300_000, 2, seed=3)):
        t_dev = torch.from_numpy(t_np).to(DEV)
        c = sm.Corpus(t_dev)
        work = torch.empty(max(sm.workspace_size(t_np.size, m_, sm.opts(lane_bytes=16)) for m_ in (1, 1024)),
                           dtype=torch.uint8, device=DEV)
        dc = torch.zeros(1, dtype=torch.int64, device=DEV)
        for m in (1, 3, 8, 20, 64, 65, 300, 1024):
            p, _ = dg.substring_pattern(t_np, m, seed=4, idx=m)
            want = oracle.find_all(t_np, p)
            c.count_async(p, dc, work)
            assert int(dc.item()) == want.size
            out = torch.empty(max(want.size, 1), dtype=torch.int64, device=DEV)
            c.find_all_async(p, out[:want.size], dc, work)
            assert int(dc.item()) == want.size
            assert np.array_equal(out[:want.size].cpu().numpy(), want), m
        c.close()


def test_every_tuning_table_entry(sm):
    """Every entry of the shipped planner table, at both ends of its pattern-length range
    (up to 1100 bytes) and an alphabet size inside its range, planned by the planner itself
    (alphabet hint, no forced option): the configurations the benchmark and the batched and
    served paths run, against the oracle."""
    n = 200_003
    texts = {}
    checked = set()
    for e in sm.tune_get():
        sigma = min(e["sigma_hi"], 256)  # 2, 7, 31, 127, 256: inside each bucket
        if sigma not in texts:
            t_np = dg.uniform_text(n, sigma, seed=71 + sigma)
            texts[sigma] = (t_np, torch.from_numpy(t_np).to(DEV))
        t_np, t_dev = texts[sigma]
        for m in {e["m_lo"], min(e["m_hi"], 1100)}:
            if (sigma, m) in checked:
                continue
            checked.add((sigma, m))
            plan = sm.plan_query(bytes(m), sm.opts(sigma_hint=sigma))
            p = dg.substring_pattern(t_np, m, seed=72, idx=m)[0]
            want = oracle.find_all(t_np, p)
            got, tot = gpu_find(sm, t_dev, p, sigma_hint=sigma)
            assert tot == want.size and np.array_equal(got, want), (sigma, m, plan)
    assert len(checked) > 150
