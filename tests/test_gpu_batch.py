"""GPU parity of the batched multi-pattern search against the CPU oracle.

Each pattern's slice of the batch output must equal the oracle's list for that
pattern alone (exact), whatever else is in the batch and in whatever order.
"""
import numpy as np
import pytest

import datagen as dg
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
DEV = "cuda:0"


@pytest.fixture(scope="module")
def sm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1012_2547_amd as sm
    sm.version()
    return sm


def mixed_patterns(text, count, seed, long_ones=True):
    ms = dg.log_uniform_lengths(count, 1, 1024, seed=seed)
    pats = []
    for i, m in enumerate(ms):
        m = int(m)
        if i % 2 == 0:
            pats.append(dg.substring_pattern(text, m, seed=seed, idx=i)[0])
        else:
            pats.append(dg.random_pattern(m, int(text.max()) + 1, seed=seed, idx=i))
    if long_ones:
        pats.append(dg.substring_pattern(text, 2500, seed=seed, idx=10_000)[0])  # beyond the batch limit
        pats.append(bytes(text[:3000]))
        pats.append(bytes(len(text) + 5))        # longer than the text
    pats.append(pats[0])                          # duplicate
    return pats


def check_csr(sm, t_np, pats, pos, off, cap=None):
    P = len(pats)
    assert off[0] == 0 and np.all(np.diff(off.astype(np.int64)) >= 0)
    want_all = [oracle.find_all(t_np, p) for p in pats]
    assert [int(off[i + 1] - off[i]) for i in range(P)] == [w.size for w in want_all]
    flat = np.concatenate(want_all) if want_all else np.empty(0, np.int64)
    lim = flat.size if cap is None else min(cap, flat.size)
    assert pos.size == lim
    assert np.array_equal(pos, flat[:lim])


@pytest.fixture(params=[0, 1, 2, 3], ids=["auto", "own", "shared", "single"])
def policy(sm, request):
    sm.batch_set_write_policy(request.param)
    yield request.param
    sm.batch_set_write_policy(0)


@pytest.mark.parametrize("sigma", [2, 4, 64])
def test_batch_count_and_find_all(sm, sigma, policy):
    t_np = dg.uniform_text(300_001, sigma, seed=21 + sigma)
    pats = mixed_patterns(t_np, 160, seed=sigma)
    c = sm.Corpus(t_np)
    counts = c.batch_count(pats)
    want = np.array([oracle.count(t_np, p) for p in pats], dtype=np.uint64)
    assert np.array_equal(counts, want)
    pos, off = c.batch_find_all(pats)
    check_csr(sm, t_np, pats, pos, off)
    c.close()


def test_batch_order_invariance_and_truncation(sm, policy):
    t_np = dg.zipf_text(200_000, 64, 1.0, seed=5)
    pats = mixed_patterns(t_np, 120, seed=9)
    c = sm.Corpus(t_np)
    pos, off = c.batch_find_all(pats)
    perm = np.random.default_rng(1).permutation(len(pats))
    pos2, off2 = c.batch_find_all([pats[i] for i in perm])
    for k, i in enumerate(perm):
        a = pos[off[i]:off[i + 1]]
        b = pos2[off2[k]:off2[k + 1]]
        assert np.array_equal(a, b), i
    total = int(off[-1])
    for cap in (0, 1, total // 3, total - 1):
        pc, oc = c.batch_find_all(pats, cap=cap)
        assert np.array_equal(oc, off)
        assert np.array_equal(pc, pos[:cap])
    c.close()


def test_batch_dense_and_periodic(sm, policy):
    n = 200_003
    t_np = np.full(n, ord("a"), dtype=np.uint8)
    t_np[4095::4096] = ord("b")
    pats = [b"a" * m for m in (1, 2, 3, 4, 16, 64, 65, 200, 1024)] + \
           [b"a" * (m - 1) + b"b" for m in (2, 4, 16, 64, 256, 1024)] + [b"b", b"ab", b"ba"]
    c = sm.Corpus(t_np)
    pos, off = c.batch_find_all(pats)
    check_csr(sm, t_np, pats, pos, off)
    c.close()


def test_batch_async_forms(sm):
    t_np = dg.uniform_text(500_000, 4, seed=77)
    t_dev = torch.from_numpy(t_np).to(DEV)
    pats = mixed_patterns(t_np, 100, seed=3, long_ones=False)
    c = sm.Corpus(t_dev)
    work = torch.empty(c.batch_workspace_size(pats), dtype=torch.uint8, device=DEV)
    d_counts = torch.zeros(len(pats), dtype=torch.int64, device=DEV)
    c.batch_count_async(pats, d_counts, work)
    counts = d_counts.cpu().numpy().astype(np.uint64)
    want = np.array([oracle.count(t_np, p) for p in pats], dtype=np.uint64)
    assert np.array_equal(counts, want)
    total = int(want.sum())
    d_out = torch.full((total + 7,), -1, dtype=torch.int64, device=DEV)
    d_off = torch.zeros(len(pats) + 1, dtype=torch.int64, device=DEV)
    c.batch_find_all_async(pats, d_out[:total], d_off, work)
    off = d_off.cpu().numpy().astype(np.uint64)
    pos = d_out[:total].cpu().numpy()
    assert np.all(d_out[total:].cpu().numpy() == -1)
    check_csr(sm, t_np, pats, pos, off)
    c.close()


def test_batch_matches_single_path(sm):
    t_np = dg.uniform_text(1 << 20, 16, seed=31)
    t_dev = torch.from_numpy(t_np).to(DEV)
    pats = mixed_patterns(t_np, 64, seed=12, long_ones=False)
    c = sm.Corpus(t_dev)
    pos, off = c.batch_find_all(pats)
    for i, p in enumerate(pats):
        single = sm.find_all(t_dev, p).cpu().numpy()
        assert np.array_equal(pos[off[i]:off[i + 1]], single), i
    c.close()


def test_batch_prefix_filter_many_patterns(sm):
    """Thousands of patterns per q-class: shared hash buckets, exact 1- and 2-byte
    keys, duplicates, and a 1024-pattern group boundary."""
    t_np = dg.zipf_text(150_001, 256, 1.1, seed=41)
    pats = []
    for i in range(1500):
        pats.append(dg.random_pattern(3, 256, seed=42, idx=i))           # hashed q = 3
    for i in range(1300):
        pats.append(dg.substring_pattern(t_np, 8 + i % 40, seed=43, idx=i)[0])  # q = 8, two groups
    for i in range(300):
        pats.append(dg.substring_pattern(t_np, 2, seed=44, idx=i)[0])    # exact q = 2
    pats += [b"\x00", b"\x01", b"\x00"]                                   # q = 1, duplicate
    pats += pats[:50]                                                     # duplicates
    c = sm.Corpus(t_np)
    counts = c.batch_count(pats)
    want = np.array([oracle.count(t_np, p) for p in pats], dtype=np.uint64)
    assert np.array_equal(counts, want)
    sub = pats[1500:1600] + pats[-60:]
    pos, off = c.batch_find_all(sub)
    check_csr(sm, t_np, sub, pos, off)
    c.close()


@pytest.mark.parametrize("k", [1, 2, 3, 4, 40])
def test_batch_filter_threshold_and_dense_classes(sm, k):
    """k patterns per length 4..7 and 8..12 on a 4-letter text (dense prefix
    hits): classes below the filter threshold use the per-pattern scanners."""
    t_np = dg.uniform_text(250_003, 4, seed=50 + k)
    pats = []
    for m in list(range(1, 13)) + [64, 65, 300]:
        for i in range(k):
            pats.append(dg.substring_pattern(t_np, m, seed=51, idx=m * 100 + i)[0] if i % 2 == 0
                        else dg.random_pattern(m, 4, seed=51, idx=m * 100 + i))
    c = sm.Corpus(t_np)
    counts = c.batch_count(pats)
    want = np.array([oracle.count(t_np, p) for p in pats], dtype=np.uint64)
    assert np.array_equal(counts, want)
    pos, off = c.batch_find_all(pats)
    check_csr(sm, t_np, pats, pos, off)
    c.close()


def test_batch_filter_write_overflowing_rounds(sm, policy):
    """1500 four-byte patterns on a 4-letter text: about 16 hits per pattern per
    4096 starts, so a round of the shared write pass holds far more hits than its
    LDS list and is split over pattern ranges."""
    t_np = dg.uniform_text(120_001, 4, seed=61)
    pats = [dg.random_pattern(4, 4, seed=62, idx=i) for i in range(1500)]
    pats += [dg.substring_pattern(t_np, 9 + i % 7, seed=63, idx=i)[0] for i in range(40)]
    c = sm.Corpus(t_np)
    pos, off = c.batch_find_all(pats)
    check_csr(sm, t_np, pats, pos, off)
    b = c.batch_open(pats)
    d = torch.empty(b.total, dtype=torch.int64, device=DEV)
    half = b.total // 2 + 3
    b.write_async(0, half, d[:half])
    b.write_async(half, b.total, d[half:])
    assert np.array_equal(d.cpu().numpy(), pos)
    b.close()
    c.close()


@pytest.mark.parametrize("policy", [0, 2])
def test_batch_filter_stash_and_rescan_items(sm, policy):
    """The filter's count step keeps each (chunk, group) item's hits when they fit; the
    write pass copies those out and scans the other items again. A run of zero bytes
    overflows the few items it covers (three zero patterns, sparse over the whole text,
    hit every start there); every other item keeps its hits. Written whole and in
    windows cut inside the zero patterns' slices."""
    n = 16 << 20
    t_np = dg.uniform_text(n, 4, seed=81)
    t_np[(5 << 20):(5 << 20) + 40_000] = 0
    pats = [dg.substring_pattern(t_np, 9 + i % 6, seed=82, idx=i)[0] for i in range(300)]
    pats += [bytes(9), bytes(12), bytes(10)]
    pats += pats[:5] + [bytes(12)]                                        # duplicates
    sm.batch_set_write_policy(policy)
    try:
        c = sm.Corpus(t_np)
        pos, off = c.batch_find_all(pats)
        check_csr(sm, t_np, pats, pos, off)
        assert off[301] - off[300] > 30_000                                 # the zero run
        b = c.batch_open(pats)
        d = torch.empty(b.total, dtype=torch.int64, device=DEV)
        cuts = [0, int(off[300]) + 777, int(off[302]) + 5, b.total]
        for lo, hi in zip(cuts[:-1], cuts[1:]):
            b.write_async(lo, hi, d[lo:hi])
        assert np.array_equal(d.cpu().numpy(), pos)
        b.close()
        c.close()
    finally:
        sm.batch_set_write_policy(0)


def test_batch_shared_write_dense_tile_of_one_pattern(sm):
    """A pattern sparse on average but with a hit at every start of one tile (a run
    of zero bytes): its tile overflows the shared write pass's list even alone and
    is written over the tile's quarters."""
    t_np = (dg.uniform_text(8 << 20, 5, seed=71) + 1).astype(np.uint8)   # bytes 1..5
    t_np[3 * 16384 + 100: 5 * 16384] = 0                                   # zero run over two tiles
    pats = [b"\x00\x00\x00\x00", b"\x00\x00\x00\x01", b"\x01\x02\x03\x04", b"\x02\x03\x04\x05",
            b"\x05\x04\x03\x02", b"\x00\x00\x00\x00\x00\x00\x00\x00\x00\x00"]
    sm.batch_set_write_policy(2)
    try:
        c = sm.Corpus(t_np)
        pos, off = c.batch_find_all(pats)
        check_csr(sm, t_np, pats, pos, off)
        c.close()
    finally:
        sm.batch_set_write_policy(0)


def test_batch_count_profiling_records(sm):
    """While kernel timing is on, each batched count pass is recorded with its shared
    filter launches and the n x patterns they cover; the counts stay exact; recording
    off leaves nothing to collect."""
    t_np = dg.uniform_text(300_000, 4, seed=91)
    t_dev = torch.from_numpy(t_np).to(DEV)
    pats = [dg.random_pattern(3 + i % 5, 4, seed=92, idx=i) for i in range(400)]
    c = sm.Corpus(t_dev)
    work = torch.empty(c.batch_workspace_size(pats), dtype=torch.uint8, device=DEV)
    d_counts = torch.zeros(len(pats), dtype=torch.int64, device=DEV)
    want = np.array([oracle.count(t_np, p) for p in pats], dtype=np.uint64)
    sm.prof_collect()
    sm.prof_enable(True, every=5)  # batched passes are recorded whatever the stride
    try:
        for _ in range(3):
            c.batch_count_async(pats, d_counts, work)
    finally:
        sm.prof_enable(False)
    pr = sm.prof_collect()
    assert np.array_equal(d_counts.cpu().numpy().astype(np.uint64), want)
    assert pr["batch_calls"] == 3
    assert pr["filter_launches"] >= 3 and pr["filter_ms"] > 0
    assert 0 < pr["filter_ms"] <= pr["batch_ms"]
    assert pr["filter_pattern_bytes"] > 0 and pr["filter_pattern_bytes"] % t_np.size == 0
    assert pr["filter_pattern_bytes"] <= 3 * len(pats) * t_np.size
    c.batch_count_async(pats, d_counts, work)
    assert sm.prof_collect()["batch_calls"] == 0
    c.close()
