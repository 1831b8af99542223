"""GPU parity at the sizes the benchmark runs at, element by element against the oracle.

A text of n = 2^32 + 4099 bytes (i.i.d. uniform over 4 symbols, the alphabet of the
batched and serving workloads) carries runs of zero bytes across the offsets 2^31 and
2^32 and at its end, so that patterns of zero bytes occur at every start around those
offsets (positions 2^31 - 1, 2^31, 2^32 - 1, 2^32, ... and n - m). Every scanner is
forced in turn on patterns of 5 to 1024 bytes (dense, sparse, straddling and
substring patterns), with the tile-count scan spread over many workgroups (more than
4096 tiles at every lane width), and the batched (every write route) and served forms
are checked on the same patterns. The oracle is the naive definition on 16 host
threads; the lists must be equal, so any slip in 64-bit position arithmetic shows.
A second test covers every scanner and lane width on a 64 MiB text (more than 4096
tiles of 4096 starts), with truncation inside the list; a third takes the serving
workload's largest corpus size, 2^33 + 4099 bytes, through the single-pattern, batched and
served forms.
"""
import os

import numpy as np
import pytest

import datagen as dg
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
DEV = "cuda:0"
THREADS = min(16, os.cpu_count() or 1)

N_BIG = (1 << 32) + 4099
RUN = 640          # length of each zero run
B31, B32 = 1 << 31, 1 << 32


@pytest.fixture(scope="module")
def sm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1012_2547_amd as sm
    sm.version()
    return sm


def gpu_find(sm, t_dev, pat, algo=0, lane=0, q=0, tpw=0, cap=None):
    o = sm.opts(algo=algo, lane_bytes=lane, q=q, tiles_per_wg=tpw)
    n, m = t_dev.numel(), len(pat)
    work = torch.empty(max(sm.workspace_size(n, m, o), 256), dtype=torch.uint8, device=DEV)
    dc = torch.zeros(1, dtype=torch.int64, device=DEV)
    sm.count_async(t_dev, pat, dc, work, o)
    total_c = int(dc.item())
    if cap is None:
        cap = total_c
    out = torch.full((max(cap, 1),), -7, dtype=torch.int64, device=DEV)
    sm.find_all_async(t_dev, pat, out[:cap], dc, work, o)
    total = int(dc.item())
    assert total == total_c, (algo, lane, m, total, total_c)
    got = out[:min(total, cap)].cpu().numpy()
    assert np.all(out[min(total, cap):].cpu().numpy() == -7)
    del work, out
    return got, total


# forced scanners per pattern length: (algo, lane_bytes, q, tiles_per_wg)
SA, BNDM, SBNDM, HASHQ, BLOCK, BRUTE = 1, 2, 3, 4, 5, 6
PLANS = {
    5: [(SA, 64, 0, 1), (SA, 16, 0, 2), (BNDM, 64, 0, 1), (SBNDM, 64, 4, 1), (HASHQ, 32, 3, 1),
        (BRUTE, 32, 0, 1)],
    12: [(SA, 128, 0, 1), (BNDM, 16, 0, 1), (SBNDM, 64, 2, 2), (HASHQ, 64, 0, 1)],
    40: [(SA, 32, 0, 1), (BNDM, 64, 0, 1), (SBNDM, 64, 8, 1), (HASHQ, 16, 0, 1)],
    64: [(SA, 64, 0, 1), (BNDM, 64, 0, 1), (SBNDM, 128, 8, 1), (HASHQ, 64, 0, 2)],
    100: [(SA, 128, 0, 1), (SA, 16, 0, 1), (HASHQ, 64, 0, 1), (SBNDM, 64, 8, 1)],
    300: [(BLOCK, 0, 0, 2), (HASHQ, 64, 0, 1), (SA, 64, 0, 1), (SBNDM, 128, 4, 2)],
    1024: [(BLOCK, 0, 0, 1), (HASHQ, 128, 0, 1)],
}


@pytest.fixture(scope="module")
def big(sm):
    """The 2^32 + 4099-byte text (host and device), its patterns and their oracle lists."""
    print("fullsize: generating n = 2^32 + 4099 (sigma 4, seed 61)", flush=True)
    t_np = dg.uniform_text(N_BIG, 4, seed=61)
    for a in (B31 - RUN // 2, B32 - RUN // 2, N_BIG - RUN):
        t_np[a:a + RUN] = 0
    pats = []
    for m in PLANS:
        if m <= RUN:
            pats.append((m, "zeros", bytes(m)))
        o = B32 + 2000 - m // 2                      # a substring above 2^32
        pats.append((m, "substring", bytes(t_np[o:o + m])))
        o = (3 << 30) + 12_345 * m                   # between 2^31 and 2^32
        pats.append((m, "substring_hi", bytes(t_np[o:o + m])))
    pats.append((5, "random", dg.random_pattern(5, 4, seed=62, idx=0)))
    want = {}
    for m, kind, p in pats:
        want[p] = oracle.find_all(t_np, p, threads=THREADS)
        print("fullsize: oracle m=%d %s: %d occurrences" % (m, kind, want[p].size), flush=True)
    # the plants are where they should be
    z5 = want[bytes(5)]
    for x in (B31 - 1, B31, B32 - 1, B32, N_BIG - 5):
        assert np.searchsorted(z5, x) < z5.size and z5[np.searchsorted(z5, x)] == x, x
    t_dev = torch.from_numpy(t_np).to(DEV)
    torch.cuda.synchronize()
    return t_np, t_dev, pats, want


def test_every_scanner_past_2_32(sm, big):
    t_np, t_dev, pats, want = big
    for m, kind, p in pats:
        w = want[p]
        for algo, lane, q, tpw in PLANS[m]:
            print("fullsize: m=%d %s algo=%d lane=%d q=%d tpw=%d" % (m, kind, algo, lane, q, tpw),
                  flush=True)
            got, tot = gpu_find(sm, t_dev, p, algo=algo, lane=lane, q=q, tpw=tpw)
            assert tot == w.size, (m, kind, algo, lane, tot, w.size)
            assert np.array_equal(got, w), (m, kind, algo, lane)
        # the planner's own choice, and a truncated list whose cut lies past 2^31
        got = sm.find_all(t_dev, p).cpu().numpy()
        assert np.array_equal(got, w), (m, kind, "planner")
        k = int(np.searchsorted(w, B31 + 1))
        if 0 < k < w.size:
            got, tot = gpu_find(sm, t_dev, p, cap=k)
            assert tot == w.size and np.array_equal(got, w[:k]), (m, kind, "cap")


@pytest.mark.parametrize("policy", [0, 1, 2, 3])
def test_batched_past_2_32(sm, big, policy):
    t_np, t_dev, pats, want = big
    plist = [p for _, _, p in pats] + [pats[0][2]]     # with a duplicate
    print("fullsize: batched find_all, write policy %d" % policy, flush=True)
    sm.batch_set_write_policy(policy)
    try:
        c = sm.Corpus(t_dev)
        counts = c.batch_count(plist)
        assert [int(x) for x in counts] == [want[p].size for p in plist]
        pos, off = c.batch_find_all(plist)
        for i, p in enumerate(plist):
            assert np.array_equal(pos[off[i]:off[i + 1]], want[p]), (policy, i, len(p))
        c.close()
    finally:
        sm.batch_set_write_policy(0)


def test_served_past_2_32(sm, big):
    t_np, t_dev, pats, want = big
    print("fullsize: served queries", flush=True)
    c = sm.Corpus(t_dev)
    # a small staging pool: the dense lists take several write waves
    srv = sm.Server(pool_bytes=32 << 20, host_bytes=256 << 20, max_batch=8)
    cid = srv.add_corpus(c)
    tickets = [(p, srv.submit(cid, p)) for _, _, p in pats]
    for p, tk in tickets:
        assert np.array_equal(srv.result(tk), want[p]), len(p)
    srv.close()
    c.close()


N_HUGE = (1 << 33) + 4099
B33 = 1 << 33


def test_positions_past_2_33(sm):
    """The serving workload's largest corpus (sigma 4, 8 GiB): a text of 2^33 + 4099 bytes
    with zero runs across 2^33 and at its end. The planner's scanners, a forced dense
    Shift-And (hit bitmaps), the batched form and a served query, each against the oracle
    element by element."""
    print("fullsize: generating n = 2^33 + 4099 (sigma 4, seed 65)", flush=True)
    t_np = dg.uniform_text(N_HUGE, 4, seed=65)
    for a in (B33 - RUN // 2, N_HUGE - RUN):
        t_np[a:a + RUN] = 0
    pats = [bytes(9), bytes(t_np[B33 + 1000:B33 + 1064]), bytes(t_np[(3 << 31) + 17:(3 << 31) + 217]),
            dg.substring_pattern(t_np, 16, seed=66, idx=0)[0], bytes(t_np[N_HUGE - 700:N_HUGE - 600])]
    want = {}
    for p in pats:
        want[p] = oracle.find_all(t_np, p, threads=THREADS)
        print("fullsize: oracle m=%d: %d occurrences" % (len(p), want[p].size), flush=True)
    z = want[bytes(9)]
    for x in (B33 - 1, B33, N_HUGE - 9):
        k = int(np.searchsorted(z, x))
        assert k < z.size and z[k] == x, x
    t_dev = torch.from_numpy(t_np).to(DEV)
    try:
        for p in pats:
            print("fullsize 2^33: planner's scanner, m=%d" % len(p), flush=True)
            got, tot = gpu_find(sm, t_dev, p)
            assert tot == want[p].size and np.array_equal(got, want[p]), len(p)
        print("fullsize 2^33: forced Shift-And, 128-start lanes", flush=True)
        got, tot = gpu_find(sm, t_dev, bytes(9), algo=SA, lane=128)
        assert tot == z.size and np.array_equal(got, z)
        print("fullsize 2^33: batched and served", flush=True)
        c = sm.Corpus(t_dev)
        pos, off = c.batch_find_all(pats)
        for i, p in enumerate(pats):
            assert np.array_equal(pos[off[i]:off[i + 1]], want[p]), ("batched", i)
        srv = sm.Server(pool_bytes=64 << 20, host_bytes=256 << 20, max_batch=4)
        cid = srv.add_corpus(c)
        tickets = [(p, srv.submit(cid, p)) for p in pats]
        for p, tk in tickets:
            assert np.array_equal(srv.result(tk), want[p]), ("served", len(p))
        srv.close()
        c.close()
    finally:
        del t_dev
        torch.cuda.empty_cache()


def test_many_tiles_every_scanner(sm):
    """More than 4096 tiles at every lane width (the tile-count scan's workgroups read
    the super-chunk totals before their chunk), every scanner, lanes 16..128."""
    n = (1 << 26) + 77
    t_np = dg.uniform_text(n, 4, seed=63)
    t_np[(1 << 25) - 300:(1 << 25) + 300] = 0
    t_dev = torch.from_numpy(t_np).to(DEV)
    pats = [dg.substring_pattern(t_np, m, seed=64, idx=m)[0] for m in (3, 8, 20, 49, 50, 64, 65, 200, 1000)]
    pats += [bytes(m) for m in (4, 9, 64, 150)] + [bytes(t_np[n - 70:])]
    for p in pats:
        m = len(p)
        w = oracle.find_all(t_np, p, threads=THREADS)
        algos = [a for a in (SA, BNDM, SBNDM, HASHQ, BLOCK, BRUTE)
                 if (a in (SA, SBNDM, HASHQ)) or (a == BNDM and m <= 64)
                 or (a == BLOCK and 144 <= m <= 4096) or (a == BRUTE and m <= 8)]
        for a in algos:
            for lane in ((0,) if a == BLOCK else (16, 64, 128)):
                print("many tiles: m=%d algo=%d lane=%d" % (m, a, lane), flush=True)
                got, tot = gpu_find(sm, t_dev, p, algo=a, lane=lane)
                assert tot == w.size and np.array_equal(got, w), (m, a, lane)
        if w.size > 2:
            got, tot = gpu_find(sm, t_dev, p, cap=w.size // 2 + 1)
            assert tot == w.size and np.array_equal(got, w[:w.size // 2 + 1]), (m, "cap")
