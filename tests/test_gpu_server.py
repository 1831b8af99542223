"""GPU tests of the windowed batch writes and the query server.

Every result is compared with the CPU oracle for the pattern alone, so a query
answered inside a mixed batch must equal its answer in isolation, exactly.
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


def corpora_small():
    """Scaled-down versions of the three serving corpora: uniform sigma=4,
    uniform sigma=20, Zipf(s=1.1) over 256 symbols."""
    return [dg.uniform_text(300_001, 4, seed=11), dg.uniform_text(200_003, 20, seed=12),
            dg.zipf_text(250_007, 256, 1.1, seed=13)]


def query_mix(texts, count, seed):
    """(corpus, pattern) pairs: corpus uniform, m log-uniform in [4, 256], half
    substrings of the chosen corpus, half i.i.d. random over its alphabet."""
    ms = dg.log_uniform_lengths(count, 4, 256, seed=seed)
    cs = dg.choices(count, len(texts), seed=seed)
    out = []
    for i in range(count):
        t = texts[int(cs[i])]
        m = int(ms[i])
        if i % 2 == 0:
            p = dg.substring_pattern(t, m, seed=seed, idx=i)[0]
        else:
            p = dg.random_pattern(m, int(t.max()) + 1, seed=seed, idx=i)
        out.append((int(cs[i]), p))
    return out


@pytest.mark.parametrize("policy", [0, 1, 3])
def test_batch_windows_match_whole_output(sm, policy):
    """Windows cut inside the slices of dense patterns, which the automatic write plan
    (0) and policy 3 search with the single-pattern pipeline, one window at a time."""
    sm.batch_set_write_policy(policy)
    t_np = dg.uniform_text(400_000, 4, seed=3)
    t_np[:50_000] = np.tile(t_np[:7], 50_000 // 7 + 1)[:50_000]  # period 7: long patterns recur
    pats = [dg.substring_pattern(t_np, int(m), seed=4, idx=i)[0]
            for i, m in enumerate(dg.log_uniform_lengths(60, 2, 1024, seed=4))]
    pats += [dg.substring_pattern(t_np, 2600, seed=4, idx=99)[0], b"\x00\x01", bytes(t_np[:3000])]
    c = sm.Corpus(t_np)
    want = [oracle.find_all(t_np, p) for p in pats]
    flat = np.concatenate(want)
    b = c.batch_open(pats)
    assert b.total == flat.size
    assert np.array_equal(b.offsets[1:] - b.offsets[:-1], [w.size for w in want])
    rng = np.random.default_rng(5)
    assert want[62].size > 1000
    cuts = np.unique(np.concatenate([[0, b.total], rng.integers(0, b.total, 9),
                                     b.offsets[[10, 61, 62]].astype(np.int64) + 1,
                                     b.offsets[[62]].astype(np.int64) + 777]))
    d = torch.full((b.total + 8,), -1, dtype=torch.int64, device=DEV)
    got = []
    for lo, hi in zip(cuts[:-1], cuts[1:]):
        buf = d[: hi - lo]
        b.write_async(int(lo), int(hi), buf)
        got.append(buf.cpu().numpy().copy())
    assert np.array_equal(np.concatenate(got), flat)
    b.write_async(5, 5, d)  # empty window
    with pytest.raises(sm.SmError):
        b.write_async(0, b.total + 1, d)
    b.close()
    c.close()
    sm.batch_set_write_policy(0)


def test_batch_find_all_in_small_waves(sm):
    t_np = np.full(100_000, ord("a"), dtype=np.uint8)
    t_np[::97] = ord("b")
    pats = [b"a", b"aa", b"ab", b"a" * 40, b"ba", bytes(t_np[:2500]), b"a" * 2500]
    c = sm.Corpus(t_np)
    want = [oracle.find_all(t_np, p) for p in pats]
    try:
        sm.batch_set_wave_bytes(8 * 4099)  # many waves
        pos, off = c.batch_find_all(pats)
        pos2, off2 = c.batch_find_all(pats, cap=12_345)
    finally:
        sm.batch_set_wave_bytes(0)
    flat = np.concatenate(want)
    assert np.array_equal(off[1:] - off[:-1], [w.size for w in want])
    assert np.array_equal(pos, flat)
    assert np.array_equal(off2, off) and np.array_equal(pos2, flat[:12_345])
    c.close()


@pytest.mark.parametrize("slots,max_batch,pool,host,graphs,policy", [(2, 64, 0, 0, True, 0), (2, 64, 0, 0, False, 0),
                                                                     (1, 7, 1 << 16, 1 << 16, True, 0),
                                                                     (3, 256, 8 * 5000 * 3, 1 << 20, True, 2),
                                                                     (2, 32, 8 * 10000 * 2, 1 << 20, True, 3)])
def test_server_alone_vs_in_mix(sm, slots, max_batch, pool, host, graphs, policy):
    """Policy 3 sends every pattern of at most 64 bytes through the single-pattern
    pipeline in each write wave (waves launched directly, the others from graphs)."""
    sm.batch_set_write_policy(policy)
    texts = corpora_small()
    srv = sm.Server(pool_bytes=pool, host_bytes=host, max_batch=max_batch, slots=slots, graphs=graphs)
    cs = [sm.Corpus(t) for t in texts]
    ids = [srv.add_corpus(c) for c in cs]
    qs = query_mix(texts, 150, seed=14)
    qs += [(0, b"\x00\x01"), (1, b"\x05"), (2, bytes(texts[2][:2100])), (0, bytes(texts[0][:300_001]))]
    tickets = [srv.submit(ids[c], p) for c, p in qs]
    refused = 0
    for (c, p), tk in zip(qs, tickets):
        want = oracle.find_all(texts[c], p)
        if host and (want.size * 8 + 255) // 256 * 256 > host:
            # positions alone larger than the host result arena: refused, not allocated
            with pytest.raises(sm.SmError, match="ENOMEM"):
                srv.wait(tk)
            refused += 1
            srv.free(tk)
            continue
        cnt, pos, info = srv.wait(tk)
        assert cnt == want.size, (c, len(p))
        assert np.array_equal(pos, want), (c, len(p))
        assert info["corpus"] == c and info["done_ns"] >= info["start_ns"] >= info["arrival_ns"] > 0
        srv.free(tk)
    st = srv.stats()
    assert st["completed"] == len(qs) - refused and st["pending"] == 0
    assert st["rejected"] == refused
    assert st["host_peak_bytes"] <= st["host_arena_bytes"]
    assert 0 < st["p50_ns"] <= st["p99_ns"] <= st["p999_ns"] <= st["max_ns"]
    if pool:  # no wave holds more than a slot's pool share
        assert st["write_waves"] * (pool // slots) >= st["out_bytes"]
    if host and host < (1 << 20):  # the 64 KiB arena cannot hold the densest queries
        assert refused > 0
    if not graphs:
        assert st["graph_launches"] == 0
    srv.close()
    sm.batch_set_write_policy(0)
    for c in cs:
        c.close()


@pytest.mark.parametrize("slots", [1, 2, 3])
def test_server_defers_on_memory(sm, slots):
    """A host result arena far smaller than a batch's positions: batches are cut to the
    prefix that fits, the rest deferred and counted again, completed results evicted to
    pageable memory when a deferred query needs the room; pinned memory never exceeds
    the arena and every result equals the oracle's for the pattern alone."""
    t_np = dg.uniform_text(300_001, 4, seed=31)
    c = sm.Corpus(t_np)
    host = 64 << 10
    srv = sm.Server(host_bytes=host, max_batch=64, slots=slots)
    cid = srv.add_corpus(c)
    pats = [dg.substring_pattern(t_np, 3 + i % 4, seed=32, idx=i)[0] for i in range(160)]
    want = [oracle.find_all(t_np, p) for p in pats]
    assert sum(w.size for w in want) * 8 > 20 * host
    tks = [srv.submit(cid, p) for p in pats]
    for k, tk in enumerate(tks):
        cnt, pos, _ = srv.wait(tk)
        assert cnt == want[k].size and np.array_equal(pos, want[k]), k
        srv.free(tk)
    st = srv.stats()
    assert st["completed"] == len(pats) and st["rejected"] == 0
    assert st["deferred"] > 0
    assert 0 < st["host_peak_bytes"] <= host == st["host_arena_bytes"]
    # results held by the caller while more queries arrive: the others wait or are
    # evicted around them; freeing them lets everything finish
    held = [srv.submit(cid, pats[i]) for i in range(4)]
    for k, tk in enumerate(held):
        cnt, pos, _ = srv.wait(tk)
        assert np.array_equal(pos, want[k])
    more = [srv.submit(cid, p) for p in pats[4:40]]
    for tk in held:
        srv.free(tk)
    for k, tk in enumerate(more):
        assert np.array_equal(srv.result(tk), want[4 + k]), k
    srv.close()
    c.close()


def test_server_matches_single_path_and_reuses_memory(sm):
    t_np = dg.uniform_text(1 << 20, 4, seed=21)
    t_dev = torch.from_numpy(t_np).to(DEV)
    c = sm.Corpus(t_dev)
    srv = sm.Server(max_batch=32, host_bytes=1 << 22)
    cid = srv.add_corpus(c)
    pats = [dg.substring_pattern(t_np, int(m), seed=22, idx=i)[0]
            for i, m in enumerate(dg.log_uniform_lengths(96, 4, 256, seed=22))]
    for rnd in range(4):  # results freed in and out of order; arena space is reused
        tks = [srv.submit(cid, p) for p in pats]
        order = list(range(len(tks)))
        np.random.default_rng(rnd).shuffle(order)
        for k in order:
            got = srv.result(tks[k])
            single = sm.find_all(t_dev, pats[k]).cpu().numpy()  # eager work between replays
            assert np.array_equal(got, single), (rnd, k)
        torch.cuda.synchronize()
    st = srv.stats()
    # the same batches again and again: graph executables are updated, not rebuilt
    assert st["graph_launches"] > 0 and st["graph_builds"] < st["graph_launches"]
    srv.close()
    c.close()


def test_server_errors(sm):
    t_np = dg.uniform_text(10_000, 4, seed=1)
    c = sm.Corpus(t_np)
    srv = sm.Server(max_pending=4)
    cid = srv.add_corpus(c)
    with pytest.raises(sm.SmError):
        srv.submit(cid + 1, b"ab")
    with pytest.raises(sm.SmError):
        srv.submit(cid, b"")
    tk = srv.submit(cid, b"\x00\x01\x02")
    assert srv.result(tk).size == oracle.find_all(t_np, b"\x00\x01\x02").size
    with pytest.raises(sm.SmError):
        srv.free(tk)  # already freed
    with pytest.raises(sm.SmError):
        srv.wait(12345)
    srv.close()
    c.close()
