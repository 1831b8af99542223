"""The find_all entry point that allocates nothing (its workspace is the library's
static device scratch) against sm_find_all_async with a caller workspace, and
against the oracle: bit-exact, on calls in a row whose later inputs are smaller,
so that whatever an earlier call left in the shared scratch must not leak into a
later result.
"""
import numpy as np
import pytest

import datagen as dg
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
DEV = "cuda:0"
SCRATCH = 256 << 20   # SM_NOALLOC_SCRATCH_BYTES


@pytest.fixture(scope="module")
def sm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1012_2547_amd as sm
    sm.version()
    return sm


def with_workspace(sm, t, pat, cap, o=None):
    """sm_find_all_async with its own workspace: (positions, total)."""
    work = torch.empty(max(sm.workspace_size(t.numel(), len(pat), o), 256), dtype=torch.uint8, device=DEV)
    dc = torch.zeros(1, dtype=torch.int64, device=DEV)
    out = torch.full((max(cap, 1),), -7, dtype=torch.int64, device=DEV)
    sm.find_all_async(t, pat, out[:cap], dc, work, o)
    total = int(dc.item())
    return out[:min(total, cap)].cpu().numpy(), total


def no_alloc(sm, t, pat, cap, o=None):
    dc = torch.full((1,), -1, dtype=torch.int64, device=DEV)
    out = torch.full((max(cap, 1),), -7, dtype=torch.int64, device=DEV)
    sm.find_all_noalloc(t, pat, out[:cap], dc, o)
    total = int(dc.item())
    k = min(total, cap)
    assert np.all(out[k:].cpu().numpy() == -7), "written past min(total, cap)"
    return out[:k].cpu().numpy(), total


def check(sm, t_np, t, pat, cap=None, o=None):
    want = oracle.find_all(t_np, pat)
    if cap is None:
        cap = want.size
    got, total = no_alloc(sm, t, pat, cap, o)
    ref, ref_total = with_workspace(sm, t, pat, cap, o)
    assert total == ref_total == want.size, (len(pat), total, ref_total, want.size)
    assert np.array_equal(got, ref), len(pat)
    assert np.array_equal(got, want[:cap]), len(pat)


def test_no_alloc_matches_async_two_calls(sm):
    # first call: a large text with many dense tiles; second: a smaller one
    big_np = dg.uniform_text((1 << 26) + 333, 2, seed=71)
    small_np = dg.uniform_text((1 << 20) + 17, 4, seed=72)
    big, small = torch.from_numpy(big_np).to(DEV), torch.from_numpy(small_np).to(DEV)
    p1 = dg.substring_pattern(big_np, 6, seed=73, idx=0)[0]
    p2 = dg.substring_pattern(small_np, 9, seed=73, idx=1)[0]
    check(sm, big_np, big, p1)
    check(sm, small_np, small, p2)
    # the same pair under forced scanners, and truncated lists
    for algo, lane in ((1, 16), (1, 128), (2, 64), (4, 32)):
        o = sm.opts(algo=algo, lane_bytes=lane)
        check(sm, big_np, big, p1, o=o)
        check(sm, small_np, small, p2, o=o)
    check(sm, big_np, big, p1, cap=1000)
    check(sm, small_np, small, p2, cap=1)


def test_no_alloc_lengths_and_edges(sm):
    t_np = dg.uniform_text(3_000_001, 4, seed=74)
    t_np[-700:] = 0
    t = torch.from_numpy(t_np).to(DEV)
    for m in (1, 2, 8, 17, 49, 50, 64, 65, 200, 1000, 3072):
        check(sm, t_np, t, dg.substring_pattern(t_np, m, seed=75, idx=m)[0])
    check(sm, t_np, t, bytes(300))            # zero run at the text's end
    # smaller inputs after larger ones: a few bytes, m == n, m > n
    tiny_np = t_np[:40].copy()
    tiny = torch.from_numpy(tiny_np).to(DEV)
    check(sm, tiny_np, tiny, bytes(tiny_np[5:9]))
    check(sm, tiny_np, tiny, bytes(tiny_np))
    got, total = no_alloc(sm, tiny, bytes(41), 4)
    assert total == 0 and got.size == 0


def test_no_alloc_rejects_beyond_scratch(sm):
    t = torch.empty(1 << 31, dtype=torch.uint8, device=DEV)      # never read: rejected first
    assert sm.workspace_size(1 << 31, 8) > SCRATCH
    out = torch.empty(1, dtype=torch.int64, device=DEV)
    dc = torch.zeros(1, dtype=torch.int64, device=DEV)
    with pytest.raises(sm.SmError, match="static scratch"):
        sm.find_all_noalloc(t, b"abcdefgh", out, dc)
    small = torch.zeros(5000, dtype=torch.uint8, device=DEV)
    with pytest.raises(sm.SmError, match="at most 3072"):
        sm.find_all_noalloc(small, bytes(3073), out, dc)
    del t
    # the entry point still works after the rejections
    s_np = dg.uniform_text(50_000, 4, seed=76)
    check(sm, s_np, torch.from_numpy(s_np).to(DEV), dg.substring_pattern(s_np, 12, seed=77, idx=0)[0])
