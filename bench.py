"""Benchmark: single-pattern exact matching sweep on one MI355X.

Workload (the headline configuration): for each alphabet size sigma in
{2, 4, 16, 64, 256} a text of n = 2^30 i.i.d. uniform bytes over {0..sigma-1}
(text seed 1), and for each m in {2, 4, ..., 1024} 20 patterns copied from
random offsets of that text (pattern seed 2) -- the shape of the paper's
Section 2 experiments at 2^30 bytes instead of 5 MB. One step = the whole sweep:
1000 find_all calls (device text, device output; count -> tile scan -> emit), texts
resident in HBM before timing starts.

Prints ONE JSON line on stdout; progress goes to stderr.
    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "text GB/s scanned (and % of HBM peak); batched patterns×GB/s; p50/p99 query latency"
HBM_PEAK_GBS = 8000.0
PROF_EVERY = 8  # sweep calls per call whose kernels are timed with HIP events

# The paper's own timings, as context only (other hardware, other text sizes): mean
# search time of the best algorithm per pattern length on its uniform 4-symbol text
# of 5e6 bytes, one core of an Intel Core2 at 1.66 GHz (Section 2; its Rand4 table,
# Section 2.2), converted to GB/s = 5e6 / t.
PAPER_CONTEXT = {
    "hardware": "one core of an Intel Core2 at 1.66 GHz",
    "text": "uniform, 4 symbols, 5e6 bytes",
    "best_gbs_by_m": {"2": {"algo": "SA", "ms": 16.4, "gbs": 0.30},
                      "8": {"algo": "HASH3", "ms": 8.30, "gbs": 0.60},
                      "64": {"algo": "HASH8", "ms": 2.46, "gbs": 2.03},
                      "1024": {"algo": "SSEF", "ms": 0.54, "gbs": 9.26}},
    "note": "context only; not the target",
}
SIGMAS = (2, 4, 16, 64, 256)
MS = (2, 4, 8, 16, 32, 64, 128, 256, 512, 1024)
PER_CELL = 20
TEXT_SEED, PAT_SEED = 1, 2


def log(*a):
    print(*a, file=sys.stderr, flush=True)


KERNEL_SOURCES = {
    "count": ("sm_kernels.hip", "sm_device.h", "sm_internal.h"),
    "mq_count": ("sm_batch.hip", "sm_device.h", "sm_internal.h"),
}
# dense VALU issue of the chip: 256 CUs x 4 SIMD16 units x 16 lanes x 2.4 GHz (one wave64
# instruction per CU per clock)
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12


def kernel_source_hash(kernel: str = "count") -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, "paper_1012_2547_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_counters(kernel: str):
    """Per-launch counter figures of a kernel from the committed rocprofv3 --pmc
    summary, if they were taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            d = json.load(f)
    except OSError:
        return None
    e = d.get(kernel)
    if not e or e.get("source_hash") != kernel_source_hash(kernel):
        return None
    return e


def load_traffic(kernel: str):
    """HBM bytes per launch from the committed rocprofv3 --pmc summary, if it was
    taken on the current kernel source; else None."""
    e = load_counters(kernel)
    return e.get("bytes_per_launch") if e else None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n-log2", type=int, default=30)
    ap.add_argument("--per-cell", type=int, default=PER_CELL)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-threads", type=int, default=0)
    ap.add_argument("--sigmas", type=str, default="",
                    help="comma-separated subset of the sweep's alphabet sizes (profiling runs)")
    ap.add_argument("--ms", type=str, default="",
                    help="comma-separated subset of the sweep's pattern lengths (profiling runs)")
    ap.add_argument("--no-skewed", action="store_true",
                    help="skip the skewed (Zipf) and adversarial (a^n) texts")
    ap.add_argument("--skewed-n-log2", type=int, default=30)
    ap.add_argument("--no-batched", action="store_true", help="skip the batched section")
    ap.add_argument("--batched-n-log2", type=int, default=32)
    ap.add_argument("--batched-patterns", type=int, default=4096)
    ap.add_argument("--no-batched-find-all", action="store_true",
                    help="skip listing every position of the batched workload (64 GiB output waves)")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving section")
    ap.add_argument("--serve-shift", type=int, default=0,
                    help="log2 scale of the serving corpora (0: 8, 2 and 4 GiB)")
    ap.add_argument("--serve-seconds", type=float, default=2.0,
                    help="trace length per arrival rate: min(20000, max(2000, rate x seconds)) queries")
    ap.add_argument("--serve-min-queries", type=int, default=2000,
                    help="queries per arrival rate at least (so that p99 and p999 rest on many samples)")
    ap.add_argument("--serve-rates", type=str, default="250,1000,4000,16000")
    ap.add_argument("--plain-queries", type=int, default=1000,
                    help="queries of each trace (its prefix) replayed through the plain path")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first copy 1 GiB device-to-device (reference for HBM byte counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py measures one GPU only: every box in this setup has a single MI355X; "
              "--gpus %d is not supported (run with --gpus 1)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import datagen as dg
    import paper_1012_2547_amd as sm

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    n = 1 << args.n_log2
    stream = torch.cuda.current_stream()
    global SIGMAS, MS
    if args.sigmas:
        SIGMAS = tuple(int(x) for x in args.sigmas.split(","))
    if args.ms:
        MS = tuple(int(x) for x in args.ms.split(","))
    if args.calibrate_copy:
        a = torch.ones(1 << 30, dtype=torch.uint8, device=dev)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
        log("calibration copy of 2^30 bytes done")

    # ---- inputs: texts resident in HBM, patterns, exact output sizes -------
    t0 = time.time()
    host_texts, dev_texts, pats = {}, {}, {}
    for s in SIGMAS:
        h = dg.uniform_text(n, s, seed=TEXT_SEED)
        host_texts[s] = h
        dev_texts[s] = torch.from_numpy(h).to(dev)
        for mi, m in enumerate(MS):
            pats[(s, m)] = [dg.substring_pattern(h, m, seed=PAT_SEED, idx=mi * 1000 + j)[0]
                            for j in range(args.per_cell)]
    log("inputs ready in %.1fs" % (time.time() - t0))

    # corpora: device-resident texts with their byte histogram probed once; the
    # planner uses each corpus's measured effective alphabet size
    corpora = {s: sm.Corpus(dev_texts[s]) for s in SIGMAS}
    sigma_eff = {s: round(corpora[s].stats()[2], 2) for s in SIGMAS}
    calls = [(s, m, p) for s in SIGMAS for m in MS for p in pats[(s, m)]]
    work = torch.empty(sm.workspace_size_upto(n, 1024), dtype=torch.uint8,
                       device=dev)
    counts_dev = torch.zeros(len(calls), dtype=torch.int64, device=dev)
    # exact counts (sizes the output buffer; checked after every step)
    for k, (s, m, p) in enumerate(calls):
        corpora[s].count_async(p, counts_dev[k:k + 1], work, None, stream)
    torch.cuda.synchronize()
    expect = counts_dev.cpu().numpy().copy()
    cap = int(expect.max())
    out = torch.empty(cap, dtype=torch.int64, device=dev)
    occ_total = int(expect.sum())
    log("counts ready: max %d, total %d occurrences per step" % (cap, occ_total))

    def step():
        for k, (s, m, p) in enumerate(calls):
            corpora[s].find_all_async(p, out, counts_dev[k:k + 1], work, None, stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    got = counts_dev.cpu().numpy()
    assert np.array_equal(got, expect), "find_all totals differ from count totals"

    sm.prof_collect()  # clear
    # kernel times from HIP events on every PROF_EVERY-th call (each event costs the
    # stream a few microseconds, about 10 % of a call if every call carried four)
    sm.prof_enable(True, every=PROF_EVERY)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    sm.prof_enable(False)
    prof = sm.prof_collect()
    assert np.array_equal(counts_dev.cpu().numpy(), expect)

    elapsed = t2 - t1
    bytes_per_step = n * len(calls)
    gbs = bytes_per_step * args.steps / elapsed / 1e9
    ms_per_step = elapsed * 1e3 / args.steps

    # dominant kernel: the count kernel, one pass over the text (n bytes per launch).
    # Calls planned on the block filter read one aligned 16-byte block per S <= m - 15 bytes;
    # they are reported apart and left out of the roofline figure.
    calls_n = max(prof["calls"], 1)
    full_n = max(prof["calls"] - prof["sampled_calls"], 1)
    avg_count_s = (prof["count_ms"] - prof["sampled_count_ms"]) / full_n / 1e3
    count_gbs = n / avg_count_s / 1e9 if avg_count_s > 0 else 0.0
    sampled = None
    if prof["sampled_calls"]:
        avg_s = prof["sampled_count_ms"] / prof["sampled_calls"] / 1e3
        sampled = {"kernel": "block_count_kernel (one aligned 16-byte block per 16*floor((m - 15)/16) text bytes)",
                   "launches": prof["sampled_calls"], "avg_launch_us": round(avg_s * 1e6, 2),
                   "text_equivalent_gbs": round(n / avg_s / 1e9, 1)}
    algo_bytes_call = (n * len(calls) + 8 * occ_total) / len(calls)
    call_gbs = algo_bytes_call / (prof["total_ms"] / calls_n / 1e3) / 1e9
    traffic = load_traffic("count")
    roofline = {"bound": "hbm", "achieved": round(count_gbs, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(count_gbs / HBM_PEAK_GBS, 4),
                "traffic": traffic, "kernel": "count_kernel<algo, L, variant, find> (text pass)",
                "avg_launch_us": round(avg_count_s * 1e6, 2),
                "launches": prof["calls"] - prof["sampled_calls"],
                "bytes_per_launch": n,
                "avg_emit_us": round(prof["emit_ms"] / calls_n * 1e3, 2),
                "whole_call_algorithmic_gbs": round(call_gbs, 1),
                "block_filter_launches": sampled}
    log("sweep: %.1f GB/s text, count kernel %.1f GB/s (%.1f%% of HBM), emit %.1f us avg, "
        "%.2f ms/step" % (gbs, count_gbs, 100 * count_gbs / HBM_PEAK_GBS,
                          roofline["avg_emit_us"], ms_per_step))

    # per-cell rates from one extra timed pass: events at cell boundaries only, so a
    # cell's rate is its patterns' bytes over their back-to-back calls
    keys = ["s%d_m%d" % (s, m) for s in SIGMAS for m in MS]
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(len(keys) + 1)]
    ev[0].record(stream)
    k = 0
    for ci, (s, m) in enumerate((s, m) for s in SIGMAS for m in MS):
        for p in pats[(s, m)]:
            corpora[s].find_all_async(p, out, counts_dev[k:k + 1], work, None, stream)
            k += 1
        ev[ci + 1].record(stream)
    torch.cuda.synchronize()
    cell_gbs = {c: round(n * args.per_cell / (ev[ci].elapsed_time(ev[ci + 1]) / 1e3) / 1e9, 1)
                for ci, c in enumerate(keys)}

    # ---- CPU baseline: the oracle on host cores, plus full-size parity --------
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        threads = args.cpu_threads or min(16, os.cpu_count() or 1)
        sample = [(s, m, pats[(s, m)][0]) for s in SIGMAS for m in MS]
        tc = time.perf_counter()
        mismatches = 0
        for s, m, p in sample:
            want = oracle.find_all(host_texts[s], p, threads=threads)
            g = torch.empty(max(want.size, 1), dtype=torch.int64, device=dev)
            dc = torch.zeros(1, dtype=torch.int64, device=dev)
            corpora[s].find_all_async(p, g, dc, work, None, stream)
            torch.cuda.synchronize()
            if int(dc.item()) != want.size or not np.array_equal(g[:want.size].cpu().numpy(), want):
                mismatches += 1
        # the GPU checks above are not timed separately; time the oracle alone
        t_or = 0.0
        for s, m, p in sample:
            ta = time.perf_counter()
            oracle.find_all(host_texts[s], p, threads=threads)
            t_or += time.perf_counter() - ta
        cpu = {"value": round(n * len(sample) / t_or / 1e9, 3), "unit": "GB/s", "cores": threads,
               "kind": "oracle",
               "sample": "naive oracle find_all, one pattern per (sigma, m) cell of the sweep "
                         "(50 patterns) over the full 2^30-byte texts, %d threads" % threads,
               "seconds": round(t_or, 2), "fullsize_parity_mismatches": mismatches}
        log("cpu baseline: %.2f GB/s on %d threads (%.1fs); full-size parity mismatches: %d" %
            (cpu["value"], threads, t_or, mismatches))
        if mismatches:
            raise SystemExit("full-size parity failed on %d patterns" % mismatches)

    skewed = None
    if not args.no_skewed:
        skewed = skewed_section(args, dev, stream)

    batched = None
    if not args.no_batched:
        del corpora
        torch.cuda.empty_cache()
        batched = batched_section(args, dev, stream)

    batched_waves = None
    if not args.no_batched_find_all:
        torch.cuda.empty_cache()
        batched_waves = batched_find_all_section(args, dev)

    serving = None
    if not args.no_serving:
        torch.cuda.empty_cache()
        serving = serving_section(args, dev)

    res = {
        "metric": METRIC, "value": round(gbs, 1), "unit": "GB/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": "single-pattern sweep, one launch per pattern: n=2^%d uniform "
                               "sigma in %s, m in %s, %d substring patterns per cell, find_all "
                               "(count -> tile scan -> emit)" % (args.n_log2, list(SIGMAS), list(MS),
                                                              args.per_cell),
                   "text_bytes_per_step": bytes_per_step, "occurrences_per_step": occ_total},
        "pct_hbm_peak": round(100 * gbs / HBM_PEAK_GBS, 2),
        "roofline": roofline,
        "cpu_baseline": cpu,
        "cells_gbs": cell_gbs,
        "sigma_eff": sigma_eff,
        "skewed": skewed,
        "batched": batched,
        "serving": serving,
        "paper_context": PAPER_CONTEXT,
    }
    if batched_waves is not None:
        res["batched_find_all"] = batched_waves
    print(json.dumps(res), flush=True)


def skewed_section(args, dev, stream):
    """Skewed and adversarial texts at n = 2^30, m in {4, 16, 64, 256}:
    (a) order-0 Zipf(s=1.0) over 64 symbols (text seed 1), 20 substring patterns per m
        (pattern seed 2): text GB/s per m, find_all totals equal to count-pass totals;
    (b) t = a^n with b at every index = 4095 mod 4096, p = a^(m-1) b: exactly 2^18 hits, at
        4096 k + 4096 - m;
    (c) t = a^n, p = a^m: n - m + 1 hits (8 GiB of positions), at 0 .. n - m.
    (b) and (c) are checked against their closed forms on the device; each is timed over 3
    calls after one warm-up, and reports text GB/s and (n + 8 occ)/t."""
    import numpy as np
    import torch

    import datagen as dg
    import paper_1012_2547_amd as sm

    n = 1 << args.skewed_n_log2
    ms = (4, 16, 64, 256)
    work = torch.empty(sm.workspace_size_upto(n, max(ms)), dtype=torch.uint8, device=dev)
    dc = torch.zeros(1, dtype=torch.int64, device=dev)

    def timed(corpus, pats, out, reps=1):
        for p in pats[:2]:
            corpus.find_all_async(p, out, dc, work, None, stream)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            for p in pats:
                corpus.find_all_async(p, out, dc, work, None, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / 1e3 / reps

    res = {}
    # (a) Zipf
    h = dg.zipf_text(n, 64, 1.0, seed=TEXT_SEED)
    text = torch.from_numpy(h).to(dev)
    c = sm.Corpus(text)
    sig = c.stats()[2]
    cells = {}
    for m in ms:
        pats = [dg.substring_pattern(h, m, seed=PAT_SEED, idx=j)[0] for j in range(args.per_cell)]
        cnt = torch.zeros(len(pats), dtype=torch.int64, device=dev)
        for k, p in enumerate(pats):
            c.count_async(p, cnt[k:k + 1], work, None, stream)
        torch.cuda.synchronize()
        counts = cnt.cpu().numpy()
        out = torch.empty(max(int(counts.max()), 1), dtype=torch.int64, device=dev)
        fcnt = torch.zeros(len(pats), dtype=torch.int64, device=dev)
        for k, p in enumerate(pats):
            c.find_all_async(p, out, fcnt[k:k + 1], work, None, stream)
        torch.cuda.synchronize()
        if not np.array_equal(fcnt.cpu().numpy(), counts):
            raise SystemExit("zipf text: find_all totals differ from count totals at m = %d" % m)
        dt = timed(c, pats, out)
        cells["m%d" % m] = {"gbs": round(n * len(pats) / dt / 1e9, 1),
                            "mean_occ": int(counts.mean()),
                            "algo": sm.plan_query(pats[0], sm.opts(sigma_hint=int(round(sig))))["algo"]}
        del out
    c.close()
    del text, h
    res["zipf64_s1"] = {"sigma_eff": round(sig, 2), "cells": cells}
    # (b) and (c): one resident text of 'a' bytes, then b every 4096 bytes
    text = torch.full((n,), 0x61, dtype=torch.uint8, device=dev)
    out = torch.empty(n, dtype=torch.int64, device=dev)

    def check(cnt_want, first, step):
        got = int(dc.item())
        if got != cnt_want:
            return False
        chunk = 1 << 27
        for a in range(0, got, chunk):
            b = min(got, a + chunk)
            want = torch.arange(a, b, dtype=torch.int64, device=dev) * step + first
            if not torch.equal(out[a:b], want):
                return False
        return True

    for name, periodic in (("a_n", False), ("a_n_with_b_every_4096", True)):
        if periodic:
            text[4095::4096] = 0x62
        c = sm.Corpus(text)
        cells = {}
        for m in ms:
            p = b"a" * (m - 1) + b"b" if periodic else b"a" * m
            occ = n // 4096 if periodic else n - m + 1
            dt = timed(c, [p], out[:occ], reps=3)
            c.find_all_async(p, out[:occ], dc, work, None, stream)
            torch.cuda.synchronize()
            ok = check(occ, 4096 - m, 4096) if periodic else check(occ, 0, 1)
            if not ok:
                raise SystemExit("%s: positions differ from the closed form at m = %d" % (name, m))
            cells["m%d" % m] = {"gbs": round(n / dt / 1e9, 1), "occ": occ,
                                "algorithmic_gbs": round((n + 8 * occ) / dt / 1e9, 1)}
        c.close()
        res[name] = {"closed_form_parity": True, "cells": cells}
    del text, out
    log("skewed: zipf %s; a^n with b: %s; a^n: %s" % (
        {k: v["gbs"] for k, v in res["zipf64_s1"]["cells"].items()},
        {k: v["gbs"] for k, v in res["a_n_with_b_every_4096"]["cells"].items()},
        {k: v["algorithmic_gbs"] for k, v in res["a_n"]["cells"].items()}))
    return res


def batched_section(args, dev, stream):
    """Batched multi-pattern counting: n = 2^32 uniform over 4 symbols (text seed 1),
    P = 4096 patterns with m log-uniform in [2, 1024] (seed 3), patterns 0..P/2-1
    substrings of the text and the rest i.i.d. random; one batched call vs P plain
    single-pattern calls on the same resident text. Counts must agree exactly."""
    import numpy as np
    import torch

    import datagen as dg
    import paper_1012_2547_amd as sm

    n = 1 << args.batched_n_log2
    P = args.batched_patterns
    t0 = time.time()
    h = dg.uniform_text(n, 4, seed=TEXT_SEED)
    text = torch.from_numpy(h).to(dev)
    ms = dg.log_uniform_lengths(P, 2, 1024, seed=3)
    pats = [dg.substring_pattern(h, int(m), seed=3, idx=i)[0] if i < P // 2
            else dg.random_pattern(int(m), 4, seed=3, idx=i) for i, m in enumerate(ms)]
    del h
    corpus = sm.Corpus(text)
    log("batched: inputs ready in %.1fs" % (time.time() - t0))
    work = torch.empty(corpus.batch_workspace_size(pats), dtype=torch.uint8, device=dev)
    d_b = torch.zeros(P, dtype=torch.int64, device=dev)
    corpus.batch_count_async(pats, d_b, work, stream)  # warm-up
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 2
    e0.record(stream)
    for _ in range(reps):
        corpus.batch_count_async(pats, d_b, work, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    t_batch = e0.elapsed_time(e1) / 1e3 / reps
    # the shared multi-pattern filter (mq_count_kernel) timed with HIP events on the
    # stream it runs on, in passes of their own
    sm.prof_collect()
    sm.prof_enable(True, every=1)
    for _ in range(reps):
        corpus.batch_count_async(pats, d_b, work, stream)
    torch.cuda.synchronize()
    sm.prof_enable(False)
    pr = sm.prof_collect()
    filt_s = pr["filter_ms"] / max(pr["filter_launches"], 1) / 1e3
    ctr = load_counters("mq_count")
    roof = {"bound": "alu", "unit": "TOP/s", "peak": round(VALU_PEAK_TOPS, 2),
            "kernel": "mq_count_kernel (shared multi-pattern q-gram filter)",
            "launches": pr["filter_launches"], "avg_launch_us": round(filt_s * 1e6, 1),
            "filter_share_of_pass": round(pr["filter_ms"] / max(pr["batch_ms"], 1e-9), 3),
            "filter_pattern_GBps": round(pr["filter_pattern_bytes"] / max(pr["filter_ms"], 1e-9) / 1e6, 1),
            "achieved": None, "frac": None, "traffic": None, "counters": None}
    if ctr and filt_s > 0:
        # VALU lane-operations issued per launch (SQ_INSTS_VALU x 64) over the live duration
        ops = ctr["valu_insts_per_launch"] * 64
        roof["achieved"] = round(ops / filt_s / 1e12, 2)
        roof["frac"] = round(ops / filt_s / 1e12 / VALU_PEAK_TOPS, 4)
        roof["traffic"] = ctr.get("bytes_per_launch")
        roof["counters"] = {k: ctr[k] for k in ("valu_insts_per_launch", "lds_insts_per_launch",
                                                "lds_bank_conflict_cycles_per_launch",
                                                "gui_active_cycles_per_launch") if k in ctr}
    log("batched: filter %d launches, %.1f us avg, %.0f%% of the count pass" % (
        roof["launches"], roof["avg_launch_us"], 100 * roof["filter_share_of_pass"]))
    # plain: one single-pattern count per pattern
    w1 = torch.empty(sm.workspace_size_upto(n, 1024), dtype=torch.uint8,
                     device=dev)
    d_p = torch.zeros(P, dtype=torch.int64, device=dev)
    for i in range(min(P, 64)):  # warm-up
        corpus.count_async(pats[i], d_p[i:i + 1], w1, None, stream)
    torch.cuda.synchronize()
    e0.record(stream)
    for i, p in enumerate(pats):
        corpus.count_async(p, d_p[i:i + 1], w1, None, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    t_plain = e0.elapsed_time(e1) / 1e3
    cb, cp = d_b.cpu().numpy(), d_p.cpu().numpy()
    agree = bool(np.array_equal(cb, cp))
    log("batched: %d patterns x 2^%d bytes: batched %.3fs (%.0f pattern-GB/s), plain %.3fs "
        "(%.0f pattern-GB/s), counts agree: %s" % (P, args.batched_n_log2, t_batch,
                                                   P * n / t_batch / 1e9, t_plain,
                                                   P * n / t_plain / 1e9, agree))
    if not agree:
        raise SystemExit("batched and plain counts differ")
    corpus.close()
    return {"workload": "n=2^%d uniform sigma=4, %d patterns m log-uniform [2,1024], half "
                        "substrings, count mode" % (args.batched_n_log2, P),
            "batched_s": round(t_batch, 4), "plain_s": round(t_plain, 4),
            "batched_pattern_GBps": round(P * n / t_batch / 1e9, 1),
            "plain_pattern_GBps": round(P * n / t_plain / 1e9, 1),
            "speedup_vs_plain": round(t_plain / t_batch, 2),
            "occurrences": int(cb.sum()), "counts_agree_with_plain": agree,
            "roofline": roof}


def batched_find_all_section(args, dev):
    """Every position of the batched workload (n = 2^32 uniform sigma=4, 4096 patterns,
    m log-uniform [2, 1024], half substrings): one count step (sm_batch_open), then
    the CSR output written in windows of 2^33 positions (64 GiB of device staging per
    wave). Pattern-bytes/s counts the count step and every wave. Sampled patterns'
    slices are compared with the plain single-pattern path wherever a wave holds
    them; the plain path (one find_all per pattern, all positions written) is timed
    on the same text."""
    import numpy as np
    import torch

    import datagen as dg
    import paper_1012_2547_amd as sm

    n = 1 << args.batched_n_log2
    P = args.batched_patterns
    h = dg.uniform_text(n, 4, seed=TEXT_SEED)
    text = torch.from_numpy(h).to(dev)
    ms = dg.log_uniform_lengths(P, 2, 1024, seed=3)
    pats = [dg.substring_pattern(h, int(m), seed=3, idx=i)[0] if i < P // 2
            else dg.random_pattern(int(m), 4, seed=3, idx=i) for i, m in enumerate(ms)]
    del h
    corpus = sm.Corpus(text)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b = corpus.batch_open(pats)
    torch.cuda.synchronize()
    t_count = time.perf_counter() - t0
    off = b.offsets.astype(np.int64)
    total = b.total
    W = 1 << 33
    buf = torch.empty(min(W, max(total, 1)), dtype=torch.int64, device=dev)
    # sampled patterns: every 128th, plus the largest output
    sample = sorted(set(list(range(0, P, 128)) + [int(np.argmax(off[1:] - off[:-1]))]))
    stream = torch.cuda.current_stream()
    checked = mismatched = 0
    t_waves = 0.0
    nw = 0
    for lo in range(0, total, W):
        hi = min(total, lo + W)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        b.write_async(lo, hi, buf[:hi - lo], stream)
        torch.cuda.synchronize()
        t_waves += time.perf_counter() - t1
        nw += 1
        for i in sample:
            a0, a1 = max(off[i], lo), min(off[i + 1], hi)
            if a0 >= a1:
                continue
            single = sm.find_all(text, pats[i])
            got = buf[a0 - lo:a1 - lo]
            ref = single[a0 - off[i]:a1 - off[i]]
            checked += 1
            if not torch.equal(got, ref):
                mismatched += 1
            del single
    t_total = t_count + t_waves
    b.close()
    del buf
    # plain path: one single-pattern find_all per pattern on the same resident text,
    # each into a buffer of its own count (every position written, as above)
    counts = off[1:] - off[:-1]
    out = torch.empty(max(int(counts.max()), 1), dtype=torch.int64, device=dev)
    work = torch.empty(sm.workspace_size_upto(n, 1024), dtype=torch.uint8, device=dev)
    dc = torch.zeros(1, dtype=torch.int64, device=dev)
    for p in pats[:64]:  # warm-up
        corpus.find_all_async(p, out, dc, work, None, stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for p in pats:
        corpus.find_all_async(p, out, dc, work, None, stream)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t1
    del out, work
    log("batched find_all: %d positions (%.1f GiB) in %d waves; count %.3fs + waves %.3fs; "
        "%.0f pattern-GB/s; %.0f GB/s of positions; plain path %.3fs; sampled slices %d, mismatches %d" % (
            total, total * 8 / 2**30, nw, t_count, t_waves, P * n / t_total / 1e9,
            total * 8 / t_waves / 1e9 if t_waves else 0, t_plain, checked, mismatched))
    corpus.close()
    if mismatched:
        raise SystemExit("batched find_all disagrees with the plain path on %d slices" % mismatched)
    return {"workload": "n=2^%d uniform sigma=4, %d patterns m log-uniform [2,1024], find_all in "
                        "waves of 2^33 positions" % (args.batched_n_log2, P),
            "positions": total, "waves": nw, "count_s": round(t_count, 3), "waves_s": round(t_waves, 3),
            "pattern_GBps": round(P * n / t_total / 1e9, 1),
            "positions_GBps": round(total * 8 / t_waves / 1e9, 1) if t_waves else None,
            "plain_s": round(t_plain, 3), "speedup_vs_plain": round(t_plain / t_total, 2),
            "sampled_slices": checked, "mismatches": mismatched}


def _digest(pos) -> tuple:
    """(count, first, last, sum of 64 evenly strided positions): cheap order-sensitive
    summary used to compare the server's answer with the plain path's."""
    k = int(pos.size)
    if k == 0:
        return (0, -1, -1, 0)
    return (k, int(pos[0]), int(pos[-1]), int(pos[::max(1, k // 64)].sum()))


def _pct(v, p):
    import numpy as np
    return float(np.percentile(np.asarray(v, dtype=np.float64), p, method="higher")) if len(v) else None


def serving_section(args, dev):
    """Open-loop serving: three resident corpora (uniform sigma=4 of 8 GiB seed 11,
    uniform sigma=20 of 2 GiB seed 12 (protein-like), Zipf(s=1.1) over 256 symbols
    of 4 GiB seed 13); per arrival rate a Poisson trace of min(20000, max(2000, rate x T))
    queries (seed 14 + rate index), corpus uniform, m log-uniform in [4, 256], even
    queries substrings of their corpus and odd ones i.i.d. random over its
    alphabet. Latency = arrival -> positions in host memory. The prefix of each
    trace is replayed through the plain path (one synchronous find_all per query,
    in arrival order) and both answers must agree exactly (digest of every query)."""
    import threading

    import numpy as np
    import torch

    import datagen as dg
    import paper_1012_2547_amd as sm

    t0 = time.time()
    sh = args.serve_shift
    specs = [("uniform sigma=4", 33 + sh, 4, lambda n: dg.uniform_text(n, 4, seed=11)),
             ("uniform sigma=20", 31 + sh, 20, lambda n: dg.uniform_text(n, 20, seed=12)),
             ("zipf K=256 s=1.1", 32 + sh, 256, lambda n: dg.zipf_text(n, 256, 1.1, seed=13))]
    hosts, corpora, names = [], [], []
    for name, lg, _, gen in specs:
        h = gen(1 << lg)
        hosts.append(h)
        corpora.append(sm.Corpus(torch.from_numpy(h).to(dev)))
        names.append("%s n=2^%d" % (name, lg))
    sig = [sp[2] for sp in specs]
    rates = [float(x) for x in args.serve_rates.split(",") if x]
    traces = []
    for k, lam in enumerate(rates):
        N = int(min(20000, max(args.serve_min_queries, round(lam * args.serve_seconds))))
        seed = 14 + k
        arr = dg.poisson_arrivals(N, lam, seed)
        cs = dg.choices(N, len(corpora), seed)
        ms = dg.log_uniform_lengths(N, 4, 256, seed)
        qs = []
        for i in range(N):
            c, m = int(cs[i]), int(ms[i])
            p = (dg.substring_pattern(hosts[c], m, seed, i)[0] if i % 2 == 0
                 else dg.random_pattern(m, sig[c], seed, i))
            qs.append((c, p))
        traces.append((lam, arr, qs))
    del hosts
    log("serving: corpora and %d queries ready in %.1fs" % (sum(len(t[2]) for t in traces),
                                                           time.time() - t0))

    srv = sm.Server(host_bytes=8 << 30)
    ids = [srv.add_corpus(c) for c in corpora]
    out = {"workload": "3 resident corpora (%s); Poisson arrivals; m log-uniform [4,256]; half "
                       "substrings, half random; latency = arrival -> positions on host"
                       % "; ".join(names),
           "server": {"slots": 2, "max_batch": 256, "pool_GiB": 16, "host_arena_GiB": 8},
           "rates": []}

    def replay_server(arr, qs):
        N = len(qs)
        tickets = [0] * N
        digests = [None] * N
        lat = np.zeros(N, dtype=np.int64)
        bsz = np.zeros(N, dtype=np.int64)
        sem = threading.Semaphore(0)
        start = sm.now_ns() + 20_000_000
        sched = start + (arr * 1e9).astype(np.int64)

        def submitter():
            for i in range(N):
                t = int(sched[i])
                while True:
                    d = t - sm.now_ns()
                    if d <= 0:
                        break
                    if d > 300_000:
                        time.sleep((d - 200_000) / 1e9)
                tickets[i] = srv.submit(ids[qs[i][0]], qs[i][1], t)
                sem.release()

        th = threading.Thread(target=submitter)
        th.start()
        for i in range(N):
            sem.acquire()
            cnt, pos, info = srv.wait(tickets[i])
            digests[i] = _digest(pos)
            lat[i] = info["done_ns"] - info["arrival_ns"]
            bsz[i] = info["batch_size"]
            srv.free(tickets[i])
        th.join()
        return lat, digests, bsz

    def replay_plain(arr, qs):
        N = len(qs)
        lat = np.zeros(N, dtype=np.int64)
        digests = [None] * N
        start = sm.now_ns() + 20_000_000
        sched = start + (arr[:N] * 1e9).astype(np.int64)
        for i in range(N):
            t = int(sched[i])
            while sm.now_ns() < t:
                d = t - sm.now_ns()
                if d > 300_000:
                    time.sleep((d - 200_000) / 1e9)
            c, p = qs[i]
            pos = corpora[c].find_all(p)  # synchronous: count, then positions to the host
            lat[i] = sm.now_ns() - t
            digests[i] = _digest(pos)
        return lat, digests

    # warm-up: one query per corpus through both paths
    for c in range(len(corpora)):
        srv.result(srv.submit(ids[c], b"\x01\x02\x03\x00"))
        corpora[c].find_all(b"\x01\x02\x03\x00")
    for lam, arr, qs in traces:
        srv.reset_stats()
        t1 = time.time()
        lat, dig, bsz = replay_server(arr, qs)
        st = srv.stats()
        wall = time.time() - t1
        K = min(len(qs), args.plain_queries)
        plat, pdig = replay_plain(arr, qs[:K])
        agree = all(a == b for a, b in zip(dig[:K], pdig))
        span_s = st["span_ns"] / 1e9 if st["span_ns"] else wall
        row = {
            "rate_qps": lam, "queries": len(qs),
            "p50_ms": round(st["p50_ns"] / 1e6, 3), "p99_ms": round(st["p99_ns"] / 1e6, 3),
            "p999_ms": round(st["p999_ns"] / 1e6, 3), "max_ms": round(st["max_ns"] / 1e6, 3),
            "achieved_qps": round(st["qps"], 1),
            "pattern_GBps": round(st["text_bytes"] / span_s / 1e9, 1),
            "out_GBps": round(st["out_bytes"] / span_s / 1e9, 2),
            "batches": st["batches"], "mean_batch": round(float(bsz.mean()), 1),
            "write_waves": st["write_waves"], "deferred": st["deferred"], "evicted": st["evicted"],
            "rejected": st["rejected"], "mem_waits": st["mem_waits"],
            "host_peak_GiB": round(st["host_peak_bytes"] / 2**30, 3),
            "host_arena_GiB": round(st["host_arena_bytes"] / 2**30, 3),
            "graph_launches": st["graph_launches"], "graph_builds": st["graph_builds"],
            "prefix": {"queries": K,
                       "server_p50_ms": round(_pct(lat[:K], 50) / 1e6, 3),
                       "server_p99_ms": round(_pct(lat[:K], 99) / 1e6, 3),
                       "plain_p50_ms": round(_pct(plat, 50) / 1e6, 3),
                       "plain_p99_ms": round(_pct(plat, 99) / 1e6, 3)},
            "alone_vs_in_mix_agree": bool(agree),
        }
        log("serving %6.0f qps: %5d queries, p50 %.2f ms p99 %.2f ms p999 %.2f ms, achieved %.0f qps, "
            "%.0f pattern-GB/s, mean batch %.1f; prefix %d: server p99 %.2f ms vs plain p99 %.2f ms; "
            "agree %s" % (lam, len(qs), row["p50_ms"], row["p99_ms"], row["p999_ms"],
                          row["achieved_qps"], row["pattern_GBps"], row["mean_batch"], K,
                          row["prefix"]["server_p99_ms"], row["prefix"]["plain_p99_ms"], agree))
        if not agree:
            raise SystemExit("server and plain path disagree at rate %g" % lam)
        out["rates"].append(row)
    srv.close()
    # the lowest rate's trace again with direct launches instead of HIP graphs
    lam, arr, qs = traces[0]
    srv = sm.Server(host_bytes=8 << 30, graphs=False)
    ids = [srv.add_corpus(c) for c in corpora]
    srv.reset_stats()
    lat, dig, _ = replay_server(arr, qs)
    st = srv.stats()
    srv.close()
    out["graphs_ab"] = {"rate_qps": lam, "queries": len(qs),
                        "graphs_p50_ms": out["rates"][0]["p50_ms"], "graphs_p99_ms": out["rates"][0]["p99_ms"],
                        "direct_p50_ms": round(st["p50_ns"] / 1e6, 3), "direct_p99_ms": round(st["p99_ns"] / 1e6, 3)}
    log("serving %g qps with direct launches: p50 %.2f ms p99 %.2f ms (graphs: %.2f / %.2f)" % (
        lam, st["p50_ns"] / 1e6, st["p99_ns"] / 1e6, out["rates"][0]["p50_ms"], out["rates"][0]["p99_ms"]))
    for c in corpora:
        c.close()
    return out


if __name__ == "__main__":
    main()
