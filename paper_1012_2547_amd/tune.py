"""Autotuner for the planner's (alphabet size, pattern length) -> kernel table.

For each alphabet-size bucket (representative sigma in 2, 4, 16, 64, 256) and a
grid of pattern lengths, every applicable configuration -- algorithm (Shift-And, beyond
m = 49 in its suffix form; BNDM and BNDMq; SBNDM and SBNDMq, beyond m = 64 in their
factor form; forward SBNDM; Hash-q with its gram length q; the block filter; brute
force), starts per lane
and tiles per workgroup -- is timed on an i.i.d. uniform text (tuning seed 2, distinct from the
benchmark's seed 1) with substring patterns, as whole find_all calls. The
fastest configuration of each cell becomes a table entry. The paper's own
summary (Section 3) says the best algorithm depends on exactly these two
quantities; this measures that map on MI355X.

    python -m paper_1012_2547_amd.tune --out tune_out --n-log2 30   # on a GPU
writes tune.json (entries + timings) and tune_table.inc (C initialisers for
csrc/tune_table.inc). With --sigmas / --ms only those cells are measured again
and the others are taken from --base (a tune.json of the same grid).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

SIGMAS = (2, 4, 16, 64, 256)
SIGMA_RANGES = {2: (1, 2), 4: (3, 7), 16: (8, 31), 64: (32, 127), 256: (128, 256)}
M_GRID = (1, 2, 3, 4, 6, 8, 9, 12, 16, 24, 32, 48, 64, 65, 96, 128, 144, 192, 256, 384, 512, 768, 1024)
QS = (2, 3, 4, 5, 6, 8, 10, 12, 16)


def candidates(m: int, sigma: int):
    """Every option is explicit (plain BNDM and SBNDM are q = 1), so that no entry of the
    library's built-in table fills in a value left at 0."""
    out = []
    if m <= 64:
        for algo in (1, 2, 3):
            for L in (32, 64, 128):
                for tpw in (1, 2, 4):
                    out.append(dict(algo=algo, lane_bytes=L, q=1 if algo in (2, 3) else 0, tiles_per_wg=tpw))
        if m <= 8:  # brute force over packed bytes
            for L in (32, 64, 128):
                for tpw in (1, 2, 4):
                    out.append(dict(algo=6, lane_bytes=L, q=0, tiles_per_wg=tpw))
        for q in (2, 4, 8):  # SBNDMq: the window's last q bytes read at once
            if q > m:
                continue
            for L in (32, 64, 128):
                for tpw in (1, 2, 4):
                    out.append(dict(algo=3, lane_bytes=L, q=q, tiles_per_wg=tpw))
        if m >= 8:
            for q in (2, 4):  # BNDMq: the window's last q bytes read at once
                for L in (32, 64, 128):
                    for tpw in (1, 2, 4):
                        out.append(dict(algo=2, lane_bytes=L, q=q, tiles_per_wg=tpw))
            if m <= 63:  # forward SBNDM: one extra bit for the look-ahead byte
                for L in (32, 64, 128):
                    for tpw in (1, 2, 4):
                        out.append(dict(algo=7, lane_bytes=L, q=0, tiles_per_wg=tpw))
    if m > 64:  # Shift-And's suffix form: the last 17 (or 49) bytes scanned, the rest verified
        for L in (64, 128):
            for tpw in (1, 2):
                out.append(dict(algo=1, lane_bytes=L, q=0, tiles_per_wg=tpw))
    if m > 64:  # SBNDM's factor form: the last 64 bytes searched, the rest verified
        for q in (1, 2, 4, 8):
            for L in (64, 128):
                for tpw in (1, 2):
                    out.append(dict(algo=3, lane_bytes=L, q=q, tiles_per_wg=tpw))
    for q in QS:
        if q > m or sigma ** q < m:  # too few distinct q-grams to skip anything
            continue
        for L in (64, 128):
            for tpw in (1, 2):
                out.append(dict(algo=4, lane_bytes=L, q=q, tiles_per_wg=tpw))
    if 144 <= m <= 4096:  # block filter: its tile is 256 sampled blocks
        for tpw in (1, 2, 4, 8):
            out.append(dict(algo=5, lane_bytes=0, q=0, tiles_per_wg=tpw))
    return out


def write_json(f, d):
    """The tuner's record, one table entry and one cell (with every candidate's timing)
    per line."""
    f.write('{"n": %d, "device": %s,\n"entries": [\n' % (d["n"], json.dumps(d["device"])))
    f.write(",\n".join(json.dumps(e) for e in d["entries"]))
    f.write('\n],\n"cells": [\n')
    f.write(",\n".join(json.dumps(c) for c in d["cells"]))
    f.write("\n]}\n")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default="tune_out")
    ap.add_argument("--n-log2", type=int, default=30)
    ap.add_argument("--patterns", type=int, default=6)
    ap.add_argument("--reps", type=int, default=2)
    ap.add_argument("--sigmas", type=str, default="", help="comma-separated subset of the alphabet buckets")
    ap.add_argument("--ms", type=str, default="", help="comma-separated subset of the pattern-length grid")
    ap.add_argument("--base", type=str, default="", help="tune.json holding the cells not measured")
    args = ap.parse_args()
    sigmas = tuple(int(x) for x in args.sigmas.split(",")) if args.sigmas else SIGMAS
    grid = tuple(int(x) for x in args.ms.split(",")) if args.ms else M_GRID
    if not set(sigmas) <= set(SIGMAS) or not set(grid) <= set(M_GRID):
        raise SystemExit("--sigmas / --ms must be taken from the grid")
    base = {}
    if args.base:
        with open(args.base) as f:
            for c in json.load(f)["cells"]:
                base[(c["sigma"], c["m"])] = c
    if (sigmas, grid) != (SIGMAS, M_GRID):
        missing = [(sg, m) for sg in SIGMAS for m in M_GRID
                   if (sg not in sigmas or m not in grid) and (sg, m) not in base]
        if missing:
            raise SystemExit("a subset needs --base with the other cells (missing %s)" % (missing[:3],))
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    import numpy as np
    import torch

    import datagen as dg
    import paper_1012_2547_amd as sm

    os.makedirs(args.out, exist_ok=True)
    dev = torch.device("cuda:0")
    n = 1 << args.n_log2
    stream = torch.cuda.current_stream()
    work = torch.empty(sm.workspace_size_upto(n, 1024, sm.opts(lane_bytes=32)), dtype=torch.uint8,
                       device=dev)
    dc = torch.zeros(1, dtype=torch.int64, device=dev)
    results = []
    t_start = time.time()
    for sigma in sigmas:
        h = dg.uniform_text(n, sigma, seed=2)
        text = torch.from_numpy(h).to(dev)
        for m in grid:
            pats = [dg.substring_pattern(h, m, seed=3, idx=j)[0] for j in range(args.patterns)]
            counts = []
            for p in pats:
                sm.count_async(text, p, dc, work, None, stream)
                counts.append(int(dc.item()))
            out = torch.empty(max(max(counts), 1), dtype=torch.int64, device=dev)
            best = None
            cell = []
            for cand in candidates(m, sigma):
                o = sm.opts(algo=cand["algo"], lane_bytes=cand["lane_bytes"], q=cand["q"],
                            tiles_per_wg=cand["tiles_per_wg"], sigma_hint=sigma)
                for p in pats:  # warm-up
                    sm.find_all_async(text, p, out, dc, work, o, stream)
                torch.cuda.synchronize()
                sm.prof_collect()
                sm.prof_enable(True)
                for _ in range(args.reps):
                    for p in pats:
                        sm.find_all_async(text, p, out, dc, work, o, stream)
                torch.cuda.synchronize()
                sm.prof_enable(False)
                pr = sm.prof_collect()
                us = pr["total_ms"] * 1e3 / max(pr["calls"], 1)
                gbs = n / (us * 1e-6) / 1e9
                rec = dict(cand, us=round(us, 2), gbs=round(gbs, 1),
                           count_us=round(pr["count_ms"] * 1e3 / max(pr["calls"], 1), 2))
                cell.append(rec)
                if best is None or us < best["us"]:
                    best = rec
            results.append(dict(sigma=sigma, m=m, best=best, all=cell))
            print("sigma=%3d m=%4d best %-9s L=%3d q=%2d tpw=%d  %.1f GB/s  (%.0fs)" % (
                sigma, m, sm.ALGO_NAMES[best["algo"]], best["lane_bytes"], best["q"],
                best["tiles_per_wg"], best["gbs"], time.time() - t_start), flush=True)
        del text
        torch.cuda.empty_cache()

    measured = {(r["sigma"], r["m"]) for r in results}
    results += [c for k, c in base.items() if k not in measured]
    results.sort(key=lambda r: (SIGMAS.index(r["sigma"]), M_GRID.index(r["m"])))
    entries = []
    for r in results:
        i = M_GRID.index(r["m"])
        m_hi = M_GRID[i + 1] - 1 if i + 1 < len(M_GRID) else 0xFFFFFFFF
        lo, hi = SIGMA_RANGES[r["sigma"]]
        b = r["best"]
        entries.append(dict(sigma_lo=lo, sigma_hi=hi, m_lo=r["m"], m_hi=m_hi, algo=b["algo"],
                            lane_bytes=b["lane_bytes"], q=b["q"], tiles_per_wg=b["tiles_per_wg"],
                            hbits=0, gbs=b["gbs"]))
    with open(os.path.join(args.out, "tune.json"), "w") as f:
        write_json(f, {"n": n, "device": torch.cuda.get_device_name(0), "entries": entries,
                       "cells": results})
    with open(os.path.join(args.out, "tune_table.inc"), "w") as f:
        f.write("// generated by paper_1012_2547_amd/tune.py on %s, n = 2^%d, tuning seed 2\n"
                % (torch.cuda.get_device_name(0), args.n_log2))
        f.write("// {sigma_lo, sigma_hi, m_lo, m_hi, algo, lane_bytes, q, tiles_per_wg, hbits, 0}"
                "  measured GB/s\n")
        for e in entries:
            f.write("    {%d, %d, %du, %du, %d, %d, %d, %d, %d, 0},  // %.1f\n" % (
                e["sigma_lo"], e["sigma_hi"], e["m_lo"], e["m_hi"], e["algo"], e["lane_bytes"],
                e["q"], e["tiles_per_wg"], e["hbits"], e["gbs"]))
    print("wrote %s (%d entries) in %.0fs" % (args.out, len(entries), time.time() - t_start))


if __name__ == "__main__":
    main()
