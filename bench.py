#!/usr/bin/env python3
"""Throughput of the seed filter on one MI355X: query Mbp searched per second.

One step is one pass of the whole search path (window setup, fused hit
gather / prefilter / exact shared counts / seeds, chaining, sorted
candidates) over the query span, with the index already resident in HBM.
The default workload is the 50 Mbp chromosome-shaped synthetic assembly
(41% GC, 45% soft-masked repeats, 2,000 planted duplications, 10 runs of N)
searched against itself as one span with k = 12, w = 16, minimum length 1000
and error bound 0.25.

Prints one JSON line (rank 0).  Progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def workload(name):
    from paper_1807_00205_amd import synth
    if name == "chromosome50":
        g = synth.config2()
        desc = ("50 Mbp chromosome-shaped assembly (41% GC, 45% soft-masked repeats, "
                "2,000 planted duplications of 1-50 kbp at 1-25%, 10 N-gaps of 50 kbp); "
                "whole-sequence self-search")
        return g, [g.spans[0]], desc
    if name == "uniform1":
        g = synth.config1()
        return g, [g.spans[0]], "1 Mbp uniform sequence with 20 planted duplications; self-search"
    raise SystemExit("unknown workload %s" % name)


def algorithmic_hits(ix):
    """Hits a whole-genome self-search must read once: for every eligible
    minimizer, every other eligible occurrence of its hash (both strands)."""
    import numpy as np
    h, _, _ = ix.entries()
    _, counts = np.unique(h, return_counts=True)
    c = counts.astype(np.int64)
    return int((c * c).sum() - c.sum())


def cpu_baseline(g, sample_mbp, max_error, min_len):
    import numpy as np
    import oracle
    b, off = g.concat()
    threads = max(1, min(16, os.cpu_count() or 1))
    t = time.time()
    orc = oracle.OracleIndex(b, off, 12, 16)
    build_s = time.time() - t
    L = len(g.seqs[0])
    span_len = min(L, int(sample_mbp * 1e6))
    a = (L - span_len) // 2
    t = time.time()
    orc.search([(0, a, a + span_len)], max_error, min_len, threads)
    dt = time.time() - t
    return {"value": round(span_len / dt / 1e6, 4), "unit": "Mbp/s", "cores": threads,
            "kind": "oracle",
            "sample": "span [%d, %d) of the same sequence (%.1f Mbp), search only; oracle "
                      "index built beforehand in %.1f s" % (a, a + span_len, span_len / 1e6,
                                                             build_s),
            "seconds": round(dt, 3)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="chromosome50")
    ap.add_argument("--max-error", type=float, default=0.25)
    ap.add_argument("--min-len", type=int, default=1000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-mbp", type=float, default=12.0)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the search path is built and timed on a single "
              "MI355X; use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1807_00205_amd import sdf

    torch.cuda.init()
    log("generating workload", args.workload)
    t = time.time()
    g, spans, desc = workload(args.workload)
    log("  %.1f s" % (time.time() - t))
    torch.cuda.synchronize()
    t = time.time()
    ix = sdf.Index(g.seqs, 12, 16)
    torch.cuda.synchronize()
    build_s = time.time() - t
    nm, ne, dev_bytes = ix.info()
    log("index built in %.2f s: %d minimizers, %d eligible, %.2f GB" % (build_s, nm, ne,
                                                                        dev_bytes / 1e9))
    span = spans[0]
    qbases = span[2] - span[1]
    alg_hits = algorithmic_hits(ix)
    for _ in range(args.warmup):
        r = ix.search(span, args.max_error, args.min_len, timing=True)
        ncand = len(r.candidates())
        stats = r.stats()
        r.close()
    torch.cuda.synchronize()
    kernel_ms, lat = [], []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        s0 = time.perf_counter()
        r = ix.search(span, args.max_error, args.min_len, timing=True)
        n = ctypes_count(r)
        lat.append((time.perf_counter() - s0) * 1e3)
        kernel_ms.append(float(r.timing()[1]))
        r.close()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    value = qbases * args.steps / dt / 1e6
    mean_k = float(np.mean(kernel_ms))
    # algorithmic bytes per launch: minimizer records (pos, hash, flags: 9 B),
    # two directory lookups per eligible query minimizer (8 B) and 4.125 B per
    # hit (position + strand bit)
    alg_bytes = nm * 9 + ne * 8 + alg_hits * 4.125
    achieved = alg_bytes / (mean_k * 1e-3) / 1e9
    out = {
        "metric": "query Mbp searched/sec (Jaccard filter)",
        "value": round(value, 3),
        "unit": "Mbp/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": desc, "query_bases": qbases, "k": 12, "w": 16,
                   "min_len": args.min_len, "max_error": args.max_error,
                   "path": "plain single-span search"},
        "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 4),
                       "p99": round(float(np.percentile(lat, 99)), 4)},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 5),
                     "traffic": None, "kernel": "k_tile_search",
                     "kernel_ms": round(mean_k, 4), "algorithmic_bytes": int(alg_bytes)},
        "detail": {"index_build_s": round(build_s, 3), "minimizers": nm, "eligible": ne,
                   "algorithmic_hits": alg_hits, "candidates": ncand, **stats},
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(g, args.cpu_sample_mbp, args.max_error, args.min_len)
    print(json.dumps(out), flush=True)


def ctypes_count(r):
    return len(r.candidates())


if __name__ == "__main__":
    main()
