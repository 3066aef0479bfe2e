#!/usr/bin/env python3
"""Throughput of the seed filter on one MI355X: query Mbp searched per second.

One step is one pass of the whole search path (window setup, fused hit
gather / prefilter / exact shared counts / seeds, chaining, sorted
candidates) over the query spans, with the index already resident in HBM.
The headline workload is the 3.1 Gbp synthetic assembly in 24 sequences
(41% GC, 50% soft-masked repeats, N-gaps, 5% of bases in planted
duplications) searched all-vs-all: the 24 whole sequences in one batched
search, with k = 12, w = 16, minimum length 1000 and error bound 0.25; the
same spans searched one call at a time are reported beside it.  The 50 Mbp
chromosome-shaped workload (plain single-span path), the 250 Mbp batch of
4,096 spans (batched against plain) and the serving sweep over that index
follow as further sections of the same JSON line.

Prints one JSON line.  Progress goes to stderr.
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


def measured_traffic(workload_name):
    """HBM bytes per launch of the tile kernel from the committed rocprofv3
    counter summary, or None if the kernel source changed since then."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic_k_tile_search_%s.json" % workload_name)
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        tr = json.load(fh)
    src = b"".join(open(os.path.join(ROOT, f), "rb").read() for f in tr["source_files"])
    if hashlib.sha256(src).hexdigest() != tr["source_sha256"]:
        return None
    return int(tr["traffic_bytes_per_launch"])


def cpu_baseline(g, sample_mbp, max_error, min_len, keep=None):
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
    _, cands = orc.search([(0, a, a + span_len)], max_error, min_len, threads)
    dt = time.time() - t
    if keep is not None:  # the oracle's own candidates, for the extension baseline
        keep.update(orc=orc, off=off, cands=cands, threads=threads, bytes=b)
    # one thread on a tenth of the span
    one = max(1, span_len // 10)
    t = time.time()
    orc.search([(0, a, a + one)], max_error, min_len, 1)
    dt1 = time.time() - t
    cpu = ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    cpu = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"value": round(span_len / dt / 1e6, 4), "unit": "Mbp/s", "cores": threads,
            "kind": "oracle",
            "sample": "span [%d, %d) of the same sequence (%.1f Mbp), search only; oracle "
                      "index built beforehand in %.1f s" % (a, a + span_len, span_len / 1e6,
                                                             build_s),
            "seconds": round(dt, 3),
            "single_thread_mbp_per_s": round(one / dt1 / 1e6, 4),
            "host_cpu": cpu, "host_threads_visible": os.cpu_count()}


def batched_vs_plain(steps, plain=True, cpu=True, max_error=0.25, min_len=1000):
    """4,096 spans of 1-100 kbp against the resident index of a 250 Mbp
    sequence: one batched search against the same spans searched one by one,
    with the tile kernel's roofline and the oracle's rate on a sample of the
    spans."""
    import numpy as np
    import torch
    from paper_1807_00205_amd import sdf, synth
    g = synth.config3()
    ix = sdf.Index(g.seqs, 12, 16)
    nm, ne, _ = ix.info()
    hbar = ix.hit_density()
    spans = g.spans
    qb = sum(e - b for _, b, e in spans)
    r = ix.search_batch(spans, timing=True)
    r.candidates()
    r.close()

    def timed():
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        kms = []
        for _ in range(steps):
            r = ix.search_batch(spans, timing=True)
            ncand = len(r.candidates())
            kms.append(float(r.timing()[1]))
            stats = r.stats()
            r.close()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps, kms, ncand, stats

    # the tile size from the hit-density rule, then the one sdf_autotune measures
    tb_rule, kms_rule, _, _ = timed()
    t0 = time.perf_counter()
    core, threads, tune_ms = ix.autotune(spans)
    tune_s = time.perf_counter() - t0
    # the measured schedule holds for this thread's searches from here on
    sdf.set_tuning(tile_core=core, tile_threads=threads)
    tb, kms, ncand, stats = timed()
    # the same batch captured once as a HIP graph and replayed
    stream = torch.cuda.Stream()
    t0 = time.perf_counter()
    plan = ix.plan(spans, stream=stream)
    plan_s = time.perf_counter() - t0
    r = plan.run(stream)
    r.candidates()
    r.close()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        r = plan.run(stream)
        ncand_g = len(r.candidates())
        r.close()
    torch.cuda.synchronize()
    tg = (time.perf_counter() - t0) / steps
    ginfo = plan.info()
    plan.close()
    lat = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for sp in (spans if plain else []):
        s0 = time.perf_counter()
        r = ix.search(sp)
        r.candidates()
        r.close()
        lat.append((time.perf_counter() - s0) * 1e3)
    torch.cuda.synchronize()
    tp = time.perf_counter() - t0
    sdf.set_tuning()  # back to the library's choices
    tuning = {"autotuned_core": core, "autotuned_threads": threads,
              "autotune_s": round(tune_s, 3),
              "tile_kernel_ms_per_schedule": {"%d threads, %d starts" % k: round(v, 3)
                                              for k, v in tune_ms.items()},
              "rule_mbp_per_s": round(qb / tb_rule / 1e6, 2),
              "rule_tile_kernel_ms": round(float(np.mean(kms_rule)), 4)}
    mean_k = float(np.mean(kms))
    alg = qb * alg_bytes_per_query_base(nm, ne, g.total, hbar)
    out = {"workload": "250 Mbp uniform sequence with %d planted duplications (1-5 kbp, "
                       "2-15%%); 4,096 query spans of 1-100 kbp (log-uniform), %.1f Mbp"
                       % (len(g.truth), qb / 1e6),
           "batched_mbp_per_s": round(qb / tb / 1e6, 2), "batched_ms": round(tb * 1e3, 3),
           "batched_tile_kernel_ms": round(mean_k, 4),
           "graph": {"path": "the same batch captured once as a HIP graph (sdf_plan_create) and "
                             "replayed (sdf_plan_run), candidates copied out each step",
                     "mbp_per_s": round(qb / tg / 1e6, 2), "ms": round(tg * 1e3, 3),
                     "capture_s": round(plan_s, 3), "candidates": ncand_g, **ginfo},
           "roofline": roofline(alg, mean_k, measured_traffic("batched250")),
           "hit_density": round(hbar, 4), "candidates": ncand, "stats": stats,
           "tuning": tuning}
    if plain:
        out.update({"plain_mbp_per_s": round(qb / tp / 1e6, 2), "plain_ms": round(tp * 1e3, 2),
                    "plain_latency_ms": {"p50": round(float(np.percentile(lat, 50)), 4),
                                         "p99": round(float(np.percentile(lat, 99)), 4)},
                    "speedup": round(tp / tb, 2)})
    if cpu:
        import oracle
        b, off = g.concat()
        threads_c = max(1, min(16, os.cpu_count() or 1))
        t = time.time()
        orc = oracle.OracleIndex(b, off, 12, 16)
        obuild = time.time() - t
        sample = spans[:512]
        sb = sum(e - b0 for _, b0, e in sample)
        t = time.time()
        orc.search(sample, max_error, min_len, threads_c)
        odt = time.time() - t
        orc.close()
        out["cpu_baseline"] = {"value": round(sb / odt / 1e6, 4), "unit": "Mbp/s",
                               "cores": threads_c, "kind": "oracle",
                               "sample": "the first 512 of the 4,096 spans (%.1f Mbp), search "
                                         "only; oracle index built beforehand in %.1f s"
                                         % (sb / 1e6, obuild),
                               "seconds": round(odt, 3)}
    return ix, g, out


def serving(ix, g, rates, seconds, workers):
    """Open-loop Poisson arrivals of spans of 1 kbp - 5 Mbp (log-uniform) over
    the resident 250 Mbp index: continuous batching vs one request at a time."""
    from paper_1807_00205_amd import serve, synth
    out = {"workload": "Poisson arrivals, spans 1 kbp - 5 Mbp (log-uniform) against the "
                       "resident 250 Mbp index", "workers": workers, "rates": {},
           "warm_up": "before each rate, 300 untimed requests at 1,000 req/s through both "
                      "servers (the library's per-stream memory pool reaches its sizes)"}
    for rate in rates:
        n = int(max(60, min(2000, rate * seconds)))
        warm = synth.poisson_requests(500 + int(rate), 1000.0, 300, [len(g.seqs[0])])
        serve.measure(ix, warm, workers=workers, max_batch=4096)
        serve.measure(ix, warm[:100], workers=1, max_batch=1)
        reqs = synth.poisson_requests(1000 + int(rate), rate, n, [len(g.seqs[0])])
        served = serve.measure(ix, reqs, workers=workers, max_batch=4096)
        plain = serve.measure(ix, reqs, workers=1, max_batch=1)
        out["rates"][str(rate)] = {"requests": n,
                                   "served": {k: round(v, 3) if isinstance(v, float) else v
                                              for k, v in served.items()},
                                   "plain_fifo": {k: round(v, 3) if isinstance(v, float) else v
                                                  for k, v in plain.items()}}
        log("  rate %s: served p50 %.2f p99 %.2f ms %.0f Mbp/s, plain p50 %.2f p99 %.2f ms "
            "%.0f Mbp/s" % (rate, served["p50_ms"], served["p99_ms"], served["mbp_per_s"],
                            plain["p50_ms"], plain["p99_ms"], plain["mbp_per_s"]))
    return out


def estimate_mode(ix, span, max_error, min_len, qbases, steps=3):
    """The same search with each run's seed chosen by the winnowed MinHash
    estimate: wall time per search, the estimate kernel's share, and the
    seed and candidate counts next to the shared-count seeds."""
    import numpy as np
    import torch
    r = ix.search(span, max_error, min_len, timing=True, estimate=True)
    ncand = len(r.candidates())
    nseed = r.stats()["seeds"]
    r.close()
    torch.cuda.synchronize()
    ts, tk, tc = [], [], []
    for _ in range(steps):
        t0 = time.perf_counter()
        r = ix.search(span, max_error, min_len, timing=True, estimate=True)
        ctypes_count(r)
        ts.append(time.perf_counter() - t0)
        tm = r.timing()
        tk.append(float(tm[1]))
        tc.append(float(tm[2]))
        r.close()
    dt = float(np.median(ts))
    return {"path": "plain single-span search, seeds by the estimate (SDF_SEED_ESTIMATE)",
            "mbp_per_s": round(qbases / dt / 1e6, 2), "ms_per_search": round(dt * 1e3, 3),
            "tile_kernel_ms": round(float(np.median(tk)), 3),
            "estimate_and_chaining_ms": round(float(np.median(tc)), 3),
            "seeds": nseed, "candidates": ncand}


def extend_mode(ix, span, max_error, min_len, steps=3, cpu=None, cpu_sample=200):
    """The same search with every candidate extended to a potential
    duplication region (Section 3.2, SDF_EXTEND): wall time per search, the
    extension's GPU time, regions per second, how far regions grew, and the
    oracle's extension rate on a seeded sample of its own candidates."""
    import numpy as np
    import torch
    from paper_1807_00205_amd import sdf
    r = ix.search(span, max_error, min_len, timing=True, extend=True)
    cands = r.candidates()
    reg = r.regions()
    st = r.stats(extension=True)
    r.close()
    torch.cuda.synchronize()
    ts, te, tk = [], [], []
    for _ in range(steps):
        t0 = time.perf_counter()
        r = ix.search(span, max_error, min_len, timing=True, extend=True)
        r.regions()
        ts.append(time.perf_counter() - t0)
        tm = r.timing()
        te.append(float(tm[5]))
        tk.append(float(tm[1]))
        r.close()
    ext_ms = float(np.median(te))
    before = (cands["q_end"] - cands["q_begin"]).astype(np.int64)
    after = (reg["q_end"] - reg["q_begin"]).astype(np.int64)
    stops = {}
    for c in (reg["stop"] & 255).tolist() + (reg["stop"] >> 8).tolist():
        name = {1: "sequence_end", 2: "length_cap", 3: "overlap", 4: "estimate"}.get(c, str(c))
        stops[name] = stops.get(name, 0) + 1
    out = {"path": "plain single-span search, every candidate extended (SDF_EXTEND, 1 Mbp cap)",
           "ms_per_search": round(float(np.median(ts)) * 1e3, 3),
           "tile_kernel_ms": round(float(np.median(tk)), 3),
           "extension_ms": round(ext_ms, 3),
           "regions": len(reg),
           "regions_per_s": round(len(reg) / (ext_ms * 1e-3), 1) if ext_ms > 0 else None,
           "insertions": st["ext_insertions"], "continued_attempts": st["ext_continued"],
           "ranked_hashes": st["ext_ranks"],
           "workgroup_ms": {"gather_and_rank": round(st["ext_rank_us"] / 1e3, 1),
                            "phases": round(st["ext_phase_us"] / 1e3, 1),
                            "slowest_region": round(st["ext_slowest_region_us"] / 1e3, 2)},
           "insertions_per_s": round(st["ext_insertions"] / (ext_ms * 1e-3), 1) if ext_ms > 0 else None,
           "region_len_median": [int(np.median(before)), int(np.median(after))],
           "region_len_max": [int(before.max()), int(after.max())] if len(reg) else [0, 0],
           "phase_stops": stops}
    # the q-gram filter of the same section on the extended regions (q and p_G
    # are not given by the paper: q = 5, p_G = 0.005 here)
    ix.qgram_filter(reg[:16], 5, 0.005, max_error)
    tq = []
    for _ in range(steps):
        t0 = time.perf_counter()
        _, ok = ix.qgram_filter(reg, 5, 0.005, max_error)
        tq.append(time.perf_counter() - t0)
    # final SDs of every extended region (Section 3.3)
    ix.align_regions(reg[:64])
    tf = []
    for _ in range(steps):
        t0 = time.perf_counter()
        fin, fops = ix.align_regions(reg, 11, min_len, max_error)
        tf.append(time.perf_counter() - t0)
    fms = float(np.median(tf)) * 1e3
    out["final_sds"] = {"regions": len(reg), "sds": len(fin), "ms_host_to_host": round(fms, 3),
                        "regions_per_s": round(len(reg) / (fms * 1e-3), 1),
                        "aligned_columns": int(fin["aln_len"].sum()),
                        "mean_identity": round(float((fin["matches"] / np.maximum(1, fin["aln_len"])).mean()), 4)
                        if len(fin) else None,
                        "cigar_ops": len(fops)}
    if cpu:
        import oracle
        rng = np.random.default_rng(2)
        sel = np.sort(rng.choice(len(reg), min(cpu_sample, len(reg)), replace=False))
        rr = reg[sel]
        qo = cpu["off"][rr["q_seq"]].astype(np.uint64)
        to = cpu["off"][rr["t_seq"]].astype(np.uint64)
        rows = np.stack([rr["q_begin"] + qo, rr["q_end"] + qo, rr["t_begin"] + to,
                         rr["t_end"] + to, rr["strand"].astype(np.uint64)], axis=1)
        t = time.time()
        oracle.sd_align(cpu["bytes"], cpu["off"], rows, 11, min_len, max_error, cpu["threads"],
                        pad_frac=sdf.PAD_FRAC)
        dt = time.time() - t
        out["final_sds"]["cpu_baseline"] = {
            "value": round(len(sel) / dt, 2), "unit": "regions/s", "cores": cpu["threads"],
            "kind": "oracle", "sample": "%d seeded random extended regions of this search" % len(sel),
            "seconds": round(dt, 3)}
    out["qgram_filter"] = {"q": 5, "gap_rate": 0.005,
                           "ms_host_to_host": round(float(np.median(tq)) * 1e3, 3),
                           "pass": int(ok.sum()), "regions": len(reg),
                           "bases_read": int(((reg["q_end"] - reg["q_begin"]) +
                                              (reg["t_end"] - reg["t_begin"])).sum())}
    if cpu:
        rng = np.random.default_rng(1)
        oc, off = cpu["cands"], cpu["off"]
        sel = np.sort(rng.choice(len(oc), min(cpu_sample, len(oc)), replace=False))
        c = oc[sel]
        qo = off[c["q_seq"]].astype(np.uint64)
        to = off[c["t_seq"]].astype(np.uint64)
        rows = np.stack([c["q_begin"] + qo, c["q_end"] + qo, c["t_begin"] + to, c["t_end"] + to,
                         c["strand"].astype(np.uint64)], axis=1)
        import oracle
        tau, _, _ = oracle.params(max_error, min_len, 12)
        t = time.time()
        cpu["orc"].extend(rows, tau, 1000000, cpu["threads"])
        dt = time.time() - t
        out["cpu_baseline"] = {"value": round(len(sel) / dt, 2), "unit": "regions/s",
                               "cores": cpu["threads"], "kind": "oracle",
                               "sample": "%d seeded random candidates of the oracle's search "
                                         "of the CPU-baseline span, extended" % len(sel),
                               "seconds": round(dt, 3)}
    return out


def sensitivity_trial_set(delta, trials, seed, max_error=0.25, min_len=1000, split="bounded"):
    """One delta of the simulated-sensitivity experiment (Section 4.1.1):
    `trials` pairs (uniform random X of 1-100 kbp, its duplicate Y with error
    delta), all in one index, each X searched against it in one batched
    search with every candidate extended (Section 3.2).  A trial is found
    when one extended region pairs X with Y (strand 0) and covers more than
    95% of the bases of both; `found_filter` asks the same of the union of
    the candidates alone."""
    import numpy as np
    from paper_1807_00205_amd import sdf, synth
    rng = synth.rng_for(seed * 1000 + int(round(delta * 100)))
    lens = rng.integers(1000, 100001, size=trials)
    seqs, dms = [], []
    for L in lens.tolist():
        x, y, dm, _ = synth.sd_pair(rng, L, delta, split=split)
        seqs += [x, y]
        dms.append(dm)
    ix = sdf.Index(seqs, 12, 16)
    t0 = time.perf_counter()
    r = ix.search_batch([(2 * i, 0, len(seqs[2 * i])) for i in range(trials)], max_error,
                        min_len, extend=True)
    cands, regs = r.candidates(), r.regions()
    r.close()
    fin, _ = ix.align_regions(regs, 11, min_len, max_error)  # final SDs (Section 3.3)
    dt = time.perf_counter() - t0
    ix.close()
    lx = np.array([len(seqs[2 * i]) for i in range(trials)], np.float64)
    ly = np.array([len(seqs[2 * i + 1]) for i in range(trials)], np.float64)
    found = np.zeros(trials, bool)
    pair = (regs["q_seq"] % 2 == 0) & (regs["t_seq"] == regs["q_seq"] + 1) & (regs["strand"] == 0)
    for g in regs[pair]:
        i = int(g["q_seq"]) // 2
        if ((g["q_end"] - g["q_begin"]) > 0.95 * lx[i] and
                (g["t_end"] - g["t_begin"]) > 0.95 * ly[i]):
            found[i] = True
    cov_q = [[] for _ in range(trials)]
    cov_t = [[] for _ in range(trials)]
    cp = (cands["q_seq"] % 2 == 0) & (cands["t_seq"] == cands["q_seq"] + 1) & (cands["strand"] == 0)
    for c in cands[cp]:
        i = int(c["q_seq"]) // 2
        cov_q[i].append((int(c["q_begin"]), int(c["q_end"])))
        cov_t[i].append((int(c["t_begin"]), int(c["t_end"])))

    def union(iv):
        tot, end = 0, -1
        for a, b in sorted(iv):
            if b > end:
                tot += b - max(a, end)
                end = b
        return tot
    found_f = np.array([union(cov_q[i]) > 0.95 * lx[i] and union(cov_t[i]) > 0.95 * ly[i]
                        for i in range(trials)])
    found_sd = np.zeros(trials, bool)
    fp = (fin["q_seq"] % 2 == 0) & (fin["t_seq"] == fin["q_seq"] + 1) & (fin["strand"] == 0)
    for s_ in fin[fp]:
        i = int(s_["q_seq"]) // 2
        if ((s_["q_end"] - s_["q_begin"]) > 0.95 * lx[i] and
                (s_["t_end"] - s_["t_begin"]) > 0.95 * ly[i]):
            found_sd[i] = True
    return {"delta": delta, "trials": trials, "found": int(found.sum()),
            "found_final_sd": int(found_sd.sum()),
            "found_filter": int(found_f.sum()), "search_extend_align_s": round(dt, 3),
            "mean_len": int(lx.mean()), "mean_delta_M": round(float(np.mean(dms)), 4)}


def sensitivity(trials, seed=41):
    res = {"workload": "Section 4.1.1 simulation: %d pairs per delta in 0.01..0.30, X uniform "
                       "random of 1-100 kbp, Y = X with delta_M substitutions and delta_G gap "
                       "bases (gaps open at 0.005 per base); max_error 0.25, min_len 1000; "
                       "found = one extended region covers > 95%% of both copies; "
                       "found_final_sd = one final SD (Section 3.3) does" % trials}
    for split in ("bounded", "exact"):
        out = [sensitivity_trial_set(round(0.01 * d, 2), trials, seed, split=split)
               for d in range(1, 31)]
        tot = sum(x["trials"] for x in out)
        res[split] = {"sensitivity": round(sum(x["found"] for x in out) / tot, 5),
                      "sensitivity_final_sd": round(sum(x["found_final_sd"] for x in out) / tot, 5),
                      "sensitivity_filter_only": round(sum(x["found_filter"] for x in out) / tot, 5),
                      "per_delta": out}
    return res


def alg_bytes_per_query_base(nm, ne, total, hbar):
    """Algorithmic HBM bytes per query base of the search: each query
    minimizer's record (position, hash, flags: 9 B), the two directory
    entries of each eligible one (8 B) and its hits (target position and
    strand bit, 4.125 B each; a query minimizer meets hbar = sum n_h^2 /
    sum n_h target occurrences of its hash, its own included)."""
    rho_all = nm / total
    rho_elig = ne / total
    return rho_all * 9.0 + rho_elig * (8.0 + 4.125 * hbar)


def roofline(alg_bytes, kernel_ms, traffic=None, kernel="k_tile_search"):
    achieved = alg_bytes / (kernel_ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": traffic,
            "kernel": kernel, "kernel_ms": round(kernel_ms, 4),
            "algorithmic_bytes": int(alg_bytes)}


def host_cpu():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return ""


def genome_headline(args):
    """3.1 Gbp in 24 sequences, all-vs-all: every whole sequence is a query
    span, all 24 searched in one batched search against the resident index
    (K timed steps), next to the same 24 spans searched one call at a time."""
    import numpy as np
    import torch
    from paper_1807_00205_amd import sdf, synth
    log("generating the 3.1 Gbp assembly")
    t = time.time()
    g = synth.config5()
    gen_s = time.time() - t
    log("  %.1f s" % gen_s)
    torch.cuda.synchronize()
    t = time.time()
    ix = sdf.Index(g.seqs, 12, 16)
    torch.cuda.synchronize()
    build_s = time.time() - t
    nm, ne, dev = ix.info()
    hbar = ix.hit_density()
    total = g.total
    log("index built in %.2f s: %d minimizers, %d eligible, %.2f GB, hit density %.2f" % (
        build_s, nm, ne, dev / 1e9, hbar))
    spans = g.spans
    qb = sum(e - b for _, b, e in spans)
    for _ in range(max(1, args.warmup)):  # the first call also grows the memory pool
        r = ix.search_batch(spans, args.max_error, args.min_len, timing=True)
        r.candidates()
        r.close()
    torch.cuda.synchronize()
    kms, lat = [], []
    t0 = time.perf_counter()
    for step in range(args.steps):
        s0 = time.perf_counter()
        r = ix.search_batch(spans, args.max_error, args.min_len, timing=True)
        nc = len(r.candidates())
        lat.append((time.perf_counter() - s0) * 1e3)
        kms.append(float(r.timing()[1]))
        if step == 0:
            stats = r.stats()
        r.close()
        log("  step %d: %.1f ms" % (step, lat[-1]))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    # plain: the same 24 spans, one search call each
    torch.cuda.synchronize()
    t = time.perf_counter()
    plain_lat = []
    for sp in spans:
        s0 = time.perf_counter()
        r = ix.search(sp, args.max_error, args.min_len)
        r.candidates()
        r.close()
        plain_lat.append((time.perf_counter() - s0) * 1e3)
    torch.cuda.synchronize()
    tp = time.perf_counter() - t
    ix.close()
    mean_k = float(np.mean(kms))
    alg = qb * alg_bytes_per_query_base(nm, ne, total, hbar)
    out = {
        "metric": "query Mbp searched/sec (Jaccard filter)",
        "value": round(qb * args.steps / dt / 1e6, 3),
        "unit": "Mbp/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "3.1 Gbp synthetic assembly in 24 sequences of 50-250 Mbp (41%% GC, "
                               "50%% soft-masked repeats, 10 N-gaps of 50 kbp per sequence, %d "
                               "planted duplications of 1-300 kbp at 1-25%%, half between "
                               "sequences, half reverse-complemented); all-vs-all" % len(g.truth),
                   "query_bases": qb, "spans": len(spans), "k": 12, "w": 16,
                   "min_len": args.min_len, "max_error": args.max_error,
                   "path": "batched: the 24 whole sequences in one search"},
        "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 3),
                       "p99": round(float(np.percentile(lat, 99)), 3)},
        "roofline": roofline(alg, mean_k, measured_traffic("genome3100")),
        "plain": {"path": "the same 24 spans, one sdf_search call each",
                  "mbp_per_s": round(qb / tp / 1e6, 3), "seconds": round(tp, 3),
                  "latency_ms_per_call": {"p50": round(float(np.percentile(plain_lat, 50)), 3),
                                          "p99": round(float(np.percentile(plain_lat, 99)), 3)}},
        "detail": {"generate_s": round(gen_s, 1), "index_build_s": round(build_s, 3),
                   "index_gb": round(dev / 1e9, 3), "minimizers": nm, "eligible": ne,
                   "hit_density": round(hbar, 4),
                   "algorithmic_bytes_per_query_base": round(
                       alg_bytes_per_query_base(nm, ne, total, hbar), 4),
                   "candidates": nc, **stats},
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) on 64 sampled 100 kbp spans")
        import oracle
        b, off = g.concat()
        threads = max(1, min(16, os.cpu_count() or 1))
        t = time.time()
        orc = oracle.OracleIndex(b, off, 12, 16)
        obuild = time.time() - t
        rng = synth.rng_for(55)
        sample = synth.draw_spans(rng, [len(s) for s in g.seqs], 64, 100_000, 100_000)
        t = time.time()
        orc.search(sample, args.max_error, args.min_len, threads)
        odt = time.time() - t
        orc.close()
        sb = sum(e - b for _, b, e in sample)
        out["cpu_baseline"] = {"value": round(sb / odt / 1e6, 5), "unit": "Mbp/s",
                               "cores": threads, "kind": "oracle",
                               "sample": "64 spans of 100 kbp drawn with seed 55 from the same "
                                         "assembly (6.4 Mbp), searched against the whole "
                                         "3.1 Gbp index; search only, oracle index built "
                                         "beforehand in %.1f s" % obuild,
                               "seconds": round(odt, 3), "host_cpu": host_cpu(),
                               "host_threads_visible": os.cpu_count()}
        del b, off
    del g
    return out


def chromosome_section(args, steps):
    """The 50 Mbp chromosome-shaped workload, whole sequence as one span
    (plain single-span path), with its roofline, the oracle's rate on a
    12 Mbp span, seeds by the estimate and every candidate extended."""
    import numpy as np
    import torch
    from paper_1807_00205_amd import sdf
    g, spans, desc = workload("chromosome50")
    ix = sdf.Index(g.seqs, 12, 16)
    nm, ne, _ = ix.info()
    hbar = ix.hit_density()
    span = spans[0]
    qbases = span[2] - span[1]
    tuned_core, tuned_threads, tuned_ms = ix.autotune([span], args.max_error, args.min_len)
    sdf.set_tuning(tile_core=tuned_core, tile_threads=tuned_threads)
    for _ in range(2):
        r = ix.search(span, args.max_error, args.min_len, timing=True)
        r.candidates()
        r.close()
    torch.cuda.synchronize()
    kernel_ms, lat = [], []
    t0 = time.perf_counter()
    for _ in range(steps):
        s0 = time.perf_counter()
        r = ix.search(span, args.max_error, args.min_len, timing=True)
        ncand = ctypes_count(r)
        lat.append((time.perf_counter() - s0) * 1e3)
        kernel_ms.append(float(r.timing()[1]))
        stats = r.stats()
        r.close()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    # the same search captured once as a HIP graph and replayed: no launch
    # gaps or count read-backs between its kernels
    stream = torch.cuda.Stream()
    plan = ix.plan([span], args.max_error, args.min_len, stream=stream)
    r = plan.run(stream)
    r.candidates()
    r.close()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        r = plan.run(stream)
        ncand_g = len(r.candidates())
        r.close()
    torch.cuda.synchronize()
    tg = (time.perf_counter() - t0) / steps
    ginfo = plan.info()
    plan.close()
    sdf.set_tuning()
    mean_k = float(np.mean(kernel_ms))
    alg = qbases * alg_bytes_per_query_base(nm, ne, g.total, hbar)
    out = {"workload": desc, "path": "plain single-span search",
           "mbp_per_s": round(qbases * steps / dt / 1e6, 3),
           "ms_per_search": round(dt / steps * 1e3, 4),
           "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 4),
                          "p99": round(float(np.percentile(lat, 99)), 4)},
           "roofline": roofline(alg, mean_k, measured_traffic("chromosome50")),
           "graph": {"path": "the same search captured once as a HIP graph (sdf_plan_create) "
                             "and replayed (sdf_plan_run), candidates copied out each step",
                     "mbp_per_s": round(qbases / tg / 1e6, 3), "ms_per_search": round(tg * 1e3, 4),
                     "candidates": ncand_g, **ginfo},
           "detail": {"autotuned_core": tuned_core, "autotuned_threads": tuned_threads,
                      "tile_kernel_ms_per_schedule": {"%d threads, %d starts" % k: round(v, 3)
                                                      for k, v in tuned_ms.items()},
                      "minimizers": nm, "eligible": ne, "hit_density": round(hbar, 4),
                      "candidates": ncand, **stats}}
    if not args.no_estimate:
        log("seeds by the winnowed MinHash estimate")
        out["estimate"] = estimate_mode(ix, span, args.max_error, args.min_len, qbases)
    keep = {}
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle), 50 Mbp workload")
        out["cpu_baseline"] = cpu_baseline(g, args.cpu_sample_mbp, args.max_error, args.min_len,
                                           keep)
    if not args.no_extend:
        log("extension of every candidate (Section 3.2)")
        out["extend"] = extend_mode(ix, span, args.max_error, args.min_len,
                                    cpu=keep if keep else None)
    keep.clear()
    ix.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--max-error", type=float, default=0.25)
    ap.add_argument("--min-len", type=int, default=1000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-mbp", type=float, default=12.0)
    ap.add_argument("--headline-only", action="store_true",
                    help="only the 3.1 Gbp all-vs-all (for profiler runs)")
    ap.add_argument("--only", default="",
                    help="run one section without the headline: chromosome50, batched250 or "
                         "serving (for profiler runs)")
    ap.add_argument("--no-chromosome", action="store_true", help="skip the 50 Mbp section")
    ap.add_argument("--no-batch", action="store_true", help="skip batched vs plain")
    ap.add_argument("--no-estimate", action="store_true",
                    help="skip the search with seeds chosen by the winnowed MinHash estimate")
    ap.add_argument("--no-extend", action="store_true",
                    help="skip the search with every candidate extended (SDF_EXTEND)")
    ap.add_argument("--no-batch-plain", action="store_true",
                    help="in the batched section, skip the 4,096 one-by-one calls")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving sweep")
    ap.add_argument("--serve-rates", default="10,30,100,300,1000")
    ap.add_argument("--serve-seconds", type=float, default=6.0)
    ap.add_argument("--serve-workers", type=int, default=2)
    ap.add_argument("--sensitivity", type=int, default=0, metavar="TRIALS",
                    help="also run the simulated-sensitivity experiment with TRIALS pairs per "
                         "delta (the paper uses 1,000; about 3 s per delta at 1,000)")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="first copy this many MiB device-to-device (a reference kernel "
                         "of known traffic for hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the search path is built and timed on a single "
              "MI355X; use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1807_00205_amd import sdf
    sdf.lib()

    torch.cuda.init()
    if args.calibrate_copy_mib:
        nbytes = args.calibrate_copy_mib << 20
        src = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.only:
        out = {"section": args.only}
        if args.only == "chromosome50":
            out["chromosome50"] = chromosome_section(args, args.steps)
        elif args.only in ("batched250", "serving"):
            ix3, g3, bat = batched_vs_plain(max(1, args.steps), not args.no_batch_plain,
                                            cpu=not args.no_cpu_baseline)
            out["batched"] = bat
            if args.only == "serving":
                rates = [float(x) for x in args.serve_rates.split(",") if x]
                out["serving"] = serving(ix3, g3, rates, args.serve_seconds, args.serve_workers)
            ix3.close()
        else:
            raise SystemExit("unknown section %s" % args.only)
        print(json.dumps(out), flush=True)
        return
    log("headline: 3.1 Gbp all-vs-all")
    out = genome_headline(args)
    if not args.headline_only:
        # further workloads; a failure in one of them is recorded, not fatal
        if not args.no_chromosome:
            log("50 Mbp chromosome-shaped workload (plain path)")
            try:
                out["chromosome50"] = chromosome_section(args, max(args.steps, 10))
            except Exception as e:  # noqa: BLE001
                out["chromosome50"] = {"error": repr(e)}
        if not args.no_batch or not args.no_serve:
            log("batched vs plain (250 Mbp, 4,096 spans)")
            try:
                ix3, g3, bat = batched_vs_plain(max(1, args.steps // 2), not args.no_batch_plain,
                                                cpu=not args.no_cpu_baseline)
                if not args.no_batch:
                    out["batched"] = bat
                if not args.no_serve:
                    log("serving")
                    rates = [float(x) for x in args.serve_rates.split(",") if x]
                    out["serving"] = serving(ix3, g3, rates, args.serve_seconds,
                                             args.serve_workers)
                ix3.close()
            except Exception as e:  # noqa: BLE001
                out["batched"] = {"error": repr(e)}
        if args.sensitivity:
            log("simulated sensitivity (Section 4.1.1), %d pairs per delta" % args.sensitivity)
            out["sensitivity"] = sensitivity(args.sensitivity)
    print(json.dumps(out), flush=True)


def ctypes_count(r):
    return len(r.candidates())


if __name__ == "__main__":
    main()
