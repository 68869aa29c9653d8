#!/usr/bin/env python3
"""Throughput of the edge-centric matcher on one MI355X.

One step = every query of the workload, each one pass of the whole path
(vertex validator, arc scan with compaction, extension to full embeddings,
count).  The target graph is resident in device memory before timing starts.

Prints ONE JSON line: matches/s (whole job), validated edge candidates/s
(arcs tested against pattern arc (0,1) per second of arc-scan device time),
the roofline position of the dominant kernel (algorithmic bytes over its
average launch time, from HIP events recorded around every launch on the
stream it runs on), and the CPU oracle timed on a bounded sample.

    python bench.py [--steps K] [--warmup W] [--workload chunglu|rmat20|er1k|batch256|serve]

Default workload: the connectome-shaped graph (2e7 vertices, 1.5e8 arcs), the
largest single-GPU configuration.  Before every timed step a scratch buffer of
--flush-mib MiB (default 2048) is written, so that no part of the graph is left
in the 256 MB last-level (infinity) cache by the previous step; each step is
timed on its own between two device synchronisations, and the line reports the
median, mean with a 95% confidence interval, and minimum of the step times.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "matches/sec & validated edge candidates/sec; query p50/p99 latency at fixed QPS"
HBM_PEAK_GBS = 8000.0

# Algorithmic bytes per unit of work (what the method has to move):
#   vertex validator  13 B per vertex (label 4, in/out degree 8, flag 1)
#   arc scan          12 B per arc (tail, head, arc label) + 8 B per surviving row
#   extension         20 B per candidate (candidate id 4, label 4, arc label 4,
#                     in/out degree 8) + 4(d+1) B per written row
#   last level        20 B per candidate + 4k B per written mapping; a row
#                     counted from its filtered list's length moves its row,
#                     offsets and pivot (4d + 24 B) plus 4 B per list probe
#   filter            per grouped row its images, pivot and offsets twice
#                     (insert, redirect: 2 x 24 B + 8d B); per list entry of a
#                     group 8 B (entry, kept copy)
B_VERTEX, B_ARC, B_ROW2, B_CAND = 13, 12, 8, 20


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def workload(name):
    from synth import configs
    from synth.patterns import ISO, MONO
    if name == "rmat20":
        g = configs.c2_graph()
        runs = configs.c2_runs()
        desc = ("R-MAT scale 20 (a,b,c,d=.57,.19,.19,.05), 2^24 arcs, Zipf(1.2) vertex labels "
                "over 16, arc labels U{0..3}; 4-cycle, FFL+tail, 3-star+back arc, 4-clique minus "
                "one arc; induced iso and mono")
    elif name == "er1k":
        g = configs.c1_graph()
        runs = [(configs.c1_pattern(), ISO), (configs.c1u_pattern(), ISO),
                (configs.c1u_pattern(), MONO)]
        desc = "Erdos-Renyi 1000 vertices / 5000 arcs, labelled and unlabelled 3-cycle"
    elif name == "batch256":
        g = configs.c2_graph()
        runs = configs.c4_patterns()
        desc = ("R-MAT scale 20 graph as rmat20; 256 random patterns of 3-8 vertices (spanning "
                "tree plus pairs up to density 0.6, Zipf vertex labels, U{0..3} arc labels, iso "
                "or mono), each within a fixed oracle search bound on this graph; one batched call")
    elif name == "serve":
        g = configs.c3_graph()
        runs = [(p, m) for p, m, _, _ in configs.c5_pool()]
        desc = ("connectome-shaped graph as chunglu, resident; a pool of random 3-8 vertex "
                "queries (labels U{0..7}, arc weight >= 10, iso or mono), each within a fixed "
                "oracle search bound; Poisson arrivals at fixed rates, served by hpm_server vs "
                "one hpm_match at a time in arrival order")
    elif name == "chunglu":
        g = configs.c3_graph()
        runs = [(p, MONO) for p in configs.c3_patterns()]
        desc = ("directed Chung-Lu 2e7 vertices / 1.5e8 arcs, power-law 2.1, 30% reciprocal; "
                "three 5-vertex motifs, arc weight >= 10, mono")
    else:
        raise SystemExit(f"unknown workload {name}")
    return g, runs, desc


def kernel_bytes(stats_list, g, runs):
    """Algorithmic bytes per kernel family, summed over the given match calls."""
    out = {"vertex_validator": 0, "edge_scan": 0, "expand": 0, "last_level": 0, "filter": 0,
           "index": 0}
    for st, (p, _) in zip(stats_list, runs):
        k = p.k
        out["vertex_validator"] += B_VERTEX * g.n
        out["edge_scan"] += B_ARC * g.m + B_ROW2 * (st["survivors"] if k >= 3 else 0)
        for d in range(2, k - 1):
            out["expand"] += B_CAND * st["work"][d] + 4 * (d + 1) * st["rows"][d + 1]
        if k >= 3:
            d = k - 1
            out["last_level"] += (B_CAND * (st["work"][d] - st["counted_work"]) +
                                  (4 * d + 24 + 4 * d) * st["counted_rows"])
        # the filtered depths are not recorded per depth: take the deepest
        # row width as an upper bound of the images per row
        out["filter"] += (48 + 8 * (k - 1)) * st["filter_rows"] + 8 * st["filter_entries"]
        # arc-predicate index, per side (out and in): the flag pass reads the
        # column and writes a position (8 B per arc), the prefix scan reads the
        # positions twice and writes them once (12 B), the compaction reads
        # position, target and column (12 B) and writes each kept arc with its
        # column (8 B), the offsets read, gather and write (12 B per vertex)
        if st.get("index_arcs"):
            out["index"] += 2 * (32 * g.m + 8 * st["index_arcs"] + 12 * (g.n + 1))
    return out


def kernel_source_sha() -> str:
    import hashlib
    path = os.path.join(ROOT, "paper_2507_04130_amd", "csrc", "hpm_kernels.hip")
    return hashlib.sha256(open(path, "rb").read()).hexdigest()


def measured_traffic(workload, kernel, launches_per_step):
    """HBM bytes per launch of kernel family `kernel` from the committed counter
    summary (profiles/<workload>_traffic.txt: FETCH_SIZE and WRITE_SIZE summed
    over the family's dispatches in one step, each scaled by the same counter
    on a 1 GiB device copy), divided by the family's launches per step; None
    when the summary is missing or was taken on a different kernel source."""
    path = os.path.join(ROOT, "profiles", f"{workload}_traffic.txt")
    if not os.path.exists(path) or not launches_per_step:
        return None
    fields = {}
    for line in open(path):
        if line.startswith(f"kernel={kernel} "):
            fields = dict(kv.split("=", 1) for kv in line.split())
    if (not fields or fields.get("source_sha256") != kernel_source_sha() or
            "fetch_bytes_per_step" not in fields or "write_bytes_per_step" not in fields):
        return None
    step = float(fields["fetch_bytes_per_step"]) + float(fields["write_bytes_per_step"])
    return int(step / launches_per_step)


def cpu_baseline(g, runs, seconds_target):
    """The oracle on a seeded random subset of root vertices (bounded CPU time)."""
    import numpy as np
    import oracle
    threads = min(16, len(os.sched_getaffinity(0)))
    rng = np.random.default_rng(12345)
    key = rng.random(g.n)

    def run(frac):
        mask = (key < frac).astype(np.uint8)
        found, secs = 0, 0.0
        for p, mode in runs:
            r = oracle.match(g, p, mode, threads=threads, rows=False, root_mask=mask)
            found += r.count
            secs += r.seconds
        return found, secs

    f = 1e-4
    found, secs = run(f)
    log(f"cpu baseline pilot: frac={f} matches={found} {secs:.2f}s")
    while secs < seconds_target / 4 and f < 1.0:
        f = min(1.0, f * min(50.0, seconds_target / max(secs, 1e-3)))
        found, secs = run(f)
    log(f"cpu baseline: frac={f:.4f} matches={found} {secs:.2f}s threads={threads}")
    return {"value": found / secs if secs > 0 else None, "unit": "matches/s", "cores": threads,
            "kind": "oracle",
            "sample": f"embeddings whose image of pattern vertex 0 lies in a seeded random "
                      f"{100 * f:.2f}% of the target vertices, every query of the step; "
                      f"{found} matches in {secs:.1f} s"}


def step_statistics(step_s):
    """Median, mean with a 95% confidence interval (Student t), and minimum of
    per-step wall times, in milliseconds."""
    import numpy as np
    from scipy import stats as sst
    a = 1000.0 * np.asarray(step_s, dtype=np.float64)
    out = {"median": round(float(np.median(a)), 4), "mean": round(float(a.mean()), 4),
           "min": round(float(a.min()), 4), "max": round(float(a.max()), 4), "n": int(a.size)}
    if a.size > 1:
        half = float(sst.t.ppf(0.975, a.size - 1) * a.std(ddof=1) / np.sqrt(a.size))
        out["ci95"] = [round(out["mean"] - half, 4), round(out["mean"] + half, 4)]
    return out


def stream_peaks(torch, mib=4096, reps=5):
    """Device-memory rates on this GPU over a buffer far larger than the
    last-level cache, in GB/s of bytes moved, the best of `reps` runs each,
    timed with HIP events on the current stream: read-only (the probe
    library's streaming kernel, 16-byte non-temporal loads, at two grid
    sizes), write-only (torch fill) and copy (torch copy, read + write)."""
    import ctypes
    n = mib << 18
    a = torch.ones(n, dtype=torch.int32, device="cuda")
    b = torch.empty_like(a)
    nbytes = 4 * n
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2507_04130_amd", "libhpm_probe.so"))
    lib.hpm_probe_read.restype = ctypes.c_int
    lib.hpm_probe_read.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int32,
                                   ctypes.c_void_p, ctypes.c_void_p]
    sink = torch.empty(1 << 16, dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream

    def read(blocks):
        def fn():
            rc = lib.hpm_probe_read(a.data_ptr(), nbytes, blocks, stream, sink.data_ptr())
            assert rc == 0, rc
        return fn

    out = {"buffer_mib": mib}
    for name, fn, moved in (("read_2048_blocks", read(2048), nbytes),
                            ("read_16384_blocks", read(16384), nbytes),
                            ("write", lambda: b.fill_(2), nbytes),
                            ("copy", lambda: b.copy_(a), 2 * nbytes)):
        fn()
        best = None
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            e1.synchronize()
            ms = e0.elapsed_time(e1)
            best = ms if best is None else min(best, ms)
        out[f"{name}_gbs"] = round(moved / (best / 1000.0) / 1e9, 1)
    out["read_gbs"] = max(out["read_2048_blocks_gbs"], out["read_16384_blocks_gbs"])
    del a, b, sink
    torch.cuda.empty_cache()
    return out


def serve_trace(hpm, dg, runs, expected, qps, n, kind, srv, stream):
    """Replay one seeded Poisson trace; latency is result time minus scheduled
    arrival.  kind "served": every query is submitted to an hpm_server at its
    arrival time; "one_at_a_time": one hpm_match after another in arrival
    order, each started at its arrival or when the previous one returns."""
    import numpy as np
    from synth import configs
    arrivals, idx = configs.c5_trace(qps, n, len(runs))
    warm = min(100, n // 10)
    lat = np.zeros(n)
    got = [None] * n
    if kind == "served":
        admitted0 = srv.stats()["admitted"]
        tickets, late = [], np.zeros(n)
        t0 = time.perf_counter()
        for i in range(n):
            wait = arrivals[i] - (time.perf_counter() - t0)
            if wait > 0:
                time.sleep(wait)
            late[i] = time.perf_counter() - t0 - arrivals[i]
            p, mode = runs[idx[i]]
            tickets.append(srv.submit(p, mode))
            if i % 500 == 499:
                log(f"  {kind} {qps} q/s: {i + 1} of {n} submitted")
        q_ms, r_ms = [], []
        for i, t in enumerate(tickets):
            r = srv.poll(t, wait=True)
            assert r["status"] == 0, r
            got[i] = r["count"]
            q_ms.append(r["queue_ms"])
            r_ms.append(r["run_ms"])
            lat[i] = late[i] + (r["queue_ms"] + r["run_ms"]) / 1000.0
        st = srv.stats()
        assert st["admitted"] - admitted0 == n
        done = arrivals + lat
    else:
        st = None
        done = np.zeros(n)
        t0 = time.perf_counter()
        for i in range(n):
            wait = arrivals[i] - (time.perf_counter() - t0)
            if wait > 0:
                time.sleep(wait)
            p, mode = runs[idx[i]]
            got[i], _ = hpm.match(dg, p, mode, stream=stream)
            done[i] = time.perf_counter() - t0
            if i % 500 == 499:
                log(f"  {kind} {qps} q/s: {i + 1} of {n} done")
        lat = done - arrivals
    bad = [i for i in range(n) if got[i] != expected[idx[i]]]
    assert not bad, f"{kind} counts differ from the oracle's at {bad[:8]}"
    span = float(done[warm:].max() - arrivals[warm])
    matches = int(sum(expected[idx[i]] for i in range(warm, n)))
    out = {}
    if kind == "served":
        qms = np.array(q_ms[warm:])
        rms = np.array(r_ms[warm:])
        out.update({"queue_ms_p50": float(np.percentile(qms, 50)),
                    "run_ms_p50": float(np.percentile(rms, 50)),
                    "late_ms_p50": 1000.0 * float(np.percentile(late[warm:], 50))})
    out.update({"p50_ms": 1000.0 * float(np.percentile(lat[warm:], 50)),
           "p99_ms": 1000.0 * float(np.percentile(lat[warm:], 99)),
           "mean_ms": 1000.0 * float(lat[warm:].mean()),
           "queries_per_sec": (n - warm) / span, "matches_per_sec": matches / span,
           "matches": matches, "span_s": span, "measured": n - warm})
    if st:
        out["peak_running_so_far"] = st["peak_running"]
        out["peak_granted_gib_so_far"] = round(st["peak_granted_bytes"] / 2**30, 3)
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--flush-mib", type=int, default=2048,
                    help="scratch MiB written before every timed step (last-level cache "
                         "flush); 0 = none")
    ap.add_argument("--workload", default="chunglu",
                    choices=["rmat20", "er1k", "chunglu", "batch256", "serve"])
    ap.add_argument("--batch-workers", type=int, default=0,
                    help="host threads / streams of the batched call (batch256); 0 = tuned")
    ap.add_argument("--qps", default="10,20,50,100,200,500",
                    help="arrival rates of the serve workload (comma separated)")
    ap.add_argument("--serve-queries", type=int, default=2000,
                    help="queries per arrival rate (serve); the first 100 (at most a tenth) "
                         "are warm-up")
    ap.add_argument("--serve-workers", type=int, default=8)
    ap.add_argument("--serve-budget-gib", type=float, default=64.0)
    ap.add_argument("--overlap", type=int, default=0,
                    help="1: apply the neighbour-overlap test to depth-2 rows (HPM_F_OVERLAP)")
    ap.add_argument("--lookahead", type=int, default=0,
                    help="1: apply the frontier look-ahead to the rows of every depth "
                         "(HPM_F_LOOKAHEAD)")
    ap.add_argument("--batched-ref", type=int, default=1,
                    help="also run the step's queries as one batched call (outside the "
                         "timed region; 0 for hardware-counter runs)")
    ap.add_argument("--cpu-baseline", type=int, default=1)
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="first run one plain device copy of this many MiB (a known-size "
                         "reference for hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: sharding the matcher by arc range across "
              "GPUs is designed but not implemented, so there is no multi-GPU run.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2507_04130_amd as hpm

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_probe_mb:
        src = torch.ones(args.copy_probe_mb << 18, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy probe: {args.copy_probe_mb} MiB read and written")
        del src, dst
    t0 = time.time()
    g, runs, desc = workload(args.workload)
    log(f"workload {args.workload}: n={g.n} m={g.m} generated in {time.time() - t0:.1f}s")
    dg = hpm.Graph.from_host(g)
    log(f"graph resident: {dg.info()['device_bytes'] / 2**20:.1f} MiB")
    stream = torch.cuda.current_stream()

    extra_flags = (hpm.F_OVERLAP if args.overlap else 0) | \
        (hpm.F_LOOKAHEAD if args.lookahead else 0)
    flush_buf = (torch.empty(args.flush_mib << 18, dtype=torch.int32, device="cuda")
                 if args.flush_mib else None)

    def flush():
        # overwrite the last-level cache with unrelated lines before a step
        if flush_buf is not None:
            flush_buf.fill_(1)

    def step(timing_flags):
        counts, stats = [], []
        for p, mode in runs:
            c, _ = hpm.match(dg, p, mode, stream=stream, flags=timing_flags | extra_flags)
            counts.append(c)
            stats.append(hpm.last_stats())
        return counts, stats

    batch = args.workload == "batch256"
    serve = args.workload == "serve"
    pats = [p for p, _ in runs]
    modes = [m for _, m in runs]
    extra = {}
    if batch:
        # one batched call per step; per-kernel times come from one sequential
        # step with HIP events, the one-at-a-time comparison from another
        # without them
        from synth import configs
        expected = configs.c4_expected_counts(len(runs))
        seq_counts, all_stats = [], []
        torch.cuda.synchronize()
        t_seq = time.perf_counter()
        for i, (p, mode) in enumerate(runs):
            c, _ = hpm.match(dg, p, mode, stream=stream, flags=hpm.F_TIMING)
            seq_counts.append(c)
            all_stats.append(hpm.last_stats())
            if i % 32 == 31:
                log(f"sequential: {i + 1} queries, {time.perf_counter() - t_seq:.3f}s")
        bad = [i for i, (a, b) in enumerate(zip(seq_counts, expected)) if a != b]
        assert not bad, f"counts differ from the oracle's for patterns {bad[:8]}"
        # the one-at-a-time comparison, without the per-kernel events
        torch.cuda.synchronize()
        t_seq = time.perf_counter()
        for p, mode in runs:
            hpm.match(dg, p, mode, stream=stream)
        torch.cuda.synchronize()
        seq_s = time.perf_counter() - t_seq
        log(f"sequential step {seq_s:.3f}s; all {len(runs)} counts equal the oracle's")
        tuned_ms = None
        if args.batch_workers == 0:
            args.batch_workers, tuned_ms = hpm.batch_tune(dg, pats, modes, stream=stream)
            log(f"tuned: {args.batch_workers} workers ({tuned_ms:.1f} ms per batch)")
        for i in range(args.warmup):
            hpm.match_batch(dg, pats, modes, workers=args.batch_workers, stream=stream)
            torch.cuda.synchronize()
            log(f"batched warmup {i} done")
        t_start = time.perf_counter()
        for i in range(args.steps):
            counts, status = hpm.match_batch(dg, pats, modes, workers=args.batch_workers,
                                             stream=stream)
            log(f"batched step {i}: {time.perf_counter() - t_start:.3f}s")
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t_start
        assert counts == expected, "batched counts differ from the oracle's"
        extra = {"batch_workers": args.batch_workers, "tuned_ms_per_batch": tuned_ms,
                 "queries_per_sec": len(runs) * args.steps / elapsed,
                 "sequential_queries_per_sec": len(runs) / seq_s,
                 "sequential_ms_per_step": 1000.0 * seq_s,
                 "batch_speedup": (seq_s * args.steps) / elapsed}
        log(f"batched {args.steps} steps in {elapsed:.3f}s; sequential step {seq_s:.3f}s")
        timed_steps = 1
    elif serve:
        from synth import configs
        pool = configs.c5_pool()
        expected = [c for _, _, c, _ in pool]
        # one sequential pass with HIP events: per-kernel times, and every
        # count checked against the oracle's
        seq_counts, all_stats = [], []
        t_seq = time.perf_counter()
        for i, (p, mode) in enumerate(runs):
            c, _ = hpm.match(dg, p, mode, stream=stream, flags=hpm.F_TIMING)
            seq_counts.append(c)
            all_stats.append(hpm.last_stats())
            if i % 32 == 31:
                log(f"pool pass: {i + 1} queries, {time.perf_counter() - t_seq:.3f}s")
        seq_s = time.perf_counter() - t_seq
        bad = [i for i, (a, b) in enumerate(zip(seq_counts, expected)) if a != b]
        assert not bad, f"counts differ from the oracle's for queries {bad[:8]}"
        log(f"pool pass {seq_s:.3f}s; all {len(runs)} counts equal the oracle's")
        rates = [float(x) for x in args.qps.split(",") if x]
        # one server for the whole sweep, warmed by two passes over the pool
        # (every worker's scratch grows to its working size before timing)
        srv = hpm.Server(dg, workers=args.serve_workers,
                         budget=int(args.serve_budget_gib * 2**30))
        t_w = time.perf_counter()
        for rep in range(2):
            tk = [srv.submit(p, mode) for p, mode in runs]
            got = [srv.poll(t, wait=True)["count"] for t in tk]
            assert got == expected, "served counts differ from the oracle's"
        log(f"server warm-up: 2 x {len(runs)} queries in {time.perf_counter() - t_w:.3f}s")
        sweep = []
        for qps in rates:
            rec = {"qps": qps}
            for kind in ("served", "one_at_a_time"):
                r = serve_trace(hpm, dg, runs, expected, qps, args.serve_queries, kind, srv,
                                stream)
                rec[kind] = r
                log(f"qps {qps} {kind}: p50 {r['p50_ms']:.2f} ms p99 {r['p99_ms']:.2f} ms, "
                    f"{r['queries_per_sec']:.1f} q/s, {r['matches_per_sec']:.3e} matches/s")
            sweep.append(rec)
        srv.close()
        top = sweep[-1]["served"]
        counts = seq_counts
        elapsed = top["span_s"]
        extra = {"serve_workers": args.serve_workers,
                 "serve_budget_gib": args.serve_budget_gib,
                 "pool_size": len(runs), "queries_per_rate": args.serve_queries,
                 "sweep": sweep,
                 "p50_ms": top["p50_ms"], "p99_ms": top["p99_ms"],
                 "queries_per_sec": top["queries_per_sec"]}
        timed_steps = 1
        args.steps, args.warmup = 1, 0     # one trace replay at the highest rate
    else:
        for i in range(args.warmup):
            counts, _ = step(0)
            log(f"warmup {i}: counts={counts}")
        # One step with events around every launch, before the timed region:
        # per-family times of the whole path, and the family that dominates.
        # The last timed step then records events only around that family and
        # the arc scan (two event records per timed launch cost step time).
        _, prof_stats = step(hpm.F_TIMING)
        prof_ms = {}
        for st in prof_stats:
            for kname, ms in st["kernel_ms"].items():
                prof_ms[kname] = prof_ms.get(kname, 0.0) + ms
        costed_kinds = ("vertex_validator", "edge_scan", "expand", "last_level", "filter",
                        "index")
        dom_kind = max(costed_kinds, key=lambda k: prof_ms.get(k, 0.0))
        timed_flags = hpm.F_TIMING | hpm.F_TIMING_KINDS(dom_kind, "edge_scan")
        log(f"profile step: {({k: round(v, 3) for k, v in prof_ms.items() if v})}; "
            f"timing {dom_kind} and edge_scan in the last timed step")
        extra["kernel_ms_per_step_all_families"] = {k: round(v, 4) for k, v in prof_ms.items()}
        extra["kernel_ms_source"] = ("kernel_ms_per_step_all_families: one step with events "
                                     "around every launch, before the timed steps; "
                                     "kernel_ms_per_step and roofline: the last timed step, "
                                     f"events around {dom_kind} and edge_scan only")
        step_s = []
        for i in range(args.steps):
            flush()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            # events in the last timed step only: the family times and the
            # roofline come from that step's launches
            counts, stats = step(timed_flags if i == args.steps - 1 else 0)
            torch.cuda.synchronize()
            step_s.append(time.perf_counter() - t0)
        elapsed = sum(step_s)
        extra["step_ms"] = step_statistics(step_s)
        log(f"timed {args.steps} steps in {elapsed:.3f}s: {extra['step_ms']}")
        all_stats = stats
        timed_steps = 1
        # For reference, outside the timed region: the same step's queries
        # as one hpm_match_batch call (queries overlapped on worker streams,
        # no events), counts checked against the sequential ones.
        if len(runs) > 1 and args.batched_ref:
            bw = args.batch_workers or len(runs)
            got, _ = hpm.match_batch(dg, pats, modes, workers=bw, stream=stream)
            assert got == counts, "batched counts differ from the sequential ones"
            torch.cuda.synchronize()
            t_b = time.perf_counter()
            for _ in range(args.steps):
                hpm.match_batch(dg, pats, modes, workers=bw, stream=stream)
            torch.cuda.synchronize()
            b_s = (time.perf_counter() - t_b) / args.steps
            extra["batched_step"] = {"workers": bw, "ms_per_step": round(1000.0 * b_s, 4),
                                     "matches_per_sec": sum(counts) / b_s}
            log(f"batched step ({bw} workers): {1000.0 * b_s:.3f} ms")

    per_query_stats = prof_stats if (not batch and not serve) else all_stats[-len(runs):]
    matches_per_step = sum(counts)
    ms_per_step = 1000.0 * elapsed / args.steps
    value = matches_per_step * args.steps / elapsed
    if serve:
        matches_per_step = extra["sweep"][-1]["served"]["matches"]
        ms_per_step = 1000.0 * elapsed
        value = extra["sweep"][-1]["served"]["matches_per_sec"]

    fam_ms, fam_launch = {}, {}
    for st in all_stats:
        for kname, ms in st["kernel_ms"].items():
            fam_ms[kname] = fam_ms.get(kname, 0.0) + ms
            fam_launch[kname] = fam_launch.get(kname, 0) + st["kernel_launches"][kname]
    scan_ms = fam_ms.get("edge_scan", 0.0)
    cand_per_s = g.m * len(runs) * timed_steps / (scan_ms / 1000.0) if scan_ms > 0 else None
    surv = sum(st["survivors"] for st in all_stats)

    bytes_by = kernel_bytes(all_stats, g, runs * timed_steps)
    costed = {k: v for k, v in fam_ms.items() if k in bytes_by and v > 0}
    dom = max(costed, key=costed.get)
    launches = fam_launch[dom]
    avg_ms = fam_ms[dom] / launches
    achieved = bytes_by[dom] / (fam_ms[dom] / 1000.0) / 1e9
    peaks = stream_peaks(torch)
    log(f"stream peaks: {peaks}")
    roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": measured_traffic(args.workload, dom, launches / timed_steps),
                "kernel": dom, "launches": launches, "avg_launch_ms": round(avg_ms, 4),
                "algorithmic_bytes_per_launch": int(bytes_by[dom] / launches),
                "frac_of_measured_read_peak": round(achieved / peaks["read_gbs"], 4),
                "measured_peaks": peaks}
    scan_gbs = bytes_by["edge_scan"] / (scan_ms / 1000.0) / 1e9 if scan_ms > 0 else None

    out = {
        "metric": METRIC, "value": value, "unit": "matches/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": desc, "name": args.workload, "n": g.n, "m": g.m,
                   "overlap_test": bool(args.overlap), "lookahead": bool(args.lookahead),
                   "queries": ([f"{p.name}/{'iso' if mode == 0 else 'mono'}" for p, mode in runs]
                               if len(runs) <= 16 else f"{len(runs)} patterns"),
                   "matches_per_step": matches_per_step},
        "validated_edge_candidates_per_sec": cand_per_s,
        "survivors_per_sec": surv / (scan_ms / 1000.0) if scan_ms > 0 else None,
        "edge_scan_gbs": scan_gbs,
        "kernel_ms_per_step": {k: round(v / timed_steps, 4) for k, v in fam_ms.items()},
        "counts": counts if len(runs) <= 16 else None,
        "per_query": [] if len(runs) > 16 else [{"query": f"{p.name}/{'iso' if mode == 0 else 'mono'}", "count": st["count"],
                       "survivors": st["survivors"], "rows": st["rows"][2:p.k],
                       "work": st["work"][2:p.k], "raw_work": st["raw_work"][2:p.k],
                       "filtered_lists": st["filtered_lists"],
                       "overlap_removed": st["overlap_removed"],
                       "lookahead_removed": st["lookahead_removed"],
                       "kernel_ms": {k: round(v, 4) for k, v in st["kernel_ms"].items() if v}}
                      for st, (p, mode) in zip(per_query_stats, runs)],
        "roofline": roofline,
    }
    out.update(extra)
    if args.cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(g, runs, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
