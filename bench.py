#!/usr/bin/env python3
"""Benchmark of the MI355X exact k-NN engine (iSAX build + exact search).

Default workload (one GPU): 100,000,000 z-normalised random walks of length
256 (fp32, 102.4 GB resident in HBM), 16 segments, 8-bit symbols, leaf
capacity 2000; 100 fresh random-walk queries answered one at a time, exact
1-NN, fp32 early-abandoning distances.

A step = one index build over the resident collection + the query set
answered one query at a time.  `value` = queries/s over the query phases of
the timed steps; p50/p99 are per-query wall-clock latencies of the synchronous
call; build GB/s = collection bytes / build time.  z-normalisation runs once
before the timed region and is reported on its own.

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "exact k-NN queries/sec + p50/p99 latency at 100M×256 fp32; index build GB/s"
PAPER_QPS = 20.0  # ~50 ms per exact 1-NN query on 100 GB (2x Xeon E5-2650 v4): context

WORKLOADS = {
    1: dict(name="random-walk 100K x 256, exact 1-NN, 10 single queries", n=100_000, length=256, queries=10, k=1),
    2: dict(name="random-walk 100M x 256, exact 1-NN, 100 single queries", n=100_000_000, length=256, queries=100,
            k=1),
    3: dict(name="random-walk 100M x 256, batches of 1024 (512 fresh walks + 512 noisy rows), k=1 and k=10, "
                 "BF16 matrix-core filter", n=100_000_000, length=256, queries=1024, k=10),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def src_hash(path):
    h = hashlib.sha256()
    with open(path, "rb") as f:
        h.update(f.read())
    return h.hexdigest()[:16]


def traffic_from_profiles(kernel):
    """HBM traffic per launch measured with rocprofv3 counters, if the kernel's
    source is unchanged since the counters were taken."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    try:
        d = json.load(open(p))
        e = d.get(kernel)
        if not e:
            return None
        if e.get("source_sha") != src_hash(os.path.join(ROOT, e["source"])):
            return None
        return e.get("bytes_per_launch")
    except Exception:
        return None


def cpu_baseline(data_gpu, q_host_raw, k, length, n_total, rows, nq, threads):
    """The CPU oracle's brute-force exact k-NN timed on a bounded sample: nq
    queries against `rows` rows of the same collection, scaled to the full
    collection size (queries/s at n_total rows)."""
    import oracle
    raw = data_gpu[:rows].cpu().numpy()
    z = oracle.znorm(raw)
    qz = oracle.znorm(q_host_raw[:nq])
    t0 = time.perf_counter()
    oracle.knn_brute(z, qz, k, nthreads=threads)
    t = time.perf_counter() - t0
    qps = nq / (t * (n_total / rows))
    return {"value": qps, "unit": "queries/s", "cores": threads, "kind": "oracle",
            "sample": "fp64 brute-force k-NN (oracle) of %d queries over the first %d rows, %.1f s, "
                      "scaled by %d/%d rows" % (nq, rows, t, n_total, rows)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", type=int, default=2, choices=sorted(WORKLOADS))
    ap.add_argument("--n", type=int, default=None, help="override the collection size")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-rows", type=int, default=4_000_000)
    ap.add_argument("--cpu-queries", type=int, default=8)
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this implementation runs on one GPU; --gpus %d is not supported "
                                   "(multi-GPU sharding is a design note only)" % args.gpus}))
        sys.exit(2)

    import torch

    import datagen
    from paper_2009_00786_amd import messi

    if args.config == 3:
        return bench_batched(args)
    wl = dict(WORKLOADS[args.config])
    if args.n:
        wl["n"] = args.n
        wl["name"] += " (n=%d)" % args.n
    n, length, nq, k = wl["n"], wl["length"], wl["queries"], wl["k"]
    w, b, cap = 16, 8, 2000
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    messi.load()

    log("generating %d x %d random walks on the GPU" % (n, length))
    data = torch.empty((n, length), dtype=torch.float32, device=dev)
    chunk = 10_000_000
    for r0 in range(0, n, chunk):
        datagen.gpu_random_walks(data[r0:r0 + chunk], row0=r0)
    torch.cuda.synchronize()
    qraw = datagen.random_walks(nq, length, seed=datagen.SEED_QUERY, stream=datagen.STREAM_QUERY)
    queries = torch.from_numpy(qraw).to(dev)
    messi.znorm_(queries)

    cpu = None
    if not args.no_cpu_baseline:
        rows = min(args.cpu_rows, n)
        threads = max(1, min(16, os.cpu_count() or 1))
        log("cpu baseline: oracle brute force, %d queries x %d rows, %d threads" % (args.cpu_queries, rows, threads))
        cpu = cpu_baseline(data, qraw, k, length, n, rows, min(args.cpu_queries, nq), threads)
        log("  ", cpu)

    log("z-normalising")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    messi.znorm_(data)
    torch.cuda.synchronize()
    znorm_ms = (time.perf_counter() - t0) * 1e3

    lat = []
    step_ms, build_ms, query_ms = [], [], []
    infos = []
    agg = {}
    ix = None
    ans_i = torch.empty((nq, k), dtype=torch.int64, device=dev)
    ans_d = torch.empty((nq, k), dtype=torch.float32, device=dev)
    answers = None
    for step in range(args.warmup + args.steps):
        timed = step >= args.warmup
        if ix is not None:
            ix.close()
            ix = None
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ix = messi.Index(data, w, b, cap)
        t1 = time.perf_counter()
        for qi in range(nq):
            a = time.perf_counter()
            _, _, st = ix.knn(queries[qi:qi + 1], k, stats=True, out=(ans_i[qi:qi + 1], ans_d[qi:qi + 1]))
            e = time.perf_counter()
            if timed:
                lat.append((e - a) * 1e3)
                for key, v in st.items():
                    agg[key] = agg.get(key, 0) + v
        t2 = time.perf_counter()
        answers = (ans_i.cpu().numpy(), ans_d.cpu().numpy())
        info = ix.info()
        log("step %d%s: build %.1f ms (summarize %.2f, bucket %.2f, split %.2f, finalize %.2f; %d leaves, %d levels), "
            "queries %.1f ms" % (step, "" if timed else " (warmup)", (t1 - t0) * 1e3, info["ms_summarize"],
                                 info["ms_bucket"], info["ms_split"], info["ms_finalize"], info["n_leaves"],
                                 info["levels"], (t2 - t1) * 1e3))
        if timed:
            step_ms.append((t2 - t0) * 1e3)
            build_ms.append((t1 - t0) * 1e3)
            query_ms.append((t2 - t1) * 1e3)
            infos.append(info)

    steps = args.steps
    total_q = nq * steps
    qps = total_q / (sum(query_ms) / 1e3)
    lat_a = np.array(lat)
    coll_bytes = n * length * 4
    build_gbps = coll_bytes / (np.mean(build_ms) / 1e3) / 1e9
    summ_ms = float(np.mean([i["ms_summarize"] for i in infos]))
    split_ms = float(np.mean([i["ms_split"] for i in infos]))
    bucket_ms = float(np.mean([i["ms_bucket"] for i in infos]))
    scan_ms_per_q = agg.get("ms_scan", 0.0) / total_q
    # dominant kernel per step: summarise (one launch) vs the scan (one launch per query)
    summ_bytes = n * (length * 4 + 16 + 2)
    scan_bytes_per_q = agg.get("bytes_scan", 0) / total_q
    rf_summ = {"bound": "hbm", "achieved": summ_bytes / (summ_ms / 1e3) / 1e9, "peak": HBM_PEAK_GBS,
               "unit": "GB/s", "kernel": "summarize_kernel", "bytes_per_launch": summ_bytes,
               "ms_per_launch": summ_ms, "traffic": traffic_from_profiles("summarize_kernel")}
    rf_scan = {"bound": "hbm", "achieved": (scan_bytes_per_q / (scan_ms_per_q / 1e3) / 1e9) if scan_ms_per_q else 0.0,
               "peak": HBM_PEAK_GBS, "unit": "GB/s", "kernel": "scan_kernel", "bytes_per_launch": scan_bytes_per_q,
               "ms_per_launch": scan_ms_per_q, "traffic": traffic_from_profiles("scan_kernel")}
    for r in (rf_summ, rf_scan):
        r["frac"] = r["achieved"] / r["peak"]
    dominant = rf_scan if scan_ms_per_q * nq > summ_ms else rf_summ
    roofline = {kk: dominant[kk] for kk in ("bound", "achieved", "peak", "unit", "frac", "traffic")}
    roofline["kernel"] = dominant["kernel"]
    roofline["bytes_per_launch"] = dominant["bytes_per_launch"]
    roofline["ms_per_launch"] = dominant["ms_per_launch"]

    res = {
        "metric": METRIC,
        "value": qps,
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": float(np.mean(step_ms)),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": qps / PAPER_QPS if args.config == 2 and n == 100_000_000 else None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl["name"], "n": n, "len": length, "segments": w, "card_bits": b, "leaf_cap": cap,
                   "queries": nq, "k": k, "mode": "fp32, one query per call"},
        "p50_ms": float(np.percentile(lat_a, 50)),
        "p99_ms": float(np.percentile(lat_a, 99)),
        "build_gbps": build_gbps,
        "build_ms": float(np.mean(build_ms)),
        "znorm_ms": znorm_ms,
        "znorm_gbps": 2 * coll_bytes / (znorm_ms / 1e3) / 1e9,
        "roofline": roofline,
        "roofline_other": rf_summ if dominant is rf_scan else rf_scan,
        "phases_ms": {"summarize": summ_ms, "bucket": bucket_ms, "split": split_ms,
                      "finalize": float(np.mean([i["ms_finalize"] for i in infos])),
                      "query_prep": agg.get("ms_prep", 0) / total_q, "leaf_lb": agg.get("ms_leaf_lb", 0) / total_q,
                      "approx": agg.get("ms_approx", 0) / total_q, "order": agg.get("ms_order", 0) / total_q,
                      "scan": scan_ms_per_q, "final": agg.get("ms_final", 0) / total_q,
                      "query_device_total": agg.get("ms_total", 0) / total_q},
        "scan_breakdown_ms": {kk: agg.get(kk, 0) / total_q for kk in (
            "scan_ms_control", "scan_ms_filter", "scan_ms_distance", "scan_ms_block_mean", "scan_ms_block_max")},
        "per_query": {kk: agg.get(kk, 0) / total_q for kk in ("leaves_total", "leaves_kept", "leaves_scanned",
                                                              "series_bounded", "series_distance",
                                                              "series_abandoned", "candidates", "bytes_scan")},
        "index": {"n_leaves": infos[-1]["n_leaves"], "max_leaf": infos[-1]["max_leaf"], "levels": infos[-1]["levels"],
                  "device_bytes": infos[-1]["device_bytes"]},
        "cpu_baseline": cpu,
        "vs_baseline_note": "paper: ~50 ms per exact 1-NN query at 100 GB on 2x Xeon E5-2650 v4 (context only)",
        "answers_sha": hashlib.sha256(answers[0].tobytes()).hexdigest()[:16],
    }
    if ix is not None:
        ix.close()
    print(json.dumps(res), flush=True)


def make_batch(data, z_rows_gpu_fn, b, nq, length, seed_off=0):
    """Half fresh random walks (query stream), half dataset rows + sigma * N(0,1),
    sigma cycling over 0.01, 0.1, 1.0 (not re-normalised)."""
    import datagen
    from paper_2009_00786_amd import messi
    import torch
    half = nq // 2
    fresh_raw = datagen.random_walks(half, length, seed=datagen.SEED_QUERY, stream=datagen.STREAM_QUERY,
                                     row0=1_000_000 + b * half)
    fresh = torch.from_numpy(fresh_raw).to(data.device)
    messi.znorm_(fresh)
    ids = datagen.uniform_ints(nq - half, data.shape[0], 9, 5 + b)
    base = data[torch.from_numpy(ids).to(data.device)].cpu().numpy()
    sig = np.array([(0.01, 0.1, 1.0)[i % 3] for i in range(nq - half)])
    noisy = datagen.add_noise(base, sig, row0=b * nq)
    return torch.cat([fresh, torch.from_numpy(noisy).to(data.device)]).contiguous()


def bench_batched(args):
    """Configuration 3: batches of 1024 queries through the BF16 filter, at k = 1 and k = 10."""
    import torch

    import datagen
    from paper_2009_00786_amd import messi

    wl = dict(WORKLOADS[3])
    if args.n:
        wl["n"] = args.n
        wl["name"] += " (n=%d)" % args.n
    n, length, nq = wl["n"], wl["length"], wl["queries"]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    messi.load()
    log("generating %d x %d random walks on the GPU" % (n, length))
    data = torch.empty((n, length), dtype=torch.float32, device=dev)
    for r0 in range(0, n, 10_000_000):
        datagen.gpu_random_walks(data[r0:r0 + 10_000_000], row0=r0)
    messi.znorm_(data)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ix = messi.Index(data, 16, 8, 2000, bf16_shadow=True)
    build_ms = (time.perf_counter() - t0) * 1e3
    info = ix.info()
    log("build with BF16 shadow: %.1f ms (shadow %.1f ms)" % (build_ms, info["ms_shadow"]))
    batches = [make_batch(data, None, b, nq, length) for b in range(args.warmup + args.steps)]
    agg = {1: {}, 10: {}}
    times = {1: [], 10: []}
    for b, q in enumerate(batches):
        timed = b >= args.warmup
        for k in (1, 10):
            torch.cuda.synchronize()
            a = time.perf_counter()
            _, _, st = ix.knn(q, k, mode=messi.MODE_BF16, stats=True)
            e = time.perf_counter()
            log("batch %d k=%d: %.2f ms  (filter %.2f ms, recheck %.2f ms, %d rounds, evals %.3g, rechecks %d)" % (
                b, k, (e - a) * 1e3, st["ms_bf16_filter"], st["ms_bf16_recheck"], st["bf16_rounds"],
                st["series_distance"], st["series_recheck"]))
            if timed:
                times[k].append((e - a) * 1e3)
                for kk, v in st.items():
                    agg[k][kk] = agg[k].get(kk, 0) + v
    # the plain fp32 path on the same batch, for comparison
    torch.cuda.synchronize()
    a = time.perf_counter()
    _, _, st32 = ix.knn(batches[-1], 1, mode=messi.MODE_FP32, stats=True)
    fp32_batch_ms = (time.perf_counter() - a) * 1e3
    log("fp32 batched k=1: %.2f ms" % fp32_batch_ms)
    steps = args.steps
    total_q = 2 * nq * steps
    total_ms = sum(times[1]) + sum(times[10])
    qps = total_q / (total_ms / 1e3)
    f_ms = (agg[1].get("ms_bf16_filter", 0) + agg[10].get("ms_bf16_filter", 0))
    f_flops = agg[1].get("bf16_flops", 0) + agg[10].get("bf16_flops", 0)
    f_bytes = agg[1].get("bytes_scan", 0) + agg[10].get("bytes_scan", 0)
    launches = agg[1].get("bf16_rounds", 0) + agg[10].get("bf16_rounds", 0)
    mfma = {"bound": "mfma", "achieved": f_flops / (f_ms / 1e3) / 1e12 if f_ms else 0.0, "peak": 2500.0,
            "unit": "TFLOP/s", "traffic": None, "kernel": "bf16_filter_kernel",
            "flops_per_launch": f_flops / max(launches, 1), "ms_per_launch": f_ms / max(launches, 1)}
    mfma["frac"] = mfma["achieved"] / mfma["peak"]
    res = {
        "metric": METRIC, "value": qps, "unit": "queries/s", "n_gpus": 1, "steps": steps, "warmup": args.warmup,
        "ms_per_step": total_ms / steps, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16", "data": "synthetic",
        "config": {"workload": wl["name"], "n": n, "len": length, "segments": 16, "card_bits": 8, "leaf_cap": 2000,
                   "batch": nq, "k": [1, 10], "mode": "BF16 matrix-core filter + compensated fp32 recheck"},
        "qps_k1": nq * steps / (sum(times[1]) / 1e3), "qps_k10": nq * steps / (sum(times[10]) / 1e3),
        "batch_ms_k1": float(np.mean(times[1])), "batch_ms_k10": float(np.mean(times[10])),
        "fp32_batched_k1_ms": fp32_batch_ms, "fp32_batched_k1_qps": nq / (fp32_batch_ms / 1e3),
        "build_ms_with_shadow": build_ms, "shadow_ms": info["ms_shadow"],
        "roofline": mfma,
        "filter_hbm_gbps": f_bytes / (f_ms / 1e3) / 1e9 if f_ms else 0.0,
        "per_batch": {str(k): {kk: agg[k].get(kk, 0) / steps for kk in (
            "leaves_kept", "series_distance", "series_recheck", "candidates", "ms_bf16_filter", "ms_bf16_recheck",
            "ms_total", "ms_leaf_lb", "ms_approx", "ms_order", "ms_scan", "ms_final", "bf16_rounds")}
            for k in (1, 10)},
        "discard_rate": 1.0 - (agg[1].get("series_recheck", 0) + agg[10].get("series_recheck", 0)) /
        max(1, agg[1].get("series_distance", 0) + agg[10].get("series_distance", 0)),
        "cpu_baseline": None,
    }
    ix.close()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
