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
    4: dict(name="random-walk 100M x 256, open-loop Poisson arrivals at 200, 1000, 5000 queries/s; per query "
                 "k in {1, 10, 100} and a dataset row + sigma*N(0,1), sigma in {0.01, 0.1, 1}; BF16 continuous-batching "
                 "server vs fp32 single-query FIFO", n=100_000_000, length=256, data="walk", rates=(200, 1000, 5000),
            headline_rate=1000),
    5: dict(name="Gaussian mixture 200M x 128 (1000 centres U[0,255], sigma 20, integers clipped to [0,255]), "
                 "z-normalised; open-loop Poisson at 200, 1000, 5000 queries/s, k=10, half noisy dataset rows and "
                 "half fresh mixture draws; BF16 continuous-batching server vs fp32 single-query FIFO",
            n=200_000_000, length=128, data="mixture", rates=(200, 1000, 5000), headline_rate=1000,
            server_slots=512),
    6: dict(name="streaming series: one random walk of 100M + 255 points cut into its 100M sliding windows of 256 "
                 "(step 1), z-normalised per window and indexed; exact 1-NN, 100 single queries",
            n=100_000_000, length=256, queries=100, k=1),
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


def copy_calibration():
    """Three copies of a 4 GiB fp32 buffer into another: a plain copy kernel of
    known traffic (4 GiB read + 4 GiB written per dispatch), against which the
    FETCH_SIZE / WRITE_SIZE counters of the other kernels are scaled."""
    import torch
    n = 1 << 30
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / 3
    print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "dispatches": 3,
                      "ms_per_copy": ms, "gbps": 8 * n / (ms / 1e3) / 1e9}), flush=True)


def host_threads():
    """Host threads for the CPU baseline: every core this process may run on,
    at most 16 -- the host share a one-GPU job is given on the GPU machines
    (their nproc shows the whole host)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def host_description():
    """CPU model and host DRAM, from /proc."""
    model, mem_gb = None, None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        for line in open("/proc/meminfo"):
            if line.startswith("MemTotal"):
                mem_gb = int(line.split()[1]) * 1024 / 1e9
                break
    except OSError:
        pass
    return {"cpu_model": model, "host_dram_gb": mem_gb, "host_cpus_visible": os.cpu_count()}


def cpu_baseline(data_gpu, q_host_raw, k, length, n_total, rows, nq, threads, build_rows=2_000_000):
    """The CPU oracle timed on bounded samples of the same collection:
    brute-force exact k-NN of nq queries against `rows` rows on `threads`
    threads, scaled to the full collection (queries/s at n_total rows); and
    the plain single-threaded index build (PAA, iSAX words, leaf partition)
    over `build_rows` rows, as host GB/s of collection."""
    import oracle
    raw = data_gpu[:rows].cpu().numpy()
    z = oracle.znorm(raw)
    qz = oracle.znorm(q_host_raw[:nq])
    t0 = time.perf_counter()
    oracle.knn_brute(z, qz, k, nthreads=threads)
    t = time.perf_counter() - t0
    qps = nq / (t * (n_total / rows))
    br = min(build_rows, rows)
    t1 = time.perf_counter()
    words = oracle.words(z[:br], 16, 8)
    oracle.build_leaves(words, 8, 2000)
    tb = time.perf_counter() - t1
    out = {"value": qps, "unit": "queries/s", "cores": threads, "kind": "oracle",
           "sample": "fp64 brute-force k-NN (oracle) of %d queries over the first %d rows on %d threads, %.1f s, "
                     "scaled by %d/%d rows; plain build (oracle, 1 thread) over the first %d rows, %.1f s"
                     % (nq, rows, threads, t, n_total, rows, br, tb),
           "build_gbps_1_thread": br * length * 4 / tb / 1e9}
    out.update(host_description())
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", type=int, default=2, choices=sorted(WORKLOADS))
    ap.add_argument("--n", type=int, default=None, help="override the collection size")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-rows", type=int, default=12_000_000)
    ap.add_argument("--cpu-queries", type=int, default=100)
    ap.add_argument("--duration", type=float, default=10.0, help="seconds of arrivals per rate (configs 4, 5)")
    ap.add_argument("--rates", type=str, default=None, help="comma-separated arrival rates (configs 4, 5)")
    ap.add_argument("--no-fifo", action="store_true", help="skip the fp32 FIFO comparison (configs 4, 5)")
    ap.add_argument("--variants", action="store_true",
                    help="also serve with BF16 batches only, and without HIP graphs (configs 4, 5)")
    ap.add_argument("--no-fp32-batch", action="store_true",
                    help="skip the fp32 batched comparison call (config 3), e.g. under a profiler")
    ap.add_argument("--no-oracle-sample", action="store_true",
                    help="config 3: skip the oracle's brute force over the whole collection for a query sample")
    ap.add_argument("--oracle-sample", type=int, default=16, help="config 3: queries in that sample")
    ap.add_argument("--core-only", action="store_true",
                    help="config 2: skip the approximate, DTW and append measurements (e.g. under counters)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run plain 4 GiB device copies (reference for the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this implementation runs on one GPU; --gpus %d is not supported "
                                   "(multi-GPU sharding is a design note only)" % args.gpus}))
        sys.exit(2)

    import torch

    import datagen
    from paper_2009_00786_amd import messi

    if args.copy_calibration:
        return copy_calibration()
    if args.config == 3:
        return bench_batched(args)
    if args.config in (4, 5):
        return bench_serving(args)
    if args.config == 6:
        return bench_windows(args)
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
        threads = host_threads()
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
    ans_i2, ans_d2 = torch.empty_like(ans_i), torch.empty_like(ans_d)
    answers = None
    same_instrumented = True
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
            ix.knn(queries[qi:qi + 1], k, out=(ans_i[qi:qi + 1], ans_d[qi:qi + 1]))
            e = time.perf_counter()
            if timed:
                lat.append((e - a) * 1e3)
        t2 = time.perf_counter()
        # the same queries again with the library's HIP-event phase timing and
        # counters (the events themselves cost device time, so this pass is
        # kept out of the throughput and latency figures)
        for qi in range(nq):
            _, _, st = ix.knn(queries[qi:qi + 1], k, stats=True, out=(ans_i2[qi:qi + 1], ans_d2[qi:qi + 1]))
            if timed:
                for key, v in st.items():
                    agg[key] = agg.get(key, 0) + v
        t3 = time.perf_counter()
        answers = (ans_i.cpu().numpy(), ans_d.cpu().numpy())
        same_instrumented &= bool(torch.equal(ans_i, ans_i2) and torch.equal(ans_d, ans_d2))
        info = ix.info()
        log("step %d%s: build %.1f ms (summarize %.2f, bucket %.2f, split %.2f, finalize %.2f; %d leaves, %d levels), "
            "queries %.1f ms" % (step, "" if timed else " (warmup)", (t1 - t0) * 1e3, info["ms_summarize"],
                                 info["ms_bucket"], info["ms_split"], info["ms_finalize"], info["n_leaves"],
                                 info["levels"], (t2 - t1) * 1e3))
        if timed:
            step_ms.append((t3 - t0) * 1e3)
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
    # the dominant kernel of a step: launches x mean duration -- summarise runs
    # once per step, the scan once per query in each of the step's two query
    # passes (the timed one and the instrumented one); the scan is also the
    # kernel that bounds the headline queries/s
    # summarise: per series the row read, the 16-byte word, the 2-byte root key
    # and the fine summary's 64-byte row (when the index has one) written
    fine_row = 64 if infos[-1].get("fine_segments", 0) else 0
    summ_bytes = n * (length * 4 + 16 + 2 + fine_row)
    scan_bytes_per_q = agg.get("bytes_scan", 0) / total_q
    # The queries/s value is bound by the scan's two kernels; the roofline
    # describes the longer one.  Coarse kernel: per member of the surviving
    # leaves its 8-byte coarse word, per coarse survivor its 4-byte entry in
    # the survivor segment.  Refine kernel: per coarse survivor its segment
    # entry, 16-byte word and 4-byte series index; per word survivor its fine
    # summary; the rows it reads (the library's byte count of the scan less
    # the coarse words).
    coarse_ms_per_q = agg.get("ms_scan_coarse", 0.0) / total_q
    refine_ms_per_q = max(0.0, scan_ms_per_q - coarse_ms_per_q)
    coarse_bytes_per_q = (8 * agg.get("series_bounded", 0) + 4 * agg.get("series_word_bounded", 0)) / total_q
    refine_bytes_per_q = (agg.get("bytes_scan", 0) - 8 * agg.get("series_bounded", 0)
                          + 4 * agg.get("series_word_bounded", 0)) / total_q
    rf_summ = {"bound": "hbm", "achieved": summ_bytes / (summ_ms / 1e3) / 1e9, "peak": HBM_PEAK_GBS,
               "unit": "GB/s", "kernel": "summarize_seg_kernel", "bytes_per_launch": summ_bytes,
               "ms_per_launch": summ_ms, "traffic": traffic_from_profiles("summarize_seg_kernel")}
    if coarse_ms_per_q > 0:
        kname, kb, kms = (("flat_coarse_kernel", coarse_bytes_per_q, coarse_ms_per_q) if coarse_ms_per_q >= refine_ms_per_q
                          else ("flat_refine_kernel", refine_bytes_per_q, refine_ms_per_q))
        rf_scan = {"bound": "hbm", "achieved": kb / (kms / 1e3) / 1e9,
                   "peak": HBM_PEAK_GBS, "unit": "GB/s", "kernel": kname,
                   "bytes_per_launch": kb, "ms_per_launch": kms,
                   "traffic": traffic_from_profiles(kname)}
    else:
        rf_scan = {"bound": "hbm", "achieved": (scan_bytes_per_q / (scan_ms_per_q / 1e3) / 1e9) if scan_ms_per_q else 0.0,
                   "peak": HBM_PEAK_GBS, "unit": "GB/s", "kernel": "scan", "bytes_per_launch": scan_bytes_per_q,
                   "ms_per_launch": scan_ms_per_q, "traffic": None}
    for r in (rf_summ, rf_scan):
        r["frac"] = r["achieved"] / r["peak"]
    rf_summ["launches_per_step"], rf_scan["launches_per_step"] = 1, 2 * nq
    dominant = rf_scan
    roofline = {kk: dominant[kk] for kk in ("bound", "achieved", "peak", "unit", "frac", "traffic")}
    for key in ("kernel", "bytes_per_launch", "ms_per_launch", "launches_per_step"):
        roofline[key] = dominant[key]
    scan_all = {"bytes_per_query": scan_bytes_per_q, "ms_per_query": scan_ms_per_q,
                "achieved_gbps": (scan_bytes_per_q / (scan_ms_per_q / 1e3) / 1e9) if scan_ms_per_q else 0.0,
                "note": "both scan kernels (coarse+word, then fine bound and rows), their algorithmic bytes"}

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
        "roofline_other": rf_summ,
        "scan_all_kernels": scan_all,
        "phases_ms": {"summarize": summ_ms, "bucket": bucket_ms, "split": split_ms,
                      "finalize": float(np.mean([i["ms_finalize"] for i in infos])),
                      "query_prep": agg.get("ms_prep", 0) / total_q, "leaf_lb": agg.get("ms_leaf_lb", 0) / total_q,
                      "approx": agg.get("ms_approx", 0) / total_q, "order": agg.get("ms_order", 0) / total_q,
                      "scan": scan_ms_per_q, "scan_fixup": agg.get("ms_fixup", 0) / total_q,
                      "final": agg.get("ms_final", 0) / total_q,
                      "query_device_total": agg.get("ms_total", 0) / total_q},
        "scan_breakdown_ms": {"coarse_kernel": coarse_ms_per_q, "refine_kernel_and_gap": scan_ms_per_q - coarse_ms_per_q},
        "per_query": {kk: agg.get(kk, 0) / total_q for kk in ("leaves_total", "leaves_kept", "leaves_scanned",
                                                              "series_bounded", "series_word_bounded",
                                                              "series_fine_bounded", "series_distance",
                                                              "series_abandoned", "candidates", "bytes_scan")},
        "index": {"n_leaves": infos[-1]["n_leaves"], "max_leaf": infos[-1]["max_leaf"], "levels": infos[-1]["levels"],
                  "device_bytes": infos[-1]["device_bytes"]},
        "cpu_baseline": cpu,
        "vs_baseline_note": "value / 20 queries/s: the paper's ~50 ms per exact 1-NN query on the same workload "
                            "(100M x 256 random walks, 100 GB) on 2x Xeon E5-2650 v4 -- another machine's number, "
                            "context only; the oracle on this host is cpu_baseline",
        "vs_cpu_baseline": (qps / cpu["value"]) if cpu else None,
        "answers_sha": hashlib.sha256(answers[0].tobytes()).hexdigest()[:16],
        "instrumented_pass_same_answers": same_instrumented,
        "measurement": "a step = index build + the queries answered one at a time (timed: value, p50, p99) + "
                       "the same queries again with the library's HIP-event phase timing and counters (phases, "
                       "roofline: the scan kernel's own event pair on its stream)",
    }
    if args.core_only:
        if ix is not None:
            ix.close()
        print(json.dumps(res), flush=True)
        return
    # the paper's approximate search on the same index and queries (the best
    # leaf's members only): its own rate and how often it finds the exact answer
    apx_i = torch.empty_like(ans_i)
    apx_d = torch.empty_like(ans_d)
    apx_lat = []
    for rep in range(2):
        for qi in range(nq):
            torch.cuda.synchronize()
            a = time.perf_counter()
            ix.knn(queries[qi:qi + 1], k, mode=messi.MODE_APPROX, out=(apx_i[qi:qi + 1], apx_d[qi:qi + 1]))
            torch.cuda.synchronize()
            if rep == 1:
                apx_lat.append((time.perf_counter() - a) * 1e3)
    apx_lat = np.array(apx_lat)
    ai = apx_i.cpu().numpy()
    res["approx_mode"] = {
        "queries_per_s": len(apx_lat) / (apx_lat.sum() / 1e3), "p50_ms": float(np.percentile(apx_lat, 50)),
        "p99_ms": float(np.percentile(apx_lat, 99)),
        "recall_at_%d" % k: float(np.mean([len(set(ai[qi]) & set(answers[0][qi])) / k for qi in range(nq)])),
        "distance_ratio_mean": float(np.mean(apx_d.cpu().numpy()[:, 0] / np.maximum(answers[1][:, 0], 1e-30))),
    }
    # the paper's DTW search on the same index and queries (warping window 10%
    # of the length): its rate, its work, and DTW <= ED for every answer
    band = length // 10
    dtw_i = torch.empty_like(ans_i)
    dtw_d = torch.empty_like(ans_d)
    dtw_lat = []
    for rep in range(2):
        for qi in range(nq):
            torch.cuda.synchronize()
            a = time.perf_counter()
            ix.knn_dtw(queries[qi:qi + 1], k, band, out=(dtw_i[qi:qi + 1], dtw_d[qi:qi + 1]))
            torch.cuda.synchronize()
            if rep == 1:
                dtw_lat.append((time.perf_counter() - a) * 1e3)
    dagg = {}
    for qi in range(nq):
        _, _, st = ix.knn_dtw(queries[qi:qi + 1], k, band, stats=True)
        for key in ("ms_total", "ms_scan", "ms_final", "series_bounded", "series_distance", "series_recheck",
                    "scan_launches"):
            dagg[key] = dagg.get(key, 0) + st[key] / nq
    dtw_lat = np.array(dtw_lat)
    res["dtw_mode"] = {
        "band": band, "k": k, "queries_per_s": len(dtw_lat) / (dtw_lat.sum() / 1e3),
        "p50_ms": float(np.percentile(dtw_lat, 50)), "p99_ms": float(np.percentile(dtw_lat, 99)),
        "per_query": {"lb_keogh": dagg["series_distance"], "dtw": dagg["series_recheck"],
                      "members_bounded": dagg["series_bounded"], "rounds": dagg["scan_launches"],
                      "ms_device": dagg["ms_total"], "ms_rounds": dagg["ms_scan"], "ms_final": dagg["ms_final"]},
        "dtw_le_ed": bool(np.all(dtw_d.cpu().numpy()[:, 0] <= answers[1][:, 0])),
    }
    if cpu is not None:
        res["dtw_mode"]["cpu_baseline"] = cpu_baseline_dtw(data, qraw, k, length, band, n, threads=cpu["cores"])
    if ix is not None:
        ix.close()
        ix = None
    # appending the last 1% of the rows to an index of the first 99%
    n0 = n - n // 100
    ixa = messi.Index(data[:n0], w, b, cap)
    app_ms = []
    for rep in range(2):
        if rep:
            ixa.close()
            ixa = messi.Index(data[:n0], w, b, cap)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ixa.append(data)
        torch.cuda.synchronize()
        app_ms.append((time.perf_counter() - t0) * 1e3)
    ai2, ad2 = ixa.knn(queries, k)
    res["append"] = {"rows_before": n0, "rows_after": n, "ms": app_ms[-1],
                     "gbps": n * length * 4 / (app_ms[-1] / 1e3) / 1e9, "n_leaves": ixa.info()["n_leaves"],
                     "same_answers_as_full_build": bool(np.array_equal(ai2.cpu().numpy(), answers[0]))}
    ixa.close()
    print(json.dumps(res), flush=True)


def cpu_baseline_dtw(data_gpu, q_host_raw, k, length, band, n_total, rows=100_000, nq=10, threads=16):
    """The CPU oracle's brute-force DTW k-NN timed on a bounded sample (nq
    queries over the first `rows` rows), scaled to the full collection."""
    import oracle
    z = oracle.znorm(data_gpu[:rows].cpu().numpy())
    qz = oracle.znorm(q_host_raw[:nq])
    t0 = time.perf_counter()
    oracle.knn_brute_dtw(z, qz, k, band, nthreads=threads)
    t = time.perf_counter() - t0
    return {"value": nq / (t * (n_total / rows)), "unit": "queries/s", "cores": threads, "kind": "oracle",
            "sample": "fp64 brute-force DTW k-NN (oracle, band %d) of %d queries over the first %d rows, %.1f s, "
                      "scaled by %d/%d rows" % (band, nq, rows, t, n_total, rows)}


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


def bench_windows(args):
    """Config 6: the windows of one long random walk as the collection.  A
    step is the windows pass (z-normalised per window), the index build over
    the windows and the queries answered one at a time."""
    import torch

    import datagen
    from paper_2009_00786_amd import messi
    wl = dict(WORKLOADS[6])
    if args.n:
        wl["n"] = args.n
        wl["name"] += " (n=%d)" % args.n
    n, length, nq, k = wl["n"], wl["length"], wl["queries"], wl["k"]
    w, b, cap = 16, 8, 2000
    m = n + length - 1
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    messi.load()
    piece = 4096
    pieces = (m + piece - 1) // piece
    log("generating one random walk of %d points on the GPU (%d pieces of %d, stitched)" % (m, pieces, piece))
    walk = torch.empty((pieces, piece), dtype=torch.float32, device=dev)
    for r0 in range(0, pieces, 1_000_000):
        datagen.gpu_random_walks(walk[r0:r0 + 1_000_000], row0=r0)
    # piece r continues from the last value of piece r - 1
    ends = walk[:, -1].double()
    walk += (torch.cumsum(ends, 0) - ends).float()[:, None]
    long_series = walk.view(-1)[:m]
    rows = torch.empty((n, length), dtype=torch.float32, device=dev)
    qraw = datagen.random_walks(nq, length, seed=datagen.SEED_QUERY, stream=datagen.STREAM_QUERY)
    queries = torch.from_numpy(qraw).to(dev)
    messi.znorm_(queries)
    torch.cuda.synchronize()

    cpu = None
    if not args.no_cpu_baseline:
        r = min(args.cpu_rows, n)
        threads = host_threads()
        messi.windows(long_series[:r + length - 1], length, 1, True, out=rows[:r])
        torch.cuda.synchronize()
        log("cpu baseline: oracle brute force, %d queries x %d windows, %d threads" % (args.cpu_queries, r, threads))
        cpu = cpu_baseline(rows, qraw, k, length, n, r, min(args.cpu_queries, nq), threads)
        log("  ", cpu)

    win_ms, build_ms, query_ms, lat, infos = [], [], [], [], []
    ans_i = torch.empty((nq, k), dtype=torch.int64, device=dev)
    ans_d = torch.empty((nq, k), dtype=torch.float32, device=dev)
    ix = None
    self_ok = True
    for step in range(args.warmup + args.steps):
        timed = step >= args.warmup
        if ix is not None:
            ix.close()
            ix = None
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        ev0.record()
        messi.windows(long_series, length, 1, True, out=rows)
        ev1.record()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ix = messi.Index(rows, w, b, cap)
        t2 = time.perf_counter()
        for qi in range(nq):
            a = time.perf_counter()
            ix.knn(queries[qi:qi + 1], k, out=(ans_i[qi:qi + 1], ans_d[qi:qi + 1]))
            e = time.perf_counter()
            if timed:
                lat.append((e - a) * 1e3)
        t3 = time.perf_counter()
        # a window used as the query finds its own start at distance 0
        probe = int(datagen.uniform_ints(1, n, 62 + step, 5)[0])
        pi, pd = ix.knn(rows[probe:probe + 1].clone(), 1)
        self_ok &= int(pi[0, 0]) == probe and float(pd[0, 0]) == 0.0
        info = ix.info()
        log("step %d%s: windows %.1f ms, build %.1f ms, queries %.1f ms" % (
            step, "" if timed else " (warmup)", ev0.elapsed_time(ev1), (t2 - t1) * 1e3, (t3 - t2) * 1e3))
        if timed:
            win_ms.append(ev0.elapsed_time(ev1))
            build_ms.append((t2 - t1) * 1e3)
            query_ms.append((t3 - t2) * 1e3)
            infos.append(info)
    steps = args.steps
    qps = nq * steps / (sum(query_ms) / 1e3)
    lat_a = np.array(lat)
    wms = float(np.mean(win_ms))
    win_bytes = n * length * 4 + m * 4  # every window written, the long series read once
    roof = {"bound": "hbm", "achieved": win_bytes / (wms / 1e3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "traffic": traffic_from_profiles("znorm_strided_kernel<4, 4>")}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["kernel"] = "znorm_strided_kernel<4, 4> (windows)"
    roof["bytes_per_launch"] = win_bytes
    roof["ms_per_launch"] = wms
    res = {
        "metric": METRIC,
        "value": qps,
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": float(np.mean(win_ms) + np.mean(build_ms) + np.mean(query_ms)),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl["name"], "n": n, "len": length, "long_series_points": m, "step": 1,
                   "segments": w, "card_bits": b, "leaf_cap": cap, "queries": nq, "k": k,
                   "mode": "fp32, one query per call"},
        "p50_ms": float(np.percentile(lat_a, 50)),
        "p99_ms": float(np.percentile(lat_a, 99)),
        "windows_ms": wms,
        "windows_gbps": roof["achieved"],
        "build_ms": float(np.mean(build_ms)),
        "build_gbps": n * length * 4 / (np.mean(build_ms) / 1e3) / 1e9,
        "roofline": roof,
        "self_match": self_ok,
        "index": {"n_leaves": infos[-1]["n_leaves"], "max_leaf": infos[-1]["max_leaf"],
                  "levels": infos[-1]["levels"]},
        "cpu_baseline": cpu,
        "measurement": "a step = the windows pass (HIP events on its stream) + the index build over the windows + "
                       "the queries answered one at a time (value, p50, p99)",
    }
    print(json.dumps(res), flush=True)


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
    # the plain fp32 path on the same batch: its time, and the BF16 answers
    # against it (both exact, so bit-identical)
    fp32_batch_ms = None
    vs_fp32 = None
    last = {kk: ix.knn(batches[-1], kk, mode=messi.MODE_BF16) for kk in (1, 10)}
    if not args.no_fp32_batch:
        vs_fp32 = {"queries": 0, "index_mismatches": 0, "distance_mismatches": 0}
        for kk in (1, 10):
            torch.cuda.synchronize()
            a = time.perf_counter()
            fi, fd = ix.knn(batches[-1], kk, mode=messi.MODE_FP32)
            torch.cuda.synchronize()
            if kk == 1:
                fp32_batch_ms = (time.perf_counter() - a) * 1e3
                log("fp32 batched k=1: %.2f ms" % fp32_batch_ms)
            bi, bd = last[kk]
            vs_fp32["queries"] += nq
            vs_fp32["index_mismatches"] += int((bi != fi).any(dim=1).sum())
            vs_fp32["distance_mismatches"] += int((bd != fd).any(dim=1).sum())
    accuracy = None
    if not args.no_oracle_sample:
        accuracy = oracle_sample_batched(batches[-1], last[10], n, length, args.oracle_sample)
    steps = args.steps
    total_q = 2 * nq * steps
    total_ms = sum(times[1]) + sum(times[10])
    qps = total_q / (total_ms / 1e3)
    f_ms = (agg[1].get("ms_bf16_filter", 0) + agg[10].get("ms_bf16_filter", 0))
    f_flops = agg[1].get("bf16_flops", 0) + agg[10].get("bf16_flops", 0)
    f_bytes = agg[1].get("bytes_scan", 0) + agg[10].get("bytes_scan", 0)
    launches = agg[1].get("bf16_rounds", 0) + agg[10].get("bf16_rounds", 0)
    # The filter's two roofs: the matrix unit (its flops, 16-row tiles counted
    # whole) and HBM (the BF16 member rows and their extra k-step terms it reads,
    # once per leaf and round, plus the recheck's rows).  The binding one is the
    # roofline; the flops per byte sit below the MI355X ridge (2.5 PFLOP/s over
    # 8 TB/s), so it is HBM.
    per_launch_ms = f_ms / max(launches, 1)
    mfma = {"bound": "mfma", "achieved": f_flops / (f_ms / 1e3) / 1e12 if f_ms else 0.0, "peak": 2500.0,
            "unit": "TFLOP/s", "traffic": None, "kernel": "bf16_filter_kernel",
            "flops_per_launch": f_flops / max(launches, 1), "ms_per_launch": per_launch_ms}
    mfma["frac"] = mfma["achieved"] / mfma["peak"]
    hbm = {"bound": "hbm", "achieved": f_bytes / (f_ms / 1e3) / 1e9 if f_ms else 0.0, "peak": HBM_PEAK_GBS,
           "unit": "GB/s", "traffic": traffic_from_profiles("bf16_filter_kernel"), "kernel": "bf16_filter_kernel",
           "bytes_per_launch": f_bytes / max(launches, 1), "ms_per_launch": per_launch_ms}
    hbm["frac"] = hbm["achieved"] / hbm["peak"]
    binding, other = (hbm, mfma) if f_bytes / (HBM_PEAK_GBS * 1e9) >= f_flops / 2.5e15 else (mfma, hbm)
    res = {
        "metric": METRIC, "value": qps, "unit": "queries/s", "n_gpus": 1, "steps": steps, "warmup": args.warmup,
        "ms_per_step": total_ms / steps, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16", "data": "synthetic",
        "config": {"workload": wl["name"], "n": n, "len": length, "segments": 16, "card_bits": 8, "leaf_cap": 2000,
                   "batch": nq, "k": [1, 10], "mode": "BF16 matrix-core filter + compensated fp32 recheck"},
        "qps_k1": nq * steps / (sum(times[1]) / 1e3), "qps_k10": nq * steps / (sum(times[10]) / 1e3),
        "batch_ms_k1": float(np.mean(times[1])), "batch_ms_k10": float(np.mean(times[10])),
        "fp32_batched_k1_ms": fp32_batch_ms,
        "fp32_batched_k1_qps": nq / (fp32_batch_ms / 1e3) if fp32_batch_ms else None,
        "build_ms_with_shadow": build_ms, "shadow_ms": info["ms_shadow"],
        "roofline": binding,
        "roofline_other": other,
        "filter_hbm_gbps": f_bytes / (f_ms / 1e3) / 1e9 if f_ms else 0.0,
        "per_batch": {str(k): {kk: agg[k].get(kk, 0) / steps for kk in (
            "leaves_kept", "series_distance", "series_recheck", "candidates", "ms_bf16_filter", "ms_bf16_recheck",
            "ms_total", "ms_leaf_lb", "ms_approx", "ms_order", "ms_scan", "ms_final", "bf16_rounds",
            "bf16_stage_queries")}
            for k in (1, 10)},
        "discard_rate": 1.0 - (agg[1].get("series_recheck", 0) + agg[10].get("series_recheck", 0)) /
        max(1, agg[1].get("series_distance", 0) + agg[10].get("series_distance", 0)),
        "fp64_rechecks_per_query": {str(k): agg[k].get("candidates", 0) / (nq * steps) for k in (1, 10)},
        "bf16_vs_fp32": vs_fp32,
        "accuracy_vs_oracle": accuracy,
        "cpu_baseline": None,
    }
    ix.close()
    print(json.dumps(res), flush=True)


def oracle_sample_batched(queries_dev, answers, n, length, nsample, k=10):
    """A fixed sample of a batch's queries (every 1024/nsample-th: fresh walks
    and noisy rows alike) against the oracle's brute force over the whole
    collection, regenerated from the seeded generator chunk by chunk and
    z-normalised on the host: index mismatches and the largest relative
    distance error of the k = 10 answers.  Also, for each sampled query and
    its 10 answers plus 100 random rows, the BF16 filter's error as the oracle
    simulates it (exact BF16 products, fp32 sums in index order) over the
    stated bound E: max(observed / E) < 1 is what the filter's exactness rests on."""
    import concurrent.futures

    import torch

    import datagen
    import oracle
    nq = queries_dev.shape[0]
    pick = np.arange(0, nq, max(1, nq // nsample))[:nsample]
    q = queries_dev[torch.from_numpy(pick).to(queries_dev.device)].cpu().numpy()
    gi = answers[0][torch.from_numpy(pick).to(queries_dev.device)].cpu().numpy()
    gd = answers[1][torch.from_numpy(pick).to(queries_dev.device)].cpu().numpy()
    nth = host_threads()
    pool = concurrent.futures.ThreadPoolExecutor(nth)
    chunk = 10_000_000
    raw_dev = torch.empty((min(chunk, n), length), dtype=torch.float32, device=queries_dev.device)
    best_i = np.full((len(q), k), -1, dtype=np.int64)
    best_d = np.full((len(q), k), np.inf)
    t0 = time.perf_counter()
    for r0 in range(0, n, chunk):
        rows = min(chunk, n - r0)
        datagen.gpu_random_walks(raw_dev[:rows], row0=r0)
        raw = raw_dev[:rows].cpu().numpy()
        z = np.concatenate(list(pool.map(oracle.znorm, np.array_split(raw, nth))))
        bi, bd, _ = oracle.knn_brute(z, q, k, nthreads=nth, row_offset=r0)
        ci = np.concatenate([best_i, bi], axis=1)
        cd = np.concatenate([best_d, bd], axis=1)
        order = np.lexsort((ci, cd), axis=1)[:, :k]
        best_i = np.take_along_axis(ci, order, 1)
        best_d = np.take_along_axis(cd, order, 1)
    pool.shutdown()
    ref = np.sqrt(best_d)
    rel = np.abs(gd.astype(np.float64) - ref) / np.maximum(ref, 1e-30)
    # the filter's error model on sampled pairs
    rng_rows = datagen.uniform_ints(100 * len(q), n, 97, 5).reshape(len(q), 100)
    ratio = 0.0
    for i in range(len(q)):
        rows = np.concatenate([best_i[i], rng_rows[i]])
        x = oracle.znorm(np.concatenate([datagen.random_walks(1, length, row0=int(r)) for r in rows]))
        qq = np.repeat(q[i:i + 1], len(rows), axis=0)
        f = oracle.bf16_filter_values(qq, x).astype(np.float64)
        d = np.array([oracle.d64(q[i], xr) for xr in x])
        e = np.array([oracle.bf16_error_bound(float(np.dot(q[i].astype(np.float64), q[i])),
                                              float(np.dot(xr.astype(np.float64), xr)), length) for xr in x])
        ratio = max(ratio, float(np.max(np.abs(f - d) / e)))
    return {"sample_queries": int(len(q)), "k": k, "index_mismatches": int((gi != best_i).any(axis=1).sum()),
            "max_rel_distance_error": float(rel.max()), "max_observed_over_E": ratio,
            "oracle_seconds": time.perf_counter() - t0, "oracle_threads": nth,
            "note": "fp64 brute force over all %d rows (the oracle, host)" % n}


def serving_queries(data, wl, total, centres_dev=None):
    """Per arrival: a query vector, its k, and where it came from.  Dataset rows
    (uniform ids) + sigma * N(0,1), not re-normalised; for the mixture half of
    the arrivals are fresh mixture draws instead (z-normalised)."""
    import torch

    import datagen
    from paper_2009_00786_amd import messi
    n, length = data.shape
    sig_choice = datagen.uniform_ints(total, 3, datagen.SEED_QUERY, 12)
    sig = np.array([0.01, 0.1, 1.0])[sig_choice]
    if wl["data"] == "walk":
        ks = np.array([1, 10, 100])[datagen.uniform_ints(total, 3, datagen.SEED_QUERY, 11)].astype(np.int32)
        ids = datagen.uniform_ints(total, n, datagen.SEED_QUERY, 10)
        base = data[torch.from_numpy(ids).to(data.device)].cpu().numpy()
        return datagen.add_noise(base, sig), ks
    ks = np.full(total, 10, dtype=np.int32)
    n_fresh, n_noisy = (total + 1) // 2, total // 2
    ids = datagen.uniform_ints(n_noisy, n, datagen.SEED_QUERY, 10)
    base = data[torch.from_numpy(ids).to(data.device)].cpu().numpy()
    noisy = datagen.add_noise(base, sig[:n_noisy])
    fresh = torch.empty((n_fresh, length), dtype=torch.float32, device=data.device)
    datagen.gpu_mixture(fresh, centres_dev, seed=datagen.SEED_QUERY, stream=datagen.STREAM_QUERY)
    messi.znorm_(fresh)
    q = np.empty((total, length), dtype=np.float32)
    q[0::2] = fresh.cpu().numpy()
    q[1::2] = noisy
    return q, ks


def open_loop(sv, qs, ks, arrivals, drain_s):
    """Submit query i at arrivals[i] seconds after the start (open loop: the
    schedule never waits for the server), collect results, and return
    per-query latency = completion - scheduled arrival (ms), NaN if unfinished."""
    n = len(arrivals)
    got = {}
    base_ms = sv.clock_ms()
    t_start = time.perf_counter()
    i = 0
    while i < n:
        now = time.perf_counter() - t_start
        if now >= arrivals[i]:
            sv.submit(qs[i], int(ks[i]), i)
            i += 1
            continue
        for r in sv.poll():
            got[r["tag"]] = r
        rem = arrivals[i] - (time.perf_counter() - t_start)
        if rem > 0.0004:
            time.sleep(rem - 0.0002)
    t_last = arrivals[-1]
    while len(got) < n and time.perf_counter() - t_start < t_last + drain_s:
        for r in sv.poll():
            got[r["tag"]] = r
        time.sleep(0.0005)
    lat = np.full(n, np.nan)
    bad = {}
    for tag, r in got.items():
        lat[tag] = r["t_done_ms"] - (base_ms + arrivals[tag] * 1e3)
        if r["status"] != 0:
            bad[str(r["status"])] = bad.get(str(r["status"]), 0) + 1
    in_window = sum(1 for tag, r in got.items() if r["t_done_ms"] - base_ms <= t_last * 1e3)
    return lat, got, in_window, bad


def latency_summary(lat, window_s, in_window):
    done = np.isfinite(lat)
    frac = float(done.mean())
    # an unfinished query has unbounded latency: a percentile that falls on one is reported as null
    srt = np.sort(np.where(done, lat, np.inf))

    def pct(p):
        v = srt[min(len(srt) - 1, int(np.ceil(p / 100.0 * len(srt))) - 1)]
        return float(v) if np.isfinite(v) else None
    return {"arrivals": int(len(lat)), "completed_frac": frac, "sustained_qps": in_window / window_s,
            "p50_ms": pct(50), "p99_ms": pct(99), "saturated": frac < 0.99}


def bench_serving(args):
    """Configurations 4 and 5: open-loop Poisson arrivals against a resident
    index; the BF16 continuous-batching server vs the fp32 single-query FIFO."""
    import torch

    import datagen
    from paper_2009_00786_amd import messi

    wl = dict(WORKLOADS[args.config])
    if args.n:
        wl["n"] = args.n
        wl["name"] += " (n=%d)" % args.n
    rates = [float(r) for r in args.rates.split(",")] if args.rates else list(wl["rates"])
    n, length = wl["n"], wl["length"]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    messi.load()
    data = torch.empty((n, length), dtype=torch.float32, device=dev)
    centres_dev = None
    if wl["data"] == "walk":
        log("generating %d x %d random walks on the GPU" % (n, length))
        for r0 in range(0, n, 10_000_000):
            datagen.gpu_random_walks(data[r0:r0 + 10_000_000], row0=r0)
    else:
        log("generating %d x %d mixture rows on the GPU" % (n, length))
        centres_dev = torch.from_numpy(datagen.mixture_centres(1000, length)).to(dev)
        for r0 in range(0, n, 10_000_000):
            datagen.gpu_mixture(data[r0:r0 + 10_000_000], centres_dev, row0=r0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    messi.znorm_(data)
    torch.cuda.synchronize()
    znorm_ms = (time.perf_counter() - t0) * 1e3
    t0 = time.perf_counter()
    ix = messi.Index(data, 16, 8, 2000, bf16_shadow=True)
    build_ms = (time.perf_counter() - t0) * 1e3
    info = ix.info()
    log("build %.1f ms (shadow %.1f ms), %d leaves" % (build_ms, info["ms_shadow"], info["n_leaves"]))

    schedules = {}
    total = 0
    for r in rates:
        m = int(np.ceil(r * args.duration))
        a = datagen.poisson_arrivals(m + 1, r)
        a = a[a <= args.duration][:m]
        schedules[r] = (total, a)
        total += len(a)
    qs, ks = serving_queries(data, wl, total, centres_dev)
    log("%d arrivals over %s /s, %.0f s each" % (total, rates, args.duration))

    budget = 8 << 30
    out = {}
    results = {}
    # server slots: 4 lanes of 64 queries; the mixture's wide queries (the
    # FP32 filter's growing rounds) gain from batches of 128
    server_slots = slots = int(wl.get("server_slots", 256))
    modes = [("bf16_server", messi.MODE_BF16, slots)]
    if args.variants:
        # the same server with one of its two latency devices switched off,
        # and the slot engine in place of lanes of batches
        modes += [("bf16_batch_only", messi.MODE_BF16 | messi.SERVER_BATCH_ONLY, slots),
                  ("bf16_no_graphs", messi.MODE_BF16 | messi.SERVER_NO_GRAPHS, slots),
                  ("bf16_slots", messi.MODE_BF16 | messi.SERVER_SLOTS, slots)]
    # the FP32 server: lanes of batches on the FP32 matrix-core filter
    modes += [("fp32_server", messi.MODE_FP32, slots)]
    if not args.no_fifo:
        modes += [("fp32_fifo", messi.MODE_FP32, 1)]
    for name, mode, slots in modes:
        out[name] = {}
        for r in rates:
            off, a = schedules[r]
            sv = messi.Server(ix, budget, slots, mode)
            try:
                lat, got, in_window, bad = open_loop(sv, qs[off:off + len(a)], ks[off:off + len(a)], a, 5.0)
                sst = sv.stats()
            finally:
                sv.close()
            summ = latency_summary(lat, float(a[-1]), in_window)
            summ["errors"] = bad
            summ["server"] = sst
            out[name][str(int(r))] = summ
            results[(name, r)] = got
            log("%s at %g/s: %s" % (name, r, summ))

    # exactness: the same query must get the same answer from both servers and
    # when run alone (a fixed sample); every answer is exact, so bit-identical
    mism_modes, compared = 0, 0
    if not args.no_fifo:
        for r in rates:
            g1, g2 = results[("bf16_server", r)], results[("fp32_fifo", r)]
            for tag in set(g1) & set(g2):
                compared += 1
                if not (np.array_equal(g1[tag]["idx"], g2[tag]["idx"]) and
                        np.array_equal(g1[tag]["dist"], g2[tag]["dist"])):
                    mism_modes += 1
    r_head = float(wl["headline_rate"]) if float(wl["headline_rate"]) in schedules else rates[0]
    off, a = schedules[r_head]
    g = results[("bf16_server", r_head)]
    sample = sorted(g)[:: max(1, len(g) // 200)][:200]
    mism_alone = 0
    for tag in sample:
        qi = torch.from_numpy(qs[off + tag:off + tag + 1].copy()).to(dev)
        ai, ad = ix.knn(qi, int(ks[off + tag]))
        if not (np.array_equal(ai.cpu().numpy()[0], g[tag]["idx"]) and
                np.array_equal(ad.cpu().numpy()[0], g[tag]["dist"])):
            mism_alone += 1
    log("alone vs mix: %d/%d mismatches; bf16 server vs fp32 fifo: %d/%d" % (mism_alone, len(sample), mism_modes,
                                                                            compared))
    head = out["bf16_server"][str(int(r_head))]
    res = {
        "metric": METRIC, "value": head["sustained_qps"], "unit": "queries/s", "n_gpus": 1, "steps": len(rates),
        "warmup": 0, "ms_per_step": args.duration * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
        "config": {"workload": wl["name"], "n": n, "len": length, "segments": 16, "card_bits": 8, "leaf_cap": 2000,
                   "rates": rates, "duration_s": args.duration, "headline_rate": r_head, "budget_bytes": budget,
                   "mode": "BF16 continuous-batching server (%d slots over 4 streams; batches replayed as HIP "
                           "graphs; a lone waiting query runs alone in FP32 mode; batches move to the FP32 "
                           "matrix-core filter while BF16 batches overflow)" % server_slots},
        "p50_ms": head["p50_ms"], "p99_ms": head["p99_ms"],
        "serving": out,
        "alone_vs_mix": {"sample": len(sample), "mismatches": mism_alone},
        "bf16_vs_fp32": {"compared": compared, "mismatches": mism_modes},
        "build_ms_with_shadow": build_ms, "znorm_ms": znorm_ms, "build_gbps": n * length * 4 / (build_ms / 1e3) / 1e9,
        "index": {"n_leaves": info["n_leaves"], "max_leaf": info["max_leaf"], "levels": info["levels"],
                  "device_bytes": info["device_bytes"]},
        "roofline": None, "cpu_baseline": None,
    }
    ix.close()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
