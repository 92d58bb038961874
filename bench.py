"""Benchmark of the SSH hot path on one MI355X.

Headline workload (the largest single-GPU configuration): 10,000,000
z-normalised random-walk series of length 2048 (fp32, 81.92 GB resident in
HBM), filter W = 128, step delta = 4, shingle n = 15, 200 weighted-MinHash
hashes (K = 10 per band, L = 20 tables).  One step is one pass of the whole
hot path: sketch, shingle, CWS and band keys of the database, the hash-table
build, then a batch of 4,096 queries (perturbed copies of series among the
first 100,000, N(0, 0.1^2) noise, z-normalised) through sketch, shingle, CWS,
band keys, probe (top C = 200 candidates) and banded DTW re-rank (10 %
Sakoe-Chiba band, top k = 10).

`--workload index` puts the batched index-build configuration on the line
instead: 1,000,000 series of length 1024, W = 80, delta = 3, n = 15, 100
hashes (K = L = 10), 1,000 queries, C = 50, 5 % band.  The default run
reports that configuration's figures as extra keys.

Prints one JSON line: series hashed per second (value), DTW cells per
second, per-stage times, the roofline of the dominant kernel, single-query
latency, recall@10 against exhaustive DTW on sampled queries, and the CPU
oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import json
import math
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_VALU_TFLOPS = 78.6
FP32_VALU_TFLOPS = 157.3
# non-packed vector lane operations per second: 256 CUs x 4 SIMDs x 16 lanes x
# 2.4 GHz (157.3 TFLOP/s counts an FMA as 2 and packed fp32 as 2 lanes)
VALU_LANE_OPS = FP32_VALU_TFLOPS * 1e12 / 4

METRIC = "series hashed/s + DTW cells/s (vs roofline); p50/p99 top-10 query latency"

WORKLOADS = {
    "large": dict(
        workload="large configuration: 10,000,000 random-walk series x 2048 fp32 (81.92 GB in "
                 "HBM), W=128 delta=4 n=15, 200 CWS hashes (K=10, L=20); 4,096 queries, C=200, "
                 "DTW band 10%, top-10",
        N=10_000_000, m=2048, W=128, delta=4, n=15, K=10, L=20, nq=4096, C=200, band=0.10,
        k=10, recall_queries=8),
    "index": dict(
        workload="batched index build: 1,000,000 random-walk series x 1024 fp32, W=80 delta=3 "
                 "n=15, 100 CWS hashes (K=10, L=10); 1,000 queries, C=50, DTW band 5%, top-10",
        N=1_000_000, m=1024, W=80, delta=3, n=15, K=10, L=10, nq=1000, C=50, band=0.05, k=10,
        recall_queries=100),
}

# series per upload chunk: generated on the host, copied, then dropped
UPLOAD_ROWS = 1 << 18

# HBM traffic of one launch of a kernel on a workload, from two rocprofv3
# counter runs of this script (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch),
# each scaled by the ratio of known bytes to the same counter's reading for a
# plain device copy (--copy-calibration).  A figure is reported only while the
# kernel's source file still has the digest it was measured with.
MEASURED_TRAFFIC = {
    # (kernel, workload): (source file, sha256 of it, FETCH_SIZE KiB, WRITE_SIZE KiB,
    #                      fetch scale, write scale); the 1 GiB copy read 524307.1 KiB
    #                      on FETCH_SIZE and 1048576 KiB on WRITE_SIZE
    ("cws_kernel", "large"): ("paper_1610_07328_amd/csrc/cws.hip",
                              "25f92e0afb0880325583d2ea1fa427aac3b8de18fbe3b2218d76023454334d74",
                              147839075.125, 17735884.4375, 1048576.0 / 524307.0625, 1.0),
}


def band_cells(lq: int, lx: int, r: int) -> int:
    """Cells of an lq x lx DTW matrix inside the band |i - j| <= r."""
    total = 0
    for i in range(lq):
        lo, hi = max(0, i - r), min(lx - 1, i + r)
        if hi >= lo:
            total += hi - lo + 1
    return total


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` from the recorded counters, or None."""
    import hashlib
    rec = MEASURED_TRAFFIC.get((kernel, workload))
    if rec is None:
        return None
    src, digest, fetch_kib, write_kib, fs, ws = rec
    path = os.path.join(ROOT, src)
    if not os.path.exists(path):
        return None
    with open(path, "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != digest:
            return None
    return fetch_kib * 1024.0 * fs + write_kib * 1024.0 * ws


def copy_calibration(nbytes: int):
    """One plain device-to-device copy of nbytes (the counter calibration run)."""
    import torch
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda:0")
    b = torch.empty_like(a)
    a.fill_(1)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": nbytes}), flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="large")
    ap.add_argument("--n-series", type=int, default=0, help="override the workload's series count")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the other workload's figures")
    ap.add_argument("--latency-samples", type=int, default=200)
    ap.add_argument("--recall-queries", type=int, default=-1)
    ap.add_argument("--cpu-sample", type=int, default=100_000)
    ap.add_argument("--no-serving", action="store_true", help="skip the serving run")
    ap.add_argument("--serving-only", action="store_true", help="only the serving run")
    ap.add_argument("--no-uneven", action="store_true", help="skip the uneven-batch run")
    ap.add_argument("--uneven-only", action="store_true", help="only the uneven-batch run")
    ap.add_argument("--serve-requests", type=int, default=6000)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run one device copy of BYTES bytes (counter calibration)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-multi", action="store_true", help="skip the multi-filter sketch run")
    ap.add_argument("--multi-only", action="store_true", help="only the multi-filter sketch run")
    ap.add_argument("--seed", type=int, default=0)
    return ap.parse_args()


def log(msg: str):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# --------------------------------------------------------------------------
# CPU baseline: the oracle, unchanged, over the host's cores
# --------------------------------------------------------------------------
_W = {}


def _cpu_init(cfg, seed):
    from paper_1610_07328_amd import datagen
    _W["cfg"] = cfg
    _W["r"] = datagen.filter_r(cfg["W"], seed=seed)
    _W["draws"] = datagen.cws_draws(cfg["n"], cfg["K"] * cfg["L"], seed=seed)


def _cpu_hash(X):
    """Sketch, shingle, CWS and band keys of rows X with the oracle; returns the
    number of series hashed."""
    import oracle
    cfg, r, draws = _W["cfg"], _W["r"], _W["draws"]
    B = oracle.sketch_batch(X, r, cfg["W"], cfg["delta"])
    sets = [oracle.shingle(b, cfg["n"]) for b in B]
    smax = max([2] + [int(c.max()) for _, c in sets if len(c)])
    lnS = oracle.ln_table(smax)
    hv = np.stack([oracle.cws(c, k, *draws, lnS)[2] for c, k in sets])
    oracle.band_keys(hv, cfg["K"], cfg["L"], 0x5EED)
    return X.shape[0]


def cpu_baseline(cfg, seed: int, sample: int, Q):
    """The CPU oracle on the first `sample` series of the workload, split over the
    host's cores (at most 16, the host share of one GPU), and its DTW on 64
    queries x C random candidates of the same shape."""
    from oracle import _dtw_c
    from paper_1610_07328_amd import datagen

    cores = min(16, len(os.sched_getaffinity(0)))
    X = datagen.random_walk_rows(0, sample, cfg["m"], seed=seed)
    parts = np.array_split(X, cores * 4)
    ctx = mp.get_context("spawn")
    with cf.ProcessPoolExecutor(cores, mp_context=ctx, initializer=_cpu_init,
                                initargs=(cfg, seed)) as ex:
        list(ex.map(_cpu_hash, [X[:cores]] * cores))  # workers started and warm
        t0 = time.perf_counter()
        done = sum(ex.map(_cpu_hash, parts))
        t_hash = time.perf_counter() - t0
    nqs = 64
    q, qoff = datagen.csr(Q[:nqs])
    db, dboff = datagen.csr(X)
    rng = np.random.default_rng(0)
    cand = rng.integers(0, sample, size=(nqs, cfg["C"])).astype(np.int64)
    ncand = np.full(nqs, cfg["C"], np.int32)
    t1 = time.perf_counter()
    _dtw_c.dtw_pairs(q, qoff, db, dboff, cand, ncand, cfg["band"])
    t_dtw = time.perf_counter() - t1
    rr = int(math.floor(float(np.float32(cfg["band"])) * cfg["m"]))
    cells = nqs * cfg["C"] * band_cells(cfg["m"], cfg["m"], rr)
    try:
        cpu = [ln.split(":", 1)[1].strip() for ln in open("/proc/cpuinfo")
               if ln.startswith("model name")][0]
    except (OSError, IndexError):
        cpu = "unknown"
    return {
        "value": done / t_hash,
        "unit": "series hashed/s",
        "cores": cores,
        "kind": "oracle",
        "sample": f"first {done} series of the workload through the oracle's sketch, shingle, "
                  f"CWS and band keys (numpy float64), split over {cores} worker processes; DTW "
                  f"of {nqs} queries x {cfg['C']} candidates in the oracle's C with OpenMP",
        "cpu_model": cpu,
        "host_cpus": os.cpu_count(),
        "hash_seconds": t_hash,
        "dtw_cells_per_s": cells / t_dtw,
        "dtw_cores": _dtw_c.num_threads(),
    }


# --------------------------------------------------------------------------
# GPU runs
# --------------------------------------------------------------------------
def upload_walks(N: int, m: int, seed: int, dev):
    """The workload's random walks, generated on the host in chunks of
    UPLOAD_ROWS series and copied into one device array (the host never holds
    more than two chunks)."""
    import torch

    from paper_1610_07328_amd import datagen
    x = torch.empty(N * m, dtype=torch.float32, device=dev)
    chunks = [(lo, min(N, lo + UPLOAD_ROWS)) for lo in range(0, N, UPLOAD_ROWS)]
    with cf.ThreadPoolExecutor(1) as ex:
        nxt = ex.submit(datagen.random_walk_rows, *chunks[0], m, seed)
        for i, (lo, hi) in enumerate(chunks):
            rows = nxt.result()
            if i + 1 < len(chunks):
                nxt = ex.submit(datagen.random_walk_rows, *chunks[i + 1], m, seed)
            x[lo * m:hi * m].copy_(torch.from_numpy(rows.reshape(-1)))
            del rows
    return x


def hbm_copy_microbench(nbytes: int = 1 << 32, reps: int = 10) -> dict:
    """A plain device-to-device copy of nbytes, timed with events: the HBM rate
    a streaming kernel reaches on this GPU (bytes read plus bytes written),
    beside the 8 TB/s datasheet peak the rooflines use."""
    import torch
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda:0")
    b = torch.empty_like(a)
    a.fill_(1)
    ms = event_ms(lambda: b.copy_(a), reps)
    gbs = 2 * nbytes / (ms / 1e3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    return {"bytes_read_plus_written": 2 * nbytes, "ms": ms, "GB/s": gbs,
            "frac_of_peak": gbs / HBM_PEAK_GBS}


def event_ms(fn, reps: int) -> float:
    import torch
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    fn()
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def run_workload(name: str, args, main: bool):
    import torch

    from paper_1610_07328_amd import datagen, ssh
    from paper_1610_07328_amd.pipeline import (HashBatch, Index, Params, QueryBatch,
                                               exhaustive_topk)

    cfg = dict(WORKLOADS[name])
    if main and args.n_series > 0:
        cfg["N"] = args.n_series
    N, m, nq = cfg["N"], cfg["m"], cfg["nq"]
    p = Params(W=cfg["W"], delta=cfg["delta"], n=cfg["n"], K=cfg["K"], L=cfg["L"],
               band_frac=cfg["band"], C=cfg["C"], k=cfg["k"])
    steps = args.steps if main else 3
    warmup = args.warmup if main else 1
    dev = torch.device("cuda:0")
    seed = args.seed

    t0 = time.perf_counter()
    xd = upload_walks(N, m, seed, dev)
    off = np.arange(N + 1, dtype=np.int64) * m
    first = datagen.random_walk_rows(0, min(N, 100_000), m, seed=seed)
    Q, src = datagen.perturbed_queries(first, nq, 0.1, seed=seed)
    r = datagen.filter_r(p.W, seed=seed)
    draws = datagen.cws_draws(p.n, p.H, seed=seed)
    log(f"{name}: {N} x {m} series generated and resident in {time.perf_counter() - t0:.1f}s")

    q, qoff = datagen.csr(Q)
    qd = torch.as_tensor(q).to(dev)
    tables = ssh.CwsTables(*draws, p.n, device=dev)
    db = HashBatch(xd, off, p)
    qb = HashBatch(qd, qoff, p)
    index = Index(db)
    qry = QueryBatch(qb, index)
    torch.cuda.synchronize()

    # "cws" is the CWS kernel with the band keys folded in (one launch)
    stages = ["sketch", "shingle", "cws", "table_build", "q_hash", "probe", "rerank"]

    def step(ev=None):
        def mark(i):
            if ev is not None:
                ev[i].record()
        mark(0)
        db.sketch(r)
        mark(1)
        db.shingle()
        mark(2)
        db.cws_band_keys(tables)
        mark(3)
        index.build()
        mark(4)
        qb.run(r, tables)
        mark(5)
        qry.probe()
        mark(6)
        qry.rerank()
        mark(7)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ssh.check_device_errors()
    events = [[torch.cuda.Event(enable_timing=True) for _ in range(len(stages) + 1)]
              for _ in range(steps)]
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for s in range(steps):
        step(events[s])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    ssh.check_device_errors()
    log(f"{name}: {steps} steps in {wall:.2f}s")

    per_stage = {k: 0.0 for k in stages}
    for ev in events:
        for i, k in enumerate(stages):
            per_stage[k] += ev[i].elapsed_time(ev[i + 1]) / steps  # ms

    # workload facts for the algorithmic counts
    ncand = qry.ncand[:nq].cpu().numpy()
    rsz = qry.rsize[:nq].cpu().numpy().astype(np.float64)
    nd = db.ndist[:N].cpu().numpy().astype(np.int64)
    repaired = int(db.repair.cpu().numpy()[0]) / (warmup + steps)
    nb = int(db.plan.max_nbits)
    words = (nb + 63) // 64
    rr = int(math.floor(float(np.float32(p.band_frac)) * m))
    cells_per_pair = band_cells(m, m, rr)
    step_cells = int(ncand.sum()) * cells_per_pair
    sum_d = int(nd.sum())
    bytes_stage = {
        "sketch": N * (4 * m + 8 * words + 4) + 16 * (N + 1),
        "shingle": N * (8 * words + 4 + 4) + 16 * (N + 1) + 8 * sum_d,
        "cws": 8 * sum_d + N * (8 * p.H + 4 + 8 + 8 * p.L),
        # radix passes over the top 24 bits (N <= 2^24) or 32: keys and ids read twice, written once
        "table_build": (3 if N <= (1 << 24) else 4) * N * p.L * (8 + 12 + 12),
    }
    stage_hbm = {k: {"GB/s": b / (per_stage[k] / 1e3) / 1e9,
                     "frac_hbm": b / (per_stage[k] / 1e3) / 1e9 / HBM_PEAK_GBS}
                 for k, b in bytes_stage.items()}
    cws_evals = sum_d * p.H

    # the re-rank kernels on a full batch: every query re-ranks C seeded random
    # candidates of the same shape (plain, then pruned)
    g = np.random.default_rng(seed + 1)
    cand_full = torch.as_tensor(g.integers(0, N, size=(nq, p.C)), device=dev)
    ncand_full = torch.full((nq,), p.C, dtype=torch.int32, device=dev)
    ws_full = torch.empty(ssh.rerank_workspace_bytes(nq, p.C), dtype=torch.uint8, device=dev)
    out_full = (torch.empty((nq, p.k), dtype=torch.int64, device=dev),
                torch.empty((nq, p.k), dtype=torch.float32, device=dev))
    ws_lb = torch.empty(ssh.rerank_lb_workspace_bytes(nq, p.C, qb.x.numel()), dtype=torch.uint8,
                        device=dev)
    out_lb = (torch.empty_like(out_full[0]), torch.empty_like(out_full[1]))

    def full_rerank(prune):
        ssh.dtw_rerank(qb.x, qb.x_off, db.x, db.x_off, cand_full, ncand_full, p.band_frac, p.k,
                       ws=ws_lb if prune else ws_full, out=out_lb if prune else out_full,
                       prune=prune)

    reps = 3 if main else 5
    t_full = event_ms(lambda: full_rerank(False), reps) / 1e3
    t_lb = event_ms(lambda: full_rerank(True), reps) / 1e3
    same = bool(torch.equal(out_lb[0], out_full[0]) and
                torch.equal(out_lb[1].view(torch.int32), out_full[1].view(torch.int32)))
    full_cells = nq * p.C * cells_per_pair
    dtw_full = {"cells_per_s": full_cells / t_full, "ms": t_full * 1e3, "pairs": nq * p.C,
                "cells": full_cells, "alu_frac": full_cells * 3 / t_full / VALU_LANE_OPS,
                "lb_pruned": {"ms": t_lb * 1e3, "speedup": t_full / t_lb, "same_results": same}}
    # the pruned re-rank on the step's own candidate lists
    ws_lbs = torch.empty(ssh.rerank_lb_workspace_bytes(nq, p.C, qb.x.numel()), dtype=torch.uint8,
                         device=dev)
    t_step_plain = event_ms(lambda: ssh.dtw_rerank(qb.x, qb.x_off, db.x, db.x_off, qry.cand[:nq],
                                                   qry.ncand[:nq], p.band_frac, p.k, ws=ws_lbs,
                                                   prune=False), 5)
    t_step_lb = event_ms(lambda: ssh.dtw_rerank(qb.x, qb.x_off, db.x, db.x_off, qry.cand[:nq],
                                                qry.ncand[:nq], p.band_frac, p.k, ws=ws_lbs,
                                                prune=True), 5)
    del ws_lb, ws_lbs

    # single-query latency with the index resident
    lat = []
    if args.latency_samples > 0:
        singles = []
        for i in range(min(args.latency_samples, nq)):
            qi, qio = datagen.csr(Q[i: i + 1])
            hb = HashBatch(torch.as_tensor(qi).to(dev), qio, p)
            singles.append((hb, QueryBatch(hb, index)))
        torch.cuda.synchronize()
        for hb, qq in singles:
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            hb.run(r, tables)
            qq.probe()
            qq.rerank()
            e1.record()
            e1.synchronize()
            lat.append(e0.elapsed_time(e1))
        del singles
    lat = np.array(lat) if lat else np.array([float("nan")])

    # recall@10: the step's top-10 against exhaustive DTW over all N series, on a
    # seeded random sample of the queries
    nrec = cfg["recall_queries"] if args.recall_queries < 0 else args.recall_queries
    recall = None
    if nrec > 0:
        t_r = time.perf_counter()
        ids_step = qry.ids[:nq].cpu().numpy()
        pick = np.sort(np.random.default_rng(seed + 2).choice(nq, min(nrec, nq), replace=False))
        hits, tot, src_exact, answered = 0, 0, 0, 0
        for i in pick:
            ex_id, ex_d = exhaustive_topk(qb.x[qoff[i]:qoff[i + 1]], db.x, db.x_off, p.band_frac,
                                          p.k)
            want = set(ex_id.cpu().numpy().tolist()) - {-1}
            got = set(ids_step[i].tolist()) - {-1}
            hits += len(want & got)
            tot += len(want)
            src_exact += int(src[i] in want)
            answered += int(ncand[i] > 0)
        recall = {"recall_at_10": hits / max(tot, 1), "queries": int(len(pick)),
                  "queries_with_candidates": answered,
                  # the ground truth holds each sampled query's source series
                  "exhaustive_top10_holds_source": src_exact / len(pick),
                  "seconds": time.perf_counter() - t_r,
                  # every query is a noisy copy of a database series: how often
                  # that series is among the step's top 10, over all queries
                  "source_in_top10": float(np.mean([src[i] in set(ids_step[i].tolist())
                                                    for i in range(nq)]))}
        log(f"{name}: recall@10 {recall['recall_at_10']:.3f} on {recall['queries']} queries")

    def hash_agreement(hv, src_ids):
        """Mean share of a query's hash values equal to its source series' ones."""
        mine = hv.view(torch.int64)
        theirs = db.hv.view(torch.int64)[torch.as_tensor(src_ids, device=dev)]
        return float((mine == theirs).float().mean())

    # query noise sweep: fresh perturbed copies at lower noise through the same
    # index (hash, probe, re-rank), so the share of queries that find their
    # source shows where near duplicates survive the sketch's sign bits
    noise_sweep = []
    if nrec > 0:
        t_s = time.perf_counter()
        nq_s = min(nq, 1024)
        n_rec_s = max(1, nrec // 2)
        noise_sweep.append({"noise_std": 0.1, "queries": nq,
                            "hash_agreement_with_source": hash_agreement(qb.hv[:nq], src),
                            "source_in_top10": recall["source_in_top10"],
                            "queries_with_candidates": int((ncand > 0).sum()) / nq,
                            "recall_at_10": recall["recall_at_10"],
                            "recall_queries": recall["queries"]})
        for li, sd in enumerate((0.03, 0.01)):
            Qs, srcs = datagen.perturbed_queries(first, nq_s, sd, seed=seed + 11 + li)
            qs, qsoff = datagen.csr(Qs)
            hbs = HashBatch(torch.as_tensor(qs).to(dev), qsoff, p)
            qys = QueryBatch(hbs, index)
            hbs.run(r, tables)
            qys.probe()
            qys.rerank()
            torch.cuda.synchronize()
            ssh.check_device_errors()
            ids_s = qys.ids[:nq_s].cpu().numpy()
            nc_s = qys.ncand[:nq_s].cpu().numpy()
            pick_s = np.sort(np.random.default_rng(seed + 21 + li).choice(nq_s, n_rec_s,
                                                                          replace=False))
            hits, tot = 0, 0
            for i in pick_s:
                ex_id, _ = exhaustive_topk(hbs.x[qsoff[i]:qsoff[i + 1]], db.x, db.x_off,
                                           p.band_frac, p.k)
                want = set(ex_id.cpu().numpy().tolist()) - {-1}
                hits += len(want & (set(ids_s[i].tolist()) - {-1}))
                tot += len(want)
            noise_sweep.append({
                "noise_std": sd, "queries": nq_s,
                "hash_agreement_with_source": hash_agreement(hbs.hv[:nq_s], srcs),
                "source_in_top10": float(np.mean([srcs[i] in set(ids_s[i].tolist())
                                                  for i in range(nq_s)])),
                "queries_with_candidates": float((nc_s > 0).mean()),
                "recall_at_10": hits / max(tot, 1), "recall_queries": int(len(pick_s))})
            log(f"{name}: noise {sd}: source in top 10 for "
                f"{noise_sweep[-1]['source_in_top10']:.3f} of {nq_s} queries, recall@10 "
                f"{noise_sweep[-1]['recall_at_10']:.3f} on {len(pick_s)}")
            del hbs, qys
        recall["noise_sweep"] = noise_sweep
        recall["noise_sweep_seconds"] = time.perf_counter() - t_s

    # the integer-replication weighted MinHash (with band keys) in place of
    # CWS on the same weighted sets, after everything above has read the CWS
    # hash values
    t_wmh = event_ms(db.wmh_int_band_keys, 5)
    wmh_pairs = N * max(int(db.plan.max_nbits) - p.n + 1, 0) * p.H  # equal lengths: every set
    wmh = {"ms": t_wmh, "pairs": wmh_pairs, "pairs_per_s": wmh_pairs / (t_wmh / 1e3),
           "cws_ms": per_stage["cws"]}
    log(f"{name}: integer-replication MinHash {t_wmh:.2f} ms ({wmh['pairs_per_s']:.3g} pairs/s)")

    # dominant stage and its roofline
    dominant = max(["sketch", "shingle", "cws", "table_build", "rerank"], key=lambda k: per_stage[k])
    if dominant == "rerank":
        achieved = step_cells * 3 / (per_stage["rerank"] / 1e3) / 1e12
        peak = VALU_LANE_OPS / 1e12
        roof = {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "Tops/s",
                "frac": achieved / peak, "traffic": None, "kernel": "dtw_group_kernel"}
    else:
        kname = {"sketch": "sketch_mfma_kernel", "shingle": "shingle_kernel", "cws": "cws_kernel",
                 "table_build": "rs_scatter_kernel"}[dominant]
        achieved = bytes_stage[dominant] / (per_stage[dominant] / 1e3) / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(kname, name),
                "kernel": kname, "kernel_ms": per_stage[dominant],
                "algorithmic_bytes": bytes_stage[dominant]}
        if dominant == "cws":
            roof["token_hash_evals_per_s"] = cws_evals / (per_stage["cws"] / 1e3)
            # the same kernel against the FP64 vector peak: about 6 lane operations
            # per (token, hash) evaluation in its keyed form
            roof["valu_lane_ops_per_eval"] = 6

    res = {
        "value": N * steps / wall,
        "ms_per_step": wall * 1000.0 / steps,
        "steps": steps,
        "warmup": warmup,
        "config": {"workload": cfg["workload"], "n_series": N, "length": m, "W": p.W,
                   "delta": p.delta, "n": p.n, "K": p.K, "L": p.L, "queries": nq, "C": p.C,
                   "band_frac": p.band_frac, "k": p.k},
        # the cells of every candidate pair's band over the re-rank stage's time
        # (an effective rate when the step prunes: pruned pairs count too)
        "dtw_cells_per_s": step_cells / (per_stage["rerank"] / 1e3),
        "dtw_step_pairs": int(ncand.sum()),
        "dtw_full_batch": dtw_full,
        "rerank_step_candidates": {"plain_ms": t_step_plain, "pruned_ms": t_step_lb,
                                   "speedup": t_step_plain / t_step_lb,
                                   "step_uses": "pruned" if qry.prune else "plain"},
        "query_latency_ms": {"p50": float(np.percentile(lat, 50)),
                             "p99": float(np.percentile(lat, 99)),
                             "samples": int(lat.size), "batch": 1},
        "recall": recall,
        "stage_ms": per_stage,
        "stage_hbm": stage_hbm,
        "retrieved_set": {"mean": float(rsz.mean()), "p50": float(np.percentile(rsz, 50)),
                          "p99": float(np.percentile(rsz, 99)), "max": float(rsz.max()),
                          "pruned_frac": float(1.0 - rsz.mean() / N),
                          "queries_with_candidates": int((ncand > 0).sum())},
        "sketch_fp64_repaired_windows": repaired,
        "mean_distinct_shingles": sum_d / N,
        "wmh_int": wmh,
        "roofline": roof,
    }
    # free the device state before anything else runs
    del db, qb, index, qry, xd, tables, cand_full, ws_full
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return res, cfg, Q


UNEVEN = dict(
    workload="uneven batch: 200,000 series of lengths uniform in [256, 8192] (even ids random "
             "walk, odd ECG-like), fp32; W=80 delta=3 n=15, 100 CWS hashes (K=10, L=10); one "
             "launch per stage, autotuned sketch work item and series order, build captured in "
             "a HIP graph",
    N=200_000, lo=256, hi=8192, plain_sample=2000)


def run_uneven(args):
    """The batched index build of an uneven batch (paper_1610_07328_amd.batching): tuned,
    graph-captured and replayed, against eager launches, the untuned default and the plain
    per-series form."""
    import torch

    from paper_1610_07328_amd import datagen, ssh
    from paper_1610_07328_amd.batching import TuneCache, UnevenBuild, autotune
    from paper_1610_07328_amd.pipeline import HashBatch, Params

    cfg = UNEVEN
    seed = args.seed
    p = Params(W=80, delta=3, n=15, K=10, L=10)
    t0 = time.perf_counter()
    x, off = datagen.ragged_series(cfg["N"], cfg["lo"], cfg["hi"], seed=seed)
    N, samples = len(off) - 1, int(off[-1])
    r = datagen.filter_r(p.W, seed=seed)
    tables = ssh.CwsTables(*datagen.cws_draws(p.n, p.H, seed=seed), p.n)
    log(f"uneven: {N} series ({samples} samples) generated in {time.perf_counter() - t0:.1f}s")
    t1 = time.perf_counter()
    cache = TuneCache()
    choice, hit = autotune(x, off, p, tables, r, cache)
    t_tune = time.perf_counter() - t1
    _, hit_again = autotune(x, off, p, tables, r, TuneCache(cache.path))
    log(f"uneven: tuner chose {choice['order']} / {choice['tile_rows']} rows "
        f"({'cache' if hit else 'timed'}, {t_tune:.1f}s)")

    def timed(fn, reps=10):
        return event_ms(fn, reps)

    b = UnevenBuild(x, off, p, tables, r, order=choice["order"], tile_rows=choice["tile_rows"])
    t_eager = timed(b.run)
    b.capture()
    t_graph = timed(b.replay)
    # hashing stages alone (the part a per-series form can do)
    db = b.db

    def hash_only():
        ssh.sketch(db.x, db.x_off, r, p.W, p.delta, db.bwo, out=(db.bits, db.nbits, db.repair),
                   tile_rows=b.tile_rows)
        db.shingle()
        db.cws_band_keys(tables)

    t_hash = timed(hash_only)
    hv_batch = b.hv().cpu().numpy()
    del b, db
    torch.cuda.empty_cache()
    d = UnevenBuild(x, off, p, tables, r)
    t_default = timed(d.run)
    del d
    torch.cuda.empty_cache()
    # the plain per-series form: one launch sequence per series, on a sample
    rng = np.random.default_rng(seed + 3)
    pick = rng.choice(N, cfg["plain_sample"], replace=False)
    singles = []
    for s in pick:
        hb = HashBatch(torch.as_tensor(x[off[s]:off[s + 1]]).cuda(),
                       np.array([0, off[s + 1] - off[s]], np.int64), p)
        singles.append(hb)
    torch.cuda.synchronize()

    def plain():
        for hb in singles:
            hb.run(r, tables)

    t_plain = timed(plain, reps=2)
    same = all(np.array_equal(hb.hv[0].cpu().numpy(), hv_batch[s]) for hb, s in zip(singles, pick))
    plain_samples = int(sum(off[s + 1] - off[s] for s in pick))
    del singles
    torch.cuda.empty_cache()
    out = {"config": {"workload": cfg["workload"], "n_series": N, "samples": samples,
                      "W": p.W, "delta": p.delta, "n": p.n, "K": p.K, "L": p.L},
           "tuner": {"order": choice["order"], "tile_rows": choice["tile_rows"],
                     "build_ms_by_choice": choice["build_ms"], "seconds": t_tune,
                     "cache_hit_first": hit, "cache_hit_second": hit_again, "cache": cache.path},
           "graph_build_ms": t_graph, "eager_build_ms": t_eager, "default_build_ms": t_default,
           "series_per_s": N / (t_graph / 1e3), "samples_per_s": samples / (t_graph / 1e3),
           "batched_hash_ms": t_hash, "batched_hash_series_per_s": N / (t_hash / 1e3),
           "plain_per_series": {"series": len(pick), "ms": t_plain,
                                "series_per_s": len(pick) / (t_plain / 1e3),
                                "samples_per_s": plain_samples / (t_plain / 1e3)},
           "batched_over_plain": (N / (t_hash / 1e3)) / (len(pick) / (t_plain / 1e3)),
           "plain_equals_batched": bool(same)}
    log(f"uneven: graph build {t_graph:.2f} ms ({out['series_per_s']:.3e} series/s), "
        f"plain per-series {out['plain_per_series']['series_per_s']:.3e} series/s")
    del tables
    torch.cuda.empty_cache()
    return out


SERVING = dict(
    workload="serving: Poisson stream at 2,000 queries/s of lengths 128, 512, 1024 and 2048 "
             "(noisy copies of stride-1 windows of one random-walk stream), against one "
             "resident index of 1,000,000 z-normalised windows per length (4,000,000 series, "
             "14.8 GB), W=80 delta=3 n=15, 100 CWS hashes (K=10, L=10), C=1024, DTW band 5%, "
             "top-10; recall@10 on every 100th arrival against exhaustive DTW",
    lengths=(128, 512, 1024, 2048), windows=1_000_000, rate=2000.0, C=1024, band=0.05,
    arena=256 << 20, max_batch=64, slots=4)


def run_serving(args):
    """Continuous batching over the resident mixed-length index (paper_1610_07328_amd.serving),
    then the plain form (one query at a time) on the same arrival trace."""
    import torch

    from paper_1610_07328_amd import datagen, ssh
    from paper_1610_07328_amd.pipeline import HashBatch, Params, exhaustive_topk
    from paper_1610_07328_amd.serving import (GpuExecutor, MixedIndex, Request, RingArena,
                                              Scheduler, latency_summary)

    cfg = SERVING
    seed = args.seed
    dev = torch.device("cuda:0")
    p = Params(W=80, delta=3, n=15, K=10, L=10, band_frac=cfg["band"], C=cfg["C"], k=10)
    lens, nwin = cfg["lengths"], cfg["windows"]
    t0 = time.perf_counter()
    stream = datagen.walk_stream(nwin + max(lens) - 1, seed=seed)
    total = sum(lens) * nwin
    x = torch.empty(total, dtype=torch.float32, device=dev)
    base = 0
    for ell in lens:
        for lo in range(0, nwin, 1 << 17):
            hi = min(nwin, lo + (1 << 17))
            w = datagen.stream_windows(stream, ell, lo, hi)
            x[base + lo * ell: base + hi * ell].copy_(torch.from_numpy(w.reshape(-1)))
        base += ell * nwin
    r = datagen.filter_r(p.W, seed=seed)
    draws = datagen.cws_draws(p.n, p.H, seed=seed)
    tables = ssh.CwsTables(*draws, p.n, device=dev)
    t1 = time.perf_counter()
    ix = MixedIndex(x, [(ell, nwin) for ell in lens], p, tables, r)
    t_index = time.perf_counter() - t1
    log(f"serving: {len(lens)} x {nwin} windows resident in {t1 - t0:.1f}s, index built in "
        f"{t_index:.2f}s")
    arr, cls, src, qv = datagen.stream_queries(stream, lens, nwin, args.serve_requests,
                                               cfg["rate"], seed=seed)
    reqs = [Request(i, float(arr[i]), int(cls[i]), qv[i]) for i in range(len(qv))]
    ex = GpuExecutor(ix, cfg["arena"], slots=cfg["slots"], max_batch=cfg["max_batch"],
                     max_len=max(lens))
    # warm-up on the first 200 arrivals (kernel loading, first launches)
    Scheduler(ex, RingArena(cfg["arena"]), cfg["max_batch"], cfg["slots"]).run(reqs[:200])
    torch.cuda.synchronize()

    def serve(max_batch, slots):
        arena = RingArena(cfg["arena"])
        res, st = Scheduler(ex, arena, max_batch, slots).run(reqs)
        ssh.check_device_errors()
        lat = latency_summary(reqs, res)
        last = max(rr.completion for rr in res if not rr.refused)
        return res, {"latency_ms": lat, "throughput_qps": lat["served"] / last,
                     "batches": st.batches, "mean_batch": float(np.mean(st.batch_sizes)),
                     "max_batch": int(max(st.batch_sizes)), "inflight_max": st.inflight_max,
                     "arena_peak_bytes": st.arena_peak, "arena_bytes": arena.capacity,
                     "refused": st.refused, "wall_s": st.wall}

    res, batched = serve(cfg["max_batch"], cfg["slots"])
    log(f"serving: p50 {batched['latency_ms']['p50']:.3f} ms, p99 "
        f"{batched['latency_ms']['p99']:.3f} ms, {batched['batches']} batches")
    res_plain, plain = serve(1, 1)
    log(f"serving, plain form: p50 {plain['latency_ms']['p50']:.3f} ms, p99 "
        f"{plain['latency_ms']['p99']:.3f} ms")
    same = all(np.array_equal(a.ids, b.ids) and np.array_equal(a.dist.view(np.uint32),
                                                                 b.dist.view(np.uint32))
               for a, b in zip(res, res_plain))

    # capacity: every request of a burst arrives at once
    burst = [Request(q.rid, 0.0, q.cls, q.values) for q in reqs[:2000]]

    def capacity(max_batch, slots):
        res_b, st = Scheduler(ex, RingArena(cfg["arena"]), max_batch, slots).run(burst)
        last = max(rr.completion for rr in res_b)
        return {"requests": len(burst), "makespan_s": last, "throughput_qps": len(burst) / last,
                "mean_batch": float(np.mean(st.batch_sizes))}

    cap_batched = capacity(cfg["max_batch"], cfg["slots"])
    cap_plain = capacity(1, 1)
    log(f"serving capacity: {cap_batched['throughput_qps']:.0f} q/s batched, "
        f"{cap_plain['throughput_qps']:.0f} q/s one at a time")

    # recall@10 on every 100th arrival against exhaustive DTW over the class's windows
    t_r = time.perf_counter()
    offs_c = np.concatenate([[0], np.cumsum([ell * nwin for ell in lens])])
    sample = [q for q in reqs if q.rid % 100 == 0]
    truth = {}
    src_in = 0
    for j, q in enumerate(sample):
        ell = lens[q.cls]
        dbx = x[offs_c[q.cls]:offs_c[q.cls + 1]]
        dbo = torch.arange(nwin + 1, dtype=torch.int64, device=dev) * ell
        ex_id, ex_d = exhaustive_topk(torch.as_tensor(q.values).to(dev), dbx, dbo, p.band_frac,
                                      p.k)
        ex_id, ex_d = ex_id.cpu().numpy(), ex_d.cpu().numpy()
        truth[q.rid] = set(ex_id.tolist()) - {-1}
        src_in += int(src[q.rid] in truth[q.rid])
    # how many of the 100 hash values each sampled query shares with its source
    # window: the MinHash estimate of their weighted Jaccard similarity, which
    # sets the chance that a table's K values all agree
    qx = np.concatenate([q.values for q in sample])
    qoff = np.concatenate([[0], np.cumsum([len(q.values) for q in sample])]).astype(np.int64)
    hb = HashBatch(torch.as_tensor(qx).to(dev), qoff, p)
    hb.run(r, tables)
    agree = [float((hb.hv[j] == ix.hv[int(ix.base[q.cls] + src[q.rid])]).float().mean())
             for j, q in enumerate(sample)]
    del hb

    def recall_of(answers):
        hits = sum(len(truth[q.rid] & (set(answers[q.rid].tolist()) - {-1})) for q in sample)
        return hits / max(sum(len(truth[q.rid]) for q in sample), 1)

    recall = {"recall_at_10": recall_of({q.rid: res[q.rid].ids for q in sample}),
              "queries": len(sample),
              "exhaustive_top10_holds_source": src_in / max(len(sample), 1),
              "hash_agreement_with_source": {"mean": float(np.mean(agree)),
                                             "median": float(np.median(agree))}}
    # the same sample through the paper's own table setting: 20 tables, each
    # keyed by one weighted MinHash (K = 1, L = 20), on a second resident index
    pp = Params(W=80, delta=3, n=15, K=1, L=20, band_frac=cfg["band"], C=cfg["C"], k=10)
    draws20 = datagen.cws_draws(pp.n, pp.H, seed=seed)
    tables20 = ssh.CwsTables(*draws20, pp.n, device=dev)
    ix20 = MixedIndex(x, [(ell, nwin) for ell in lens], pp, tables20, r)
    ex20 = GpuExecutor(ix20, cfg["arena"], slots=1, max_batch=len(sample), max_len=max(lens))
    ex20.start(time.perf_counter())
    h = ex20.launch(sample, 0, 0)
    torch.cuda.synchronize()
    ssh.check_device_errors()
    ans20 = {rr.rid: rr.ids for rr in ex20.finish(h)}
    recall["paper_tables_K1_L20"] = {"recall_at_10": recall_of(ans20), "queries": len(sample)}
    recall["seconds"] = time.perf_counter() - t_r
    log(f"serving: recall@10 {recall['recall_at_10']:.3f} (K=10, L=10), "
        f"{recall['paper_tables_K1_L20']['recall_at_10']:.3f} (K=1, L=20) on {len(sample)} queries")
    del ex20, ix20, tables20
    out = {"config": {"workload": cfg["workload"], "lengths": list(lens), "windows": nwin,
                      "rate_qps": cfg["rate"], "requests": len(reqs), "C": p.C,
                      "band_frac": p.band_frac, "k": p.k, "max_batch": cfg["max_batch"],
                      "slots": cfg["slots"], "arena_bytes": cfg["arena"]},
           "continuous_batching": batched, "plain_one_at_a_time": plain,
           "same_answers_batched_and_plain": bool(same),
           "capacity_burst": {"continuous_batching": cap_batched, "plain_one_at_a_time": cap_plain},
           "recall": recall,
           "index_build_s": t_index}
    del ex, ix, x, tables
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return out


MULTI_SHAPES = [(80, 3), (128, 4)]
MULTI_F = 64
MULTI_N, MULTI_M = 1_000_000, 1024


def run_multi(args):
    """F = 64 sign sketches of the index configuration's series at once
    (ssh_sketch_multi), for each matrix-core filter shape: time per call with
    HIP events on the launching stream, the MFMA roofline of the product, the
    float64 repair fraction, and the same 64 streams from 64 single-filter
    launches (ssh_sketch) for comparison and as a bit-for-bit check."""
    import numpy as np
    import torch

    from paper_1610_07328_amd import datagen, ssh
    dev = torch.device("cuda")
    N, m, F = (args.n_series or MULTI_N), MULTI_M, MULTI_F
    x = upload_walks(N, m, args.seed, dev)
    off = np.arange(N + 1, dtype=np.int64) * m
    doff = torch.as_tensor(off).to(dev)
    res = {}
    for W, delta in MULTI_SHAPES:
        p = ssh.plan(off, W, delta, 1)
        dbwo = torch.as_tensor(p.bit_word_off).to(dev)
        nwin = N * ssh.num_bits(m, W, delta)
        R = datagen.filters_R(F, W, seed=args.seed)
        filt = ssh.MultiFilter(R, delta)
        out = ssh.sketch_multi(x, doff, filt, dbwo)
        torch.cuda.synchronize()
        ssh.check_device_errors()
        out[2].zero_()
        reps = 5
        ms = event_ms(lambda: ssh.sketch_multi(x, doff, filt, dbwo, out=out), reps)
        repaired = int(out[2].cpu().numpy()[0]) / (reps + 1)
        # the same streams from F single-filter launches
        single = ssh.sketch(x, doff, R[0], W, delta, dbwo)
        ms1 = event_ms(lambda: ssh.sketch(x, doff, R[0], W, delta, dbwo, out=single), reps)
        words = int(p.bit_word_off[-1])
        same = True
        for f in range(F):
            b1, _, _ = ssh.sketch(x, doff, R[f], W, delta, dbwo)
            same &= bool(torch.equal(b1[:words].view(torch.int64), out[0][f, :words].view(torch.int64)))
        torch.cuda.synchronize()
        flops = 2.0 * W * F * nwin
        tfs = flops / (ms * 1e-3) / 1e12
        hbm = (N * m * 4 * ((F + 31) // 32) + F * words * 8) / (ms * 1e-3) / 1e9
        res[f"W{W}_delta{delta}"] = {
            "config": {"workload": f"multi-filter sign sketch: {N:,} random-walk series x {m}, "
                                   f"W={W} delta={delta}, F={F} Gaussian filters", "N": N, "m": m,
                       "W": W, "delta": delta, "F": F},
            "ms": ms, "windows": nwin, "pairs_per_s": F * nwin / (ms * 1e-3),
            "roofline": {"bound": "mfma", "achieved": tfs, "peak": 2500.0, "unit": "TFLOP/s",
                         "frac": tfs / 2500.0, "traffic": None, "kernel": "sketch_multi_kernel",
                         "flops_per_call": flops},
            "hbm_GBps": hbm,
            "fp64_repaired_fraction": repaired / (F * nwin),
            "single_filter_ms": ms1,
            "speedup_over_single_filter_launches": F * ms1 / ms,
            "streams_equal_single_filter": same,
        }
        log(f"multi: W={W} delta={delta} F={F}: {ms:.2f} ms ({tfs:.0f} TFLOP/s, "
            f"{F * ms1 / ms:.2f}x {F} single-filter launches, streams equal: {same})")
        del out, single, filt, dbwo
        torch.cuda.empty_cache()
    del x
    torch.cuda.empty_cache()
    return res


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              f"(the index would shard by series across GPUs; only one GPU is measured).",
              file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration > 0:
        copy_calibration(args.copy_calibration)
        return

    import torch

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.serving_only:
        print(json.dumps({"serving": run_serving(args)}), flush=True)
        return
    if args.uneven_only:
        print(json.dumps({"uneven_batch": run_uneven(args)}), flush=True)
        return
    if args.multi_only:
        print(json.dumps({"multi_filter_sketch": run_multi(args)}), flush=True)
        return

    res, cfg, Q = run_workload(args.workload, args, main=True)
    out = {
        "metric": METRIC,
        "value": res["value"],
        "unit": "series hashed/s",
        "n_gpus": 1,
        "steps": res["steps"],
        "warmup": res["warmup"],
        "ms_per_step": res["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f16 dot / f32 acc / f64 repair + f64 CWS + f32 DTW",
        "data": "synthetic",
        "config": res["config"],
    }
    out.update({k: v for k, v in res.items() if k not in out and k != "value"})
    if not args.no_extra:
        other = "index" if args.workload == "large" else "large"
        extra, _, _ = run_workload(other, args, main=False)
        out["other_workload"] = extra
    if not args.no_uneven:
        out["uneven_batch"] = run_uneven(args)
    if not args.no_multi:
        out["multi_filter_sketch"] = run_multi(args)
    if not args.no_serving:
        out["serving"] = run_serving(args)
        out["query_latency_ms_served"] = out["serving"]["continuous_batching"]["latency_ms"]
    out["hbm_copy_microbench"] = hbm_copy_microbench()
    log(f"HBM copy micro-benchmark: {out['hbm_copy_microbench']['GB/s']:.0f} GB/s")
    if not args.no_cpu_baseline:
        log("cpu baseline")
        out["cpu_baseline"] = cpu_baseline(cfg, args.seed, min(args.cpu_sample, cfg["N"]), Q)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
