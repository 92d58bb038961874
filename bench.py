"""Benchmark of the SSH hot path on one MI355X.

Workload (batched index build): 1,000,000 z-normalised random-walk series of
length 1024 (fp32, resident in HBM), filter W = 80, step delta = 3, shingle
n = 15, 100 weighted-MinHash hashes (K = 10 per band, L = 10 tables).  One
step is one pass of the whole hot path: sketch, shingle, CWS and band keys of
the database, the hash-table build, then a batch of 1,000 queries (perturbed
database series, N(0, 0.1^2) noise, z-normalised) through sketch, shingle,
CWS, band keys, probe (top C = 50 candidates) and banded DTW re-rank (5 %
Sakoe-Chiba band, top k = 10).

Prints one JSON line: series hashed per second (value), DTW cells per
second, per-stage times, the roofline of the dominant kernel and the CPU
oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
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

# HBM traffic of one launch of a kernel on this workload, from two rocprofv3
# counter runs of this script (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch),
# each scaled by the ratio of known bytes to the same counter's reading for a
# plain device copy (--copy-calibration).  A figure is reported only while the
# kernel's source file still has the digest it was measured with.
MEASURED_TRAFFIC = {
    # kernel: (source file, sha256 of it, FETCH_SIZE KiB, WRITE_SIZE KiB,
    #          fetch scale, write scale); the 1 GiB copy read 524306.6 KiB on
    #          FETCH_SIZE and 1048576 KiB on WRITE_SIZE
    "cws_kernel": ("paper_1610_07328_amd/csrc/cws.hip",
                   "ccb9483ee387c2dfa4db072c851ec8119f7e73577ec1befb94fc91647033061b",
                   3571453.9375, 903875.46875, 1048576.0 / 524306.5625, 1.0),
}


def band_cells(lq: int, lx: int, r: int) -> int:
    """Cells of an lq x lx DTW matrix inside the band |i - j| <= r."""
    total = 0
    for i in range(lq):
        lo, hi = max(0, i - r), min(lx - 1, i + r)
        if hi >= lo:
            total += hi - lo + 1
    return total


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the recorded counters, or None."""
    import hashlib
    rec = MEASURED_TRAFFIC.get(kernel)
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
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n-series", type=int, default=1_000_000)
    ap.add_argument("--length", type=int, default=1024)
    ap.add_argument("--nq", type=int, default=1000)
    ap.add_argument("--latency-samples", type=int, default=200)
    ap.add_argument("--cpu-sample", type=int, default=80000)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run one device copy of BYTES bytes (counter calibration)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--seed", type=int, default=0)
    return ap.parse_args()


def cpu_baseline(X, r, draws, p, Q, sample: int):
    """The CPU oracle on the first `sample` series (and 16 queries) of the workload."""
    import oracle
    from oracle import _dtw_c

    Xs = X[:sample]
    t0 = time.perf_counter()
    B = oracle.sketch_batch(Xs, r, p.W, p.delta)
    sets = [oracle.shingle(b, p.n) for b in B]
    smax = max(2, max(int(c.max()) for _, c in sets if len(c)))
    lnS = oracle.ln_table(smax)
    hv = np.stack([oracle.cws(c, k, *draws, lnS)[2] for c, k in sets])
    oracle.band_keys(hv, p.K, p.L, p.key_seed)
    t_hash = time.perf_counter() - t0
    # DTW: 16 queries x C candidates in the same band
    from paper_1610_07328_amd import datagen
    nqs = 16
    q, qoff = datagen.csr(Q[:nqs])
    db, dboff = datagen.csr(Xs)
    rng = np.random.default_rng(0)
    cand = rng.integers(0, sample, size=(nqs, p.C)).astype(np.int64)
    ncand = np.full(nqs, p.C, np.int32)
    t1 = time.perf_counter()
    oracle.rerank(q, qoff, db, dboff, cand, ncand, p.band_frac, p.k)
    t_dtw = time.perf_counter() - t1
    rr = int(math.floor(float(np.float32(p.band_frac)) * X.shape[1]))
    cells = nqs * p.C * band_cells(X.shape[1], X.shape[1], rr)
    return {
        "value": sample / t_hash,
        "unit": "series hashed/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"first {sample} series of the workload through sketch, shingle, CWS and "
                  f"band keys (numpy float64, one thread); DTW re-rank of {nqs} queries x "
                  f"{p.C} candidates in C with OpenMP",
        "dtw_cells_per_s": cells / t_dtw,
        "dtw_cores": _dtw_c.num_threads(),
        "seconds": t_hash + t_dtw,
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              f"(the index would shard by series across GPUs; only one GPU is measured).", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration > 0:
        copy_calibration(args.copy_calibration)
        return

    import torch

    from paper_1610_07328_amd import datagen, ssh
    from paper_1610_07328_amd.pipeline import HashBatch, Index, Params, QueryBatch

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    p = Params(W=80, delta=3, n=15, K=10, L=10, band_frac=0.05, C=50, k=10)
    N, m, nq = args.n_series, args.length, args.nq
    t0 = time.perf_counter()
    X = datagen.random_walks(N, m, seed=args.seed)
    Q, _ = datagen.perturbed_queries(X[: min(N, 100_000)], nq, 0.1, seed=args.seed)
    r = datagen.filter_r(p.W, seed=args.seed)
    draws = datagen.cws_draws(p.n, p.H, seed=args.seed)
    print(f"[bench] generated {N} x {m} series in {time.perf_counter() - t0:.1f}s", file=sys.stderr,
          flush=True)

    dev = torch.device("cuda:0")
    x, off = datagen.csr(X)
    xd = torch.as_tensor(x).to(dev)
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

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ssh.check_device_errors()

    events = [[torch.cuda.Event(enable_timing=True) for _ in range(len(stages) + 1)]
              for _ in range(args.steps)]
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for s in range(args.steps):
        step(events[s])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    ssh.check_device_errors()

    per_stage = {name: 0.0 for name in stages}
    for ev in events:
        for i, name in enumerate(stages):
            per_stage[name] += ev[i].elapsed_time(ev[i + 1]) / args.steps  # ms
    ms_per_step = wall * 1000.0 / args.steps

    # workload facts for the algorithmic byte counts
    ncand = qry.ncand[:nq].cpu().numpy()
    rsz = qry.rsize[:nq].cpu().numpy().astype(np.float64)
    nd = db.ndist[:N].cpu().numpy().astype(np.int64)
    repaired = int(db.repair.cpu().numpy()[0]) / (args.warmup + args.steps)
    nb = int(db.plan.max_nbits)
    words = (nb + 63) // 64
    S = nb - p.n + 1
    rr = int(math.floor(float(np.float32(p.band_frac)) * m))
    cells_per_pair = band_cells(m, m, rr)
    cells = int(ncand.sum()) * cells_per_pair
    sum_d = int(nd.sum())

    bytes_stage = {
        "sketch": N * (4 * m + 8 * words + 4) + 16 * (N + 1),
        "shingle": N * (8 * words + 4 + 4) + 16 * (N + 1) + 8 * sum_d,
        "cws": 8 * sum_d + N * (8 * p.H + 4 + 8 + 8 * p.L),
        # radix passes over the top 24 bits (N <= 2^20) or 32: keys and ids read twice, written once
        "table_build": (3 if N <= (1 << 20) else 4) * N * p.L * (8 + 12 + 12),
    }
    stage_roofline = {}
    for name, b in bytes_stage.items():
        t = per_stage[name] / 1e3
        stage_roofline[name] = {"GB/s": b / t / 1e9, "frac_hbm": b / t / 1e9 / HBM_PEAK_GBS}

    # CWS float64 evaluations: one per (series, distinct token, hash)
    cws_evals = sum_d * p.H
    dominant = max(["sketch", "shingle", "cws", "table_build", "rerank"],
                   key=lambda k: per_stage[k])
    if dominant == "rerank":
        # 3 VALU lane-ops per cell (subtract, 3-way min, FMA) against the lane-op peak
        achieved = cells * 3 / (per_stage["rerank"] / 1e3) / 1e12
        peak = VALU_LANE_OPS / 1e12
        roof = {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "Tops/s",
                "frac": achieved / peak, "traffic": None, "kernel": "dtw_kernel"}
    else:
        kname = {"sketch": "sketch_mfma_kernel", "shingle": "shingle_kernel", "cws": "cws_kernel",
                 "table_build": "rs_scatter_kernel"}[dominant]
        achieved = bytes_stage[dominant] / (per_stage[dominant] / 1e3) / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(kname),
                "kernel": kname, "kernel_ms": per_stage[dominant],
                "algorithmic_bytes": bytes_stage[dominant]}
        if dominant == "cws":
            roof["token_hash_evals_per_s"] = cws_evals / (per_stage["cws"] / 1e3)

    # DTW kernel throughput on a full batch: every query re-ranks C seeded
    # random candidates in the same band (outside the timed step)
    g = np.random.default_rng(args.seed + 1)
    cand_full = torch.as_tensor(g.integers(0, N, size=(nq, p.C)), device=dev)
    ncand_full = torch.full((nq,), p.C, dtype=torch.int32, device=dev)
    ws_full = torch.empty(max(ssh.rerank_workspace_bytes(nq, p.C), 1), dtype=torch.uint8, device=dev)
    out_full = (torch.empty((nq, p.k), dtype=torch.int64, device=dev),
                torch.empty((nq, p.k), dtype=torch.float32, device=dev))

    def full_rerank():
        ssh.dtw_rerank(qb.x, qb.x_off, db.x, db.x_off, cand_full, ncand_full, p.band_frac,
                       p.k, ws=ws_full, out=out_full)

    full_rerank()
    torch.cuda.synchronize()
    reps = 5
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        full_rerank()
    e1.record()
    e1.synchronize()
    t_full = e0.elapsed_time(e1) / reps / 1e3
    full_cells = nq * p.C * cells_per_pair
    dtw_full = {"cells_per_s": full_cells / t_full, "ms": t_full * 1e3,
                "pairs": nq * p.C, "cells": full_cells,
                "alu_frac": full_cells * 3 / t_full / VALU_LANE_OPS}

    # the same batch through the LB_Keogh-pruned re-rank (same results, less work)
    ws_lb = torch.empty(max(ssh.rerank_lb_workspace_bytes(nq, p.C, qb.x.numel()), 1), dtype=torch.uint8,
                        device=dev)
    out_lb = (torch.empty_like(out_full[0]), torch.empty_like(out_full[1]))

    def full_rerank_lb():
        ssh.dtw_rerank(qb.x, qb.x_off, db.x, db.x_off, cand_full, ncand_full, p.band_frac,
                       p.k, ws=ws_lb, out=out_lb, prune=True)

    full_rerank_lb()
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        full_rerank_lb()
    e1.record()
    e1.synchronize()
    t_lb = e0.elapsed_time(e1) / reps / 1e3
    same = bool(torch.equal(out_lb[0], out_full[0]) and
                torch.equal(out_lb[1].view(torch.int32), out_full[1].view(torch.int32)))
    dtw_full["lb_pruned"] = {"ms": t_lb * 1e3, "speedup": t_full / t_lb, "same_results": same}

    # weighted MinHash by integer replication over the same index histograms
    # (outside the step: an alternative to the CWS stage, integer arithmetic only)
    hv_int = torch.empty((N, p.H), dtype=torch.uint64, device=dev)

    def wmh_index():
        ssh.wmh_int(db.codes, db.counts, db.hoff, db.ndist, p.H, p.wmh_seed, out=hv_int)

    wmh_index()
    torch.cuda.synchronize()
    e0.record()
    for _ in range(3):
        wmh_index()
    e1.record()
    e1.synchronize()
    t_wmh = e0.elapsed_time(e1) / 3 / 1e3
    pairs = int(torch.clamp(db.nbits[:N].to(torch.int64) - p.n + 1, min=0).sum().item())
    wmh_int_index = {"ms": t_wmh * 1e3, "series_per_s": N / t_wmh,
                     "pair_hash_evals_per_s": pairs * p.H / t_wmh,
                     "cws_stage_ms": per_stage["cws"]}
    del hv_int

    # single-query latency with the index resident
    lat = []
    if args.latency_samples > 0:
        Q1 = Q[: args.latency_samples]
        singles = []
        for i in range(Q1.shape[0]):
            qi, qio = datagen.csr(Q1[i: i + 1])
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
    lat = np.array(lat) if lat else np.array([float("nan")])

    out = {
        "metric": "series hashed/s",
        "value": N * args.steps / wall,
        "unit": "series/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f16 dot / f32 acc / f64 repair + f64 CWS + f32 DTW",
        "data": "synthetic",
        "config": {"workload": "batched index build: 1,000,000 random-walk series x 1024 fp32, "
                               "W=80 delta=3 n=15, 100 CWS hashes (K=10, L=10); 1,000 queries, "
                               "C=50, DTW band 5%, top-10",
                   "n_series": N, "length": m, "W": p.W, "delta": p.delta, "n": p.n,
                   "K": p.K, "L": p.L, "queries": nq, "C": p.C, "band_frac": p.band_frac,
                   "k": p.k},
        "dtw_cells_per_s": cells / (per_stage["rerank"] / 1e3),
        "dtw_full_batch": dtw_full,
        "query_latency_ms": {"p50": float(np.percentile(lat, 50)),
                             "p99": float(np.percentile(lat, 99)),
                             "samples": int(lat.size), "batch": 1},
        "stage_ms": per_stage,
        "stage_hbm": stage_roofline,
        "retrieved_set": {"mean": float(rsz.mean()), "p50": float(np.percentile(rsz, 50)),
                          "p99": float(np.percentile(rsz, 99)), "max": float(rsz.max()),
                          "pruned_frac": float(1.0 - rsz.mean() / N)},
        "sketch_fp64_repaired_windows": repaired,
        "mean_distinct_shingles": sum_d / N,
        "wmh_int_index": wmh_int_index,
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(X, r, draws, p, Q, min(args.cpu_sample, N))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
