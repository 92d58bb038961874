"""Batched index build over series of uneven lengths (Algorithm 1 for a whole
batch): the launch plan, an autotuner with an on-disk cache, and a HIP graph
of the build.

* Plan.  Every stage is one launch over the whole batch.  The sketch runs on a
  resident grid whose wavefronts stride over the series, so a batch can be
  ordered longest first: wavefront w then takes series w, w + G, w + 2G, ...
  of descending length and every wavefront gets about the same work (the
  other stages give each series its own wavefront or workgroup).  Ids of the
  ordered batch map back to the caller's through `perm`.
* Autotuner.  For a batch it times every combination of the sketch's work
  item (`ssh_sketch_tiled`: 8, 12, 16 or 20 rows of 16 windows) and the series
  order (as given, longest first) over a whole build, keeps the fastest, and
  stores the choice in a JSON file keyed by (GPU architecture, W, delta, n,
  H, length bucket), so later batches of that kind skip the timing.  Every
  choice gives the same bits; only the time differs.
* Graph.  The build's launches (sketch, shingle, CWS with band keys, table
  build) are captured once into a HIP graph and replayed; no step allocates
  or synchronises, so the graph holds kernels only.

Nothing here computes: every step runs in the library's kernels.
"""
from __future__ import annotations

import json
import math
import os
import time

import numpy as np

ORDERS = ("given", "longest_first")


def longest_first(lengths: np.ndarray) -> np.ndarray:
    """Permutation listing series by descending length (ties by id)."""
    return np.argsort(-np.asarray(lengths, np.int64), kind="stable")


def length_bucket(lengths: np.ndarray) -> int:
    """Power of two at or below the batch's mean length."""
    mean = float(np.mean(lengths)) if len(lengths) else 1.0
    return 1 << max(0, int(math.floor(math.log2(max(mean, 1.0)))))


def default_cache_path() -> str:
    return os.environ.get("SSH_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "paper_1610_07328_amd",
                                       "tune.json"))


class TuneCache:
    """Autotuner choices on disk: {key: {"tile_rows": .., "order": .., ...}}."""

    def __init__(self, path: str | None = None):
        self.path = path or default_cache_path()
        self.data = {}
        if os.path.exists(self.path):
            with open(self.path) as f:
                self.data = json.load(f)

    @staticmethod
    def key(arch: str, W: int, delta: int, n: int, H: int, bucket: int) -> str:
        return f"{arch}|W={W}|delta={delta}|n={n}|H={H}|len={bucket}"

    def get(self, key: str):
        return self.data.get(key)

    def put(self, key: str, choice: dict):
        self.data[key] = choice
        os.makedirs(os.path.dirname(os.path.abspath(self.path)), exist_ok=True)
        tmp = self.path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(self.data, f, indent=1, sort_keys=True)
        os.replace(tmp, self.path)


def reorder(x: np.ndarray, off: np.ndarray, perm: np.ndarray):
    """Series of a CSR batch in the order perm; returns (x, off)."""
    lens = np.diff(off)[perm]
    noff = np.zeros(len(perm) + 1, np.int64)
    np.cumsum(lens, out=noff[1:])
    nx = np.empty(int(noff[-1]), np.float32)
    for j, i in enumerate(perm):
        nx[noff[j]:noff[j + 1]] = x[off[i]:off[i + 1]]
    return nx, noff


class UnevenBuild:
    """The index build of one batch in a given order with a given sketch item.

    x, off: the batch on the host (float32 values, int64 offsets);
    p: pipeline.Params; tables: ssh.CwsTables; r: the filter."""

    def __init__(self, x: np.ndarray, off: np.ndarray, p, tables, r, order: str = "given",
                 tile_rows: int = 0, device="cuda"):
        import torch

        from .pipeline import HashBatch, Index

        if order not in ORDERS:
            raise ValueError(f"unknown order {order!r}")
        self.p, self.tables, self.r = p, tables, r
        self.order, self.tile_rows = order, tile_rows
        N = len(off) - 1
        if order == "longest_first":
            self.perm = longest_first(np.diff(off))
            hx, hoff = reorder(x, off, self.perm)
        else:
            self.perm = np.arange(N, dtype=np.int64)
            hx, hoff = x, off
        self.db = HashBatch(torch.as_tensor(hx).to(device), hoff, p)
        self.index = Index(self.db)
        self.graph = None

    def run(self):
        """The build, one launch per stage on the current stream."""
        from . import ssh
        db = self.db
        ssh.sketch(db.x, db.x_off, self.r, self.p.W, self.p.delta, db.bwo,
                   out=(db.bits, db.nbits, db.repair), tile_rows=self.tile_rows)
        db.shingle()
        db.cws_band_keys(self.tables)
        self.index.build()

    def capture(self):
        """Capture run() into a HIP graph (after one eager run on a side stream,
        which loads every kernel)."""
        import torch
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            self.run()
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, capture_error_mode="relaxed"):
            self.run()
        torch.cuda.synchronize()
        self.graph = g
        return g

    def replay(self):
        self.graph.replay()

    # results in the caller's series order (for checks; moves data only)
    def _caller_order(self, t):
        import torch
        inv = torch.as_tensor(np.argsort(self.perm), device=t.device)
        return t[: self.db.N].view(torch.int64)[inv].view(torch.uint64)

    def hv(self):
        return self._caller_order(self.db.hv)

    def keys(self):
        return self._caller_order(self.db.keys)


def autotune(x: np.ndarray, off: np.ndarray, p, tables, r, cache: TuneCache | None = None,
             reps: int = 3, device="cuda"):
    """The fastest (tile_rows, order) for this kind of batch, from the cache or
    by timing every combination over a whole build.  Returns (choice, hit)."""
    import torch

    from . import ssh
    cache = cache or TuneCache()
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    key = TuneCache.key(arch, p.W, p.delta, p.n, p.H, length_bucket(np.diff(off)))
    hit = cache.get(key)
    if hit is not None:
        return hit, True
    timings = {}
    tiles = [t for t in ssh.SKETCH_TILES if ssh.sketch_tile_supported(p.W, p.delta, t)]
    for order in ORDERS:
        b = UnevenBuild(x, off, p, tables, r, order=order, device=device)
        for t in tiles or [0]:
            b.tile_rows = t
            b.run()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                b.run()
            e1.record()
            e1.synchronize()
            timings[f"{order}/{t}"] = e0.elapsed_time(e1) / reps
        del b
        torch.cuda.empty_cache()
    best = min(timings, key=timings.get)
    order, t = best.split("/")
    choice = {"order": order, "tile_rows": int(t), "build_ms": timings, "tuned_at": time.time()}
    cache.put(key, choice)
    return choice, False
