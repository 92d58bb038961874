"""The SSH hot path as reusable device state: index build and query batches.

Holds preallocated device buffers so that repeated passes (benchmark steps,
serving) launch kernels only.  Every stage is one call into the C ABI through
paper_1610_07328_amd.ssh; nothing here computes.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import torch

from . import ssh


@dataclass
class Params:
    W: int
    delta: int
    n: int
    K: int
    L: int
    key_seed: int = 0x5EED
    wmh_seed: int = 0x1D5EED  # seed of the integer-replication MinHash
    band_frac: float = 0.05
    C: int = 50
    k: int = 10

    @property
    def H(self) -> int:
        return self.K * self.L


class HashBatch:
    """Device buffers for sketch -> shingle -> CWS -> band keys of one ragged batch."""

    def __init__(self, x: torch.Tensor, x_off_host: np.ndarray, p: Params, out=None):
        """out: optional (hv [N, H], keys [N, L]) device views to hash into."""
        dev = x.device
        self.p = p
        self.N = len(x_off_host) - 1
        self.x = x
        self.x_off_host = np.ascontiguousarray(x_off_host, np.int64)
        self.x_off = torch.as_tensor(self.x_off_host).to(dev)
        plan = ssh.plan(self.x_off_host, p.W, p.delta, p.n)
        self.plan = plan
        self.bwo = torch.as_tensor(plan.bit_word_off).to(dev)
        self.hoff = torch.as_tensor(plan.hist_off).to(dev)
        nw = max(int(plan.bit_word_off[-1]), 1)
        cap = max(int(plan.hist_off[-1]), 1)
        N1 = max(self.N, 1)
        self.bits = torch.empty(nw, dtype=torch.uint64, device=dev)
        self.nbits = torch.empty(N1, dtype=torch.int32, device=dev)
        self.repair = torch.zeros(1, dtype=torch.uint64, device=dev)
        self.codes = torch.empty(cap, dtype=torch.uint32, device=dev)
        self.counts = torch.empty(cap, dtype=torch.uint32, device=dev)
        self.ndist = torch.empty(N1, dtype=torch.int32, device=dev)
        if out is not None:
            self.hv, self.keys = out
        else:
            self.hv = torch.empty((N1, p.H), dtype=torch.uint64, device=dev)
            self.keys = torch.empty((N1, p.L), dtype=torch.uint64, device=dev)

    # individual stages (return nothing; results stay in the buffers)
    def sketch(self, r: np.ndarray):
        ssh.sketch(self.x, self.x_off, r, self.p.W, self.p.delta, self.bwo,
                   out=(self.bits, self.nbits, self.repair))

    def shingle(self):
        ssh.shingle(self.bits, self.bwo, self.nbits, self.p.n, self.hoff,
                    out=(self.codes, self.counts, self.ndist))

    def cws(self, tables: ssh.CwsTables):
        ssh.cws(self.codes, self.counts, self.hoff, self.ndist, tables, out=self.hv)

    def band_keys(self, seed: int | None = None):
        ssh.band_keys(self.hv[: self.N], self.p.K, self.p.L,
                      self.p.key_seed if seed is None else seed, out=self.keys)

    def cws_band_keys(self, tables: ssh.CwsTables, seed: int | None = None):
        """CWS and band keys in one kernel pass (same results as cws() then band_keys());
        seed overrides the band-key seed of the parameters."""
        ssh.cws_band_keys(self.codes, self.counts, self.hoff, self.ndist, tables, self.p.K,
                          self.p.L, self.p.key_seed if seed is None else seed,
                          out=(self.hv, self.keys))

    def wmh_int_band_keys(self):
        """Integer-replication MinHash, then band keys: the hash values and keys
        feed the same tables, probe and re-rank as the CWS ones."""
        ssh.wmh_int(self.codes, self.counts, self.hoff, self.ndist, self.p.H, self.p.wmh_seed,
                    out=self.hv)
        self.band_keys()

    def run(self, r: np.ndarray, tables: ssh.CwsTables | None = None, method: str = "cws"):
        """Sketch, shingle and hash the batch; method "cws" (needs tables) or
        "wmh_int" (integer-replication MinHash)."""
        if method not in ("cws", "wmh_int"):
            raise ValueError(f"unknown hash method {method!r}")
        if method == "cws" and tables is None:
            raise ValueError("method 'cws' needs CWS tables")
        self.sketch(r)
        self.shingle()
        if method == "cws":
            self.cws_band_keys(tables)
        else:
            self.wmh_int_band_keys()
        return self.hv[: self.N], self.keys[: self.N]


class Index:
    """Hash tables over a resident database batch."""

    def __init__(self, db: HashBatch):
        self.db = db
        N, L = db.N, db.p.L
        dev = db.x.device
        self.tab_keys = torch.empty((L, max(N, 1)), dtype=torch.uint64, device=dev)
        self.tab_ids = torch.empty((L, max(N, 1)), dtype=torch.uint32, device=dev)
        self.ws = torch.empty(max(ssh.table_workspace_bytes(N, L), 1), dtype=torch.uint8,
                              device=dev)

    def build(self):
        ssh.table_build(self.db.keys[: self.db.N], ws=self.ws, out=(self.tab_keys, self.tab_ids))


# When the step's re-rank prunes (LB_Kim, LB_Keogh and early abandoning,
# dtw_rerank_lb; the same results as the plain re-rank).  The bounds cost
# O(length) per pair against the DTW's O(length x radius), so they pay for wide
# bands: on the 2048-sample, 10 % band configuration (radius 204) the pruned
# re-rank of 4,096 queries' candidates takes half the time, on the 1024-sample,
# 5 % band one (radius 51) twice the time.  A small batch is bound by its
# launches and dependent passes, which pruning adds to: single queries keep the
# plain re-rank.
PRUNE_RADIUS = 128
PRUNE_MIN_PAIRS = 8192


class QueryBatch:
    """Probe + DTW re-rank buffers for a batch of queries against an Index.

    prune: None prunes when the batch's widest band radius is at least
    PRUNE_RADIUS and it re-ranks at least PRUNE_MIN_PAIRS (query, candidate)
    slots; True / False force the pruned / plain re-rank."""

    def __init__(self, qh: HashBatch, index: Index, prune: bool | None = None):
        self.qh = qh
        self.index = index
        p = qh.p
        nq = qh.N
        dev = qh.x.device
        lq = int(np.diff(qh.x_off_host).max()) if nq else 0
        radius = int(np.floor(float(np.float32(p.band_frac)) * lq))
        auto = radius >= PRUNE_RADIUS and nq * p.C >= PRUNE_MIN_PAIRS
        self.prune = auto if prune is None else bool(prune)
        self.cand = torch.empty((max(nq, 1), p.C), dtype=torch.int64, device=dev)
        self.ncand = torch.empty(max(nq, 1), dtype=torch.int32, device=dev)
        self.rsize = torch.empty(max(nq, 1), dtype=torch.int64, device=dev)
        self.ids = torch.empty((max(nq, 1), p.k), dtype=torch.int64, device=dev)
        self.dist = torch.empty((max(nq, 1), p.k), dtype=torch.float32, device=dev)
        need = (ssh.rerank_lb_workspace_bytes(nq, p.C, qh.x.numel()) if self.prune
                else ssh.rerank_workspace_bytes(nq, p.C))
        self.ws = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
        self.pws = torch.empty(max(ssh.probe_workspace_bytes(nq, p.L, p.C), 1), dtype=torch.uint8,
                               device=dev)

    def probe(self):
        ix, db, q = self.index, self.index.db, self.qh
        N = db.N
        ssh.probe(ix.tab_keys[:, :N], ix.tab_ids[:, :N], db.keys[:N], db.hv[:N], q.keys[: q.N],
                  q.hv[: q.N], q.p.C, out=(self.cand, self.ncand, self.rsize), ws=self.pws)

    def rerank(self):
        db, q = self.index.db, self.qh
        ssh.dtw_rerank(q.x, q.x_off, db.x, db.x_off, self.cand[: q.N], self.ncand[: q.N],
                       q.p.band_frac, q.p.k, ws=self.ws, out=(self.ids, self.dist),
                       prune=self.prune)


def exhaustive_topk(q: torch.Tensor, db_x: torch.Tensor, db_off: torch.Tensor, band_frac: float,
                    k: int, chunk: int = ssh.MAX_C):
    """Exact top-k of one query over every series of the database by banded DTW.

    Ground truth for recall: a search that visits every series.  Only the
    library's re-rank runs: the database is cut into rows of `chunk`
    candidates (the query repeated once per row), each row keeps its k best by
    (distance, id), and the survivors go through the same re-rank again until
    one row remains.  A pair's distance does not depend on the batch it is
    computed in, so the result is the global top-k by (distance, id).
    Returns (ids int64 [k], dist float32 [k]) on the device.
    """
    dev = q.device
    lq = q.numel()
    N = db_off.numel() - 1
    ids = torch.arange(N, dtype=torch.int64, device=dev)
    while True:
        n = ids.numel()
        rows = max(1, (n + chunk - 1) // chunk)
        C = min(chunk, max(n, k))
        cand = torch.full((rows * C,), -1, dtype=torch.int64, device=dev)
        cand[:n] = ids
        cand = cand.view(rows, C)
        ncand = torch.full((rows,), C, dtype=torch.int32, device=dev)
        if n % C:
            ncand[-1] = n % C
        qx = q.repeat(rows)
        qoff = torch.arange(rows + 1, dtype=torch.int64, device=dev) * lq
        out_id, out_d = ssh.dtw_rerank(qx, qoff, db_x, db_off, cand, ncand, band_frac, k)
        if rows == 1:
            return out_id[0], out_d[0]
        keep = out_id.reshape(-1)
        ids = keep[keep >= 0]
