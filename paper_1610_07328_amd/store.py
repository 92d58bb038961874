"""A resident index that grows and shrinks, and its file format.

SSH's hashing is data independent (Section 1): the filter and the
weighted-MinHash draws are fixed in advance, so a series can be hashed and
placed in the tables at any time without touching the others, and taken out
again.  DynamicIndex keeps the series, their hash values and keys and the L
tables in HBM and updates them through the C ABI:

* insert: the new series are hashed (sketch, shingle, CWS and band keys) into
  the next rows and merged into the tables (ssh_table_insert); the tables are
  then those a build over every series gives;
* delete: the series are marked dead and every table keeps its other entries
  (ssh_table_delete); ids are never reused, so a probe answers with the ids
  the series were inserted under;
* save / load: the whole index in one directory, raw arrays plus a JSON
  manifest; the draws and the filter travel with it, so queries are hashed
  the same way after a load.

Nothing here computes: every step runs in the library's kernels.
"""
from __future__ import annotations

import json
import os

import numpy as np
import torch

from . import ssh
from .pipeline import HashBatch, Params

FORMAT = "ssh-index-1"


class DynamicIndex:
    """Series, hash values, keys and tables of a growing set of series."""

    def __init__(self, p: Params, draws, r: np.ndarray, device="cuda"):
        self.p = p
        self.dev = torch.device(device)
        self.draws = tuple(np.ascontiguousarray(a) for a in draws)
        self.r = np.ascontiguousarray(r, np.float32)
        self.tables = ssh.CwsTables(*self.draws, p.n, device=self.dev)
        self.x = torch.empty(0, dtype=torch.float32, device=self.dev)
        self.off = np.zeros(1, np.int64)          # host copy of the series offsets
        self.x_off = torch.zeros(1, dtype=torch.int64, device=self.dev)
        self.hv = torch.empty((0, p.H), dtype=torch.uint64, device=self.dev)
        self.keys = torch.empty((0, p.L), dtype=torch.uint64, device=self.dev)
        self.dead = torch.zeros(0, dtype=torch.uint8, device=self.dev)
        self.tab_keys = torch.empty((p.L, 0), dtype=torch.uint64, device=self.dev)
        self.tab_ids = torch.empty((p.L, 0), dtype=torch.uint32, device=self.dev)
        self.n_live = 0

    @property
    def n_total(self) -> int:
        """Series ever inserted (ids 0 .. n_total - 1)."""
        return len(self.off) - 1

    # ---- updates ---------------------------------------------------------
    def insert(self, x_new: np.ndarray, off_new: np.ndarray) -> np.ndarray:
        """Append series (CSR on the host); returns their ids."""
        p = self.p
        M = len(off_new) - 1
        base = self.n_total
        if M == 0:
            return np.zeros(0, np.int64)
        xs = torch.as_tensor(np.ascontiguousarray(x_new, np.float32)).to(self.dev)
        hv_new = torch.empty((M, p.H), dtype=torch.uint64, device=self.dev)
        keys_new = torch.empty((M, p.L), dtype=torch.uint64, device=self.dev)
        hb = HashBatch(xs, np.ascontiguousarray(off_new, np.int64), p, out=(hv_new, keys_new))
        hb.run(self.r, self.tables)
        rebuild = self.n_live == base and ssh.table_sort_bits(base) != ssh.table_sort_bits(base + M)
        if not rebuild:
            # raises when the sort width changes and deleted series left holes
            self.tab_keys, self.tab_ids = ssh.table_insert(self.tab_keys, self.tab_ids, keys_new,
                                                           id_base=base)
        self.x = torch.cat([self.x, xs])
        self.off = np.concatenate([self.off, self.off[-1] + np.asarray(off_new[1:], np.int64)])
        self.x_off = torch.as_tensor(self.off).to(self.dev)
        self.hv = torch.cat([self.hv.view(torch.int64), hv_new.view(torch.int64)]).view(torch.uint64)
        self.keys = torch.cat([self.keys.view(torch.int64),
                               keys_new.view(torch.int64)]).view(torch.uint64)
        self.dead = torch.cat([self.dead, torch.zeros(M, dtype=torch.uint8, device=self.dev)])
        self.n_live += M
        if rebuild:  # crossing 2^24 series without deletions: the same tables, built anew
            self.tab_keys, self.tab_ids = ssh.table_build(self.keys)
        return np.arange(base, base + M, dtype=np.int64)

    def delete(self, ids) -> int:
        """Take series out of the tables; returns how many were live."""
        ids = np.unique(np.asarray(ids, np.int64))
        ids = ids[(ids >= 0) & (ids < self.n_total)]
        if len(ids) == 0:
            return 0
        was = self.dead[torch.as_tensor(ids, device=self.dev)].cpu().numpy()
        fresh = ids[was == 0]
        if len(fresh) == 0:
            return 0
        self.dead[torch.as_tensor(fresh, device=self.dev)] = 1
        n_live = self.n_live - len(fresh)
        self.tab_keys, self.tab_ids = ssh.table_delete(self.tab_keys, self.tab_ids, self.dead,
                                                       n_live)
        self.n_live = n_live
        return len(fresh)

    # ---- queries ---------------------------------------------------------
    def hash_queries(self, q: np.ndarray, qoff: np.ndarray):
        """Query batch hashed like the indexed series: (HashBatch, hv, keys)."""
        hb = HashBatch(torch.as_tensor(np.ascontiguousarray(q, np.float32)).to(self.dev),
                       np.ascontiguousarray(qoff, np.int64), self.p)
        hv, keys = hb.run(self.r, self.tables)
        return hb, hv, keys

    def probe(self, q_keys, q_hv, C: int):
        """ssh_probe over the live entries; ids are the inserted ids."""
        return ssh.probe(self.tab_keys, self.tab_ids, self.keys, self.hv, q_keys, q_hv, C)

    def search(self, q: np.ndarray, qoff: np.ndarray, C: int | None = None, k: int | None = None):
        """Hash, probe and DTW re-rank a query batch: (ids, dist, cand, ncand, r_size)."""
        C = C or self.p.C
        k = k or self.p.k
        hb, hv, keys = self.hash_queries(q, qoff)
        cand, ncand, rs = self.probe(keys, hv, C)
        ids, dist = ssh.dtw_rerank(hb.x, hb.x_off, self.x, self.x_off, cand, ncand,
                                   self.p.band_frac, k)
        return ids, dist, cand, ncand, rs

    # ---- files -----------------------------------------------------------
    def save(self, path: str):
        """Write the index to directory `path` (raw little-endian arrays and a
        JSON manifest of their dtypes and shapes)."""
        os.makedirs(path, exist_ok=True)
        arrays = {
            "x": self.x, "off": torch.as_tensor(self.off), "hv": self.hv.view(torch.int64),
            "keys": self.keys.view(torch.int64), "dead": self.dead,
            "tab_keys": self.tab_keys.contiguous().view(torch.int64),
            "tab_ids": self.tab_ids.contiguous().view(torch.int32),
            "r": torch.as_tensor(self.r), "draw_r": torch.as_tensor(self.draws[0]),
            "draw_lnc": torch.as_tensor(self.draws[1]), "draw_beta": torch.as_tensor(self.draws[2]),
        }
        manifest = {"format": FORMAT, "params": vars(self.p), "n_live": self.n_live,
                    "arrays": {}}
        for name, t in arrays.items():
            a = t.detach().cpu().numpy()
            a.tofile(os.path.join(path, name + ".bin"))
            manifest["arrays"][name] = {"dtype": a.dtype.str, "shape": list(a.shape)}
        with open(os.path.join(path, "manifest.json"), "w") as f:
            json.dump(manifest, f, indent=1)

    @classmethod
    def load(cls, path: str, device="cuda") -> "DynamicIndex":
        with open(os.path.join(path, "manifest.json")) as f:
            man = json.load(f)
        if man.get("format") != FORMAT:
            raise ValueError(f"{path}: not an index of format {FORMAT}")

        def arr(name):
            m = man["arrays"][name]
            return np.fromfile(os.path.join(path, name + ".bin"),
                               dtype=np.dtype(m["dtype"])).reshape(m["shape"])

        p = Params(**man["params"])
        ix = cls(p, (arr("draw_r"), arr("draw_lnc"), arr("draw_beta")), arr("r"), device)
        dev = ix.dev
        ix.x = torch.as_tensor(arr("x")).to(dev)
        ix.off = arr("off").astype(np.int64)
        ix.x_off = torch.as_tensor(ix.off).to(dev)
        ix.hv = torch.as_tensor(arr("hv")).to(dev).view(torch.uint64)
        ix.keys = torch.as_tensor(arr("keys")).to(dev).view(torch.uint64)
        ix.dead = torch.as_tensor(arr("dead")).to(dev)
        ix.tab_keys = torch.as_tensor(arr("tab_keys")).to(dev).view(torch.uint64)
        ix.tab_ids = torch.as_tensor(arr("tab_ids")).to(dev).view(torch.uint32)
        ix.n_live = int(man["n_live"])
        return ix
