"""Helpers shared by the GPU parity tests: data movement, format conversion and
the DTW result comparison."""
from __future__ import annotations

import math

import numpy as np
import torch


def to_dev(a, dtype=None):
    t = torch.as_tensor(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def to_np(t: torch.Tensor) -> np.ndarray:
    return t.detach().cpu().numpy()


def unpack_bits(words: np.ndarray, bwo: np.ndarray, nbits: np.ndarray, s: int) -> np.ndarray:
    """Bit i of series s is bit (i & 63) of word bwo[s] + (i >> 6)."""
    w = np.ascontiguousarray(words[bwo[s]: bwo[s + 1]], dtype=np.uint64)
    b = np.unpackbits(w.view(np.uint8), bitorder="little")
    return b[: int(nbits[s])]


def ragged(series_list):
    lens = np.array([len(s) for s in series_list], np.int64)
    off = np.zeros(len(series_list) + 1, np.int64)
    np.cumsum(lens, out=off[1:])
    x = np.concatenate([np.asarray(s, np.float32) for s in series_list]) if len(series_list) else \
        np.zeros(0, np.float32)
    return x.astype(np.float32), off


# DTW distances agree within this relative tolerance; top-k ids agree except
# where the oracle's k-th and (k+1)-th distances are that close
DTW_RTOL = 1e-5


def compare_rerank(ids, dist, oids, odist, all_odist, cand, ncand):
    """GPU top-k (ids, dist) against the oracle's (oids, odist, all_odist)."""
    for i in range(ids.shape[0]):
        for j in range(ids.shape[1]):
            if oids[i, j] < 0:
                assert ids[i, j] == -1 and math.isinf(dist[i, j])
                continue
            if math.isinf(odist[i, j]):
                assert math.isinf(dist[i, j])
            else:
                assert abs(dist[i, j] - odist[i, j]) <= DTW_RTOL * max(odist[i, j], 1e-30), (i, j)
        # same ids except where the oracle's k-th and (k+1)-th are near ties
        got, want = set(ids[i][ids[i] >= 0].tolist()), set(oids[i][oids[i] >= 0].tolist())
        if got != want:
            row = np.sort(all_odist[i, : ncand[i]])
            kk = ids.shape[1]
            assert kk < len(row) and abs(row[kk] - row[kk - 1]) <= DTW_RTOL * row[kk], i
