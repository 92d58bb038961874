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
# where the oracle's distances are that close
DTW_RTOL = 1e-5


def _close(a: float, b: float) -> bool:
    if math.isinf(a) or math.isinf(b):
        return math.isinf(a) and math.isinf(b)
    return abs(a - b) <= DTW_RTOL * max(abs(b), 1e-30)


def compare_pair_distances(pair_d, all_odist, ncand) -> float:
    """Every live pair's float32 distance (the re-rank workspace [nq][C])
    against the oracle's float64 one; columns past ncand hold +inf.  Returns
    the largest relative error over the finite pairs."""
    worst = 0.0
    nq, C = all_odist.shape
    for i in range(nq):
        nc = int(min(ncand[i], C))
        for c in range(C):
            got, want = float(pair_d[i, c]), float(all_odist[i, c])
            if c >= nc:
                assert math.isinf(got), (i, c, got)
                continue
            assert _close(got, want), (i, c, got, want)
            if math.isfinite(want) and want > 0:
                worst = max(worst, abs(got - want) / want)
    return worst


def compare_rerank(ids, dist, oids, odist, all_odist, cand, ncand):
    """GPU top-k (ids, dist) against the oracle's (oids, odist, all_odist).

    Position by position: the GPU's distance matches the oracle's at that
    position, the id's own oracle distance is that value too (so an id may
    differ from the oracle's only inside a near tie), and the GPU's order is
    ascending by (distance, id)."""
    k = ids.shape[1]
    for i in range(ids.shape[0]):
        own = {}
        for c in range(int(min(ncand[i], cand.shape[1]))):
            own.setdefault(int(cand[i, c]), float(all_odist[i, c]))
        for j in range(k):
            if oids[i, j] < 0:
                assert ids[i, j] == -1 and math.isinf(dist[i, j]), (i, j)
                continue
            assert ids[i, j] >= 0, (i, j)
            assert _close(float(dist[i, j]), float(odist[i, j])), (i, j, dist[i, j], odist[i, j])
            if ids[i, j] != oids[i, j]:
                mine = own[int(ids[i, j])]
                assert _close(mine, float(odist[i, j])), (i, j, int(ids[i, j]), int(oids[i, j]))
            if j > 0 and ids[i, j - 1] >= 0:
                a, b = (float(dist[i, j - 1]), int(ids[i, j - 1])), (float(dist[i, j]), int(ids[i, j]))
                assert a <= b, (i, j, a, b)
