"""Helpers shared by the GPU parity tests: data movement and format conversion only."""
from __future__ import annotations

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
