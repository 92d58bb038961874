"""Check hash tables laid out as (tab_keys, tab_ids) arrays against the oracle's
buckets (Algorithm 1).  The layout's sort order is the library's own choice;
what is checked is what Algorithm 1 fixes: every table holds every id once,
each entry carries its series' key, and the entries of one key, read in
storage order, are exactly that key's bucket (ascending ids)."""
from __future__ import annotations

import numpy as np


def layout_buckets(tk: np.ndarray, ti: np.ndarray):
    """Buckets of one table read from its layout: {key: ids in storage order}."""
    tk = np.asarray(tk, dtype=np.uint64)
    ti = np.asarray(ti, dtype=np.int64)
    order = np.argsort(tk, kind="stable")  # groups equal keys, keeps storage order
    sk, sid = tk[order], ti[order]
    cuts = np.nonzero(sk[1:] != sk[:-1])[0] + 1
    starts = np.concatenate(([0], cuts))
    return {int(sk[s]): ids for s, ids in zip(starts, np.split(sid, cuts))}


def assert_tables_match(tk: np.ndarray, ti: np.ndarray, keys: np.ndarray, buckets=None):
    """tk, ti: [L, N] layout; keys: [N, L]; buckets: oracle.build_tables(keys)."""
    keys = np.asarray(keys, dtype=np.uint64)
    N, L = keys.shape
    assert tk.shape == (L, N) and ti.shape == (L, N)
    for l in range(L):
        ids = np.asarray(ti[l], dtype=np.int64)
        assert np.array_equal(np.sort(ids), np.arange(N)), f"table {l}: not a permutation"
        assert np.array_equal(np.asarray(tk[l], np.uint64), keys[ids, l]), f"table {l}: key moved"
        if buckets is not None:
            got = layout_buckets(tk[l], ti[l])
            want = buckets[l]
            assert got.keys() == want.keys(), f"table {l}: bucket keys differ"
            for k, v in want.items():
                assert np.array_equal(got[k], v), f"table {l}: bucket {k:#x} differs"
