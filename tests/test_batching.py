"""Host side of the batched build (CPU): batch order, length buckets, the
autotuner's cache, and the tiled sketch entry point's validation."""
import ctypes

import numpy as np

from paper_1610_07328_amd import datagen
from paper_1610_07328_amd.batching import TuneCache, length_bucket, longest_first, reorder


def test_longest_first_is_a_stable_descending_order():
    lens = np.array([5, 9, 9, 1, 7, 9])
    perm = longest_first(lens)
    assert perm.tolist() == [1, 2, 5, 4, 0, 3]


def test_reorder_moves_whole_series():
    x, off = datagen.ragged_series(50, 3, 40, seed=1)
    perm = longest_first(np.diff(off))
    nx, noff = reorder(x, off, perm)
    for j, i in enumerate(perm):
        assert np.array_equal(nx[noff[j]:noff[j + 1]], x[off[i]:off[i + 1]])


def test_length_bucket():
    assert length_bucket(np.array([256, 8192])) == 4096
    assert length_bucket(np.array([1024])) == 1024
    assert length_bucket(np.array([1023])) == 512


def test_tune_cache_round_trip(tmp_path):
    path = str(tmp_path / "sub" / "tune.json")
    c = TuneCache(path)
    k = TuneCache.key("gfx950", 80, 3, 15, 100, 4096)
    assert c.get(k) is None
    c.put(k, {"order": "longest_first", "tile_rows": 12})
    assert TuneCache(path).get(k) == {"order": "longest_first", "tile_rows": 12}
    assert k == "gfx950|W=80|delta=3|n=15|H=100|len=4096"


def test_ragged_series_same_with_worker_processes():
    a = datagen.ragged_series(9000, 64, 300, seed=4)
    b = datagen.ragged_series(9000, 64, 300, seed=4, procs=1)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_sketch_tiled_validation_matches_binding():
    from paper_1610_07328_amd import ssh
    L = ssh.lib()
    r = np.ones(128, np.float32)
    for W, d in [(80, 3), (64, 4), (128, 4), (30, 5), (80, 4), (100, 3)]:
        for rows in [0, 4, 8, 12, 16, 20, 24]:
            st = L.ssh_sketch_tiled(None, None, 0, r.ctypes.data, W, d, None, None, None, None,
                                    rows, None)
            assert (st == 0) == ssh.sketch_tile_supported(W, d, rows), (W, d, rows, st)
            if st != 0:
                assert st == -2
