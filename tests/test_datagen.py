"""Input generators (CPU): the row-range random-walk generator gives exactly
the rows of the whole-batch generator, so a batch too large for host memory
can be generated and uploaded piece by piece, and any sample of it drawn again."""
import numpy as np

from paper_1610_07328_amd import datagen


def test_random_walk_rows_equal_the_whole_batch():
    N, m = 9000, 48
    X = datagen.random_walks(N, m, seed=5)
    for lo, hi in [(0, 1), (0, 4096), (4095, 4097), (4100, 8192), (8191, 9000), (3, 8999)]:
        assert np.array_equal(datagen.random_walk_rows(lo, hi, m, seed=5), X[lo:hi]), (lo, hi)


def test_random_walk_rows_are_znormalised():
    Y = datagen.random_walk_rows(100, 200, 256, seed=1).astype(np.float64)
    assert np.allclose(Y.mean(axis=1), 0.0, atol=1e-5)
    assert np.allclose(Y.std(axis=1), 1.0, atol=1e-5)
