"""Seeded synthetic inputs for the SSH hot path.

This module only draws inputs: series, queries, the random filter and the
random numbers of consistent weighted sampling.  It holds none of the
method's arithmetic (no sketching, shingling, hashing or DTW), so that the
HIP path and the CPU oracle can both consume its outputs without sharing
any code.

The series follow the paper's evaluation protocol (Experiments, Datasets):
every series is z-normalised.  The UCR random-walk and ECG recordings used
by the paper are not available, so the generators below stand in for them:

* random walk: x_t = x_{t-1} + N(0, 1), then z-normalised;
* ECG-like: Gaussian pulses (sigma = 6 samples) every 200 +- 20 samples with
  amplitude 1 +- 0.2, a 0.3 * sin baseline wander of period 2000 samples,
  N(0, 0.05^2) noise, then z-normalised.

Z-normalisation is done in float64 with the population standard deviation
and the result is stored as float32.  A constant series becomes all zeros.

Random numbers that the method itself draws are produced here and passed
to both implementations as inputs:

* the sketch filter r ~ N(0, 1)^W (Section 4.1), float32, and F such
  filters at once for the multi-filter sketch;
* for weighted MinHash by Ioffe's improved consistent weighted sampling
  (Section 4.3, cited work), one triple per (code, hash):
  r ~ Gamma(2, 1), ln c with c ~ Gamma(2, 1), and beta ~ U[0, 1),
  each a float64 array of shape [2**n, H] (code-major).

Every stream comes from numpy's PCG64 seeded through SeedSequence, with a
separate child stream per purpose so that changing one size never changes
another stream.
"""
from __future__ import annotations

import concurrent.futures as _fut
import os

import numpy as np

# child-stream indices of SeedSequence(seed).spawn(...)
_DATA, _FILTER, _CWS, _QUERY, _ARRIVAL, _LENGTHS, _FILTERS = range(7)
_N_CHILDREN = 8
# series are drawn in blocks of this many, each block from its own stream,
# so a sample of the first B series is identical whatever the total N is
SERIES_BLOCK = 4096


def _child(seed: int, which: int) -> np.random.SeedSequence:
    return np.random.SeedSequence(seed).spawn(_N_CHILDREN)[which]


def _rng(seed: int, which: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(_child(seed, which)))


def znorm(a: np.ndarray) -> np.ndarray:
    """Z-normalise the rows of ``a`` in float64 (population sigma)."""
    a = np.asarray(a, dtype=np.float64)
    mu = a.mean(axis=-1, keepdims=True)
    sd = a.std(axis=-1, keepdims=True)
    out = np.zeros_like(a)
    np.divide(a - mu, sd, out=out, where=sd > 0)
    return out


def _rw_block(ss: np.random.SeedSequence, rows: int, m: int) -> np.ndarray:
    g = np.random.Generator(np.random.PCG64(ss))
    steps = g.standard_normal((rows, m))
    return znorm(np.cumsum(steps, axis=1)).astype(np.float32)


def _ecg_block(ss: np.random.SeedSequence, rows: int, m: int) -> np.ndarray:
    g = np.random.Generator(np.random.PCG64(ss))
    t = np.arange(m, dtype=np.float64)
    out = np.empty((rows, m), dtype=np.float32)
    npulse = m // 180 + 3
    lag = np.arange(81)
    for i in range(rows):
        tau0 = g.uniform(0.0, 200.0)
        gaps = g.uniform(180.0, 220.0, size=npulse)
        taus = tau0 + np.concatenate(([0.0], np.cumsum(gaps[:-1])))
        amps = g.uniform(0.8, 1.2, size=npulse)
        phi = g.uniform(0.0, 2.0 * np.pi)
        # pulse p covers samples [max(0, tau - 40), min(m, tau + 41)); pulses are
        # at least 180 samples apart, so no sample gets two of them
        lo = np.maximum(0.0, taus - 40.0).astype(np.int64)
        hi = np.minimum(float(m), taus + 41.0).astype(np.int64)
        idx = lo[:, None] + lag[None, :]
        keep = idx < hi[:, None]
        pi, tt = np.nonzero(keep)[0], idx[keep]
        sig = np.zeros(m)
        sig[tt] = amps[pi] * np.exp(-((t[tt] - taus[pi]) ** 2) / (2.0 * 36.0))
        sig += 0.3 * np.sin(2.0 * np.pi * t / 2000.0 + phi)
        sig += g.normal(0.0, 0.05, size=m)
        out[i] = znorm(sig[None, :])[0].astype(np.float32)
    return out


def _blocks(seed: int, N: int, m: int, fn, threads: int | None) -> np.ndarray:
    nblk = (N + SERIES_BLOCK - 1) // SERIES_BLOCK
    kids = _child(seed, _DATA).spawn(nblk)
    out = np.empty((N, m), dtype=np.float32)

    def work(b):
        lo = b * SERIES_BLOCK
        hi = min(N, lo + SERIES_BLOCK)
        out[lo:hi] = fn(kids[b], hi - lo, m)

    threads = threads or min(16, os.cpu_count() or 1)
    if nblk == 1 or threads == 1:
        for b in range(nblk):
            work(b)
    else:
        with _fut.ThreadPoolExecutor(threads) as ex:
            list(ex.map(work, range(nblk)))
    return out


def random_walks(N: int, m: int, seed: int = 0, threads: int | None = None) -> np.ndarray:
    """[N, m] float32 z-normalised random walks."""
    return _blocks(seed, N, m, _rw_block, threads)


def random_walk_rows(lo: int, hi: int, m: int, seed: int = 0,
                     threads: int | None = None) -> np.ndarray:
    """Rows [lo, hi) of random_walks(N, m, seed) for any N >= hi, without drawing
    the others: each block of SERIES_BLOCK series has its own stream, so only
    the blocks that overlap [lo, hi) are drawn.  Lets a batch too large for host
    memory be generated and uploaded piece by piece, and any sample of it be
    drawn again on the host."""
    b0, b1 = lo // SERIES_BLOCK, (hi + SERIES_BLOCK - 1) // SERIES_BLOCK
    kids = _child(seed, _DATA).spawn(b1)
    out = np.empty((hi - lo, m), dtype=np.float32)

    def work(b):
        a = b * SERIES_BLOCK
        rows = _rw_block(kids[b], SERIES_BLOCK, m)
        s0, s1 = max(a, lo), min(a + SERIES_BLOCK, hi)
        out[s0 - lo:s1 - lo] = rows[s0 - a:s1 - a]

    threads = threads or min(16, os.cpu_count() or 1)
    if b1 - b0 == 1 or threads == 1:
        for b in range(b0, b1):
            work(b)
    else:
        with _fut.ThreadPoolExecutor(threads) as ex:
            list(ex.map(work, range(b0, b1)))
    return out


def ecg_like(N: int, m: int, seed: int = 0, threads: int | None = None) -> np.ndarray:
    """[N, m] float32 z-normalised ECG-like series."""
    return _blocks(seed, N, m, _ecg_block, threads)


def _ragged_fill(args):
    """Worker of ragged_series: series [a, b) into the shared value array."""
    from multiprocessing import shared_memory
    name, total, seed, N, a, b, lens, offs = args
    shm = shared_memory.SharedMemory(name=name)
    try:
        x = np.ndarray((total,), dtype=np.float32, buffer=shm.buf)
        kids = _child(seed, _DATA).spawn(b)  # child i is the same whatever the count
        for i in range(a, b):
            fn = _rw_block if i % 2 == 0 else _ecg_block
            x[offs[i - a]:offs[i - a] + lens[i - a]] = fn(kids[i], 1, int(lens[i - a]))[0]
    finally:
        shm.close()
    return b - a


def ragged_series(N: int, m_lo: int, m_hi: int, seed: int = 0, procs: int | None = None):
    """Series of lengths uniform in [m_lo, m_hi]; even ids random walk, odd ECG-like.

    Returns (x: float32[sum m], x_off: int64[N + 1]).  Large batches are drawn
    by worker processes into shared memory (each series has its own stream,
    so the result does not depend on how the work is split).
    """
    g = _rng(seed, _LENGTHS)
    lens = g.integers(m_lo, m_hi + 1, size=N).astype(np.int64)
    off = np.zeros(N + 1, dtype=np.int64)
    np.cumsum(lens, out=off[1:])
    total = int(off[-1])
    procs = procs or min(16, os.cpu_count() or 1)
    if N < 8192 or procs == 1:
        x = np.empty(total, dtype=np.float32)
        kids = _child(seed, _DATA).spawn(N)
        for i in range(N):
            fn = _rw_block if i % 2 == 0 else _ecg_block
            x[off[i]:off[i + 1]] = fn(kids[i], 1, int(lens[i]))[0]
        return x, off
    import multiprocessing as mp
    from multiprocessing import shared_memory
    shm = shared_memory.SharedMemory(create=True, size=max(4 * total, 4))
    try:
        step = (N + 4 * procs - 1) // (4 * procs)
        jobs = [(shm.name, total, seed, N, a, min(N, a + step), lens[a:a + step],
                 off[a:a + step]) for a in range(0, N, step)]
        with _fut.ProcessPoolExecutor(procs, mp_context=mp.get_context("spawn")) as ex:
            assert sum(ex.map(_ragged_fill, jobs)) == N
        x = np.ndarray((total,), dtype=np.float32, buffer=shm.buf).copy()
    finally:
        shm.close()
        shm.unlink()
    return x, off


def csr(series: np.ndarray):
    """[N, m] array -> (flat float32 values, int64 offsets [N + 1])."""
    series = np.ascontiguousarray(series, dtype=np.float32)
    N, m = series.shape
    return series.reshape(-1), np.arange(N + 1, dtype=np.int64) * m


def perturbed_queries(db: np.ndarray, nq: int, noise_std: float = 0.1, seed: int = 0):
    """Queries znorm(db[src] + N(0, noise_std^2)); returns (queries [nq, m] f32, src ids)."""
    g = _rng(seed, _QUERY)
    src = g.permutation(db.shape[0])[:nq].astype(np.int64)
    noisy = db[src].astype(np.float64) + g.normal(0.0, noise_std, size=(nq, db.shape[1]))
    return znorm(noisy).astype(np.float32), src


def filter_r(W: int, seed: int = 0) -> np.ndarray:
    """The sketch filter r ~ N(0, 1)^W as float32 (Section 4.1)."""
    return _rng(seed, _FILTER).standard_normal(W).astype(np.float32)


def filters_R(F: int, W: int, seed: int = 0) -> np.ndarray:
    """F independent sketch filters, [F, W] float32 with N(0, 1) entries (the
    filter of Section 4.1 drawn F times, for the multi-filter sketch)."""
    return _rng(seed, _FILTERS).standard_normal((F, W)).astype(np.float32)


def cws_draws(n: int, H: int, seed: int = 0):
    """ICWS random numbers for every (code, hash): r, ln c, beta; each float64 [2**n, H].

    r and c are Gamma(2, 1) variates, drawn as -ln(u1 u2) from two uniforms;
    beta is uniform on [0, 1).  The log of c is what the sampler consumes,
    so it is drawn directly in that form.
    """
    g = _rng(seed, _CWS)
    D = 1 << n
    r = g.gamma(2.0, 1.0, size=(D, H))
    c = g.gamma(2.0, 1.0, size=(D, H))
    beta = g.random(size=(D, H))
    # Gamma(2, 1) is positive with probability one; guard the measure-zero case
    r = np.maximum(r, np.finfo(np.float64).tiny)
    c = np.maximum(c, np.finfo(np.float64).tiny)
    return r, np.log(c), beta


def walk_stream(length: int, seed: int = 0) -> np.ndarray:
    """One random-walk stream x_t = x_{t-1} + N(0, 1) of `length` samples
    (float64, not normalised): the recording that subsequence search cuts into
    windows (Experiments: every length-l window of a long series)."""
    return np.cumsum(_rng(seed, _DATA).standard_normal(length))


def stream_windows(stream: np.ndarray, ell: int, lo: int, hi: int,
                   threads: int | None = None) -> np.ndarray:
    """Windows stream[s : s + ell] for s in [lo, hi), each z-normalised in
    float64 (population sigma) and stored as float32: [hi - lo, ell]."""
    from numpy.lib.stride_tricks import sliding_window_view
    win = sliding_window_view(stream, ell)
    out = np.empty((hi - lo, ell), dtype=np.float32)
    step = max(1, (1 << 22) // ell)

    def work(a):
        b = min(hi, a + step)
        out[a - lo:b - lo] = znorm(win[a:b]).astype(np.float32)

    starts = range(lo, hi, step)
    threads = threads or min(16, os.cpu_count() or 1)
    if len(starts) == 1 or threads == 1:
        for a in starts:
            work(a)
    else:
        with _fut.ThreadPoolExecutor(threads) as ex:
            list(ex.map(work, starts))
    return out


def stream_queries(stream: np.ndarray, lengths, n_windows: int, count: int, rate: float,
                   noise_std: float = 0.1, seed: int = 0):
    """A Poisson query stream over the windows of `stream`.

    Arrival gaps are exponential with mean 1/rate; each query's length is drawn
    uniformly from `lengths` and its source window uniformly from the first
    n_windows windows of that length; the query is znorm(window +
    N(0, noise_std^2)), the window itself z-normalised first.  Returns
    (arrivals [count] s, class index [count], source window [count], list of
    float32 query arrays)."""
    arrivals = poisson_arrivals(rate, count, seed)
    g = _rng(seed, _LENGTHS)
    cls = g.integers(0, len(lengths), size=count)
    gq = _rng(seed, _QUERY)
    src = gq.integers(0, n_windows, size=count)
    out = []
    for c, s in zip(cls, src):
        ell = lengths[c]
        w = znorm(stream[s:s + ell][None, :])[0]
        out.append(znorm((w + gq.normal(0.0, noise_std, size=ell))[None, :])[0].astype(np.float32))
    return arrivals, cls.astype(np.int64), src.astype(np.int64), out


def poisson_arrivals(rate: float, count: int, seed: int = 0) -> np.ndarray:
    """Arrival times (s) of a Poisson stream with exponential gaps."""
    g = _rng(seed, _ARRIVAL)
    return np.cumsum(g.exponential(1.0 / rate, size=count))
