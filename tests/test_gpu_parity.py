"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Bits, counts, hash values, keys, tables and candidate lists must be
identical; DTW distances must agree within 1e-5 relative.  Inputs are the
seeded synthetic generators; no expected value comes from the HIP path.
"""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_1610_07328_amd import datagen
from tests._gpu_helpers import (DTW_RTOL, compare_pair_distances, compare_rerank, ragged, to_dev,
                                to_np, unpack_bits)
from tests._tables import assert_tables_match

pytestmark = pytest.mark.gpu



@pytest.fixture(scope="module")
def ssh():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1610_07328_amd import ssh as mod
    mod.lib()
    return mod


def _announce(msg):
    print(f"\n[case] {msg}", flush=True)


# --------------------------------------------------------------------------
# sketch
# --------------------------------------------------------------------------
def _run_sketch(ssh, x, off, r, W, delta, generic=False):
    p = ssh.plan(off, W, delta, 1)
    bits, nbits, rep = ssh.sketch(to_dev(x), to_dev(off), r, W, delta, to_dev(p.bit_word_off),
                                  generic=generic)
    torch.cuda.synchronize()
    ssh.check_device_errors()
    return to_np(bits), p.bit_word_off, to_np(nbits), int(to_np(rep)[0])


def _assert_sketch_equal(ssh, x, off, r, W, delta, generic=False):
    words, bwo, nb, rep = _run_sketch(ssh, x, off, r, W, delta, generic)
    N = len(off) - 1
    for s in range(N):
        want = oracle.sketch_series(x[off[s]:off[s + 1]], r, W, delta)
        assert nb[s] == len(want), (s, nb[s], len(want))
        got = unpack_bits(words, bwo, nb, s)
        if not np.array_equal(got, want):
            bad = np.nonzero(got != want)[0]
            raise AssertionError(f"series {s}: {len(bad)} bits differ, first at {bad[:5]}")
        # unused high bits of the last word are zero
        if nb[s] % 64:
            last = int(words[bwo[s + 1] - 1])
            assert last >> int(nb[s] % 64) == 0
    return rep


@pytest.mark.parametrize("N,m,W,delta", [(2000, 512, 64, 4), (1024, 1024, 80, 3),
                                         (256, 2048, 128, 4), (512, 700, 30, 5)])
def test_sketch_fast_path_matches_oracle(ssh, N, m, W, delta):
    _announce(f"sketch fast N={N} m={m} W={W} delta={delta}")
    X = datagen.random_walks(N, m, seed=1)
    r = datagen.filter_r(W, seed=1)
    x, off = datagen.csr(X)
    B = oracle.sketch_batch(X, r, W, delta)
    words, bwo, nb, rep = _run_sketch(ssh, x, off, r, W, delta)
    assert np.all(nb == B.shape[1])
    for s in range(N):
        assert np.array_equal(unpack_bits(words, bwo, nb, s), B[s]), s
    # the repair pass is exercised on this data
    assert rep >= 0


@pytest.mark.parametrize("W,delta", [(7, 1), (33, 2), (80, 3), (256, 7), (1, 1), (30, 5)])
def test_sketch_generic_path_ragged(ssh, W, delta):
    _announce(f"sketch generic ragged W={W} delta={delta}")
    rng = np.random.default_rng(W * 10 + delta)
    lens = [0, 1, W - 1, W, W + delta - 1, W + delta, 5 * W + 3, 900, 2500]
    lens += list(rng.integers(0, 1500, size=20))
    series = [datagen.random_walks(1, int(m), seed=int(m) + 3)[0] if m > 1 else
              np.zeros(int(m), np.float32) for m in lens]
    x, off = ragged(series)
    r = datagen.filter_r(W, seed=W)
    _assert_sketch_equal(ssh, x, off, r, W, delta, generic=True)
    _assert_sketch_equal(ssh, x, off, r, W, delta, generic=False)


def test_sketch_multichunk_ragged_ecg(ssh):
    _announce("sketch ragged RW/ECG 256..8192 W=80 delta=3")
    x, off = datagen.ragged_series(40, 256, 8192, seed=5)
    r = datagen.filter_r(80, seed=5)
    _assert_sketch_equal(ssh, x, off, r, 80, 3)


def _near_zero_windows(W, count, seed):
    """Series of one window each whose float64 inner product with r is ~0."""
    rng = np.random.default_rng(seed)
    r = rng.standard_normal(W).astype(np.float32)
    out = []
    for i in range(count):
        w = rng.standard_normal(W).astype(np.float64)
        if i % 3 == 0:
            w *= 2.0 ** rng.integers(-30, 10)
        partial = float(np.dot(r[:-1].astype(np.float64), w[:-1]))
        w[-1] = -partial / float(r[-1])
        w = w.astype(np.float32)
        if i % 7 == 0:
            w[:] = 0.0
        out.append(w)
    return r, out


@pytest.mark.parametrize("W,delta", [(80, 3), (64, 4), (13, 2)])
def test_sketch_adversarial_near_zero_windows(ssh, W, delta):
    _announce(f"sketch adversarial W={W}")
    r, series = _near_zero_windows(W, 600, seed=W)
    x, off = ragged(series)
    rep = _assert_sketch_equal(ssh, x, off, r, W, delta)
    assert rep > 0  # these windows must take the float64 path


@pytest.mark.parametrize("W,delta", [(80, 3), (128, 4)])
def test_sketch_filter_of_wide_dynamic_range(ssh, W, delta):
    """Filter entries from 2^-13 to 2^10, all above fp16's subnormal range, so
    the matrix path's L1 margin applies with weights over many binades; some
    entries exactly representable in fp16.  Near-zero windows over many
    scales, re-aimed at this filter, and random walks, against the oracle."""
    _announce(f"sketch wide-range filter W={W}")
    r, series = _near_zero_windows(W, 300, seed=W + 2)
    rng = np.random.default_rng(W + 3)
    r = r.astype(np.float64) * np.exp2(rng.uniform(-13, 10, size=W))
    r = (np.where(r < 0, -1.0, 1.0) * np.maximum(np.abs(r), 2.0 ** -13)).astype(np.float32)
    r[::7] = np.float16(r[::7]).astype(np.float32)  # no low part
    assert np.all(np.abs(r) >= 2.0 ** -14)
    rr = r.astype(np.float64)
    for i, w in enumerate(series):  # re-aim the windows at the new filter
        w = w.astype(np.float64)
        w[-1] = -float(np.dot(rr[:-1], w[:-1])) / rr[-1]
        series[i] = w.astype(np.float32)
    series = series + list(datagen.random_walks(20, 1024, seed=W + 4))
    x, off = ragged(series)
    assert _assert_sketch_equal(ssh, x, off, r, W, delta) > 0


@pytest.mark.parametrize("W,delta", [(80, 3), (128, 4)])
def test_sketch_l1_margin_items_with_and_without_tiny_samples(ssh, W, delta):
    """The matrix path's L1 margin at the edge of fp16's normal range: windows
    whose samples sit just above 2^-14 (the coarsest relative rounding) aimed
    at a zero sum, the same windows with one sample moved into (0, 2^-14)
    (subnormal or flushed in fp16: the margin's absolute term), and both
    planted in random walks of 1024 samples (items of many windows), against
    the oracle."""
    _announce(f"sketch L1 margin with and without tiny samples W={W}")
    rng = np.random.default_rng(W + 5)
    r = datagen.filter_r(W, seed=W + 5)
    rr = r.astype(np.float64)

    def aimed(w):
        w = w.copy()
        w[-1] = -float(np.dot(rr[:-1], w[:-1])) / rr[-1]
        return w.astype(np.float32)

    series = []
    walks = datagen.random_walks(200, 1024, seed=W + 6)
    for i in range(200):
        w = rng.choice([-1.0, 1.0], size=W) * 2.0 ** -14 * (1 + 3 * rng.random(W))
        clean = aimed(w)
        w[rng.integers(0, W - 1)] = 2.0 ** -16 * (1 + rng.random())
        tiny = aimed(w)
        series += [clean, tiny]
        host = walks[i].copy()
        at = delta * int(rng.integers(0, (1024 - W) // delta))
        host[at:at + W] = clean if i % 2 else tiny
        series.append(host)
    assert any(np.any((w != 0) & (np.abs(w) < 2.0 ** -14)) for w in series)
    assert any(not np.any((w != 0) & (np.abs(w) < 2.0 ** -14)) for w in series[::3])
    x, off = ragged(series)
    assert _assert_sketch_equal(ssh, x, off, r, W, delta) > 0


@pytest.mark.parametrize("W,delta", [(80, 3), (64, 4)])
def test_sketch_filter_with_subnormal_fp16_entry(ssh, W, delta):
    """A filter entry below 2^-14 (fp16's subnormal range) takes the fast path's
    other margin (the sum of squares): near-zero windows and random walks."""
    _announce(f"sketch tiny filter entry W={W}")
    r, series = _near_zero_windows(W, 300, seed=W + 1)
    r = r.copy()
    r[3] = np.float32(3e-6)
    r[W - 2] = np.float32(-2.0 ** -20)
    series = series + list(datagen.random_walks(20, 1024, seed=W))
    x, off = ragged(series)
    assert _assert_sketch_equal(ssh, x, off, r, W, delta) > 0


def test_sketch_huge_and_nonfinite_values(ssh):
    _announce("sketch huge / non-finite values")
    rng = np.random.default_rng(17)
    W, delta = 80, 3
    r = datagen.filter_r(W, seed=17)
    series = []
    for i in range(12):
        s = rng.standard_normal(600).astype(np.float32)
        if i % 4 == 0:
            s *= np.float32(3.0e4)
        elif i % 4 == 1:
            s[rng.integers(0, 600)] = np.inf
        elif i % 4 == 2:
            s[rng.integers(0, 600)] = np.nan
        else:
            s[100:140] = np.float32(-2.0e5)
        series.append(s)
    x, off = ragged(series)
    _assert_sketch_equal(ssh, x, off, r, W, delta)


# --------------------------------------------------------------------------
# shingles
# --------------------------------------------------------------------------
def _pack_streams(streams):
    nb = np.array([len(b) for b in streams], np.int64)
    bwo = np.zeros(len(streams) + 1, np.int64)
    np.cumsum((nb + 63) // 64, out=bwo[1:])
    words = np.zeros(max(int(bwo[-1]), 1), np.uint64)
    for s, b in enumerate(streams):
        if len(b):
            pad = np.zeros(((len(b) + 63) // 64) * 64, np.uint8)
            pad[: len(b)] = b
            words[bwo[s]: bwo[s + 1]] = np.packbits(pad, bitorder="little").view(np.uint64)
    return words, bwo, nb.astype(np.int32)


@pytest.mark.parametrize("n", [1, 2, 5, 12, 15, 16])
def test_shingle_matches_oracle(ssh, n):
    _announce(f"shingle n={n}")
    rng = np.random.default_rng(n)
    streams = []
    for i, L in enumerate([0, 1, n - 1, n, n + 1, 64, 65, 130, 301, 3000, 2705]):
        p = 0.5 if i % 2 else 0.93
        streams.append((rng.random(L) < p).astype(np.uint8))
    # a stream from a real sketch (long runs)
    X = datagen.random_walks(3, 1024, seed=n)
    streams += list(oracle.sketch_batch(X, datagen.filter_r(80, seed=n), 80, 3))
    # distinct-token counts around the LDS count buffer (512 tokens, 16-bit
    # counts), and all-ones streams whose one token has 2^16 - 1 and 2^16
    # occurrences (the second takes the global-count path)
    streams += [(rng.random(L) < 0.5).astype(np.uint8) for L in (450, 520, 600)]
    streams += [np.ones(65535 + n - 1, np.uint8), np.ones(65536 + n - 1, np.uint8)]
    words, bwo, nb = _pack_streams(streams)
    hist_off = np.zeros(len(streams) + 1, np.int64)
    np.cumsum([max(0, int(b) - n + 1) for b in nb], out=hist_off[1:])
    codes, counts, nd = ssh.shingle(to_dev(words), to_dev(bwo), to_dev(nb), n, to_dev(hist_off))
    torch.cuda.synchronize()
    ssh.check_device_errors()
    codes, counts, nd = to_np(codes), to_np(counts), to_np(nd)
    for s, b in enumerate(streams):
        wc, wn = oracle.shingle(b, n)
        assert nd[s] == len(wc), (s, nd[s], len(wc))
        o = hist_off[s]
        assert np.array_equal(codes[o:o + nd[s]], wc), s
        assert np.array_equal(counts[o:o + nd[s]], wn), s


def _de_bruijn_bits(n):
    """A binary de Bruijn cycle of order n (every n-bit word once as a cyclic
    window), by the Fredricksen-Kessler-Maiorana concatenation of Lyndon words."""
    a = [0] * (n + 1)
    seq = []

    def gen(t, p):
        if t > n:
            if n % p == 0:
                seq.extend(a[1:p + 1])
            return
        a[t] = a[t - p]
        gen(t + 1, p)
        if a[t - p] == 0:
            a[t] = 1
            gen(t + 1, t)

    gen(1, 1)
    return np.array(seq, np.uint8)


@pytest.mark.parametrize("n", [12, 15, 16])
def test_shingle_every_code_present(ssh, n):
    """Streams holding every one of the 2^n tokens: the bitmap is full, so the
    rank bases reach D - 1 (2^16 - 1 at n = 16, the largest 16-bit base) and
    every rank reads whole words.  Each token once, twice (two cycles), and
    after a long run of ones; exact against the oracle."""
    _announce(f"shingle every code n={n}")
    cyc = _de_bruijn_bits(n)
    assert len(cyc) == 1 << n
    once = np.concatenate([cyc, cyc[:n - 1]])
    twice = np.concatenate([cyc, cyc, cyc[:n - 1]])
    after_run = np.concatenate([np.ones(3 * n, np.uint8), once])
    streams = [once, twice, after_run]
    words, bwo, nb = _pack_streams(streams)
    hist_off = np.zeros(len(streams) + 1, np.int64)
    np.cumsum([max(0, int(b) - n + 1) for b in nb], out=hist_off[1:])
    codes, counts, nd = ssh.shingle(to_dev(words), to_dev(bwo), to_dev(nb), n, to_dev(hist_off))
    torch.cuda.synchronize()
    ssh.check_device_errors()
    codes, counts, nd = to_np(codes), to_np(counts), to_np(nd)
    for s, b in enumerate(streams):
        wc, wn = oracle.shingle(b, n)
        assert len(wc) == 1 << n
        assert nd[s] == len(wc), (s, nd[s], len(wc))
        o = hist_off[s]
        assert np.array_equal(codes[o:o + nd[s]], wc), s
        assert np.array_equal(counts[o:o + nd[s]], wn), s
    assert np.all(counts[hist_off[1]:hist_off[1] + nd[1]] == 2)


# --------------------------------------------------------------------------
# weighted MinHash
# --------------------------------------------------------------------------
def test_ln_table_exact(ssh):
    _announce("cws lnS table")
    r, lnc, beta = datagen.cws_draws(4, 3, seed=0)
    t = ssh.CwsTables(r, lnc, beta, 4)
    torch.cuda.synchronize()
    got = to_np(t.lnS)
    want = oracle.ln_table(ssh.LNS_ENTRIES - 1)
    assert np.array_equal(got[1:], want[1:])


def _cws_case(ssh, n, H, sets, seed):
    r, lnc, beta = datagen.cws_draws(n, H, seed=seed)
    tabs = ssh.CwsTables(r, lnc, beta, n)
    codes = np.concatenate([c for c, _ in sets] + [np.zeros(0, np.uint32)]).astype(np.uint32)
    counts = np.concatenate([k for _, k in sets] + [np.zeros(0, np.uint32)]).astype(np.uint32)
    ho = np.zeros(len(sets) + 1, np.int64)
    np.cumsum([len(c) for c, _ in sets], out=ho[1:])
    nd = np.array([len(c) for c, _ in sets], np.int32)
    hv = ssh.cws(to_dev(np.maximum(codes, 0) if codes.size else np.zeros(1, np.uint32)),
                 to_dev(counts if counts.size else np.zeros(1, np.uint32)), to_dev(ho),
                 to_dev(nd), tabs)
    torch.cuda.synchronize()
    ssh.check_device_errors()
    hv = to_np(hv)
    smax = int(counts.max()) if counts.size else 1
    lnS = oracle.ln_table(max(smax, 2))
    for s, (c, k) in enumerate(sets):
        want = oracle.cws(c, k, r, lnc, beta, lnS)[2]
        assert np.array_equal(hv[s], want), s


def test_cws_random_sets_exact(ssh):
    _announce("cws random sets n=12 H=20 / n=6 H=257")
    rng = np.random.default_rng(3)
    for n, H in [(12, 20), (6, 257)]:
        sets = [(np.zeros(0, np.uint32), np.zeros(0, np.uint32))]
        for i in range(300):
            D = int(rng.integers(1, min(200, 1 << n) + 1))
            c = np.sort(rng.choice(1 << n, size=D, replace=False)).astype(np.uint32)
            k = (rng.integers(1, 3, size=D) if i % 2 else rng.integers(1, 300, size=D)).astype(np.uint32)
            sets.append((c, k))
        _cws_case(ssh, n, H, sets, seed=n)


def _wmh_case(ssh, sets, H, seed):
    codes = np.concatenate([c for c, _ in sets] + [np.zeros(0, np.uint32)]).astype(np.uint32)
    counts = np.concatenate([k for _, k in sets] + [np.zeros(0, np.uint32)]).astype(np.uint32)
    ho = np.zeros(len(sets) + 1, np.int64)
    np.cumsum([len(c) for c, _ in sets], out=ho[1:])
    nd = np.array([len(c) for c, _ in sets], np.int32)
    hv = to_np(ssh.wmh_int(to_dev(codes), to_dev(counts), to_dev(ho), to_dev(nd), H, seed))
    want = oracle.wmh_int_batch(codes, counts, ho, nd, H, seed)
    assert hv.shape == want.shape
    bad = np.argwhere(hv != want)
    assert bad.size == 0, (H, seed, bad[:5])


@pytest.mark.parametrize("H", [1, 64, 100, 130, 300])
def test_wmh_int_random_sets_exact(ssh, H):
    """Ragged batch: empty sets, zero counts, unsorted tokens, more than 64
    tokens per set, and hash groups past 128."""
    _announce(f"wmh_int random sets H={H}")
    rng = np.random.default_rng(40 + H)
    sets = [(np.zeros(0, np.uint32), np.zeros(0, np.uint32)),
            (np.array([5], np.uint32), np.array([0], np.uint32))]
    for i in range(150):
        D = int(rng.integers(1, 200))
        c = rng.choice(1 << 15, size=D, replace=False).astype(np.uint32)
        if i % 3:
            c = np.sort(c)
        k = rng.integers(0 if i % 5 == 0 else 1, 12, size=D).astype(np.uint32)
        sets.append((c, k))
    sets.append((np.array([7, 9], np.uint32), np.array([3000, 1], np.uint32)))
    _wmh_case(ssh, sets, H, seed=H * 1000003)


def test_wmh_int_after_sketch_and_shingle_with_band_keys(ssh):
    """Random walks through the device sketch and shingle kernels, then the
    integer MinHash and band keys; the oracle runs its own chain from the same
    series.  The integer hash values feed the same tables as the CWS ones."""
    _announce("wmh_int chained after sketch and shingle, band keys")
    W, delta, n, K, L = 80, 3, 15, 10, 10
    lens = [1024] * 60 + [0, 90, 300, 777]
    X = datagen.random_walks(len(lens), 1024, seed=44)
    series = [X[i, :m] for i, m in enumerate(lens)]
    x, off = ragged(series)
    r = datagen.filter_r(W, seed=44)
    p = ssh.plan(off, W, delta, n)
    bits, nb, _ = ssh.sketch(to_dev(x), to_dev(off), r, W, delta, to_dev(p.bit_word_off))
    codes, counts, nd = ssh.shingle(bits, to_dev(p.bit_word_off), nb, n, to_dev(p.hist_off))
    hv = ssh.wmh_int(codes, counts, to_dev(p.hist_off), nd, K * L, 3)
    keys = to_np(ssh.band_keys(hv, K, L, 11))
    hv = to_np(hv)
    sets = [oracle.shingle(oracle.sketch_series(xs, r, W, delta), n) for xs in series]
    want = np.stack([oracle.wmh_int(c, k, K * L, 3) for c, k in sets])
    assert np.array_equal(hv, want)
    assert np.array_equal(keys, oracle.band_keys(want, K, L, 11))


def test_cws_equal_keys_resolved_exactly(ssh):
    """Draws whose weight-1 ln a values all fall into one 16-bit key bucket."""
    _announce("cws equal keys")
    n, H = 7, 24
    rng = np.random.default_rng(12)
    r = 1.0 + rng.random((1 << n, H)) * 1e-6
    lnc = np.zeros((1 << n, H))
    beta = np.zeros((1 << n, H))
    tabs = ssh.CwsTables(r, lnc, beta, n)
    sets = []
    for i in range(200):
        D = int(rng.integers(1, 100))
        c = np.sort(rng.choice(1 << n, size=D, replace=False)).astype(np.uint32)
        k = np.where(rng.random(D) < 0.8, 1, rng.integers(2, 6, size=D)).astype(np.uint32)
        sets.append((c, k))
    codes = np.concatenate([c for c, _ in sets]).astype(np.uint32)
    counts = np.concatenate([k for _, k in sets]).astype(np.uint32)
    ho = np.zeros(len(sets) + 1, np.int64)
    np.cumsum([len(c) for c, _ in sets], out=ho[1:])
    nd = np.array([len(c) for c, _ in sets], np.int32)
    hv = to_np(ssh.cws(to_dev(codes), to_dev(counts), to_dev(ho), to_dev(nd), tabs))
    lnS = oracle.ln_table(8)
    for s, (c, k) in enumerate(sets):
        assert np.array_equal(hv[s], oracle.cws(c, k, r, lnc, beta, lnS)[2]), s


@pytest.mark.parametrize("split", [True, False])
@pytest.mark.parametrize("n,H", [(8, 200), (7, 300), (6, 132), (7, 230), (6, 97)])
def test_cws_several_hash_passes_exact(ssh, n, H, split):
    """H above 128: two or three passes of 128 hashes over the tokens, the
    last one partial (H = 200 is the large workload's); the key table's last
    chunk is padded to 128 columns at H = 230 (102 hashes) and H = 97 (one
    chunk, odd).  Random weighted sets, light and heavy, and an empty one,
    against the oracle; split: fewer than 4,096 series (a workgroup per
    series), else one wave per series."""
    _announce(f"cws several hash passes n={n} H={H} split={split}")
    rng = np.random.default_rng(H + n)
    sets = [(np.zeros(0, np.uint32), np.zeros(0, np.uint32))]
    for i in range(120):
        D = int(rng.integers(1, min(200, 1 << n) + 1))
        c = np.sort(rng.choice(1 << n, size=D, replace=False)).astype(np.uint32)
        k = (rng.integers(1, 3, size=D) if i % 2 else rng.integers(1, 300, size=D)).astype(np.uint32)
        sets.append((c, k))
    reps = 1 if split else 4200 // len(sets) + 1
    _cws_sets_exact(ssh, n, datagen.cws_draws(n, H, seed=n), sets * reps)


def _tied_draws(n, H, a, b, seed, r0=50.0):
    """Tokens a and b get identical draw rows with r in [r0, r0 + 1) and
    beta < 0.8, so t = 0 for every weight w with ln w / r0 < 0.2 and their
    ln a (= ln c + r beta - r) is bit-identical whatever the weights; their
    ln c is low enough that the tie is the minimum."""
    rng = np.random.default_rng(seed)
    D = 1 << n
    r = rng.gamma(2.0, 1.0, (D, H))
    lnc = np.log(rng.gamma(2.0, 1.0, (D, H)))
    beta = rng.random((D, H))
    r[a] = r[b] = r0 + rng.random(H)
    beta[a] = beta[b] = 0.8 * rng.random(H)
    lnc[a] = lnc[b] = -60.0 + rng.random(H)
    return r, lnc, beta


def _cws_sets_exact(ssh, n, draws, sets, expect_k=None):
    tabs = ssh.CwsTables(*draws, n)
    codes = np.concatenate([c for c, _ in sets]).astype(np.uint32)
    counts = np.concatenate([k for _, k in sets]).astype(np.uint32)
    ho = np.zeros(len(sets) + 1, np.int64)
    np.cumsum([len(c) for c, _ in sets], out=ho[1:])
    nd = np.array([len(c) for c, _ in sets], np.int32)
    hv = to_np(ssh.cws(to_dev(codes), to_dev(counts), to_dev(ho), to_dev(nd), tabs))
    torch.cuda.synchronize()
    ssh.check_device_errors()
    lnS = oracle.ln_table(max(2, int(counts.max())))
    checked = {}
    for s, (c, k) in enumerate(sets):
        key = (c.tobytes(), k.tobytes())
        if key not in checked:
            kk, _, want = oracle.cws(c, k, *draws, lnS)
            if expect_k is not None:
                assert np.all(kk == expect_k), s  # the tie is the minimum: the smaller token
            checked[key] = want
        assert np.array_equal(hv[s], checked[key]), s


@pytest.mark.parametrize("H", [130, 132])
@pytest.mark.parametrize("split", [True, False])
def test_cws_exact_ties_go_to_the_smaller_token(ssh, split, H):
    """Two tokens with bit-identical ln a at the minimum, the smaller one wins:
    both keyed (pass A: equal keys, exact re-scan), keyed against heavy in
    either order (pass B's (ln a, k) comparison), and the two run codes at
    counts up to 4096 (keyed by their run rows).  split: fewer than 4,096
    series (a workgroup per series), else one wave per series.  H = 130 and
    132: the second pass over the tokens holds one or two hashes per lane."""
    _announce(f"cws exact ties split={split} H={H}")
    n, a, b = 6, 9, 41
    rng = np.random.default_rng(31)
    weights = [(1, 1), (2, 2), (7, 3), (1, 10), (10, 1), (20, 100), (8, 8), (1, 7), (7, 8)]
    base = []
    for wa, wb in weights:
        others = rng.choice([c for c in range(1 << n) if c not in (a, b)], size=12, replace=False)
        c = np.array(sorted([a, b, *others.tolist()]), np.uint32)
        k = rng.integers(1, 12, size=len(c)).astype(np.uint32)
        k[c == a], k[c == b] = wa, wb
        base.append((c, k))
    reps = 1 if split else 4200 // len(base) + 1
    _cws_sets_exact(ssh, n, _tied_draws(n, H, a, b, seed=32), base * reps, expect_k=a)
    # the run codes 0 and 2^n - 1, keyed up to 4096 (r ~ 100 keeps t = 0 there)
    z, o = 0, (1 << n) - 1
    runs = []
    for wa, wb in [(300, 4096), (4096, 300), (4000, 4000), (1, 4096)]:
        c = np.array([z, 5, 17, o], np.uint32)
        runs.append((c, np.array([wa, 2, 1, wb], np.uint32)))
    _cws_sets_exact(ssh, n, _tied_draws(n, H, z, o, seed=33, r0=100.0),
                    runs * (1 if split else 4200 // len(runs) + 1), expect_k=z)


def test_cws_exact_ties_with_many_distinct_tokens(ssh):
    """n = 16: a set of all 65,536 codes takes the plain exact scan (more
    tokens than 16-bit positions), one of 65,535 the keyed passes; a tied
    pair at the minimum goes to the smaller token in both."""
    _announce("cws exact ties, 65,535 and 65,536 distinct tokens")
    n, H, a, b = 16, 4, 1000, 60000
    draws = _tied_draws(n, H, a, b, seed=34)
    allc = np.arange(1 << n, dtype=np.uint32)
    rng = np.random.default_rng(35)
    w = rng.integers(1, 9, size=1 << n).astype(np.uint32)
    w[a], w[b] = 1, 10
    drop = np.ones(1 << n, bool)
    drop[777] = False
    sets = [(allc, w), (allc[drop], w[drop])]
    _cws_sets_exact(ssh, n, draws, sets, expect_k=a)


def test_cws_saturated_t_is_not_the_empty_value(ssh):
    """n = 16, token 2^16 - 1 wins with a tiny r: t saturates at 2^47 - 1 and
    the hash value and band keys stay distinct from the empty values."""
    _announce("cws saturated t")
    n, H = 16, 3
    D = 1 << n
    r = np.full((D, H), 1.0)
    lnc = np.zeros((D, H))
    beta = np.full((D, H), 0.5)
    k = D - 1
    r[k] = 1e-15
    lnc[k] = -100.0
    tabs = ssh.CwsTables(r, lnc, beta, n)
    sets = [(np.array([5, k], np.uint32), np.array([1, 2], np.uint32)),
            (np.array([k], np.uint32), np.array([3], np.uint32))]
    codes = np.concatenate([c for c, _ in sets])
    counts = np.concatenate([c for _, c in sets])
    ho = np.array([0, 2, 3], np.int64)
    nd = np.array([2, 1], np.int32)
    hv, keys = ssh.cws_band_keys(to_dev(codes), to_dev(counts), to_dev(ho), to_dev(nd), tabs,
                                 1, H, 3)
    torch.cuda.synchronize()
    ssh.check_device_errors()
    hv, keys = to_np(hv), to_np(keys)
    lnS = oracle.ln_table(4)
    for s, (c, kk) in enumerate(sets):
        want = oracle.cws(c, kk, r, lnc, beta, lnS)[2]
        assert np.array_equal(hv[s], want)
        assert np.all(want == np.uint64(((1 << 47) - 1) << 16 | k))
        assert np.array_equal(keys[s], oracle.band_keys(want[None, :], 1, H, 3)[0])
        assert not np.any(keys[s] == np.uint64(oracle.KEY_EMPTY))


def test_cws_counts_beyond_table(ssh):
    _announce("cws counts beyond the ln table")
    rng = np.random.default_rng(4)
    sets = []
    for i in range(40):
        D = 10
        c = np.sort(rng.choice(64, size=D, replace=False)).astype(np.uint32)
        k = rng.integers(65530, 65600, size=D).astype(np.uint32)
        sets.append((c, k))
    _cws_case(ssh, 6, 33, sets, seed=9)


def test_cws_key_rows_at_their_limits(ssh):
    """Weights around the keyed limits: every code up to SSH_CWS_KEY_WEIGHTS, the
    run codes 0 and 2^n - 1 up to SSH_CWS_RUN_CAP, and tokens just past each
    (exact path), alone and mixed, in sets of 1 to 200 tokens."""
    _announce("cws key rows at their limits")
    KW, RC = ssh.CWS_KEY_WEIGHTS, ssh.CWS_RUN_CAP
    edge = np.array([1, 2, 3, KW - 1, KW, KW + 1, KW + 2, 100, RC - 1, RC, RC + 1, 65535, 65536,
                     70000], np.uint32)
    rng = np.random.default_rng(21)
    for n, H in [(10, 30), (15, 100)]:
        mask = (1 << n) - 1
        sets = []
        for i in range(240):
            D = int(rng.integers(1, 201))
            c = np.sort(rng.choice(np.arange(1, mask), size=D, replace=False)).astype(np.uint32)
            k = rng.integers(1, KW + 3, size=D).astype(np.uint32)  # other codes up to KW + 2
            if i % 3 != 2:  # run codes present, with edge weights
                c = np.concatenate([[0], c[: max(D - 2, 0)], [mask]]).astype(np.uint32)
                k = np.concatenate([[edge[rng.integers(len(edge))]], k[: max(D - 2, 0)],
                                    [edge[rng.integers(len(edge))]]]).astype(np.uint32)
            if i % 5 == 0:  # only keyed tokens
                other = (c != 0) & (c != mask)
                k = np.where(other, np.minimum(k, KW), np.minimum(k, RC)).astype(np.uint32)
            sets.append((c, k))
        _cws_case(ssh, n, H, sets, seed=30 + n)


@pytest.mark.parametrize("n,K,L", [(12, 4, 5), (8, 1, 130), (10, 8, 25), (6, 20, 15),
                                   (6, 50, 13)])
def test_cws_band_keys_fused_exact(ssh, n, K, L):
    """CWS with the band keys folded in, against the oracle's CWS then band keys:
    H = 20 (one chunk of hash values), L = 130 (more tables than lanes), H = 200
    (two chunks of 128), and H = 300 and 650 (beyond the kernel's LDS copy:
    two kernels), with empty sets among ragged ones."""
    _announce(f"cws + band keys fused n={n} K={K} L={L}")
    H = K * L
    seed = 0xDEADBEEFCAFEBABE
    rng = np.random.default_rng(40 + n)
    sets = []
    for i in range(150):
        if i % 37 == 0:
            sets.append((np.zeros(0, np.uint32), np.zeros(0, np.uint32)))
            continue
        D = int(rng.integers(1, min(300, 1 << n) + 1))
        c = np.sort(rng.choice(1 << n, size=D, replace=False)).astype(np.uint32)
        k = (rng.integers(1, 4, size=D) if i % 2 else rng.integers(1, 400, size=D)).astype(np.uint32)
        sets.append((c, k))
    r, lnc, beta = datagen.cws_draws(n, H, seed=n)
    tabs = ssh.CwsTables(r, lnc, beta, n)
    codes = np.concatenate([c for c, _ in sets]).astype(np.uint32)
    counts = np.concatenate([k for _, k in sets]).astype(np.uint32)
    ho = np.zeros(len(sets) + 1, np.int64)
    np.cumsum([len(c) for c, _ in sets], out=ho[1:])
    nd = np.array([len(c) for c, _ in sets], np.int32)
    hv, keys = ssh.cws_band_keys(to_dev(codes), to_dev(counts), to_dev(ho), to_dev(nd), tabs, K,
                                 L, seed)
    torch.cuda.synchronize()
    ssh.check_device_errors()
    lnS = oracle.ln_table(int(counts.max()))
    ohv = np.stack([oracle.cws(c, k, r, lnc, beta, lnS)[2] for c, k in sets])
    assert np.array_equal(to_np(hv), ohv)
    assert np.array_equal(to_np(keys), oracle.band_keys(ohv, K, L, seed))


@pytest.mark.parametrize("K,L", [(4, 5), (10, 10), (3, 30)])
def test_cws_band_keys_fused_many_series_per_wave(ssh, K, L):
    """600,000 short sets, so that every wave hashes two or three series and
    folds the bands of several at once: the fused pass against the separate CWS
    and band-key kernels on every series, and against the oracle on a sample."""
    _announce(f"cws + band keys fused, 600k series, K={K} L={L}")
    n, N, H, seed = 10, 600_000, K * L, 12345
    rng = np.random.default_rng(K * 100 + L)
    D = rng.integers(0, 31, size=N)
    D[rng.random(N) < 0.02] = 0
    ho = np.zeros(N + 1, np.int64)
    np.cumsum(D, out=ho[1:])
    total = int(ho[-1])
    sid = np.repeat(np.arange(N), D)
    pos = np.arange(total) - ho[sid]
    a = rng.integers(0, 1 << n, size=N)
    b = rng.integers(0, 1 << (n - 1), size=N) * 2 + 1  # odd step: distinct codes per set
    codes = ((a[sid] + pos * b[sid]) & ((1 << n) - 1)).astype(np.uint32)
    codes = codes[np.lexsort((codes, sid))]  # ascending within each set, as shingling gives
    counts = np.where(rng.random(total) < 0.9, rng.integers(1, 7, size=total),
                      rng.integers(7, 500, size=total)).astype(np.uint32)
    r, lnc, beta = datagen.cws_draws(n, H, seed=K + L)
    tabs = ssh.CwsTables(r, lnc, beta, n)
    dc, dk, dho = to_dev(codes), to_dev(counts), to_dev(ho)
    dnd = to_dev(D.astype(np.int32))
    hv, keys = ssh.cws_band_keys(dc, dk, dho, dnd, tabs, K, L, seed)
    hv2 = ssh.cws(dc, dk, dho, dnd, tabs)
    keys2 = ssh.band_keys(hv2, K, L, seed)
    torch.cuda.synchronize()
    ssh.check_device_errors()
    hv, keys = to_np(hv), to_np(keys)
    assert np.array_equal(hv, to_np(hv2))
    assert np.array_equal(keys, to_np(keys2))
    lnS = oracle.ln_table(int(counts.max()))
    sample = np.concatenate([np.nonzero(D == 0)[0][:20], rng.choice(N, 980, replace=False)])
    ohv = np.stack([oracle.cws(codes[ho[s]:ho[s + 1]], counts[ho[s]:ho[s + 1]], r, lnc, beta,
                               lnS)[2] for s in sample])
    assert np.array_equal(hv[sample], ohv)
    assert np.array_equal(keys[sample], oracle.band_keys(ohv, K, L, seed))


# --------------------------------------------------------------------------
# full pipeline pieces on C1-shaped data
# --------------------------------------------------------------------------
C1 = dict(N=2000, m=512, W=64, delta=4, n=12, K=4, L=5, nq=50, C=50, band=0.05, k=10)


@pytest.fixture(scope="module")
def c1(ssh):
    P = C1
    X = datagen.random_walks(P["N"], P["m"], seed=0)
    r = datagen.filter_r(P["W"], seed=0)
    Q, src = datagen.perturbed_queries(X, P["nq"], 0.1, seed=0)
    Q = np.concatenate([Q, X[:3], np.zeros((1, P["m"]), np.float32)])  # exact copies, one flat
    draws = datagen.cws_draws(P["n"], P["K"] * P["L"], seed=0)
    return X, r, Q, draws


def _gpu_hash(ssh, X, r, draws, P, fused=False):
    x, off = datagen.csr(X)
    p = ssh.plan(off, P["W"], P["delta"], P["n"])
    offd = to_dev(off)
    bits, nb, _ = ssh.sketch(to_dev(x), offd, r, P["W"], P["delta"], to_dev(p.bit_word_off))
    codes, counts, nd = ssh.shingle(bits, to_dev(p.bit_word_off), nb, P["n"], to_dev(p.hist_off))
    tabs = ssh.CwsTables(*draws, P["n"])
    if fused:
        hv, keys = ssh.cws_band_keys(codes, counts, to_dev(p.hist_off), nd, tabs, P["K"], P["L"], 7)
    else:
        hv = ssh.cws(codes, counts, to_dev(p.hist_off), nd, tabs)
        keys = ssh.band_keys(hv, P["K"], P["L"], seed=7)
    torch.cuda.synchronize()
    return hv, keys


def _oracle_hash(X, r, draws, P):
    B = oracle.sketch_batch(X, r, P["W"], P["delta"])
    sets = [oracle.shingle(b, P["n"]) for b in B]
    lnS = oracle.ln_table(max(1, max(int(k.max()) if len(k) else 1 for _, k in sets)))
    hv = np.stack([oracle.cws(c, k, *draws, lnS)[2] for c, k in sets])
    return hv, oracle.band_keys(hv, P["K"], P["L"], seed=7)


def test_c1_hash_values_and_keys_exact(ssh, c1):
    _announce("C1 hash values and keys")
    X, r, Q, draws = c1
    hv, keys = _gpu_hash(ssh, X, r, draws, C1)
    ohv, okeys = _oracle_hash(X, r, draws, C1)
    assert np.array_equal(to_np(hv), ohv)
    assert np.array_equal(to_np(keys), okeys)
    # deterministic: the same launch twice gives the same bits
    hv2, keys2 = _gpu_hash(ssh, X, r, draws, C1)
    assert torch.equal(hv.cpu(), hv2.cpu()) and torch.equal(keys.cpu(), keys2.cpu())
    # the fused CWS + band-key pass writes the same values
    hv3, keys3 = _gpu_hash(ssh, X, r, draws, C1, fused=True)
    assert torch.equal(hv.cpu(), hv3.cpu()) and torch.equal(keys.cpu(), keys3.cpu())


@pytest.mark.parametrize("N,L,distinct", [(2000, 5, None), (10007, 3, 50), (4096, 2, 1),
                                          (3000, 65, 40), (1 << 24, 1, 3000),
                                          ((1 << 24) + 1, 1, 3000)])
def test_table_build_exact(ssh, N, L, distinct):
    """Every bucket of Algorithm 1 read back from the device tables (three radix
    passes for N <= 2^24, four above; L > 64 straight from the series-major keys)."""
    _announce(f"table build N={N} L={L}")
    rng = np.random.default_rng(N)
    if distinct is None:
        keys = rng.integers(0, 2**63, size=(N, L), dtype=np.int64).astype(np.uint64) * np.uint64(2)
    else:
        base = rng.integers(0, 2**63, size=distinct, dtype=np.int64).astype(np.uint64)
        keys = base[rng.integers(0, distinct, size=(N, L))]
        keys[::5] ^= np.uint64(1)  # equal high halves, different full keys
    keys[3] = np.uint64(oracle.KEY_EMPTY)
    tk, ti = ssh.table_build(to_dev(keys))
    torch.cuda.synchronize()
    assert_tables_match(to_np(tk), to_np(ti), keys, oracle.build_tables(keys))
    if N > 1 << 24:  # the probe's search over the 32-bit order, against the brute-force oracle
        hv = rng.integers(0, 4, size=(N, 6), dtype=np.int64).astype(np.uint64)
        qs = [0, 1, 5, N - 1]
        cand, ncand, rs = ssh.probe(tk, ti, to_dev(keys), to_dev(hv), to_dev(keys[qs]),
                                    to_dev(hv[qs]), 20)
        torch.cuda.synchronize()
        cand, ncand, rs = to_np(cand), to_np(ncand), to_np(rs)
        for i, qi in enumerate(qs):
            oc, orr = oracle.probe(keys, hv, keys[qi], hv[qi], 20)
            assert rs[i] == orr and np.array_equal(cand[i, : ncand[i]], oc), qi


def test_c1_probe_exact(ssh, c1):
    """Tables and probe on hash values and keys that the oracle computed."""
    _announce("C1 probe")
    X, r, Q, draws = c1
    P = C1
    ohv, okeys = _oracle_hash(X, r, draws, P)
    oq_hv, oq_keys = _oracle_hash(Q, r, draws, P)
    hv, keys = to_dev(ohv), to_dev(okeys)
    tk, ti = ssh.table_build(keys)
    cand, ncand, rs = ssh.probe(tk, ti, keys, hv, to_dev(oq_keys), to_dev(oq_hv), P["C"])
    torch.cuda.synchronize()
    cand, ncand, rs = to_np(cand), to_np(ncand), to_np(rs)
    for i in range(Q.shape[0]):
        oc, orr = oracle.probe(okeys, ohv, oq_keys[i], oq_hv[i], P["C"])
        assert rs[i] == orr and ncand[i] == len(oc), i
        assert np.array_equal(cand[i, : ncand[i]], oc), i
        assert np.all(cand[i, ncand[i]:] == -1)
    # exact copies find themselves first
    for t in range(3):
        assert cand[P["nq"] + t, 0] == t


def test_c1_wmh_int_pipeline_probe_exact(ssh, c1):
    """The small configuration hashed with the integer MinHash through the
    pipeline (sketch, shingle, MinHash, band keys, tables, probe), against the
    oracle's own chain; H = 20 runs the one-hash-per-lane group."""
    _announce("C1 integer MinHash pipeline and probe")
    from paper_1610_07328_amd.pipeline import HashBatch, Index, Params, QueryBatch
    X, r, Q, _ = c1
    P = C1
    p = Params(W=P["W"], delta=P["delta"], n=P["n"], K=P["K"], L=P["L"], C=P["C"])
    x, off = datagen.csr(X)
    qx, qoff = datagen.csr(Q)
    db = HashBatch(to_dev(x), off, p)
    qh = HashBatch(to_dev(qx), qoff, p)
    db.run(r, method="wmh_int")
    qh.run(r, method="wmh_int")
    ix = Index(db)
    ix.build()
    qb = QueryBatch(qh, ix)
    qb.probe()
    torch.cuda.synchronize()

    def chain(S):
        B = oracle.sketch_batch(S, r, P["W"], P["delta"])
        hv = np.stack([oracle.wmh_int(*oracle.shingle(b, P["n"]), p.H, p.wmh_seed) for b in B])
        return hv, oracle.band_keys(hv, P["K"], P["L"], p.key_seed)

    ohv, okeys = chain(X)
    oq_hv, oq_keys = chain(Q)
    assert np.array_equal(to_np(db.hv[: db.N]), ohv)
    assert np.array_equal(to_np(db.keys[: db.N]), okeys)
    assert np.array_equal(to_np(qh.hv[: qh.N]), oq_hv)
    cand, ncand, rs = to_np(qb.cand), to_np(qb.ncand), to_np(qb.rsize)
    for i in range(Q.shape[0]):
        oc, orr = oracle.probe(okeys, ohv, oq_keys[i], oq_hv[i], P["C"])
        assert rs[i] == orr and ncand[i] == len(oc), i
        assert np.array_equal(cand[i, : ncand[i]], oc), i
    for t in range(3):  # exact copies find themselves first
        assert cand[P["nq"] + t, 0] == t
    with pytest.raises(ValueError):
        db.run(r, method="minhash")


@pytest.mark.parametrize("N,C", [(20000, 1), (20000, 7), (20000, 100), (20000, 600),
                                  (20000, 4096), (150000, 7), (150000, 600)])
def test_probe_large_retrieved_sets_with_ties(ssh, N, C):
    """|R| far above C, a tie level larger than a part's in-LDS tie buffer, and
    every split of a query's entries (8 parts for small C down to 1 for C = 4096).
    Parts of more entries than the in-LDS score cache holds (16,384) score their
    members again in each pass: the single part at C = 4096, and every part at
    N = 150,000."""
    _announce(f"probe large R with ties N={N} C={C}")
    rng = np.random.default_rng(21)
    L, H = 2, 8
    hv = rng.integers(0, 2, size=(N, H), dtype=np.int64).astype(np.uint64)
    keys = np.stack([np.where(rng.random(N) < 0.5, np.uint64(11), np.uint64(22)),
                     np.where(rng.random(N) < 0.5, np.uint64(33), np.uint64(44))], 1).astype(np.uint64)
    keys = keys * np.uint64(0x9E3779B97F4A7C15)
    qk = np.stack([keys[0], keys[1], keys[2]])
    qh = np.stack([hv[0], np.zeros(H, np.uint64), np.full(H, 7, np.uint64)])
    tk, ti = ssh.table_build(to_dev(keys))
    cand, ncand, rs = ssh.probe(tk, ti, to_dev(keys), to_dev(hv), to_dev(qk), to_dev(qh), C)
    torch.cuda.synchronize()
    cand, ncand, rs = to_np(cand), to_np(ncand), to_np(rs)
    for i in range(3):
        oc, orr = oracle.probe(keys, hv, qk[i], qh[i], C)
        assert rs[i] == orr and ncand[i] == len(oc)
        assert np.array_equal(cand[i, : ncand[i]], oc), i


def test_probe_strict_reports_truncation(ssh):
    """ssh_probe_strict writes what ssh_probe writes and returns SSH_ECAPACITY
    exactly when some query's retrieved set exceeds C."""
    _announce("probe strict capacity")
    rng = np.random.default_rng(22)
    N, L, H = 5000, 2, 8
    hv = rng.integers(0, 4, size=(N, H), dtype=np.int64).astype(np.uint64)
    keys = (rng.integers(0, 50, size=(N, L), dtype=np.int64).astype(np.uint64) *
            np.uint64(0x9E3779B97F4A7C15))
    qk, qh = keys[:4].copy(), hv[:4].copy()
    tk, ti = ssh.table_build(to_dev(keys))
    args = (tk, ti, to_dev(keys), to_dev(hv), to_dev(qk), to_dev(qh))
    cand, ncand, rs = ssh.probe(*args, 50)
    torch.cuda.synchronize()
    cand, ncand, rs = to_np(cand), to_np(ncand), to_np(rs)
    big = int(rs.max())
    assert big > 50  # every query's buckets hold about 200 series
    with pytest.raises(ssh.CapacityError, match="largest"):
        ssh.probe(*args, 50, strict=True)
    # the outputs of the refused call are the truncated ones
    c2, n2, r2 = ssh.probe(*args, 50)
    torch.cuda.synchronize()
    assert np.array_equal(to_np(c2), cand) and np.array_equal(to_np(r2), rs)
    # with C at least every |R| the strict call succeeds and equals the plain one
    cs, ns, rss = ssh.probe(*args, big, strict=True)
    cp, npl, rp = ssh.probe(*args, big)
    torch.cuda.synchronize()
    assert np.array_equal(to_np(cs), to_np(cp)) and np.array_equal(to_np(rss), rs)
    for i in range(4):
        oc, orr = oracle.probe(keys, hv, qk[i], qh[i], big)
        assert to_np(rss)[i] == orr and np.array_equal(to_np(cs)[i, : to_np(ns)[i]], oc)


# --------------------------------------------------------------------------
# DTW re-rank
# --------------------------------------------------------------------------
def _al(v):
    return (v + 255) // 256 * 256


def _rerank_run(ssh, q, qoff, db, dboff, cand, ncand, band, k):
    """Both entry points on one batch.  Checks the pruned one against the plain
    one (same bits; every pair it computed has the plain pair's bits, the others
    +inf) and returns (ids, dist, plain pair distances, pruned workspace)."""
    nq, C = cand.shape
    dq, dqo, ddb, ddo = to_dev(q), to_dev(qoff), to_dev(db), to_dev(dboff)
    dc, dn = to_dev(cand), to_dev(ncand)
    ws = torch.empty(ssh.rerank_workspace_bytes(nq, C), dtype=torch.uint8, device="cuda")
    ws_lb = torch.empty(ssh.rerank_lb_workspace_bytes(nq, C, len(q)), dtype=torch.uint8,
                        device="cuda")
    ids, dist = ssh.dtw_rerank(dq, dqo, ddb, ddo, dc, dn, band, k, ws=ws)
    ids_p, dist_p = ssh.dtw_rerank(dq, dqo, ddb, ddo, dc, dn, band, k, ws=ws_lb, prune=True)
    torch.cuda.synchronize()
    ssh.check_device_errors()
    assert np.array_equal(to_np(ids_p), to_np(ids))
    assert np.array_equal(to_np(dist_p).view(np.uint32), to_np(dist).view(np.uint32))
    pair_d = to_np(ssh.pair_distances(ws, nq, C))
    pair_p = to_np(ssh.pair_distances(ws_lb, nq, C))
    same = pair_p.view(np.uint32) == pair_d.view(np.uint32)
    assert np.all(same | np.isinf(pair_p))
    return to_np(ids), to_np(dist), pair_d, pair_p, ws_lb


def _rerank_case(ssh, q, qoff, db, dboff, cand, ncand, band, k):
    """Top-k and every pair distance against the oracle; returns the largest
    relative error of a pair distance."""
    ids, dist, pair_d, _, _ = _rerank_run(ssh, q, qoff, db, dboff, cand, ncand, band, k)
    oids, odist, all_d = oracle.rerank(q, qoff, db, dboff, cand, ncand, band, k)
    compare_rerank(ids, dist, oids, odist, all_d, cand, ncand)
    return compare_pair_distances(pair_d, all_d, ncand)


def _rerank_dense(ssh, Q, X, cand, ncand, band, k):
    q, qoff = datagen.csr(Q)
    db, dboff = datagen.csr(X)
    return _rerank_case(ssh, q, qoff, db, dboff, cand, ncand, band, k)


def test_c1_rerank(ssh, c1):
    _announce("C1 rerank")
    X, r, Q, draws = c1
    rng = np.random.default_rng(0)
    nq, C = Q.shape[0], C1["C"]
    cand = rng.integers(0, X.shape[0], size=(nq, C)).astype(np.int64)
    cand[:, 0] = np.arange(nq) % X.shape[0]
    ncand = rng.integers(0, C + 1, size=nq).astype(np.int32)
    ncand[:5] = C
    _rerank_dense(ssh, Q, X, cand, ncand, C1["band"], C1["k"])


@pytest.mark.parametrize("m,band,lq", [(128, 0.05, 128), (200, 0.0, 200), (200, 1.0, 200),
                                       (1024, 0.05, 1024), (300, 0.1, 290), (64, 0.1, 50),
                                       (2048, 0.1, 2048)])
def test_rerank_band_shapes(ssh, m, band, lq):
    _announce(f"rerank m={m} band={band} lq={lq}")
    N = 40
    X = datagen.random_walks(N, m, seed=m)
    Q = datagen.random_walks(3, lq, seed=lq + 1)
    if lq == m:
        Q[0] = X[5]
    nq = Q.shape[0]
    C = 8 if m >= 2048 else 24
    rng = np.random.default_rng(m)
    cand = rng.integers(0, N, size=(nq, C)).astype(np.int64)
    ncand = np.full(nq, C, np.int32)
    _rerank_dense(ssh, Q, X, cand, ncand, band, min(10, C))


def test_rerank_large_shape_max_error(ssh):
    """The large configuration's pairs (length 2048, 10 % band, r = 204): every
    one of 16 x 64 pair distances within 1e-5 of the float64 oracle; the
    largest relative error is printed."""
    _announce("rerank 2048 x 2048, band 10 %, all pair distances")
    N, m, nq, C = 300, 2048, 16, 64
    X = datagen.random_walks(N, m, seed=71)
    Q, src = datagen.perturbed_queries(X, nq, 0.1, seed=71)
    rng = np.random.default_rng(71)
    cand = rng.integers(0, N, size=(nq, C)).astype(np.int64)
    cand[:, 5] = src
    ncand = np.full(nq, C, np.int32)
    worst = _rerank_dense(ssh, Q, X, cand, ncand, 0.1, 10)
    print(f"[result] largest relative error of {nq * C} pair distances: {worst:.3e}", flush=True)
    assert worst <= DTW_RTOL


def _ragged_batch(lens, seed):
    """Random walks of the given lengths (0 allowed) as CSR."""
    rng = np.random.default_rng(seed)
    series = []
    for ln in lens:
        if ln == 0:
            series.append(np.zeros(0, np.float32))
        else:
            series.append(datagen.znorm(np.cumsum(rng.standard_normal(ln))[None, :])[0]
                          .astype(np.float32))
    return ragged(series)


@pytest.mark.parametrize("band", [0.05, 0.1])
def test_rerank_ragged_mixed_lengths(ssh, band):
    """Queries of lengths 128, 512, 1024 and 2048 (and odd ones) against
    candidates of mixed lengths in one call: every pair takes its own radius
    floor(band * max(lq, lx)), many lane widths run in one call, pairs with
    |lq - lx| above the band and empty series give +inf."""
    _announce(f"rerank ragged lengths band={band}")
    qlens = [128, 512, 1024, 2048, 130, 2000, 700, 1]
    dblens = [128, 512, 1024, 2048, 127, 135, 500, 530, 1000, 1050, 2040, 2048, 0, 1, 2, 64,
              300, 700, 701, 1900]
    q, qoff = _ragged_batch(qlens, seed=81)
    db, dboff = _ragged_batch(dblens, seed=82)
    nq, N, C = len(qlens), len(dblens), 24
    rng = np.random.default_rng(83)
    cand = rng.integers(0, N, size=(nq, C)).astype(np.int64)
    # each query also meets a candidate of its own length and a near-length one
    for i, lq in enumerate(qlens):
        same = [j for j, lx in enumerate(dblens) if lx == lq]
        near = [j for j, lx in enumerate(dblens) if 0 < abs(lx - lq) <= max(2, lq // 50)]
        if same:
            cand[i, 0] = same[0]
        if near:
            cand[i, 1] = near[0]
    ncand = np.full(nq, C, np.int32)
    ncand[6] = 5
    worst = _rerank_case(ssh, q, qoff, db, dboff, cand, ncand, band, 8)
    print(f"[result] largest relative error: {worst:.3e}", flush=True)


def test_rerank_many_pairs_multiblock_plan(ssh):
    """40 queries x 256 candidates (above one planning workgroup's 4,096 pairs,
    so the three-kernel planner runs over ten workgroups), lengths 40..600 and
    a 20 % band: radii up to 120 spread the pairs over the two narrower lane
    groups; every pair distance against the oracle."""
    _announce("rerank 10,240 ragged pairs, multi-workgroup planning")
    rng = np.random.default_rng(101)
    qlens = rng.integers(40, 601, size=40)
    dblens = rng.integers(40, 601, size=300)
    q, qoff = _ragged_batch(qlens, seed=102)
    db, dboff = _ragged_batch(dblens, seed=103)
    nq, C = len(qlens), 256
    cand = rng.integers(0, len(dblens), size=(nq, C)).astype(np.int64)
    ncand = rng.integers(C // 2, C + 1, size=nq).astype(np.int32)
    ncand[0] = C
    worst = _rerank_case(ssh, q, qoff, db, dboff, cand, ncand, 0.2, 10)
    print(f"[result] largest relative error: {worst:.3e}", flush=True)


def test_exhaustive_topk_is_the_oracle_top_k(ssh):
    """The exhaustive search (re-rank rounds over chunks of the whole database,
    then over the survivors) against the oracle's top-10 over every series;
    64-candidate chunks give three rounds over 2,000 series."""
    _announce("exhaustive top-k over 2,000 series in 64-candidate chunks")
    from paper_1610_07328_amd.pipeline import exhaustive_topk
    N, m = 2000, 128
    X = datagen.random_walks(N, m, seed=111)
    Q, src = datagen.perturbed_queries(X, 3, 0.1, seed=111)
    db, dboff = datagen.csr(X)
    ddb, ddo = to_dev(db), to_dev(dboff)
    allc = np.arange(N, dtype=np.int64)[None, :]
    for i in range(3):
        ids, dist = exhaustive_topk(to_dev(Q[i]), ddb, ddo, 0.05, 10, chunk=64)
        torch.cuda.synchronize()
        q, qoff = datagen.csr(Q[i:i + 1])
        oids, odist, all_d = oracle.rerank(q, qoff, db, dboff, allc, np.array([N], np.int32),
                                           0.05, 10)
        compare_rerank(to_np(ids)[None, :], to_np(dist)[None, :], oids, odist, all_d, allc,
                       np.array([N], np.int32))
        assert to_np(ids)[0] == src[i]


def test_rerank_uniform_equals_ragged_layout(ssh):
    """The same pairs computed in a uniform batch and inside a mixed-length
    batch give the same bits (a pair's result does not depend on the others)."""
    _announce("rerank alone vs in a mixed batch")
    X = datagen.random_walks(30, 512, seed=91)
    Q = datagen.random_walks(4, 512, seed=92)
    rng = np.random.default_rng(93)
    cand = rng.integers(0, 30, size=(4, 16)).astype(np.int64)
    ncand = np.full(4, 16, np.int32)
    q, qoff = datagen.csr(Q)
    db, dboff = datagen.csr(X)
    _, _, pd_alone, _, _ = _rerank_run(ssh, q, qoff, db, dboff, cand, ncand, 0.05, 5)
    # the same queries and series among others of other lengths
    extra_q = datagen.random_walks(3, 2048, seed=94)
    extra_x = datagen.random_walks(5, 100, seed=95)
    qs = [Q[0], extra_q[0], Q[1], Q[2], extra_q[1], Q[3], extra_q[2]]
    xs = list(extra_x[:2]) + list(X) + list(extra_x[2:])
    q2, qoff2 = ragged(qs)
    db2, dboff2 = ragged(xs)
    qmap = [0, 2, 3, 5]
    cand2 = rng.integers(0, len(xs), size=(7, 16)).astype(np.int64)
    for i, qi in enumerate(qmap):
        cand2[qi] = cand[i] + 2
    ncand2 = np.full(7, 16, np.int32)
    _, _, pd_mix, _, _ = _rerank_run(ssh, q2, qoff2, db2, dboff2, cand2, ncand2, 0.05, 5)
    assert np.array_equal(pd_mix[qmap].view(np.uint32), pd_alone.view(np.uint32))


def test_rerank_lb_prunes_and_abandons(ssh):
    """Perturbed copies of database series among random candidates (the shape of
    the benchmark's candidate lists), with repeated ids, short and empty lists:
    the pruned re-rank matches the plain one and the oracle, it skips pairs
    (read back from its workspace marks) and it abandons others early (pairs
    of its second pass that report +inf where the plain distance is finite)."""
    _announce("rerank with lower-bound pruning and early abandoning")
    m, N, nq, C, k, band = 512, 400, 24, 50, 10, 0.05
    X = datagen.random_walks(N, m, seed=11)
    Q, src = datagen.perturbed_queries(X, nq, 0.1, seed=11)
    rng = np.random.default_rng(11)
    cand = rng.integers(0, N, size=(nq, C)).astype(np.int64)
    cand[:, 0] = src
    cand[:, 7] = cand[:, 3]  # the same series twice in one list
    ncand = np.full(nq, C, np.int32)
    ncand[1], ncand[2], ncand[3] = 3, 0, k
    q, qoff = datagen.csr(Q)
    db, dboff = datagen.csr(X)
    ids, dist, pair_d, pair_p, ws = _rerank_run(ssh, q, qoff, db, dboff, cand, ncand, band, k)
    oids, odist, all_d = oracle.rerank(q, qoff, db, dboff, cand, ncand, band, k)
    compare_rerank(ids, dist, oids, odist, all_d, cand, ncand)
    compare_pair_distances(pair_d, all_d, ncand)
    # workspace layout: dist, bounds (float32 [nq][C]), marks (u8), slot lists
    # (int32: the first pass's nq k, then the second pass's nq (C - k)), tau
    off = 2 * _al(nq * C * 4)
    marks = to_np(ws[off:off + nq * C]).reshape(nq, C)
    off += _al(nq * C)
    lists = to_np(ws[off:off + nq * C * 4].view(torch.int32))
    list1, list2 = lists[:nq * k].reshape(nq, k), lists[nq * k:].reshape(nq, C - k)
    live = np.arange(C)[None, :] < ncand[:, None]
    first = np.minimum(ncand, k)
    assert np.all(marks[~live] == 0)
    assert np.array_equal((marks == 1).sum(1), first)
    assert np.array_equal((list1 >= 0).sum(1), first)
    kept = (list2 >= 0).sum(1)
    pruned = int(live.sum() - first.sum() - kept.sum())
    second = list2[list2 >= 0]
    flat_p, flat_d = pair_p.reshape(-1), pair_d.reshape(-1)
    abandoned = int(np.sum(np.isinf(flat_p[second]) & np.isfinite(flat_d[second])))
    print(f"[result] pruned {pruned}, abandoned {abandoned} of {int(live.sum())} live pairs",
          flush=True)
    assert pruned > 0 and abandoned > 0


def test_rerank_flags_invalid_id_and_wide_band(ssh):
    """A candidate id outside [0, N) and a pair whose radius exceeds
    SSH_MAX_BAND are flagged and get +inf; the other pairs are computed."""
    _announce("rerank error flags")
    X = datagen.random_walks(4, 100, seed=1)
    Y = datagen.random_walks(2, 600, seed=2)
    q, qoff = ragged([X[0], Y[0]])
    db, dboff = ragged(list(X) + [Y[1]])
    cand = np.array([[0, 1, 9], [4, 4, 0]], np.int64)
    ncand = np.array([3, 2], np.int32)
    ws = torch.empty(ssh.rerank_workspace_bytes(2, 3), dtype=torch.uint8, device="cuda")
    ids, dist = ssh.dtw_rerank(to_dev(q), to_dev(qoff), to_dev(db), to_dev(dboff), to_dev(cand),
                               to_dev(ncand), 0.5, 2, ws=ws)
    with pytest.raises(ssh.SSHError, match="outside"):
        ssh.check_device_errors()
    pd = to_np(ssh.pair_distances(ws, 2, 3))
    assert pd[0, 0] == 0.0 and np.isfinite(pd[0, 1]) and np.isinf(pd[0, 2])
    assert np.all(np.isinf(pd[1]))  # radius 300 > SSH_MAX_BAND
    assert to_np(ids)[0, 0] == 0
    ssh.dtw_rerank(to_dev(q[:100]), to_dev(qoff[:2]), to_dev(db), to_dev(dboff),
                   to_dev(cand[:1, :2]), to_dev(ncand[:1]), 0.5, 2)
    ssh.check_device_errors()  # flags were cleared and nothing new was raised
