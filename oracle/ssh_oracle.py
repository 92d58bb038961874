"""Float64 CPU oracle of the SSH pipeline.  Test infrastructure only.

Each function follows one passage of the paper (Luo & Shrivastava, "SSH
(Sketch, Shingle, & Hash) for Indexing Massive-Scale Time Series"):

* sketch   -- Section 4.1, the sign stream B_X and its worked example;
* shingle  -- Section 4.2, the weighted set S_X of n-grams (eq. "set");
* cws      -- Section 4.3 / Section 2 (Weighted Minwise Hashing, eqs.
              WJaccardDef and CollProb), realised with Ioffe's improved
              consistent weighted sampling, the method the paper cites;
* wmh_int  -- Section 2 (eq. CollProb) by integer replication of the
              weights, hashed with a running minimum as in Section 4
              (Discussions and Practical Issues);
* band_keys, build_tables -- Algorithm 1 (Pre-Processing), d hash tables;
* probe    -- Algorithm 2 (Query Process), the retrieved set R;
* dtw, rerank -- Section 2.1 (DTW) and the last step of Algorithm 2.

Where the paper is silent or garbled, the reading taken is stated in the
docstring of the function that depends on it.
"""
from __future__ import annotations

import decimal
import math

import numpy as np

from . import _dtw_c

U64 = (1 << 64) - 1
EMPTY = U64            # hash value of a series with no shingle
KEY_EMPTY = U64        # band key of a series with no shingle
HV_T_MAX = (1 << 47) - 1  # keeps every hash value below EMPTY, even with k* = 2^16 - 1
GOLDEN_GAMMA = 0x9E3779B97F4A7C15


# ----------------------------------------------------------------------------
# Section 4.1: sliding-window sign sketch
# ----------------------------------------------------------------------------
def num_bits(m: int, W: int, delta: int) -> int:
    """Length N_B of the sign stream.

    The paper writes N_B = (m - W) / delta, but its own worked example
    (m = 4, W = 2, delta = 2) produces two bits, so the count of window
    start positions i * delta with i * delta + W <= m is used:
    floor((m - W) / delta) + 1, and 0 when m < W.
    """
    return (m - W) // delta + 1 if m >= W else 0


def sketch_series(x, r, W: int, delta: int) -> np.ndarray:
    """Bits B_X of one series, 1 for +1 and 0 for -1 (Section 4.1).

    Window i covers x[i*delta : i*delta + W] (0-based, as in the worked
    example).  The inner product r . window is accumulated in float64, term
    by term in ascending filter index; every term is the exact product of
    two float32 values.  Bit i is 1 when that sum is >= 0 (a zero inner
    product gives +1, as the definition's ">= 0" says).
    """
    x = np.asarray(x, dtype=np.float32).astype(np.float64)
    r = np.asarray(r, dtype=np.float32).astype(np.float64)
    assert r.shape[0] == W
    nb = num_bits(x.shape[0], W, delta)
    if nb == 0:
        return np.zeros(0, dtype=np.uint8)
    s = np.zeros(nb, dtype=np.float64)
    for k in range(W):
        s = s + r[k] * x[k: k + delta * (nb - 1) + 1: delta]
    return (s >= 0).astype(np.uint8)


def sketch_batch(X, r, W: int, delta: int) -> np.ndarray:
    """Bits of every row of a [N, m] array; the same arithmetic as sketch_series."""
    X = np.asarray(X, dtype=np.float32).astype(np.float64)
    r = np.asarray(r, dtype=np.float32).astype(np.float64)
    nb = num_bits(X.shape[1], W, delta)
    if nb == 0:
        return np.zeros((X.shape[0], 0), dtype=np.uint8)
    s = np.zeros((X.shape[0], nb), dtype=np.float64)
    for k in range(W):
        s = s + r[k] * X[:, k: k + delta * (nb - 1) + 1: delta]
    return (s >= 0).astype(np.uint8)


# ----------------------------------------------------------------------------
# Section 4.2: n-gram shingles -> weighted set
# ----------------------------------------------------------------------------
def num_shingles(nbits: int, n: int) -> int:
    """Number of n-gram start positions in a stream of nbits bits."""
    return nbits - n + 1 if nbits >= n else 0


def shingle(bits, n: int):
    """Weighted set S_X of a bit stream (Section 4.2, eq. "set").

    Every one of the N_B - n + 1 substrings of length n is a token; its
    weight is the number of times it occurs.  A token is encoded as the
    integer whose binary digits, most significant first, are the n bits in
    stream order (+1 -> 1, -1 -> 0).  Returns (codes ascending, counts), both
    uint32.
    """
    b = np.asarray(bits, dtype=np.int64)
    S = num_shingles(b.shape[0], n)
    if S == 0:
        return np.zeros(0, np.uint32), np.zeros(0, np.uint32)
    codes = np.zeros(S, dtype=np.int64)
    for q in range(n):
        codes = codes * 2 + b[q: q + S]
    u, c = np.unique(codes, return_counts=True)
    return u.astype(np.uint32), c.astype(np.uint32)


# ----------------------------------------------------------------------------
# Section 4.3: weighted MinHash by consistent weighted sampling
# ----------------------------------------------------------------------------
def ln_table(s_max: int) -> np.ndarray:
    """ln(s) for s = 0..s_max, each the float64 nearest to the exact value.

    Computed with Python's decimal module at 60 significant digits and then
    rounded once to float64; entry 0 is -inf and never used.  A rounding
    that the 60-digit value cannot decide raises.
    """
    ctx = decimal.Context(prec=60)
    out = np.empty(s_max + 1, dtype=np.float64)
    out[0] = -np.inf
    for s in range(1, s_max + 1):
        d = ctx.ln(decimal.Decimal(s))
        f = float(d)
        if s > 1:
            eps = abs(d) * decimal.Decimal("1e-50")
            if float(d - eps) != f or float(d + eps) != f:
                raise ArithmeticError(f"ln({s}) too close to a rounding boundary")
        out[s] = f
    return out


def hv_encode(kstar: np.ndarray, tstar: np.ndarray) -> np.ndarray:
    """Pack a sample (k*, t*) into one uint64: min(t*, 2^47 - 1) << 16 | k*.

    The cap keeps the value at most 2^63 - 1, so a sample never reads as the
    EMPTY value (2^64 - 1) of a series without shingles, whatever k* is.
    """
    t = np.minimum(np.asarray(tstar, dtype=np.float64), float(HV_T_MAX)).astype(np.uint64)
    return (t << np.uint64(16)) | np.asarray(kstar, dtype=np.uint64)


def cws(codes, counts, r_tab, lnc_tab, beta_tab, lnS):
    """H weighted-MinHash samples of one weighted set (Ioffe's ICWS).

    For every hash j and every token k with weight S_k > 0, with the draws
    r = r_tab[k, j] ~ Gamma(2,1), ln c = lnc_tab[k, j] (c ~ Gamma(2,1)) and
    beta = beta_tab[k, j] ~ U[0,1):
        t    = floor(ln S_k / r + beta)
        ln y = r * (t - beta)
        ln a = ln c - ln y - r            (a = c / (y e^r), in logs)
    The sample is k* = argmin_k ln a with t* its t.  Every operation is one
    correctly rounded float64 step in exactly this order; ln S_k comes from
    ``lnS`` (correctly rounded).  A tie in ln a goes to the smaller token.

    Returns (k* [H] int64, t* [H] float64, hv [H] uint64).  A set with no
    token returns k* = -1 and hv = EMPTY.
    """
    codes = np.asarray(codes, dtype=np.int64)
    counts = np.asarray(counts, dtype=np.int64)
    H = r_tab.shape[1]
    if codes.shape[0] == 0:
        return (np.full(H, -1, np.int64), np.zeros(H), np.full(H, EMPTY, np.uint64))
    assert np.all(np.diff(codes) > 0) and np.all(counts > 0)
    R = r_tab[codes]
    B = beta_tab[codes]
    LC = lnc_tab[codes]
    ls = lnS[counts][:, None]
    t = np.floor(ls / R + B)
    ln_y = R * (t - B)
    ln_a = (LC - ln_y) - R
    idx = np.argmin(ln_a, axis=0)  # first minimum = smallest token
    kstar = codes[idx]
    tstar = t[idx, np.arange(H)]
    return kstar, tstar, hv_encode(kstar, tstar)


# ----------------------------------------------------------------------------
# Algorithm 1: d hash tables keyed by bands of K hash values
# ----------------------------------------------------------------------------
def mix64(z):
    """SplitMix64 output function (Steele, Lea & Flood 2014) on uint64 arrays."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def wmh_int(codes, counts, H: int, seed: int) -> np.ndarray:
    """Weighted MinHash of one weighted set by integer replication -> hv [H].

    Section 2, eq. CollProb: a hash whose collision probability is the
    generalized Jaccard similarity.  A token c of integer weight n stands for
    the n distinct elements (c, 1) .. (c, n), so the weighted set becomes a
    plain set and one min-hash over it is such a hash; Section 4 (Discussions
    and Practical Issues) hashes the tokens with a running minimum.  Element
    (c, j) is the integer c * 2^32 + j; hash k ranks it by
    mix(s_k XOR element), s_k = mix(seed + (k+1) * gamma), and keeps the
    element of smallest rank (the first one in input order on equal ranks).
    A set whose weights sum to zero gets EMPTY.
    """
    codes = np.asarray(codes, dtype=np.uint64)
    counts = np.asarray(counts, dtype=np.int64)
    total = int(counts.sum())
    if total == 0:
        return np.full(H, EMPTY, dtype=np.uint64)
    # the replicated elements in input order: token by token, j ascending
    starts = np.cumsum(counts) - counts
    j = np.arange(total, dtype=np.int64) - np.repeat(starts, counts) + 1
    elem = (np.repeat(codes, counts) << np.uint64(32)) | j.astype(np.uint64)
    k = np.arange(H, dtype=object)
    s = mix64(np.array([(seed + (kk + 1) * GOLDEN_GAMMA) & U64 for kk in k], dtype=np.uint64))
    rank = mix64(s[:, None] ^ elem[None, :])
    return elem[np.argmin(rank, axis=1)]  # argmin: first of equal minima


def wmh_int_batch(codes, counts, hist_off, n_distinct, H: int, seed: int) -> np.ndarray:
    """wmh_int of every series of a ragged batch (layout of ssh_shingle) -> [N, H]."""
    N = len(hist_off) - 1
    out = np.empty((N, H), dtype=np.uint64)
    for i in range(N):
        a = int(hist_off[i])
        d = int(n_distinct[i])
        out[i] = wmh_int(codes[a:a + d], counts[a:a + d], H, seed)
    return out


def band_keys(hv, K: int, L: int, seed: int) -> np.ndarray:
    """Band keys of hash-value rows hv [N, K*L] -> keys [N, L] uint64.

    Table l is keyed by the K values hv[:, l*K : (l+1)*K] folded with the
    SplitMix64 mix: h = mix(seed + (l+1) * gamma); h = mix(h ^ hv_j) for each j
    of the band in order.  KEY_EMPTY is reserved for series without shingles,
    so a fold that lands on it is moved to KEY_EMPTY - 1.
    """
    hv = np.asarray(hv, dtype=np.uint64)
    N = hv.shape[0]
    assert hv.shape[1] == K * L
    keys = np.empty((N, L), dtype=np.uint64)
    empty = hv[:, 0] == np.uint64(EMPTY)
    with np.errstate(over="ignore"):
        for l in range(L):
            h0 = np.uint64((seed + (l + 1) * GOLDEN_GAMMA) & U64)
            h = np.full(N, mix64(h0), dtype=np.uint64)
            for t in range(K):
                h = mix64(h ^ hv[:, l * K + t])
            h = np.where(h == np.uint64(KEY_EMPTY), np.uint64(KEY_EMPTY - 1), h)
            keys[:, l] = np.where(empty, np.uint64(KEY_EMPTY), h)
    return keys


def build_tables(keys):
    """The L hash tables of Algorithm 1, each a map from key to bucket.

    Algorithm 1 inserts every series into every table under its key for that
    table.  Series are inserted in id order, so a bucket is the ascending list
    of the ids that share one full key (series without shingles sit in the
    KEY_EMPTY bucket, which no query key equals).  How a table is laid out in
    memory is not part of the method.  Returns a list of L dicts
    {key (int): int64 array of ids, ascending}.
    """
    keys = np.asarray(keys, dtype=np.uint64)
    N, L = keys.shape
    tables = []
    for l in range(L):
        col = keys[:, l].tolist()
        buckets = {}
        for i in range(N):
            buckets.setdefault(col[i], []).append(i)
        tables.append({k: np.asarray(v, dtype=np.int64) for k, v in buckets.items()})
    return tables


# ----------------------------------------------------------------------------
# Algorithm 2: probe the d tables, rank the retrieved set R
# ----------------------------------------------------------------------------
def probe(db_keys, db_hv, q_keys, q_hv, C: int):
    """Candidates of one query (Algorithm 2, the loop over hash tables).

    R is the union over tables l of the series whose key in table l equals
    the query's.  Members of R are ranked by the number of the H hash values
    they share with the query (the MinHash estimate of weighted Jaccard,
    eq. CollProb), ties by ascending id; the first C are returned.
    Returns (cand int64 [<= C], |R|).  A query without shingles retrieves
    nothing.
    """
    db_keys = np.asarray(db_keys, dtype=np.uint64)
    q_keys = np.asarray(q_keys, dtype=np.uint64)
    if q_keys[0] == np.uint64(KEY_EMPTY):
        return np.zeros(0, np.int64), 0
    R = set()
    for l in range(db_keys.shape[1]):
        R.update(np.nonzero(db_keys[:, l] == q_keys[l])[0].tolist())
    R = sorted(R)
    if not R:
        return np.zeros(0, np.int64), 0
    ids = np.array(R, dtype=np.int64)
    score = (np.asarray(db_hv)[ids] == np.asarray(q_hv)[None, :]).sum(axis=1)
    order = sorted(range(len(ids)), key=lambda i: (-int(score[i]), int(ids[i])))
    return ids[order[:C]], len(ids)


# ----------------------------------------------------------------------------
# Section 2.1: DTW, and the top-k re-rank that ends Algorithm 2
# ----------------------------------------------------------------------------
def band_radius(band_frac: float, lq: int, lx: int) -> int:
    """Sakoe-Chiba radius r = floor(band_frac * max(lq, lx)), band_frac as float32."""
    return int(math.floor(float(np.float32(band_frac)) * max(lq, lx)))


def dtw(q, x, r: int) -> float:
    """Banded DTW distance in float64 (plain C dynamic program)."""
    return _dtw_c.dtw(q, x, r)


def rerank(q, q_off, db, db_off, cand, ncand, band_frac: float, k: int):
    """Top-k of every query's candidates by DTW distance, ties by ascending id.

    cand is [nq, C] with ncand[i] valid entries per row.  Returns
    (ids int64 [nq, k] padded with -1, dist float64 [nq, k] padded with +inf,
    all distances float64 [nq, C] with +inf past ncand).
    """
    cand = np.asarray(cand, dtype=np.int64)
    nq = len(ncand)
    dist = _dtw_c.dtw_pairs(q, q_off, db, db_off, cand, ncand, band_frac)
    out_id = np.full((nq, k), -1, np.int64)
    out_d = np.full((nq, k), np.inf)
    for i in range(nq):
        rows = sorted((float(dist[i, c]), int(cand[i, c])) for c in range(int(ncand[i])))
        for j, (d, c) in enumerate(rows[:k]):
            out_id[i, j] = c
            out_d[i, j] = d
    return out_id, out_d, dist
