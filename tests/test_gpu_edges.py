"""Degenerate inputs and the device-side error reports, through the C ABI.

Degenerate series (empty, shorter than the filter, shorter than one shingle)
go through every stage and must match the oracle, including the reserved empty
hash value and key.  Capacity and draw errors are forced from the host: the
kernels detect them, skip the affected series and raise a flag that
ssh_check_device_errors reports; every kernel still runs to completion.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1610_07328_amd import datagen
from tests._gpu_helpers import ragged, to_dev, to_np, unpack_bits
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


W, DELTA, N_SH, K, L = 80, 3, 15, 10, 10


def test_degenerate_series_end_to_end(ssh):
    """Lengths 0, below W, at W, below one shingle, and ordinary ones, in one batch."""
    _announce("degenerate series end to end")
    nbits_needed = (N_SH - 1) * DELTA + W  # shortest series with one shingle
    lens = [0, 1, W - 1, W, W + 1, nbits_needed - 1, nbits_needed, nbits_needed + 1, 1024, 0, 700]
    X = datagen.random_walks(len(lens), 1024, seed=11)
    series = [X[i, :m] for i, m in enumerate(lens)]
    series[-2] = np.zeros(0, np.float32)
    x, off = ragged(series)
    r = datagen.filter_r(W, seed=11)
    draws = datagen.cws_draws(N_SH, K * L, seed=11)
    p = ssh.plan(off, W, DELTA, N_SH)
    bwo, hoff = p.bit_word_off, p.hist_off
    bits, nb, _ = ssh.sketch(to_dev(x), to_dev(off), r, W, DELTA, to_dev(bwo))
    codes, counts, nd = ssh.shingle(bits, to_dev(bwo), nb, N_SH, to_dev(hoff))
    tabs = ssh.CwsTables(*draws, N_SH)
    hv = ssh.cws(codes, counts, to_dev(hoff), nd, tabs)
    keys = ssh.band_keys(hv, K, L, seed=3)
    torch.cuda.synchronize()
    ssh.check_device_errors()
    words, nb, codes, counts, nd = to_np(bits), to_np(nb), to_np(codes), to_np(counts), to_np(nd)
    hv, keys = to_np(hv), to_np(keys)
    lnS = oracle.ln_table(1024)
    for s, xs in enumerate(series):
        ob = oracle.sketch_series(xs, r, W, DELTA)
        assert nb[s] == len(ob), s
        assert np.array_equal(unpack_bits(words, bwo, nb, s), ob), s
        oc, ok = oracle.shingle(ob, N_SH)
        assert nd[s] == len(oc), s
        assert np.array_equal(codes[hoff[s]:hoff[s] + nd[s]], oc), s
        assert np.array_equal(counts[hoff[s]:hoff[s] + nd[s]], ok), s
        _, _, ohv = oracle.cws(oc, ok, *draws, lnS)
        assert np.array_equal(hv[s], ohv), s
        okey = oracle.band_keys(ohv[None, :], K, L, 3)[0]
        assert np.array_equal(keys[s], okey), s
        if len(oc) == 0:
            assert np.all(hv[s] == np.uint64(oracle.EMPTY))
            assert np.all(keys[s] == np.uint64(oracle.KEY_EMPTY))
    # tables over them, and a query without shingles retrieves nothing
    tk, ti = ssh.table_build(to_dev(keys))
    assert_tables_match(to_np(tk), to_np(ti), keys, oracle.build_tables(keys))
    empty_q = int(np.nonzero(nd == 0)[0][0])
    full_q = int(np.argmax(nd))
    qk = to_dev(keys[[empty_q, full_q]])
    qh = to_dev(hv[[empty_q, full_q]])
    cand, ncand, rs = ssh.probe(tk, ti, to_dev(keys), to_dev(hv), qk, qh, 8)
    torch.cuda.synchronize()
    cand, ncand, rs = to_np(cand), to_np(ncand), to_np(rs)
    assert ncand[0] == 0 and rs[0] == 0 and np.all(cand[0] == -1)
    oc, orr = oracle.probe(keys, hv, keys[full_q], hv[full_q], 8)
    assert rs[1] == orr and np.array_equal(cand[1, :ncand[1]], oc)


def test_sketch_capacity_error_is_reported(ssh):
    """A stream capacity below ceil(N_B / 64) words: flagged, the series gets no bits."""
    _announce("sketch capacity error")
    X = datagen.random_walks(3, 1024, seed=12)
    x, off = datagen.csr(X)
    r = datagen.filter_r(W, seed=12)
    p = ssh.plan(off, W, DELTA, N_SH)
    bwo = p.bit_word_off.copy()
    bwo[2:] -= 1  # series 1 loses one word of its capacity
    bits, nb, _ = ssh.sketch(to_dev(x), to_dev(off), r, W, DELTA, to_dev(bwo))
    torch.cuda.synchronize()
    with pytest.raises(ssh.SSHError, match="bit_word_off"):
        ssh.check_device_errors()
    nb = to_np(nb)
    assert nb[1] == 0
    words = to_np(bits)
    for s in (0, 2):
        ob = oracle.sketch_series(X[s], r, W, DELTA)
        assert nb[s] == len(ob) and np.array_equal(unpack_bits(words, bwo, nb, s), ob)
    ssh.check_device_errors()  # the flag was cleared by the report


def test_shingle_capacity_error_is_reported(ssh):
    """A token capacity below N_B - n + 1: flagged, the series gets no tokens."""
    _announce("shingle capacity error")
    X = datagen.random_walks(3, 512, seed=13)
    x, off = datagen.csr(X)
    r = datagen.filter_r(W, seed=13)
    p = ssh.plan(off, W, DELTA, N_SH)
    bits, nb, _ = ssh.sketch(to_dev(x), to_dev(off), r, W, DELTA, to_dev(p.bit_word_off))
    hoff = p.hist_off.copy()
    hoff[1:] -= 1
    hoff[0] = 0  # series 0 loses one slot
    codes, counts, nd = ssh.shingle(bits, to_dev(p.bit_word_off), nb, N_SH, to_dev(hoff))
    torch.cuda.synchronize()
    with pytest.raises(ssh.SSHError, match="hist_off"):
        ssh.check_device_errors()
    assert to_np(nd)[0] == 0
    ssh.check_device_errors()


def test_cws_draw_out_of_range_is_reported(ssh):
    """r must be in (0, 1e5): a zero draw is flagged by the prepare kernel."""
    _announce("cws draw out of range")
    r, lnc, beta = datagen.cws_draws(6, 8, seed=14)
    r = r.copy()
    r[5, 3] = 0.0
    ssh.CwsTables(r, lnc, beta, 6)
    torch.cuda.synchronize()
    with pytest.raises(ssh.SSHError, match="draw"):
        ssh.check_device_errors()
    ssh.check_device_errors()
