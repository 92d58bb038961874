"""CPU checks of the C ABI: the library loads, exports every declared symbol,
its host-only helpers agree with the oracle's size rules, and argument
validation rejects bad calls before touching the device."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ssh.h")


@pytest.fixture(scope="module")
def ssh():
    from paper_1610_07328_amd import ssh as mod
    if not os.path.exists(mod.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    mod.lib()
    return mod


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\*?\s+\*?([a-z_0-9]+)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if n not in {"if", "return"}))


def test_header_declares_the_pipeline():
    names = _declared_functions()
    for want in ["ssh_sketch", "ssh_shingle", "ssh_cws", "ssh_band_keys", "ssh_cws_band_keys", "dtw_rerank",
                 "ssh_table_build", "ssh_probe", "ssh_plan", "ssh_cws_prepare", "ssh_wmh_int"]:
        assert want in names


def test_every_declared_symbol_is_exported(ssh):
    lib = ctypes.CDLL(ssh.LIB_PATH)
    names = _declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
        assert n in ssh.SIGNATURES, n


def test_size_helpers_match_oracle(ssh):
    for m in [0, 1, 63, 64, 65, 100, 512, 1024, 2048, 8192]:
        for W, d in [(64, 4), (80, 3), (128, 4), (30, 5), (1, 1)]:
            assert ssh.num_bits(m, W, d) == oracle.num_bits(m, W, d)
    for nb in [0, 1, 11, 12, 13, 315]:
        for n in [1, 12, 15, 16]:
            assert ssh.num_shingles(nb, n) == oracle.num_shingles(nb, n)


def test_plan_offsets(ssh):
    rng = np.random.default_rng(0)
    lens = np.concatenate([[0, 79, 80, 83], rng.integers(0, 3000, 50)])
    off = np.zeros(len(lens) + 1, np.int64)
    np.cumsum(lens, out=off[1:])
    p = ssh.plan(off, 80, 3, 15)
    nb = [oracle.num_bits(int(m), 80, 3) for m in lens]
    assert np.array_equal(np.diff(p.bit_word_off), [(b + 63) // 64 for b in nb])
    assert np.array_equal(np.diff(p.hist_off), [oracle.num_shingles(b, 15) for b in nb])
    assert p.max_nbits == max(nb)


def test_validation_rejects_without_device_work(ssh):
    L = ssh.lib()
    EINVAL, EUNSUP = -1, -2
    r = np.ones(8, np.float32)
    dummy = ctypes.c_void_p(16)
    # bad W, delta, N
    assert L.ssh_sketch(dummy, dummy, 4, r.ctypes.data, 0, 1, dummy, dummy, dummy, None, None) == EINVAL
    assert L.ssh_sketch(dummy, dummy, 4, r.ctypes.data, 8, 0, dummy, dummy, dummy, None, None) == EINVAL
    assert L.ssh_sketch(dummy, dummy, -1, r.ctypes.data, 8, 1, dummy, dummy, dummy, None, None) == EINVAL
    assert b"W" in L.ssh_last_error() or b"delta" in L.ssh_last_error() or b"N" in L.ssh_last_error()
    big = np.ones(300, np.float32)
    assert L.ssh_sketch(dummy, dummy, 4, big.ctypes.data, 300, 1, dummy, dummy, dummy, None, None) == EINVAL
    # shingle length beyond 16
    assert L.ssh_shingle(dummy, dummy, dummy, 4, 17, dummy, dummy, dummy, dummy, None) == EINVAL
    # probe cap, rerank k and band
    assert L.ssh_probe(dummy, dummy, 10, 2, dummy, dummy, 4, dummy, dummy, 1, 0, dummy, dummy,
                       dummy, dummy, 1 << 20, None) == EINVAL
    assert L.ssh_probe(dummy, dummy, 10, 2, dummy, dummy, 4, dummy, dummy, 1, 5000, dummy, dummy,
                       dummy, dummy, 1 << 20, None) == EINVAL
    # too small a probe workspace
    assert L.ssh_probe(dummy, dummy, 10, 2, dummy, dummy, 4, dummy, dummy, 3, 50, dummy, dummy,
                       dummy, dummy, 8, None) == EINVAL
    assert L.dtw_rerank(dummy, dummy, 1, dummy, dummy, 10, dummy, dummy, 8, 0.1, 9,
                        dummy, dummy, dummy, 1 << 20, None) == EINVAL
    assert L.dtw_rerank(dummy, dummy, 1, dummy, dummy, 10, dummy, dummy, 8, 1.5, 4,
                        dummy, dummy, dummy, 1 << 20, None) == EINVAL
    assert L.dtw_rerank(dummy, dummy, 2, dummy, dummy, 10, dummy, dummy, 8, 0.1, 4,
                        dummy, dummy, dummy, 16, None) == EINVAL
    assert b"workspace" in L.ssh_last_error()
    # nq * C must stay below 2^31 (int32 pair indices)
    assert L.dtw_rerank(dummy, dummy, 1 << 20, dummy, dummy, 10, dummy, dummy, 4096, 0.1, 4,
                        dummy, dummy, dummy, 1 << 20, None) == EUNSUP
    # the allocation-free re-rank refuses a batch beyond its static scratch, before any device work
    assert L.dtw_rerank_noalloc(dummy, dummy, 1 << 16, dummy, dummy, 10, dummy, dummy, 4096, 0.1,
                                4, dummy, dummy, None) == -4  # SSH_ECAPACITY
    assert b"SSH_NOALLOC_SCRATCH_BYTES" in L.ssh_last_error()
    assert L.dtw_rerank_noalloc(dummy, dummy, 1, dummy, dummy, 10, dummy, dummy, 8, 0.1, 9,
                                dummy, dummy, None) == EINVAL
    # table updates: the sort width may not change, id_base may not reuse ids,
    # n_live within [0, N]; all refused before any device work
    assert L.ssh_table_insert(dummy, dummy, (1 << 24) - 5, dummy, 10, 4, (1 << 24) - 5, dummy,
                              dummy, dummy, 1 << 30, None) == EUNSUP
    assert L.ssh_table_insert(dummy, dummy, 100, dummy, 10, 4, 99, dummy, dummy, dummy, 1 << 30,
                              None) == EINVAL
    assert L.ssh_table_delete(dummy, dummy, 100, 4, dummy, 100, 101, dummy, dummy, dummy,
                              1 << 20, None) == EINVAL
    assert L.ssh_table_delete(dummy, dummy, (1 << 24) + 5, 4, dummy, (1 << 24) + 5, 1000, dummy,
                              dummy, dummy, 1 << 30, None) == EUNSUP
    # the pruned re-rank validates the same way, and its workspace must be large enough
    assert L.dtw_rerank_lb(dummy, dummy, 1, dummy, dummy, 10, dummy, dummy, 8, 0.1, 9,
                           dummy, dummy, dummy, 1 << 20, None) == EINVAL
    assert L.dtw_rerank_lb(dummy, dummy, 1, dummy, dummy, 10, dummy, dummy, 8, 1.5, 4,
                           dummy, dummy, dummy, 1 << 20, None) == EINVAL
    assert L.dtw_rerank_lb(dummy, dummy, 2, dummy, dummy, 10, dummy, dummy, 8, 0.1, 4,
                           dummy, dummy, dummy, 16, None) == EINVAL
    assert b"workspace" in L.ssh_last_error()
    # a filter value that fp16 staging cannot represent is refused
    bad = np.array([1.0, np.inf, 0.5], np.float32)
    assert L.ssh_sketch(dummy, dummy, 4, bad.ctypes.data, 3, 1, dummy, dummy, dummy, None, None) == EINVAL
    # empty batches are not errors
    assert L.ssh_sketch(None, None, 0, r.ctypes.data, 8, 1, None, None, None, None, None) == 0
    # key-table sizes: chunks of 128 hashes, a chunk above 96 hashes padded to 128
    rows = lambda n: ssh.CWS_KEY_WEIGHTS * (1 << n) + 2 * ssh.CWS_RUN_CAP + 1
    assert L.ssh_cws_key_table_elems(15, 100) == rows(15) * 128
    assert L.ssh_cws_key_table_elems(15, 200) == rows(15) * (128 + 72)
    assert L.ssh_cws_key_table_elems(15, 257) == rows(15) * (128 + 128 + 2)
    assert L.ssh_cws_key_table_elems(4, 95) == rows(4) * 96
    assert L.ssh_cws_key_table_elems(4, 96) == rows(4) * 96
    assert L.ssh_cws_key_table_elems(4, 97) == rows(4) * 128
    assert L.ssh_cws_key_table_elems(4, 3) == rows(4) * 4
    assert L.ssh_cws_key_table_elems(0, 10) == 0 and L.ssh_cws_key_table_elems(4, 0) == 0
    # CWS tables with n out of range
    t = ssh._CwsTablesC(17, 4, 16, 16, 16, 16, 16, 16, 16)
    assert L.ssh_cws_prepare(ctypes.byref(t), None) == EINVAL
    # a null scratch table is refused
    t = ssh._CwsTablesC(4, 12, 16, 16, 16, 16, 16, 16, None)
    assert L.ssh_cws_prepare(ctypes.byref(t), None) == EINVAL
    assert b"null table" in L.ssh_last_error()
    # fused CWS + band keys: K * L must equal H, and no null output
    t = ssh._CwsTablesC(4, 12, 16, 16, 16, 16, 16, 16, 16)
    assert L.ssh_cws_band_keys(dummy, dummy, dummy, dummy, 4, ctypes.byref(t), 5, 2, 7, dummy,
                               dummy, None) == EINVAL
    assert b"K * L" in L.ssh_last_error()
    assert L.ssh_cws_band_keys(dummy, dummy, dummy, dummy, 4, ctypes.byref(t), 0, 12, 7, dummy,
                               dummy, None) == EINVAL
    assert L.ssh_cws_band_keys(dummy, dummy, dummy, dummy, 4, ctypes.byref(t), 3, 4, 7, dummy,
                               None, None) == EINVAL
    assert L.ssh_cws_band_keys(None, None, None, None, 0, ctypes.byref(t), 3, 4, 7, None,
                               None, None) == 0
    # integer-replication MinHash: H range, null pointers, empty batch
    assert L.ssh_wmh_int(dummy, dummy, dummy, dummy, 4, 0, 1, dummy, None) == EINVAL
    assert L.ssh_wmh_int(dummy, dummy, dummy, dummy, 4, 65537, 1, dummy, None) == EINVAL
    assert L.ssh_wmh_int(dummy, dummy, dummy, dummy, -1, 8, 1, dummy, None) == EINVAL
    assert L.ssh_wmh_int(dummy, None, dummy, dummy, 4, 8, 1, dummy, None) == EINVAL
    assert b"null pointer" in L.ssh_last_error()
    assert L.ssh_wmh_int(None, None, None, None, 0, 8, 1, None, None) == 0
    assert L.ssh_status_str(EUNSUP) == b"SSH_EUNSUPPORTED"


def test_multi_filter_sketch_validation(ssh):
    """ssh_sketch_multi and its prepare step refuse bad shapes, filter counts,
    depths, filters and workspaces before any device work."""
    L = ssh.lib()
    EINVAL, EUNSUP = -1, -2
    dummy = ctypes.c_void_p(16)
    R = np.random.default_rng(3).standard_normal((32, 80)).astype(np.float32)
    nbytes = L.ssh_sketch_multi_workspace_bytes(32, 80)
    # float32 rows and fp16 rows padded to 96 taps, and two margin constants per filter
    assert nbytes >= 32 * 96 * 6 + 32 * 8
    assert L.ssh_sketch_multi_workspace_bytes(0, 80) == 0
    assert L.ssh_sketch_multi_workspace_bytes(16, 0) == 0
    # shapes without a matrix-core kernel, filter counts, depths
    assert L.ssh_sketch_multi(dummy, dummy, 4, dummy, 32, 81, 3, dummy, 10, dummy, dummy, None,
                              0, None) == EUNSUP
    assert L.ssh_sketch_multi(dummy, dummy, 4, dummy, 24, 80, 3, dummy, 10, dummy, dummy, None,
                              0, None) == EINVAL
    assert L.ssh_sketch_multi(dummy, dummy, 4, dummy, 80, 80, 3, dummy, 10, dummy, dummy, None,
                              0, None) == EINVAL
    assert L.ssh_sketch_multi(dummy, dummy, 4, dummy, 32, 80, 3, dummy, 10, dummy, dummy, None,
                              8, None) == EINVAL
    assert L.ssh_sketch_multi(dummy, None, 4, dummy, 32, 80, 3, dummy, 10, dummy, dummy, None,
                              0, None) == EINVAL
    assert b"null pointer" in L.ssh_last_error()
    assert L.ssh_sketch_multi(None, None, 0, None, 32, 80, 3, None, 0, None, None, None, 0,
                              None) == 0
    # prepare: workspace size, F, shape, and filter values fp16 cannot carry
    assert L.ssh_sketch_multi_prepare(R.ctypes.data, 32, 80, 3, dummy, nbytes - 1, None) == EINVAL
    assert b"workspace" in L.ssh_last_error()
    assert L.ssh_sketch_multi_prepare(R.ctypes.data, 8, 80, 3, dummy, nbytes, None) == EINVAL
    assert L.ssh_sketch_multi_prepare(R.ctypes.data, 32, 80, 4, dummy, nbytes, None) == EUNSUP
    for v in (np.inf, np.nan, 16384.0):
        bad = R.copy()
        bad[31, 0] = v
        assert L.ssh_sketch_multi_prepare(bad.ctypes.data, 32, 80, 3, dummy, nbytes, None) == EINVAL


def test_workspace_sizes(ssh):
    assert ssh.table_workspace_bytes(1_000_000, 10) >= 1_000_000 * 10 * 12
    # distances, class bytes and class lists of every pair
    assert ssh.rerank_workspace_bytes(50, 50) >= 50 * 50 * 9
    # distances, bounds, marks, lists, planning, and two envelopes of the query values
    assert ssh.rerank_lb_workspace_bytes(50, 50, 50 * 1024) >= 50 * 50 * 18 + 2 * 50 * 1024 * 4
    assert ssh.rerank_lb_workspace_bytes(50, 50, 50 * 1024) > ssh.rerank_lb_workspace_bytes(50, 50, 0)
    # the partial rankings of every part of every query, and the runs
    assert ssh.probe_workspace_bytes(1000, 10, 50) >= 1000 * 8 * 50 * 8 + 1000 * 21 * 8
    assert ssh.probe_workspace_bytes(1, 10, 4096) >= 4096 * 8


def test_band_keys_binding_checks_shapes(ssh):
    """band_keys refuses hash values that are not [N, K*L] and a short output
    before any device call (the C call takes no H)."""
    import torch
    hv = torch.zeros((4, 12), dtype=torch.uint64)
    with pytest.raises(ssh.SSHError, match="K\\*L"):
        ssh.band_keys(hv, 5, 2, 1)
    with pytest.raises(ssh.SSHError, match="N\\*L"):
        ssh.band_keys(hv, 4, 3, 1, out=torch.zeros(11, dtype=torch.uint64))
