"""Python binding of the SSH HIP library (libssh_hip.so).

Argument marshalling only: every function allocates its outputs with
PyTorch on the current device, passes raw pointers and the current HIP
stream to the C ABI declared in include/ssh.h, and raises SSHError on a
non-zero status.  All computation runs in the library's kernels; there is no
fallback, and importing this module fails loudly when the library has not
been built.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libssh_hip.so")

HV_EMPTY = (1 << 64) - 1
KEY_EMPTY = (1 << 64) - 1
LNS_ENTRIES = 65536
CWS_KEY_WEIGHTS = 31
CWS_RUN_CAP = 4096
MAX_C = 4096

_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_u64 = ctypes.c_uint64
_f32 = ctypes.c_float
_sz = ctypes.c_size_t


class SSHError(RuntimeError):
    pass


class _CwsTablesC(ctypes.Structure):
    _fields_ = [("n", _i32), ("H", _i32), ("r", _vp), ("lnc", _vp), ("beta", _vp),
                ("a1", _vp), ("lnS", _vp), ("k16", _vp), ("rb", _vp)]


# name -> (restype, argtypes); mirrors include/ssh.h
SIGNATURES = {
    "ssh_status_str": (ctypes.c_char_p, [_i32]),
    "ssh_last_error": (ctypes.c_char_p, []),
    "ssh_num_bits": (_i32, [_i64, _i32, _i32]),
    "ssh_num_shingles": (_i32, [_i32, _i32]),
    "ssh_plan": (_i32, [_vp, _i64, _i32, _i32, _i32, _vp, _vp, _vp]),
    "ssh_sketch": (_i32, [_vp, _vp, _i64, _vp, _i32, _i32, _vp, _vp, _vp, _vp, _vp]),
    "ssh_sketch_generic": (_i32, [_vp, _vp, _i64, _vp, _i32, _i32, _vp, _vp, _vp, _vp, _vp]),
    "ssh_sketch_tiled": (_i32, [_vp, _vp, _i64, _vp, _i32, _i32, _vp, _vp, _vp, _vp, _i32, _vp]),
    "ssh_sketch_multi_workspace_bytes": (_sz, [_i32, _i32]),
    "ssh_sketch_multi_prepare": (_i32, [_vp, _i32, _i32, _i32, _vp, _sz, _vp]),
    "ssh_sketch_multi": (_i32, [_vp, _vp, _i64, _vp, _i32, _i32, _i32, _vp, _i64, _vp, _vp, _vp,
                                _i32, _vp]),
    "ssh_shingle": (_i32, [_vp, _vp, _vp, _i64, _i32, _vp, _vp, _vp, _vp, _vp]),
    "ssh_cws_key_table_elems": (_i64, [_i32, _i32]),
    "ssh_cws_prepare": (_i32, [ctypes.POINTER(_CwsTablesC), _vp]),
    "ssh_cws": (_i32, [_vp, _vp, _vp, _vp, _i64, ctypes.POINTER(_CwsTablesC), _vp, _vp]),
    "ssh_band_keys": (_i32, [_vp, _i64, _i32, _i32, _u64, _vp, _vp]),
    "ssh_cws_band_keys": (_i32, [_vp, _vp, _vp, _vp, _i64, ctypes.POINTER(_CwsTablesC), _i32,
                                 _i32, _u64, _vp, _vp, _vp]),
    "ssh_wmh_int": (_i32, [_vp, _vp, _vp, _vp, _i64, _i32, _u64, _vp, _vp]),
    "ssh_table_workspace_bytes": (_sz, [_i64, _i32]),
    "ssh_table_build": (_i32, [_vp, _i64, _i32, _vp, _vp, _vp, _sz, _vp]),
    "ssh_table_insert_workspace_bytes": (_sz, [_i64, _i32]),
    "ssh_table_insert": (_i32, [_vp, _vp, _i64, _vp, _i64, _i32, _i64, _vp, _vp, _vp, _sz, _vp]),
    "ssh_table_delete_workspace_bytes": (_sz, [_i64, _i32]),
    "ssh_table_delete": (_i32, [_vp, _vp, _i64, _i32, _vp, _i64, _i64, _vp, _vp, _vp, _sz, _vp]),
    "ssh_probe_workspace_bytes": (_sz, [_i32, _i32, _i32]),
    "ssh_probe": (_i32, [_vp, _vp, _i64, _i32, _vp, _vp, _i32, _vp, _vp, _i32, _i32, _vp, _vp,
                         _vp, _vp, _sz, _vp]),
    "ssh_probe_strict": (_i32, [_vp, _vp, _i64, _i32, _vp, _vp, _i32, _vp, _vp, _i32, _i32, _vp,
                                _vp, _vp, _vp, _sz, _vp]),
    "ssh_rerank_workspace_bytes": (_sz, [_i32, _i32]),
    "dtw_rerank": (_i32, [_vp, _vp, _i32, _vp, _vp, _i64, _vp, _vp, _i32, _f32, _i32, _vp,
                          _vp, _vp, _sz, _vp]),
    "dtw_rerank_noalloc": (_i32, [_vp, _vp, _i32, _vp, _vp, _i64, _vp, _vp, _i32, _f32, _i32,
                                  _vp, _vp, _vp]),
    "ssh_rerank_lb_workspace_bytes": (_sz, [_i32, _i32, _i64]),
    "dtw_rerank_lb": (_i32, [_vp, _vp, _i32, _vp, _vp, _i64, _vp, _vp, _i32, _f32, _i32, _vp,
                             _vp, _vp, _sz, _vp]),
    "ssh_check_device_errors": (_i32, []),
}

_lib = None


def lib() -> ctypes.CDLL:
    """Load the library once; raise if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise SSHError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(status: int, what: str) -> None:
    if status != 0:
        L = lib()
        raise SSHError(f"{what}: {L.ssh_status_str(status).decode()}: "
                       f"{L.ssh_last_error().decode()}")


def _dev(t: torch.Tensor, dtype, name: str) -> int:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise SSHError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise SSHError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise SSHError(f"{name} must be contiguous")
    return t.data_ptr()


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _u64_view(t: torch.Tensor) -> torch.Tensor:
    return t  # torch.uint64 tensors carry raw 64-bit patterns


# --------------------------------------------------------------------------
# host helpers
# --------------------------------------------------------------------------
def num_bits(m: int, W: int, delta: int) -> int:
    return int(lib().ssh_num_bits(m, W, delta))


def num_shingles(nbits: int, n: int) -> int:
    return int(lib().ssh_num_shingles(nbits, n))


@dataclass
class Plan:
    bit_word_off: np.ndarray  # int64 [N+1]
    hist_off: np.ndarray      # int64 [N+1]
    max_nbits: int


def plan(x_off: np.ndarray, W: int, delta: int, n: int) -> Plan:
    x_off = np.ascontiguousarray(x_off, dtype=np.int64)
    N = x_off.shape[0] - 1
    bwo = np.empty(N + 1, np.int64)
    ho = np.empty(N + 1, np.int64)
    mx = ctypes.c_int32(0)
    _check(lib().ssh_plan(x_off.ctypes.data, N, W, delta, n, bwo.ctypes.data, ho.ctypes.data,
                          ctypes.addressof(mx)), "ssh_plan")
    return Plan(bwo, ho, int(mx.value))


def check_device_errors() -> None:
    _check(lib().ssh_check_device_errors(), "device error flags")


# --------------------------------------------------------------------------
# pipeline stages
# --------------------------------------------------------------------------
SKETCH_TILES = (8, 12, 16, 20)
_FAST_SHAPES = ((80, 3), (64, 4), (128, 4), (30, 5))


def sketch_tile_supported(W: int, delta: int, rows: int) -> bool:
    """Whether ssh_sketch_tiled offers `rows` for this (W, delta)."""
    return (W, delta) in _FAST_SHAPES and rows in SKETCH_TILES


def sketch(x: torch.Tensor, x_off: torch.Tensor, r: np.ndarray, W: int, delta: int,
           bit_word_off: torch.Tensor, generic: bool = False, out=None, tile_rows: int = 0):
    """Returns (bits uint64 [words], nbits int32 [N], repaired uint64 [1]).
    tile_rows > 0 picks the matrix-core work item (ssh_sketch_tiled)."""
    N = x_off.numel() - 1
    dev = x.device
    total_words = int(bit_word_off[-1].item()) if out is None else None
    if out is None:
        bits = torch.empty(max(total_words, 1), dtype=torch.uint64, device=dev)
        nbits = torch.empty(max(N, 1), dtype=torch.int32, device=dev)
        rep = torch.zeros(1, dtype=torch.uint64, device=dev)
    else:
        bits, nbits, rep = out
    r = np.ascontiguousarray(r, dtype=np.float32)
    if r.shape[0] != W:
        raise SSHError("filter length differs from W")
    args = [_dev(x, torch.float32, "x"), _dev(x_off, torch.int64, "x_off"), N, r.ctypes.data,
            W, delta, _dev(bits, torch.uint64, "bits"),
            _dev(bit_word_off, torch.int64, "bit_word_off"), _dev(nbits, torch.int32, "nbits"),
            _dev(rep, torch.uint64, "repair_count")]
    if tile_rows > 0:
        _check(lib().ssh_sketch_tiled(*args, tile_rows, _stream()), "ssh_sketch_tiled")
    else:
        fn = lib().ssh_sketch_generic if generic else lib().ssh_sketch
        _check(fn(*args, _stream()), "ssh_sketch")
    return bits, nbits[:N], rep


class MultiFilter:
    """F filters prepared for ssh_sketch_multi (a device block holding them
    as the kernels read them, written once)."""

    def __init__(self, R: np.ndarray, delta: int, device="cuda"):
        R = np.ascontiguousarray(R, dtype=np.float32)
        if R.ndim != 2:
            raise SSHError("filters must be a [F, W] array")
        self.F, self.W = R.shape
        self.delta = delta
        nbytes = lib().ssh_sketch_multi_workspace_bytes(self.F, self.W)
        if nbytes == 0:
            raise SSHError("F or W out of range")
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
        _check(lib().ssh_sketch_multi_prepare(R.ctypes.data, self.F, self.W, delta,
                                              self.ws.data_ptr(), nbytes, _stream()),
               "ssh_sketch_multi_prepare")


def sketch_multi(x: torch.Tensor, x_off: torch.Tensor, filters: MultiFilter,
                 bit_word_off: torch.Tensor, kdepth: int = 0, out=None):
    """Returns (bits uint64 [F, words], nbits int32 [N], repaired uint64 [1]):
    row f of bits is the stream set of filter f, laid out as ssh_sketch's."""
    N = x_off.numel() - 1
    dev = x.device
    total_words = int(bit_word_off[-1].item())
    if out is None:
        bits = torch.empty((filters.F, max(total_words, 1)), dtype=torch.uint64, device=dev)
        nbits = torch.empty(max(N, 1), dtype=torch.int32, device=dev)
        rep = torch.zeros(1, dtype=torch.uint64, device=dev)
    else:
        bits, nbits, rep = out
    stride = bits.shape[1] if bits.dim() == 2 else total_words
    _check(lib().ssh_sketch_multi(_dev(x, torch.float32, "x"), _dev(x_off, torch.int64, "x_off"),
                                  N, filters.ws.data_ptr(), filters.F, filters.W, filters.delta,
                                  _dev(bits, torch.uint64, "bits"), stride,
                                  _dev(bit_word_off, torch.int64, "bit_word_off"),
                                  _dev(nbits, torch.int32, "nbits"),
                                  _dev(rep, torch.uint64, "repair_count"), kdepth, _stream()),
           "ssh_sketch_multi")
    return bits, nbits[:N], rep


def shingle(bits, bit_word_off, nbits, n: int, hist_off, out=None):
    """Returns (codes uint32, counts uint32, n_distinct int32 [N])."""
    N = hist_off.numel() - 1
    dev = bits.device
    if out is None:
        cap = max(int(hist_off[-1].item()), 1)
        codes = torch.empty(cap, dtype=torch.uint32, device=dev)
        counts = torch.empty(cap, dtype=torch.uint32, device=dev)
        nd = torch.empty(max(N, 1), dtype=torch.int32, device=dev)
    else:
        codes, counts, nd = out
    _check(lib().ssh_shingle(_dev(bits, torch.uint64, "bits"),
                             _dev(bit_word_off, torch.int64, "bit_word_off"),
                             _dev(nbits, torch.int32, "nbits"), N, n,
                             _dev(codes, torch.uint32, "codes"),
                             _dev(counts, torch.uint32, "counts"),
                             _dev(hist_off, torch.int64, "hist_off"),
                             _dev(nd, torch.int32, "n_distinct"), _stream()), "ssh_shingle")
    return codes, counts, nd[:N]


class CwsTables:
    """Device copies of the ICWS draws plus the prepared a1, lnS, key and (r, beta) tables."""

    def __init__(self, r: np.ndarray, lnc: np.ndarray, beta: np.ndarray, n: int,
                 device="cuda"):
        D, H = r.shape
        if D != (1 << n) or lnc.shape != r.shape or beta.shape != r.shape:
            raise SSHError("draw tables must be [2**n, H]")
        self.n, self.H = n, H
        f64 = dict(dtype=torch.float64, device=device)
        self.r = torch.as_tensor(np.ascontiguousarray(r), **f64)
        self.lnc = torch.as_tensor(np.ascontiguousarray(lnc), **f64)
        self.beta = torch.as_tensor(np.ascontiguousarray(beta), **f64)
        self.a1 = torch.empty((D, H), **f64)
        self.lnS = torch.empty(LNS_ENTRIES, **f64)
        nkeys = int(lib().ssh_cws_key_table_elems(n, H))
        if nkeys <= 0:
            raise SSHError(f"no key table for n={n}, H={H}")
        self.k16 = torch.empty(nkeys, dtype=torch.int16, device=device)
        self.rb = torch.empty((D, H, 2), **f64)
        self._c = _CwsTablesC(n, H, self.r.data_ptr(), self.lnc.data_ptr(), self.beta.data_ptr(),
                              self.a1.data_ptr(), self.lnS.data_ptr(), self.k16.data_ptr(),
                              self.rb.data_ptr())
        _check(lib().ssh_cws_prepare(ctypes.byref(self._c), _stream()), "ssh_cws_prepare")


def cws(codes, counts, hist_off, n_distinct, tables: CwsTables, out=None):
    """Returns hv uint64 [N, H]."""
    N = hist_off.numel() - 1
    hv = out if out is not None else torch.empty((max(N, 1), tables.H), dtype=torch.uint64,
                                                 device=codes.device)
    _check(lib().ssh_cws(_dev(codes, torch.uint32, "codes"), _dev(counts, torch.uint32, "counts"),
                         _dev(hist_off, torch.int64, "hist_off"),
                         _dev(n_distinct, torch.int32, "n_distinct"), N,
                         ctypes.byref(tables._c), _dev(hv, torch.uint64, "hv"), _stream()),
           "ssh_cws")
    return hv[:N]


def band_keys(hv: torch.Tensor, K: int, L: int, seed: int, out=None):
    """Band keys of hash-value rows hv [N, K*L]; returns keys [N, L] (uint64)."""
    if hv.dim() != 2 or hv.shape[1] != K * L:
        raise SSHError(f"band_keys: hv must be [N, K*L] = [N, {K * L}], got {tuple(hv.shape)}")
    N = hv.shape[0]
    keys = out if out is not None else torch.empty((max(N, 1), L), dtype=torch.uint64,
                                                   device=hv.device)
    if keys.numel() < N * L:
        raise SSHError(f"band_keys: keys holds {keys.numel()} values, needs N*L = {N * L}")
    _check(lib().ssh_band_keys(_dev(hv, torch.uint64, "hv"), N, K, L, seed & ((1 << 64) - 1),
                               _dev(keys, torch.uint64, "keys"), _stream()), "ssh_band_keys")
    return keys.view(-1)[: N * L].view(N, L)


def cws_band_keys(codes, counts, hist_off, n_distinct, tables: CwsTables, K: int, L: int,
                  seed: int, out=None):
    """CWS hash values and band keys in one pass; returns (hv [N, H], keys [N, L])."""
    N = hist_off.numel() - 1
    dev = codes.device
    hv, keys = out if out is not None else (
        torch.empty((max(N, 1), tables.H), dtype=torch.uint64, device=dev),
        torch.empty((max(N, 1), L), dtype=torch.uint64, device=dev))
    if hv.numel() < N * tables.H or keys.numel() < N * L:
        raise SSHError("cws_band_keys: output buffers too small")
    _check(lib().ssh_cws_band_keys(
        _dev(codes, torch.uint32, "codes"), _dev(counts, torch.uint32, "counts"),
        _dev(hist_off, torch.int64, "hist_off"), _dev(n_distinct, torch.int32, "n_distinct"), N,
        ctypes.byref(tables._c), K, L, seed & ((1 << 64) - 1), _dev(hv, torch.uint64, "hv"),
        _dev(keys, torch.uint64, "keys"), _stream()), "ssh_cws_band_keys")
    return hv.view(-1)[: N * tables.H].view(N, tables.H), keys.view(-1)[: N * L].view(N, L)


def wmh_int(codes, counts, hist_off, n_distinct, H: int, seed: int, out=None):
    """Weighted MinHash by integer replication; returns hv [N, H] (uint64)."""
    N = hist_off.numel() - 1
    hv = out if out is not None else torch.empty((max(N, 1), H), dtype=torch.uint64,
                                                 device=codes.device)
    if hv.numel() < N * H:
        raise SSHError("wmh_int: output buffer too small")
    _check(lib().ssh_wmh_int(
        _dev(codes, torch.uint32, "codes"), _dev(counts, torch.uint32, "counts"),
        _dev(hist_off, torch.int64, "hist_off"), _dev(n_distinct, torch.int32, "n_distinct"), N,
        H, seed & ((1 << 64) - 1), _dev(hv, torch.uint64, "hv"), _stream()), "ssh_wmh_int")
    return hv.view(-1)[: N * H].view(N, H)


def table_sort_bits(N: int) -> int:
    """Top key bits the tables of N series are ordered by (the probe's search width)."""
    return 24 if N <= (1 << 24) else 32


def table_workspace_bytes(N: int, L: int) -> int:
    return int(lib().ssh_table_workspace_bytes(N, L))


def table_build(keys: torch.Tensor, ws: torch.Tensor | None = None, out=None):
    """Returns (tab_keys uint64 [L, N], tab_ids uint32 [L, N])."""
    N, L = keys.shape
    dev = keys.device
    if out is None:
        tk = torch.empty((L, max(N, 1)), dtype=torch.uint64, device=dev)
        ti = torch.empty((L, max(N, 1)), dtype=torch.uint32, device=dev)
    else:
        tk, ti = out
    need = table_workspace_bytes(N, L)
    if ws is None:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
    _check(lib().ssh_table_build(_dev(keys, torch.uint64, "keys"), N, L,
                                 _dev(tk, torch.uint64, "tab_keys"),
                                 _dev(ti, torch.uint32, "tab_ids"), _dev(ws, torch.uint8, "ws"),
                                 ws.numel(), _stream()), "ssh_table_build")
    return tk[:, :N], ti[:, :N]


def table_insert(tab_keys, tab_ids, new_keys, id_base: int | None = None, out=None, ws=None):
    """Tables of N entries plus M new series with ids id_base..id_base+M-1 (default
    N) -> (tab_keys [L, N+M], tab_ids)."""
    L, N = tab_keys.shape
    M = new_keys.shape[0]
    dev = new_keys.device
    if out is None:
        out = (torch.empty((L, max(N + M, 1)), dtype=torch.uint64, device=dev),
               torch.empty((L, max(N + M, 1)), dtype=torch.uint32, device=dev))
    need = int(lib().ssh_table_insert_workspace_bytes(M, L))
    if ws is None or ws.numel() < need:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
    tk = tab_keys.contiguous() if N > 0 else tab_keys
    ti = tab_ids.contiguous() if N > 0 else tab_ids
    _check(lib().ssh_table_insert(
        tk.data_ptr() if N > 0 else None, ti.data_ptr() if N > 0 else None, N,
        _dev(new_keys, torch.uint64, "new_keys") if M > 0 else None, M, L,
        N if id_base is None else id_base,
        _dev(out[0], torch.uint64, "out_keys"), _dev(out[1], torch.uint32, "out_ids"),
        _dev(ws, torch.uint8, "ws"), ws.numel(), _stream()), "ssh_table_insert")
    return out[0][:, :N + M], out[1][:, :N + M]


def table_delete(tab_keys, tab_ids, dead: torch.Tensor, n_live: int, out=None, ws=None):
    """Tables without the series marked in dead (uint8 [id_bound]) -> [L, n_live] tables."""
    L, N = tab_keys.shape
    dev = tab_keys.device
    if out is None:
        out = (torch.empty((L, max(n_live, 1)), dtype=torch.uint64, device=dev),
               torch.empty((L, max(n_live, 1)), dtype=torch.uint32, device=dev))
    need = int(lib().ssh_table_delete_workspace_bytes(N, L))
    if ws is None or ws.numel() < need:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
    _check(lib().ssh_table_delete(
        _dev(tab_keys.contiguous(), torch.uint64, "tab_keys"),
        _dev(tab_ids.contiguous(), torch.uint32, "tab_ids"), N, L, _dev(dead, torch.uint8, "dead"),
        dead.numel(), n_live, _dev(out[0], torch.uint64, "out_keys"),
        _dev(out[1], torch.uint32, "out_ids"), _dev(ws, torch.uint8, "ws"), ws.numel(),
        _stream()), "ssh_table_delete")
    return out[0][:, :n_live], out[1][:, :n_live]


def probe_workspace_bytes(nq: int, L: int, C: int) -> int:
    return int(lib().ssh_probe_workspace_bytes(nq, L, C))


class CapacityError(SSHError):
    """A strict probe retrieved more than C series for some query."""


def probe(tab_keys, tab_ids, db_keys, db_hv, q_keys, q_hv, C: int, out=None, ws=None,
          strict: bool = False):
    """Returns (cand int64 [nq, C], ncand int32 [nq], r_size int64 [nq]).
    strict=True calls ssh_probe_strict: it synchronises and raises CapacityError
    when a query's retrieved set exceeds C (the outputs are still written)."""
    L, N = tab_keys.shape
    H = db_hv.shape[1]
    nq = q_keys.shape[0]
    dev = q_keys.device
    need = probe_workspace_bytes(nq, L, C)
    if ws is None or ws.numel() < need:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
    if out is None:
        cand = torch.empty((max(nq, 1), C), dtype=torch.int64, device=dev)
        ncand = torch.empty(max(nq, 1), dtype=torch.int32, device=dev)
        rs = torch.empty(max(nq, 1), dtype=torch.int64, device=dev)
    else:
        cand, ncand, rs = out
    tk = tab_keys.contiguous() if N > 0 else tab_keys
    fn = lib().ssh_probe_strict if strict else lib().ssh_probe
    st = fn(_dev(tk, torch.uint64, "tab_keys"), _dev(tab_ids.contiguous(), torch.uint32, "tab_ids"),
            N, L, _dev(db_keys, torch.uint64, "db_keys"), _dev(db_hv, torch.uint64, "db_hv"), H,
            _dev(q_keys, torch.uint64, "q_keys"), _dev(q_hv, torch.uint64, "q_hv"), nq, C,
            _dev(cand, torch.int64, "cand"), _dev(ncand, torch.int32, "ncand"),
            _dev(rs, torch.int64, "r_size"), _dev(ws, torch.uint8, "ws"), ws.numel(), _stream())
    if st == -4:  # SSH_ECAPACITY
        raise CapacityError(lib().ssh_last_error().decode())
    _check(st, "ssh_probe_strict" if strict else "ssh_probe")
    return cand[:nq], ncand[:nq], rs[:nq]


def rerank_workspace_bytes(nq: int, C: int) -> int:
    return int(lib().ssh_rerank_workspace_bytes(nq, C))


def rerank_lb_workspace_bytes(nq: int, C: int, q_values: int) -> int:
    """Workspace of the pruned re-rank; q_values = q_off[nq] (query values of the batch)."""
    return int(lib().ssh_rerank_lb_workspace_bytes(nq, C, q_values))


def dtw_rerank(q, q_off, db, db_off, cand, ncand, band_frac: float, k: int,
               ws: torch.Tensor | None = None, out=None, prune: bool = False):
    """Returns (ids int64 [nq, k], dist float32 [nq, k]).  Queries and series
    may have any lengths (CSR offsets); each pair's band radius is
    floor(band_frac * max(lq, lx)).  With prune, the same results through
    dtw_rerank_lb (lower bounds and early abandoning skip far candidates).
    A caller-supplied ws keeps every pair's distance in its first nq*C float32
    values (see pair_distances)."""
    nq, C = cand.shape
    N = db_off.numel() - 1
    dev = q.device
    if out is None:
        oid = torch.empty((max(nq, 1), k), dtype=torch.int64, device=dev)
        od = torch.empty((max(nq, 1), k), dtype=torch.float32, device=dev)
    else:
        oid, od = out
    if ws is None:
        nws = rerank_lb_workspace_bytes(nq, C, q.numel()) if prune else \
            rerank_workspace_bytes(nq, C)
        ws = torch.empty(max(nws, 1), dtype=torch.uint8, device=dev)
    fn = lib().dtw_rerank_lb if prune else lib().dtw_rerank
    _check(fn(_dev(q, torch.float32, "q"), _dev(q_off, torch.int64, "q_off"), nq,
              _dev(db, torch.float32, "db"), _dev(db_off, torch.int64, "db_off"), N,
              _dev(cand, torch.int64, "cand"), _dev(ncand, torch.int32, "ncand"), C,
              float(band_frac), k, _dev(oid, torch.int64, "out_id"),
              _dev(od, torch.float32, "out_dist"), _dev(ws, torch.uint8, "ws"), ws.numel(),
              _stream()), "dtw_rerank_lb" if prune else "dtw_rerank")
    return oid[:nq], od[:nq]


NOALLOC_SCRATCH_BYTES = 32 << 20


def dtw_rerank_noalloc(q, q_off, db, db_off, cand, ncand, band_frac: float, k: int, out):
    """dtw_rerank through the allocation-free entry point: the library takes
    its workspace from a static per-device array, and the caller passes the
    outputs (ids int64 [nq, k], dist float32 [nq, k]).  Calls that overlap on
    one device race for that array."""
    nq, C = cand.shape
    N = db_off.numel() - 1
    oid, od = out
    _check(lib().dtw_rerank_noalloc(
        _dev(q, torch.float32, "q"), _dev(q_off, torch.int64, "q_off"), nq,
        _dev(db, torch.float32, "db"), _dev(db_off, torch.int64, "db_off"), N,
        _dev(cand, torch.int64, "cand"), _dev(ncand, torch.int32, "ncand"), C, float(band_frac),
        k, _dev(oid, torch.int64, "out_id"), _dev(od, torch.float32, "out_dist"), _stream()),
        "dtw_rerank_noalloc")
    return oid[:nq], od[:nq]


def pair_distances(ws: torch.Tensor, nq: int, C: int) -> torch.Tensor:
    """View of the [nq, C] float32 pair distances a re-rank left in its workspace."""
    return ws[: nq * C * 4].view(torch.float32).view(nq, C)
