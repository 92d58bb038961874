"""The batched build of an uneven batch on the GPU.

* Every autotuner choice (sketch work item of 8, 12, 16 or 20 rows; series as
  given or longest first) gives the same bits, hash values, keys and buckets.
* The HIP graph of the build, replayed several times with eager work and
  synchronisations between the replays, gives the eager results every time.
* The plain per-series form (one launch sequence per series) gives the same
  hash values and keys as the batched launches.
* The autotuner times the choices once, then answers from its cache.
Inputs are the seeded generators; the reference is the library's own default
path, itself checked against the oracle in test_gpu_parity and
test_gpu_fullsize.
"""
import numpy as np
import pytest
import torch

from paper_1610_07328_amd import datagen
from paper_1610_07328_amd.batching import ORDERS, TuneCache, UnevenBuild, autotune
from paper_1610_07328_amd.pipeline import HashBatch, Params
from tests._gpu_helpers import to_np, unpack_bits

pytestmark = pytest.mark.gpu

P = Params(W=80, delta=3, n=15, K=10, L=10)


@pytest.fixture(scope="module")
def batch():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1610_07328_amd import ssh
    ssh.lib()
    x, off = datagen.ragged_series(3000, 256, 8192, seed=31)
    r = datagen.filter_r(P.W, seed=31)
    tables = ssh.CwsTables(*datagen.cws_draws(P.n, P.H, seed=31), P.n)
    ref = UnevenBuild(x, off, P, tables, r)
    ref.run()
    torch.cuda.synchronize()
    ssh.check_device_errors()
    return dict(x=x, off=off, r=r, tables=tables, ref=ref, ssh=ssh)


def _buckets(build):
    """Every table's buckets as sets of the caller's ids."""
    tk, ti = to_np(build.index.tab_keys), to_np(build.index.tab_ids).astype(np.int64)
    out = []
    for l in range(tk.shape[0]):
        d = {}
        for k, i in zip(tk[l].tolist(), build.perm[ti[l]].tolist()):
            d.setdefault(k, set()).add(i)
        out.append(d)
    return out


def _bits_of(build, s_pos):
    db = build.db
    return unpack_bits(to_np(db.bits), db.plan.bit_word_off, to_np(db.nbits), s_pos)


@pytest.mark.parametrize("order", ORDERS)
def test_every_tuner_choice_gives_the_same_results(batch, order):
    ssh, ref = batch["ssh"], batch["ref"]
    hv0, k0 = to_np(ref.hv()), to_np(ref.keys())
    b0 = _buckets(ref)
    inv = None
    for t in ssh.SKETCH_TILES:
        print(f"\n[case] order={order} tile_rows={t}", flush=True)
        b = UnevenBuild(batch["x"], batch["off"], P, batch["tables"], batch["r"], order=order,
                        tile_rows=t)
        b.run()
        torch.cuda.synchronize()
        ssh.check_device_errors()
        assert np.array_equal(to_np(b.hv()), hv0)
        assert np.array_equal(to_np(b.keys()), k0)
        if inv is None:
            inv = np.argsort(b.perm)
            for s in [0, 1, 2, 1500, 2999]:
                assert np.array_equal(_bits_of(b, inv[s]), _bits_of(ref, s))
            assert _buckets(b) == b0


def test_graph_replays_equal_eager(batch):
    ssh = batch["ssh"]
    b = UnevenBuild(batch["x"], batch["off"], P, batch["tables"], batch["r"],
                    order="longest_first", tile_rows=12)
    b.run()
    torch.cuda.synchronize()
    eager = [to_np(b.db.hv), to_np(b.db.keys), to_np(b.index.tab_keys), to_np(b.index.tab_ids)]
    b.capture()
    for rep in range(3):
        print(f"\n[case] graph replay {rep}", flush=True)
        # eager work between replays that overwrites what the graph writes
        b.db.hv.fill_(0)
        b.index.tab_keys.fill_(0)
        torch.cuda.synchronize()
        b.replay()
        torch.cuda.synchronize()
        ssh.check_device_errors()
        got = [to_np(b.db.hv), to_np(b.db.keys), to_np(b.index.tab_keys), to_np(b.index.tab_ids)]
        for g, e in zip(got, eager):
            assert np.array_equal(g, e)


def test_per_series_launches_equal_the_batch(batch):
    ssh, ref = batch["ssh"], batch["ref"]
    x, off = batch["x"], batch["off"]
    hv0, k0 = to_np(ref.hv()), to_np(ref.keys())
    rng = np.random.default_rng(32)
    for s in rng.choice(len(off) - 1, 24, replace=False):
        hb = HashBatch(torch.as_tensor(x[off[s]:off[s + 1]]).cuda(),
                       np.array([0, off[s + 1] - off[s]], np.int64), P)
        hb.run(batch["r"], batch["tables"])
        torch.cuda.synchronize()
        assert np.array_equal(to_np(hb.hv[0]), hv0[s]), s
        assert np.array_equal(to_np(hb.keys[0]), k0[s]), s
    ssh.check_device_errors()


def test_autotuner_times_once_then_reads_its_cache(batch, tmp_path):
    cache = TuneCache(str(tmp_path / "tune.json"))
    choice, hit = autotune(batch["x"], batch["off"], P, batch["tables"], batch["r"], cache,
                           reps=1)
    print(f"\n[result] tuner choice {choice['order']} / {choice['tile_rows']} rows: "
          f"{choice['build_ms']}", flush=True)
    assert not hit and choice["order"] in ORDERS and choice["tile_rows"] in (8, 12, 16, 20)
    assert len(choice["build_ms"]) == 8
    again, hit2 = autotune(batch["x"], batch["off"], P, batch["tables"], batch["r"],
                           TuneCache(cache.path))
    assert hit2 and again["order"] == choice["order"] and again["tile_rows"] == choice["tile_rows"]
