"""Dynamic updates and persistence of a resident index (GPU).

* Insert-then-probe equals rebuild-then-probe, bit for bit: the merged tables
  equal a fresh build over every series, and so do the probes' answers.
* Delete-then-probe equals a rebuild over the surviving series, with the
  rebuild's ids mapped to the surviving ids; inserting after deleting keeps
  that equality.
* Save then load gives the same arrays and the same answers.
The reference is the library's own build and probe, themselves checked
against the oracle in test_gpu_parity.
"""
import numpy as np
import pytest
import torch

from paper_1610_07328_amd import datagen
from paper_1610_07328_amd.pipeline import HashBatch, Params
from tests._gpu_helpers import to_np

pytestmark = pytest.mark.gpu

P = Params(W=64, delta=4, n=12, K=2, L=10, C=40, k=5, band_frac=0.05)


@pytest.fixture(scope="module")
def env():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1610_07328_amd import ssh
    ssh.lib()
    X = datagen.random_walks(5000, 256, seed=41)
    Q, src = datagen.perturbed_queries(X, 24, 0.05, seed=41)
    draws = datagen.cws_draws(P.n, P.H, seed=41)
    r = datagen.filter_r(P.W, seed=41)
    return dict(ssh=ssh, X=X, Q=Q, draws=draws, r=r)


def _rebuild(env, rows):
    """Hash values, keys, tables and probe answers of a fresh build over X[rows]."""
    ssh = env["ssh"]
    x, off = datagen.csr(env["X"][rows])
    tables = ssh.CwsTables(*env["draws"], P.n)
    hb = HashBatch(torch.as_tensor(x).cuda(), off, P)
    hv, keys = hb.run(env["r"], tables)
    tk, ti = ssh.table_build(keys)
    q, qoff = datagen.csr(env["Q"])
    qb = HashBatch(torch.as_tensor(q).cuda(), qoff, P)
    qhv, qkeys = qb.run(env["r"], tables)
    cand, ncand, rs = ssh.probe(tk, ti, keys, hv, qkeys, qhv, P.C)
    torch.cuda.synchronize()
    return dict(hv=to_np(hv), keys=to_np(keys), tk=to_np(tk), ti=to_np(ti), cand=to_np(cand),
                ncand=to_np(ncand), rs=to_np(rs))


def _probe(env, ix):
    q, qoff = datagen.csr(env["Q"])
    _, qhv, qkeys = ix.hash_queries(q, qoff)
    cand, ncand, rs = ix.probe(qkeys, qhv, P.C)
    torch.cuda.synchronize()
    return to_np(cand), to_np(ncand), to_np(rs)


def _insert_rows(ix, X, rows):
    x, off = datagen.csr(X[rows])
    return ix.insert(x, off)


def test_insert_then_probe_equals_rebuild(env):
    from paper_1610_07328_amd.store import DynamicIndex
    print("\n[case] 3,000 series then two inserts of 1,000", flush=True)
    ix = DynamicIndex(P, env["draws"], env["r"])
    X = env["X"]
    assert np.array_equal(_insert_rows(ix, X, np.arange(0, 3000)), np.arange(3000))
    _insert_rows(ix, X, np.arange(3000, 4000))
    _insert_rows(ix, X, np.arange(4000, 5000))
    env["ssh"].check_device_errors()
    ref = _rebuild(env, np.arange(5000))
    assert np.array_equal(to_np(ix.hv), ref["hv"]) and np.array_equal(to_np(ix.keys), ref["keys"])
    assert np.array_equal(to_np(ix.tab_keys), ref["tk"])
    assert np.array_equal(to_np(ix.tab_ids), ref["ti"])
    cand, ncand, rs = _probe(env, ix)
    assert np.array_equal(cand, ref["cand"]) and np.array_equal(ncand, ref["ncand"])
    assert np.array_equal(rs, ref["rs"])
    assert ncand.sum() > 0


def test_delete_then_probe_equals_rebuild_over_survivors(env, tmp_path):
    from paper_1610_07328_amd.store import DynamicIndex
    print("\n[case] delete 900 of 4,000, insert 1,000 more, save and load", flush=True)
    ssh = env["ssh"]
    X = env["X"]
    ix = DynamicIndex(P, env["draws"], env["r"])
    _insert_rows(ix, X, np.arange(4000))
    rng = np.random.default_rng(42)
    gone = rng.choice(4000, 900, replace=False)
    assert ix.delete(gone) == 900 and ix.delete(gone[:10]) == 0
    _insert_rows(ix, X, np.arange(4000, 5000))
    ssh.check_device_errors()
    live = np.setdiff1d(np.arange(5000), gone)
    assert ix.n_live == len(live)
    ref = _rebuild(env, live)
    # the rebuild numbers the survivors 0..; map its ids to theirs
    assert np.array_equal(to_np(ix.tab_keys), ref["tk"])
    assert np.array_equal(to_np(ix.tab_ids).astype(np.int64), live[ref["ti"].astype(np.int64)])
    cand, ncand, rs = _probe(env, ix)
    assert np.array_equal(ncand, ref["ncand"]) and np.array_equal(rs, ref["rs"])
    for i in range(len(ncand)):
        assert np.array_equal(cand[i, :ncand[i]], live[ref["cand"][i, :ncand[i]]]), i
    # the whole search, then the index saved and loaded
    q, qoff = datagen.csr(env["Q"])
    ids0, d0, *_ = ix.search(q, qoff)
    ix.save(str(tmp_path / "ix"))
    jx = DynamicIndex.load(str(tmp_path / "ix"))
    for a, b in [(ix.hv, jx.hv), (ix.keys, jx.keys), (ix.tab_keys, jx.tab_keys),
                 (ix.tab_ids, jx.tab_ids), (ix.x, jx.x), (ix.dead, jx.dead)]:
        assert np.array_equal(to_np(a), to_np(b))
    ids1, d1, *_ = jx.search(q, qoff)
    torch.cuda.synchronize()
    assert np.array_equal(to_np(ids0), to_np(ids1))
    assert np.array_equal(to_np(d0).view(np.uint32), to_np(d1).view(np.uint32))
    assert not np.isin(to_np(ids0), gone).any()
