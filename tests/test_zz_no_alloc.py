"""dtw_rerank_noalloc (the allocation-free re-rank) against dtw_rerank.

Called through the C ABI on two calls in a row, the second with a smaller
batch, so that the second call runs over the first call's leftover scratch.
Ids and distances must be identical, bit for bit: both entry points run the
same kernels, only the workspace differs.
"""
import ctypes

import numpy as np
import pytest
import torch

from paper_1610_07328_amd import datagen
from tests._gpu_helpers import ragged, to_dev, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ssh():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1610_07328_amd import ssh as mod
    mod.lib()
    return mod


def _batch(nq, N, C, seed):
    rng = np.random.default_rng(seed)
    qlens = rng.choice([128, 512, 1024, 300], size=nq)
    dblens = rng.choice([128, 512, 1024, 310, 1000], size=N)
    qs = [datagen.random_walks(1, int(m), seed=seed * 1000 + i)[0] for i, m in enumerate(qlens)]
    xs = [datagen.random_walks(1, int(m), seed=seed * 2000 + i)[0] for i, m in enumerate(dblens)]
    q, qoff = ragged(qs)
    db, dboff = ragged(xs)
    cand = rng.integers(0, N, size=(nq, C)).astype(np.int64)
    ncand = rng.integers(0, C + 1, size=nq).astype(np.int32)
    ncand[0] = C
    return q, qoff, db, dboff, cand, ncand


def test_noalloc_rerank_matches_workspace_rerank_twice(ssh):
    L = ssh.lib()
    # 12,800 pairs (multi-workgroup planning), then 150 pairs (one workgroup)
    for nq, N, C, seed in [(64, 400, 200, 1), (5, 40, 30, 2)]:
        print(f"\n[case] noalloc re-rank nq={nq} C={C} seed={seed}", flush=True)
        q, qoff, db, dboff, cand, ncand = _batch(nq, N, C, seed)
        dq, dqo, ddb, ddo, dc, dn = (to_dev(a) for a in (q, qoff, db, dboff, cand, ncand))
        band, k = 0.05, 10
        ids, dist = ssh.dtw_rerank(dq, dqo, ddb, ddo, dc, dn, band, k)
        oid = torch.full((nq, k), 7, dtype=torch.int64, device="cuda")
        od = torch.full((nq, k), float("nan"), dtype=torch.float32, device="cuda")
        st = L.dtw_rerank_noalloc(dq.data_ptr(), dqo.data_ptr(), nq, ddb.data_ptr(), ddo.data_ptr(),
                                  N, dc.data_ptr(), dn.data_ptr(), C, ctypes.c_float(band), k,
                                  oid.data_ptr(), od.data_ptr(),
                                  torch.cuda.current_stream().cuda_stream)
        assert st == 0, L.ssh_last_error()
        torch.cuda.synchronize()
        ssh.check_device_errors()
        assert np.array_equal(to_np(oid), to_np(ids))
        assert np.array_equal(to_np(od).view(np.uint32), to_np(dist).view(np.uint32))
        assert np.all(to_np(oid)[ncand == 0] == -1)
