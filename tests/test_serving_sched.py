"""Continuous batching and memory admission of the server, on the CPU.

The scheduler runs against a fake executor on a simulated clock.  The fake
executor replays the oracle: a request's answer is the oracle's DTW top-k of
its query over a small database, and a batch takes a simulated service time.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1610_07328_amd import datagen
from paper_1610_07328_amd.serving import Request, RingArena, Scheduler


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def idle(self):
        self.t += 50e-6


class OracleExecutor:
    """Batches finish `base + per_request * size` seconds after launch; the
    answer of each request is the oracle's top-k over the whole database."""

    def __init__(self, clock, db, band=0.1, k=3, base=2e-3, per_request=0.5e-3,
                 bytes_per_value=64, bytes_per_batch=4096):
        self.clock = clock
        self.db, self.dboff = datagen.csr(db)
        self.N = db.shape[0]
        self.band, self.k = band, k
        self.base, self.per = base, per_request
        self.bpv, self.bpb = bytes_per_value, bytes_per_batch
        self.launches = []   # (launch time, [rids], offset)
        self.t0 = 0.0

    def start(self, t0):
        self.t0 = t0

    def bytes_for(self, reqs):
        if not reqs:
            return 0
        return self.bpb + sum(self.bpv * len(q.values) for q in reqs)

    def launch(self, reqs, offset, slot):
        now = self.clock() - self.t0
        self.launches.append((now, [q.rid for q in reqs], offset, slot))
        return (reqs, now + self.base + self.per * len(reqs))

    def done(self, h):
        return self.clock() - self.t0 >= h[1]

    def answer(self, q):
        qx, qoff = datagen.csr(q.values[None, :])
        cand = np.arange(self.N, dtype=np.int64)[None, :]
        ids, dist, _ = oracle.rerank(qx, qoff, self.db, self.dboff, cand,
                                     np.array([self.N], np.int32), self.band, self.k)
        return ids[0], dist[0]

    def finish(self, h):
        from paper_1610_07328_amd.serving import Result
        out = []
        for q in h[0]:
            ids, dist = self.answer(q)
            out.append(Result(q.rid, ids, dist, h[1]))
        return out


def _requests(n, rate, lens, seed):
    arr = datagen.poisson_arrivals(rate, n, seed=seed)
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        ln = int(rng.choice(lens))
        out.append(Request(i, float(arr[i]), 0, datagen.random_walks(1, ln, seed=1000 + i)[0]))
    return out


class CheckedArena(RingArena):
    """A ring arena that asserts its invariants on every call."""

    def alloc(self, nbytes):
        s = super().alloc(nbytes)
        assert self.used <= self.capacity
        if s is not None:
            off = self.offset(s)
            assert off + nbytes <= self.capacity  # a range never wraps
        return s


def test_ring_arena_order_wrap_and_early_free():
    a = RingArena(1000 * 256)
    x = a.alloc(300 * 256)
    y = a.alloc(500 * 256)
    assert a.alloc(300 * 256) is None          # 800 used, 300 more do not fit
    assert a.fits(200 * 256)
    z = a.alloc(200 * 256)
    assert a.used == 1000 * 256 and a.offset(z) == 800 * 256
    a.free(y)                                   # freed early: the tail waits for x
    assert a.used == 1000 * 256
    a.free(x)                                   # x and y both released
    assert a.used == 200 * 256
    w = a.alloc(600 * 256)                      # does not fit before the end: wraps to 0
    assert w is not None and a.offset(w) == 0
    assert a.alloc(300 * 256) is None
    a.free(z)
    a.free(w)
    assert a.used == 0 and a.peak == 1000 * 256


def test_scheduler_admits_by_memory_in_arrival_order():
    """Thirty requests arrive almost at once; the budget holds about two of
    them.  Every request is served with the oracle's answer, no batch is
    launched before its requests arrived, admission follows arrival order, and
    the budget is never exceeded."""
    clock = FakeClock()
    db = datagen.random_walks(40, 64, seed=3)
    ex = OracleExecutor(clock, db)
    reqs = _requests(30, 20000.0, [32, 64], seed=4)
    one = ex.bytes_for([reqs[0]])
    arena = CheckedArena(int(2.5 * ex.bytes_for([max(reqs, key=lambda q: len(q.values))])))
    sched = Scheduler(ex, arena, max_batch=8, max_inflight=4, clock=clock, idle=clock.idle)
    results, stats = sched.run(reqs)
    assert stats.refused == 0 and len(results) == 30
    assert arena.peak <= arena.capacity and one <= arena.capacity
    by_rid = {q.rid: q for q in reqs}
    launched = []
    for t, rids, off, slot in ex.launches:
        assert all(by_rid[r].arrival <= t for r in rids)
        launched.extend(rids)
    order = sorted(reqs, key=lambda q: (q.arrival, q.rid))
    assert launched == [q.rid for q in order]
    for q, r in zip(reqs, results):
        ids, dist = ex.answer(q)
        assert np.array_equal(r.ids, ids) and np.array_equal(r.dist, dist)
        assert r.completion >= q.arrival


def test_scheduler_refuses_a_request_larger_than_the_budget():
    clock = FakeClock()
    db = datagen.random_walks(10, 32, seed=5)
    ex = OracleExecutor(clock, db)
    reqs = _requests(6, 1000.0, [32], seed=6)
    big = Request(99, reqs[2].arrival, 0, datagen.random_walks(1, 4096, seed=7)[0])
    arena = RingArena(ex.bytes_for([reqs[0]]) * 3)
    results, stats = Scheduler(ex, arena, clock=clock, idle=clock.idle).run(reqs + [big])
    assert stats.refused == 1
    res = {r.rid: r for r in results}
    assert "budget" in res[99].refused and res[99].ids is None
    assert all(not res[q.rid].refused and res[q.rid].ids is not None for q in reqs)


def test_scheduler_overlaps_batches_and_admits_while_others_run():
    """Service time well above the arrival gap: several batches are in flight
    at once, later arrivals are admitted while earlier batches still run, and
    batching grows the batches instead of queueing one request at a time."""
    clock = FakeClock()
    db = datagen.random_walks(20, 32, seed=8)
    ex = OracleExecutor(clock, db, base=5e-3, per_request=0.2e-3)
    reqs = _requests(80, 4000.0, [32], seed=9)
    arena = RingArena(1 << 30)
    results, stats = Scheduler(ex, arena, max_batch=16, max_inflight=3, clock=clock,
                               idle=clock.idle).run(reqs)
    assert stats.inflight_max == 3
    assert max(stats.batch_sizes) > 1 and stats.batches < len(reqs)
    assert max(stats.batch_sizes) <= 16
    # some batch started before an earlier batch finished
    ends = {}
    for r in results:
        ends[r.batch] = r.completion
    starts = [t for t, *_ in ex.launches]
    assert any(starts[b + 1] < ends[b] for b in range(len(starts) - 1))
    assert all(math.isfinite(r.completion) for r in results)


def test_scheduler_plain_form_is_one_request_at_a_time():
    """max_batch = 1 and max_inflight = 1 is the plain per-query form: one
    request per batch, each launched only after the previous one finished."""
    clock = FakeClock()
    db = datagen.random_walks(20, 32, seed=10)
    ex = OracleExecutor(clock, db)
    reqs = _requests(12, 2000.0, [32], seed=11)
    results, stats = Scheduler(ex, RingArena(1 << 30), max_batch=1, max_inflight=1, clock=clock,
                               idle=clock.idle).run(reqs)
    assert stats.batch_sizes == [1] * 12 and stats.inflight_max == 1
    comp = sorted(r.completion for r in results)
    starts = [t for t, *_ in ex.launches]
    assert all(starts[i + 1] >= comp[i] for i in range(len(starts) - 1))
