"""Serving the SSH index: continuous batching of queries of mixed lengths.

The index and its hash tables stay resident in HBM.  Queries arrive over
time (Algorithm 2, the query process, one query at a time in the paper); the
server admits them into batches while earlier batches are still on the GPU,
as device memory and batch slots free up, so the work of several batches
overlaps on the device.

Parts:
* RingArena -- device-memory admission: a fixed budget carved in arrival
  order; a batch is admitted only when its exact byte need fits.
* Scheduler -- the continuous-batching loop over an executor; it never
  touches the GPU itself, so it runs on the CPU against a fake executor in
  the tests.
* MixedIndex -- one resident index over several length classes (stride-1
  windows of one stream, one class per query length).  Every class is
  hashed with the same sketch filter and weighted-MinHash draws, but its band
  keys are folded with a seed of its own, so a query's buckets only ever
  hold windows of its own length: one table set, one probe call and one
  ragged re-rank call serve a batch that mixes lengths.
* GpuExecutor -- runs a batch through the C ABI on one of its streams:
  hashing (sketch, shingle, CWS and band keys per class), probe and DTW
  re-rank, with every buffer carved from the arena.

Nothing here computes: every step of the method runs in the library's kernels.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

import numpy as np

ALIGN = 256


def _al(n: int) -> int:
    return (int(n) + ALIGN - 1) // ALIGN * ALIGN


# --------------------------------------------------------------------------
# requests and results
# --------------------------------------------------------------------------
@dataclass
class Request:
    rid: int
    arrival: float          # seconds after the stream starts
    cls: int                # length class index
    values: np.ndarray      # float32 query values (z-normalised)


@dataclass
class Result:
    rid: int
    ids: np.ndarray = None          # int64 [k], -1 padding (ids local to the class)
    dist: np.ndarray = None         # float32 [k], +inf padding
    completion: float = float("nan")  # seconds after the stream starts
    batch: int = -1                 # index of the batch that served it
    batch_size: int = 0
    refused: str = ""               # reason when the request could never be admitted


# --------------------------------------------------------------------------
# admission by memory
# --------------------------------------------------------------------------
class RingArena:
    """Byte ranges of a fixed budget handed out in ring order.

    Batches mostly finish in the order they started, so a ring suffices: new
    ranges are cut at the head, and the tail advances over ranges once they
    are freed (a range freed early waits until the ranges before it are freed
    too).  alloc() returns None when the range does not fit right now."""

    def __init__(self, capacity: int):
        self.capacity = int(capacity) // ALIGN * ALIGN
        self.head = 0          # next free byte (monotone, modulo capacity)
        self.tail = 0          # oldest byte still in use (monotone)
        self.live = collections.OrderedDict()  # start -> [end, freed]
        self.peak = 0

    @property
    def used(self) -> int:
        return self.head - self.tail

    def _place(self, n: int):
        """(start, padding before it) of an n-byte range at the head, or None."""
        h = self.head % self.capacity
        pad = 0 if h + n <= self.capacity else self.capacity - h  # ranges do not wrap
        if self.used + pad + n > self.capacity:
            return None
        return self.head + pad, pad

    def fits(self, nbytes: int) -> bool:
        n = _al(nbytes)
        return n <= self.capacity and self._place(n) is not None

    def alloc(self, nbytes: int):
        n = _al(nbytes)
        if n > self.capacity:
            return None
        spot = self._place(n)
        if spot is None:
            return None
        start, pad = spot
        if pad:
            self.live[self.head] = [self.head + pad, True]  # the skipped end of the ring
        self.live[start] = [start + n, False]
        self.head = start + n
        self.peak = max(self.peak, self.used)
        return start

    def offset(self, start: int) -> int:
        """Byte offset of a range inside the budget."""
        return start % self.capacity

    def free(self, start: int):
        self.live[start][1] = True
        while self.live:
            s0, (e0, freed) = next(iter(self.live.items()))
            if not freed:
                break
            del self.live[s0]
            self.tail = e0
        if not self.live:
            self.tail = self.head


# --------------------------------------------------------------------------
# the continuous-batching loop
# --------------------------------------------------------------------------
@dataclass
class _Batch:
    index: int
    requests: list
    mem: int
    handle: object
    slot: int


@dataclass
class ServeStats:
    batches: int = 0
    batch_sizes: list = field(default_factory=list)
    inflight_max: int = 0
    arena_peak: int = 0
    refused: int = 0
    wall: float = 0.0


class Scheduler:
    """Admits arrived requests into batches as slots and memory free up.

    executor must provide:
      bytes_for(requests) -> int            device bytes a batch of them needs
      launch(requests, offset, slot) -> h   start the batch asynchronously
      done(h) -> bool                       non-blocking completion test
      finish(h) -> list[Result]             results (ids, dist, completion)
    A request whose batch of one does not fit the whole arena is refused.
    Requests are admitted in arrival order; a batch holds at most max_batch
    requests and at most max_inflight batches run at once."""

    def __init__(self, executor, arena: RingArena, max_batch: int = 64, max_inflight: int = 4,
                 clock=time.perf_counter, idle=None):
        self.ex = executor
        self.arena = arena
        self.max_batch = max_batch
        self.max_inflight = max_inflight
        self.clock = clock
        self.idle = idle or (lambda: None)

    def run(self, requests):
        reqs = sorted(requests, key=lambda q: (q.arrival, q.rid))
        n = len(reqs)
        results = {}
        stats = ServeStats()
        pending = collections.deque()
        inflight = []
        free_slots = list(range(self.max_inflight))
        i = 0
        t0 = self.clock()
        if hasattr(self.ex, "start"):
            self.ex.start(t0)
        while len(results) < n:
            now = self.clock() - t0
            while i < n and reqs[i].arrival <= now:
                pending.append(reqs[i])
                i += 1
            progressed = False
            # retire finished batches, in any order
            for b in list(inflight):
                if self.ex.done(b.handle):
                    for res in self.ex.finish(b.handle):
                        res.batch, res.batch_size = b.index, len(b.requests)
                        results[res.rid] = res
                    self.arena.free(b.mem)
                    inflight.remove(b)
                    free_slots.append(b.slot)
                    progressed = True
            # admit one new batch
            if pending and free_slots:
                batch = []
                while pending and len(batch) < self.max_batch:
                    head = pending[0]
                    if self.ex.bytes_for([head]) > self.arena.capacity:
                        pending.popleft()
                        results[head.rid] = Result(head.rid, refused="needs more device memory "
                                                   "than the whole admission budget")
                        stats.refused += 1
                        progressed = True
                        continue
                    if not self.arena.fits(self.ex.bytes_for(batch + [head])):
                        break
                    batch.append(pending.popleft())
                if batch:
                    need = self.ex.bytes_for(batch)
                    mem = self.arena.alloc(need)
                    assert mem is not None
                    slot = free_slots.pop()
                    h = self.ex.launch(batch, self.arena.offset(mem), slot)
                    inflight.append(_Batch(stats.batches, batch, mem, h, slot))
                    stats.batches += 1
                    stats.batch_sizes.append(len(batch))
                    stats.inflight_max = max(stats.inflight_max, len(inflight))
                    progressed = True
            if not progressed:
                self.idle()
        stats.arena_peak = self.arena.peak
        stats.wall = self.clock() - t0
        return [results[q.rid] for q in sorted(requests, key=lambda q: q.rid)], stats


# --------------------------------------------------------------------------
# GPU side
# --------------------------------------------------------------------------
def class_seed(key_seed: int, c: int) -> int:
    """Band-key seed of length class c."""
    return (key_seed + (c + 1) * 0xD1B54A32D192ED03) & ((1 << 64) - 1)


class MixedIndex:
    """One resident index over length classes of series in one device array.

    x: float32 device array holding every class's series back to back;
    classes: list of (length, count) in that order.  Class c's series get
    global ids base[c] .. base[c] + count - 1."""

    def __init__(self, x, classes, p, tables, r):
        import torch

        from . import ssh
        from .pipeline import HashBatch

        self.p, self.tables, self.r = p, tables, r
        self.classes = list(classes)
        dev = x.device
        lens = np.concatenate([np.full(cnt, ln, np.int64) for ln, cnt in classes])
        off = np.zeros(len(lens) + 1, np.int64)
        np.cumsum(lens, out=off[1:])
        self.N = len(lens)
        self.base = np.concatenate([[0], np.cumsum([cnt for _, cnt in classes])]).astype(np.int64)
        self.x = x
        self.off = torch.as_tensor(off).to(dev)
        self.hv = torch.empty((self.N, p.H), dtype=torch.uint64, device=dev)
        self.keys = torch.empty((self.N, p.L), dtype=torch.uint64, device=dev)
        for c, (ln, cnt) in enumerate(classes):
            b = int(self.base[c])
            xs = x[off[b]:off[b + cnt]]
            hb = HashBatch(xs, np.arange(cnt + 1, dtype=np.int64) * ln, p,
                           out=(self.hv[b:b + cnt], self.keys[b:b + cnt]))
            hb.sketch(r)
            hb.shingle()
            hb.cws_band_keys(tables, seed=class_seed(p.key_seed, c))
            torch.cuda.synchronize()
            del hb
        self.tab_keys, self.tab_ids = ssh.table_build(self.keys)
        torch.cuda.synchronize()


class GpuExecutor:
    """Runs admitted batches through the C ABI, one stream per batch slot.

    Every device buffer of a batch is carved from the arena's device array at
    the offset the scheduler admitted it at; each slot has pinned host staging
    for the queries and the results."""

    def __init__(self, index: MixedIndex, arena_bytes: int, slots: int, max_batch: int,
                 max_len: int):
        import torch

        self.ix = index
        self.p = index.p
        self.dev = index.x.device
        self.mem = torch.empty(arena_bytes, dtype=torch.uint8, device=self.dev)
        self.streams = [torch.cuda.Stream(device=self.dev) for _ in range(slots)]
        self.max_batch = max_batch
        stage = 4 * max_batch * max_len + 3 * 8 * (max_batch + 1) + 3 * ALIGN
        self.stage_in = [torch.empty(stage, dtype=torch.uint8, pin_memory=True) for _ in range(slots)]
        k = self.p.k
        self.stage_out = [torch.empty(_al(max_batch * k * 8) + max_batch * k * 4, dtype=torch.uint8,
                                      pin_memory=True) for _ in range(slots)]
        self.t0_event = None
        self.t0_shift = 0.0

    # ---- sizes -----------------------------------------------------------
    def _layout(self, requests):
        from . import ssh
        p = self.p
        n = len(requests)
        order = sorted(range(n), key=lambda j: (requests[j].cls, j))
        lens = np.array([len(requests[j].values) for j in order], np.int64)
        qoff = np.zeros(n + 1, np.int64)
        np.cumsum(lens, out=qoff[1:])
        plan = ssh.plan(qoff, p.W, p.delta, p.n)
        words = max(int(plan.bit_word_off[-1]), 1)
        cap = max(int(plan.hist_off[-1]), 1)
        sizes = [
            ("x", 4 * int(qoff[-1])), ("qoff", 8 * (n + 1)), ("bwo", 8 * (n + 1)),
            ("hoff", 8 * (n + 1)), ("bits", 8 * words), ("nbits", 4 * n), ("rep", 8),
            ("codes", 4 * cap), ("counts", 4 * cap), ("nd", 4 * n), ("hv", 8 * n * p.H),
            ("keys", 8 * n * p.L), ("cand", 8 * n * p.C), ("ncand", 4 * n), ("rsize", 8 * n),
            ("pws", ssh.probe_workspace_bytes(n, p.L, p.C)),
            ("rws", ssh.rerank_workspace_bytes(n, p.C)), ("ids", 8 * n * p.k),
            ("dist", 4 * n * p.k),
        ]
        offs, pos = {}, 0
        for name, b in sizes:
            offs[name] = (pos, int(b))
            pos += _al(max(int(b), 1))
        return order, qoff, plan, offs, pos

    def bytes_for(self, requests) -> int:
        return self._layout(requests)[4] if requests else 0

    # ---- running ---------------------------------------------------------
    def start(self, t0: float):
        """Mark time zero on the device: completions are measured from this event
        and shifted by the host time (after t0) at which it was seen to pass."""
        import torch
        self.t0_event = torch.cuda.Event(enable_timing=True)
        self.t0_event.record()
        self.t0_event.synchronize()
        self.t0_shift = time.perf_counter() - t0

    def launch(self, requests, offset: int, slot: int):
        import torch

        from . import ssh
        p, ix = self.p, self.ix
        order, qoff, plan, offs, total = self._layout(requests)
        n = len(requests)

        def view(name, dtype, shape=None):
            a, b = offs[name]
            t = self.mem[offset + a: offset + a + max(b, 1)].view(dtype)
            return t if shape is None else t[: int(np.prod(shape))].view(*shape)

        # stage the queries and the three offset arrays, then one copy
        st = self.stage_in[slot]
        nx = int(qoff[-1])
        hx = st[: 4 * nx].view(torch.float32).numpy()
        for j, src in enumerate(order):
            hx[qoff[j]:qoff[j + 1]] = requests[src].values
        o1 = _al(4 * nx)
        ho = st[o1: o1 + 3 * 8 * (n + 1)].view(torch.int64).numpy()
        ho[: n + 1] = qoff
        ho[n + 1: 2 * (n + 1)] = plan.bit_word_off
        ho[2 * (n + 1):] = plan.hist_off
        s = self.streams[slot]
        with torch.cuda.stream(s):
            view("x", torch.float32)[:nx].copy_(st[: 4 * nx].view(torch.float32), non_blocking=True)
            dq = view("qoff", torch.int64)[: n + 1]
            dq.copy_(st[o1: o1 + 8 * (n + 1)].view(torch.int64), non_blocking=True)
            dbwo = view("bwo", torch.int64)[: n + 1]
            dbwo.copy_(st[o1 + 8 * (n + 1): o1 + 16 * (n + 1)].view(torch.int64), non_blocking=True)
            dho = view("hoff", torch.int64)[: n + 1]
            dho.copy_(st[o1 + 16 * (n + 1): o1 + 24 * (n + 1)].view(torch.int64), non_blocking=True)
            x = view("x", torch.float32)[:nx]
            bits = view("bits", torch.uint64)
            nbits = view("nbits", torch.int32)
            rep = view("rep", torch.uint64)[:1]
            ssh.sketch(x, dq, ix.r, p.W, p.delta, dbwo, out=(bits, nbits, rep))
            codes, counts, nd = view("codes", torch.uint32), view("counts", torch.uint32), \
                view("nd", torch.int32)
            ssh.shingle(bits, dbwo, nbits[:n], p.n, dho, out=(codes, counts, nd))
            hv = view("hv", torch.uint64, (n, p.H))
            keys = view("keys", torch.uint64, (n, p.L))
            classes = [requests[j].cls for j in order]
            a = 0
            while a < n:
                c = classes[a]
                b = a
                while b < n and classes[b] == c:
                    b += 1
                ssh.cws_band_keys(codes, counts, dho[a:b + 1], nd[a:b], ix.tables, p.K, p.L,
                                  class_seed(p.key_seed, c), out=(hv[a:b], keys[a:b]))
                a = b
            cand = view("cand", torch.int64, (n, p.C))
            ncand = view("ncand", torch.int32)[:n]
            rsize = view("rsize", torch.int64)[:n]
            ssh.probe(ix.tab_keys, ix.tab_ids, ix.keys, ix.hv, keys, hv, p.C,
                      out=(cand, ncand, rsize), ws=view("pws", torch.uint8))
            ids = view("ids", torch.int64, (n, p.k))
            dist = view("dist", torch.float32, (n, p.k))
            ssh.dtw_rerank(x, dq, ix.x, ix.off, cand, ncand, p.band_frac, p.k,
                           ws=view("rws", torch.uint8), out=(ids, dist))
            so = self.stage_out[slot]
            oi = so[: 8 * n * p.k].view(torch.int64)
            od_at = _al(self.max_batch * p.k * 8)
            od = so[od_at: od_at + 4 * n * p.k].view(torch.float32)
            oi.copy_(ids.reshape(-1), non_blocking=True)
            od.copy_(dist.reshape(-1), non_blocking=True)
            ev = torch.cuda.Event(enable_timing=True)
            ev.record(s)
        return (requests, order, slot, ev)

    def done(self, h) -> bool:
        return h[3].query()

    def finish(self, h):
        import torch
        requests, order, slot, ev = h
        p, ix = self.p, self.ix
        n = len(requests)
        completion = self.t0_shift + self.t0_event.elapsed_time(ev) / 1e3
        so = self.stage_out[slot]
        ids = so[: 8 * n * p.k].view(torch.int64).numpy().reshape(n, p.k).copy()
        od_at = _al(self.max_batch * p.k * 8)
        dist = so[od_at: od_at + 4 * n * p.k].view(torch.float32).numpy().reshape(n, p.k).copy()
        out = []
        for j, src in enumerate(order):
            q = requests[src]
            local = np.where(ids[j] >= 0, ids[j] - ix.base[q.cls], -1)
            out.append(Result(q.rid, local, dist[j], completion))
        return out


def latency_summary(requests, results):
    """p50/p99 latency (ms) of the served requests, by length and overall."""
    lat = {}
    for q, r in zip(sorted(requests, key=lambda q: q.rid), results):
        if r.refused:
            continue
        lat.setdefault(len(q.values), []).append((r.completion - q.arrival) * 1e3)
    allv = np.concatenate([np.array(v) for v in lat.values()]) if lat else np.array([np.nan])
    out = {"p50": float(np.percentile(allv, 50)), "p99": float(np.percentile(allv, 99)),
           "mean": float(allv.mean()), "served": int(allv.size)}
    out["by_length"] = {int(k): {"p50": float(np.percentile(v, 50)),
                                 "p99": float(np.percentile(v, 99)), "n": len(v)}
                        for k, v in sorted(lat.items())}
    return out
