"""Serving loop over resident columns: admission by output bytes and continuous
batching of predicate scans.

A query is a conjunction of predicates on one table (columns of equal length),
followed by a lookup of one or more columns on the qualifying rows (the scan
and lookup operations of Sec. 2.2; the conjunction pipelines each scan's
result into the next as its incoming mask, Sec. 3.3).  Every column stays
resident in device memory.  The server runs in steps:

* admission: arrived queries enter in arrival order while the device bytes
  they need fit the budget -- two result bitvectors of ceil(n/64) words, and
  later 8 bytes per qualifying row per lookup column (values plus row IDs).
  The bitvectors of scanning queries may hold only a share of the budget
  (half by default), so the lookups of finished queries always find room and
  a queue of new arrivals cannot starve them;
* scan step: admitted queries that still have predicates contribute their
  next one, with the previous result as the incoming mask, to ONE batched
  launch (a persistent kernel over all their tiles).  The oldest queries go
  first, and a step stops adding queries once it covers enough rows to fill
  the device by itself (``step_rows``): so a query advances one predicate per
  step, small scans share launches, and a large scan is not slowed by
  sharing the device with later queries;
* lookup: a query whose predicates are done counts its rows, gathers the
  values of its lookup columns, and completes.

The loop never waits for the device while it has work to enqueue: each step
and each set of lookups is followed by a fence (an event on the stream), the
host reads counts and completes queries once their fences have passed, and
keeps few scan steps in flight -- at most ``lookahead`` of them, covering at
most ``lookahead_rows`` rows -- so that new arrivals join soon.  So the host's admission, counting and lookup set-up of some queries
overlap the device's scans of others.

Latency is completion time minus arrival time.  ``run_serial`` serves the
same queries one at a time with single scans, waiting for each, the baseline
continuous batching is measured against.

The executor is an interface: ``GpuExecutor`` drives the HIP library; tests
drive the same loop with a host executor.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Callable, Dict, List, Optional, Sequence, Tuple

import numpy as np


@dataclasses.dataclass
class Query:
    qid: int
    table: str
    preds: List[Tuple[str, str, int, Optional[int]]]   # (column, op, lo, hi)
    lookups: List[str]                                   # columns whose values are returned
    arrival: float = 0.0                                 # seconds after the start of the run


@dataclasses.dataclass
class Result:
    qid: int
    count: int
    values: Dict[str, object]    # column -> values of the qualifying rows (executor's array type)
    arrival: float
    admitted: float
    done: float

    @property
    def latency(self) -> float:
        return self.done - self.arrival


class _Active:
    __slots__ = ("q", "k", "cur", "nxt", "admitted", "reserved")

    def __init__(self, q, cur, nxt, admitted, reserved):
        self.q, self.k, self.cur, self.nxt, self.admitted, self.reserved = q, 0, cur, nxt, admitted, reserved


class Server:
    """Continuous-batching server.

    executor: object with ``n_rows(table)``, ``bv_bytes(table)``, ``new_bv(table)``,
    ``scan_step(items)``, ``count_rows(pairs)``, ``read_counts(handle)``,
    ``lookup(table, column, bv, count)``, ``fence()``, ``is_done(token)`` and
    ``wait(token)``.  ``scan_step`` takes a list of (table, column, op, lo, hi,
    in_bv or None, out_bv), enqueues the scans and returns a token that marks
    them; ``count_rows`` enqueues the row counts of (table, bv) pairs, ordered
    after every scan enqueued so far, and returns a token that ``read_counts``
    turns into ints once it is done; ``lookup`` enqueues a gather of the set
    rows' values, ordered after the counts; ``fence`` marks the counts and
    lookups enqueued so far; ``is_done`` tests a token without waiting and
    ``wait`` waits for it.  Counts and lookups may run beside later scans.
    budget_bytes: device bytes the admitted queries may hold at once.  A query
    that alone exceeds the budget is still served once nothing else is admitted.
    scan_share: fraction of the budget the bitvectors of admitted queries may
    hold; the rest is kept for lookups.
    max_batch: most scans per step.  step_rows: a step takes no further query
    once its scans cover this many rows.  lookahead / lookahead_rows: most scan
    steps, and most rows scanned by them, in flight (one step always may be).
    """

    def __init__(self, executor, budget_bytes: int, max_batch: int = 256, scan_share: float = 0.5,
                 step_rows: int = 1 << 27, lookahead: int = 8, lookahead_rows: int = 1 << 30,
                 clock: Callable[[], float] = time.perf_counter, sleep: Callable[[float], None] = time.sleep):
        if (budget_bytes <= 0 or max_batch <= 0 or step_rows <= 0 or lookahead <= 0 or lookahead_rows <= 0
                or not 0.0 < scan_share <= 1.0):
            raise ValueError("budget_bytes, max_batch, step_rows, lookahead and lookahead_rows must be "
                             "positive, scan_share in (0, 1]")
        self.ex = executor
        self.budget = int(budget_bytes)
        self.scan_budget = max(1, int(budget_bytes * scan_share))
        self.max_batch = int(max_batch)
        self.step_rows = int(step_rows)
        self.lookahead = int(lookahead)
        self.lookahead_rows = int(lookahead_rows)
        self.clock = clock
        self.sleep = sleep
        self.in_use = 0
        self.scan_in_use = 0
        self.peak_in_use = 0
        self.steps = 0
        self.batch_sizes: List[int] = []

    def _scan_bytes(self, q: Query) -> int:
        return 2 * self.ex.bv_bytes(q.table)

    def run(self, queries: Sequence[Query], keep_values: bool = True) -> Dict[int, Result]:
        order = sorted(queries, key=lambda q: (q.arrival, q.qid))
        for q in order:
            if not q.preds:
                raise ValueError("query %d has no predicate" % q.qid)
        ex = self.ex
        t0 = self.clock()
        nxt_arrival = 0
        waiting: collections.deque = collections.deque()
        scanning: List[_Active] = []          # admitted, predicates left, in admission order
        steps: collections.deque = collections.deque()      # (seq, fence, rows) of scan steps in flight
        inflight_rows = 0
        counting: collections.deque = collections.deque()   # (seq, counts token, [_Active])
        blocked: collections.deque = collections.deque()    # (_Active, count): lookup waits for memory
        gathering: collections.deque = collections.deque()  # (seq, fence, [(a, count, extra, vals)])
        seq = 0
        done: Dict[int, Result] = {}
        while len(done) < len(order):
            now = self.clock() - t0
            while nxt_arrival < len(order) and order[nxt_arrival].arrival <= now:
                waiting.append(order[nxt_arrival])
                nxt_arrival += 1
            # admission in arrival order (no overtaking: a large query blocks later ones)
            while waiting:
                need = self._scan_bytes(waiting[0])
                busy = scanning or counting or blocked or gathering
                if busy and (self.in_use + need > self.budget or self.scan_in_use + need > self.scan_budget):
                    break
                q = waiting.popleft()
                self.in_use += need
                self.scan_in_use += need
                self.peak_in_use = max(self.peak_in_use, self.in_use)
                scanning.append(_Active(q, None, ex.new_bv(q.table), self.clock() - t0, need))
            enqueued = False
            # one scan step: the next predicate of the oldest scanning queries, one launch
            while steps and ex.is_done(steps[0][1]):
                inflight_rows -= steps.popleft()[2]
            batch, rows = [], 0
            if scanning and len(steps) < self.lookahead:
                for a in scanning:
                    n = ex.n_rows(a.q.table)
                    if batch and (len(batch) >= self.max_batch or rows + n > self.step_rows):
                        break
                    batch.append(a)
                    rows += n
                if steps and inflight_rows + rows > self.lookahead_rows:
                    batch = []
            if batch:
                items = []
                for a in batch:
                    col, op, lo, hi = a.q.preds[a.k]
                    if a.cur is None and a.k + 1 < len(a.q.preds):
                        a.cur = ex.new_bv(a.q.table)   # second buffer, needed from the next step on
                    items.append((a.q.table, col, op, lo, hi, a.cur if a.k > 0 else None, a.nxt))
                tok = ex.scan_step(items)
                self.steps += 1
                self.batch_sizes.append(len(items))
                for a in batch:
                    a.k += 1
                    a.cur, a.nxt = a.nxt, a.cur
                seq += 1
                steps.append((seq, tok, rows))
                inflight_rows += rows
                fin = [a for a in batch if a.k >= len(a.q.preds)]
                if fin:
                    scanning = [a for a in scanning if a.k < len(a.q.preds)]
                    seq += 1
                    counting.append((seq, ex.count_rows([(a.q.table, a.cur) for a in fin]), fin))
                enqueued = True
            # counts known: reserve lookup bytes and enqueue the gathers, oldest
            # first; the oldest query always proceeds when no gather is in flight
            while counting and ex.is_done(counting[0][1]):
                _, handle, fin = counting.popleft()
                blocked.extend(zip(fin, ex.read_counts(handle)))
            started = []
            while blocked:
                a, count = blocked[0]
                extra = 8 * int(count) * len(a.q.lookups)
                if extra and self.in_use + extra > self.budget and (gathering or started):
                    break
                blocked.popleft()
                self.in_use += extra
                self.peak_in_use = max(self.peak_in_use, self.in_use)
                vals = {c: ex.lookup(a.q.table, c, a.cur, int(count)) for c in a.q.lookups}
                started.append((a, int(count), extra, vals))
            if started:
                seq += 1
                gathering.append((seq, ex.fence(), started))
                enqueued = True
            # gathers finished: the queries complete
            while gathering and ex.is_done(gathering[0][1]):
                _, _, fin = gathering.popleft()
                t = self.clock() - t0
                for a, count, extra, vals in fin:
                    self.in_use -= extra + a.reserved
                    self.scan_in_use -= a.reserved
                    done[a.q.qid] = Result(a.q.qid, count, vals if keep_values else {}, a.q.arrival, a.admitted, t)
            if enqueued or len(done) == len(order):
                continue
            # nothing to enqueue: wait for the earliest outstanding fence, else the next arrival
            fronts = [d[0][:2] for d in (steps, counting, gathering) if d]
            if fronts:
                ex.wait(min(fronts, key=lambda f: f[0])[1])
            elif nxt_arrival < len(order):
                wait = order[nxt_arrival].arrival - (self.clock() - t0)
                if wait > 0:
                    self.sleep(wait)
        return done


def run_serial(executor, queries: Sequence[Query], keep_values: bool = True,
               clock: Callable[[], float] = time.perf_counter,
               sleep: Callable[[float], None] = time.sleep) -> Dict[int, Result]:
    """Serve the queries one at a time in arrival order, one scan launch per
    predicate, waiting for each query's count and lookups before the next."""
    order = sorted(queries, key=lambda q: (q.arrival, q.qid))
    t0 = clock()
    done = {}
    for q in order:
        wait = q.arrival - (clock() - t0)
        if wait > 0:
            sleep(wait)
        start = clock() - t0
        cur, nxt = None, executor.new_bv(q.table)
        for k, (col, op, lo, hi) in enumerate(q.preds):
            if cur is None and k + 1 < len(q.preds):
                cur = executor.new_bv(q.table)
            executor.scan_step([(q.table, col, op, lo, hi, cur if k > 0 else None, nxt)])
            cur, nxt = nxt, cur
        handle = executor.count_rows([(q.table, cur)])
        executor.wait(handle)
        count = int(executor.read_counts(handle)[0])
        vals = {c: executor.lookup(q.table, c, cur, count) for c in q.lookups}
        executor.wait(executor.fence())
        done[q.qid] = Result(q.qid, count, vals if keep_values else {}, q.arrival, start, clock() - t0)
    return done


def latency_summary(results: Dict[int, Result]) -> dict:
    lat = np.array([r.latency for r in results.values()], dtype=np.float64)
    span = max(r.done for r in results.values()) - min(r.arrival for r in results.values())
    return {
        "queries": int(lat.size),
        "p50_ms": float(np.percentile(lat, 50) * 1e3),
        "p99_ms": float(np.percentile(lat, 99) * 1e3),
        "mean_ms": float(lat.mean() * 1e3),
        "qps": float(lat.size / span) if span > 0 else float("inf"),
    }


def poisson_arrivals(n: int, qps: float, seed: int) -> np.ndarray:
    """n arrival times (seconds) of a Poisson process of rate qps."""
    rng = np.random.default_rng(seed)
    if qps <= 0 or not np.isfinite(qps):
        return np.zeros(n)
    return np.cumsum(rng.exponential(1.0 / qps, size=n))


class _Counts:
    __slots__ = ("host", "dev", "ev")

    def __init__(self, host, dev, ev):
        self.host, self.dev, self.ev = host, dev, ev


class GpuExecutor:
    """Executor over resident DeviceColumns: tables = {table: {column: DeviceColumn}}.

    Scans run on the current stream; counts and lookups on a second stream
    (default priority) that waits for the scans before them, so a finished
    query's counting and gathering overlap the next scan step on the device.
    """

    def __init__(self, tables, grid: int = 0, tiles_per_grab: int = 0):
        import torch

        from . import column as C

        self.torch = torch
        self.C = C
        self.tables = tables
        self.grid = grid
        self.grab = tiles_per_grab
        self.main = torch.cuda.current_stream()
        self.side = torch.cuda.Stream()
        self._last_scan = None
        self._n = {}
        for t, cols in tables.items():
            ns = {int(dc.n_rows) for dc in cols.values()}
            if len(ns) != 1:
                raise ValueError("table %s: columns of different lengths" % t)
            self._n[t] = ns.pop()

    def n_rows(self, table):
        return self._n[table]

    def bv_bytes(self, table):
        return 8 * self.C.nwords(self._n[table])

    def new_bv(self, table):
        return self.torch.empty(self.C.nwords(self._n[table]), dtype=self.torch.int64, device="cuda")

    def scan_step(self, items):
        # enqueued only: the launch copies the batch's work list through the
        # library's pinned staging ring, and the workspace goes back to torch's
        # stream-ordered allocator, so no later work on the stream can reuse it
        # before the scans have run
        from .batch import Batch

        specs = [(self.tables[t][c], op, lo, hi, inb) for t, c, op, lo, hi, inb, _ in items]
        outs = [it[6] for it in items]
        with self.torch.cuda.stream(self.main):
            if len(items) == 1:
                dc, op, lo, hi, inb = specs[0]
                dc.scan(op, lo, hi, in_mask=inb, out=outs[0])
            else:
                b = Batch(specs, outs)
                b.launch(self.grid, self.grab, use_graph=False)
                b.close()
            ev = self.torch.cuda.Event()
            ev.record(self.main)
        self._last_scan = ev
        return ev

    def count_rows(self, pairs):
        torch = self.torch
        with torch.cuda.stream(self.side):
            if self._last_scan is not None:
                self.side.wait_event(self._last_scan)
            cs = torch.cat([self.C.bv_popcount(bv, self._n[t]) for t, bv in pairs])
            host = torch.empty(cs.shape, dtype=cs.dtype, pin_memory=True)
            host.copy_(cs, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(self.side)
        return _Counts(host, cs, ev)

    def read_counts(self, handle):
        handle.ev.synchronize()
        return [int(v) for v in handle.host.tolist()]

    def lookup(self, table, column, bv, count):
        with self.torch.cuda.stream(self.side):
            vals, _ = self.tables[table][column].lookup_bv(bv, max(int(count), 1))
        return vals[: int(count)]

    def fence(self):
        ev = self.torch.cuda.Event()
        ev.record(self.side)
        return ev

    def is_done(self, token):
        return getattr(token, "ev", token).query()

    def wait(self, token):
        getattr(token, "ev", token).synchronize()

    def sync(self):
        """Make the current stream wait for the counts and lookups enqueued so far."""
        self.torch.cuda.current_stream().wait_stream(self.side)
