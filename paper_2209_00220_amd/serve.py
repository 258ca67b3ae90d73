"""Serving loop over resident columns: admission by output bytes and continuous
batching of predicate scans.

A query is a conjunction of predicates on one table (columns of equal length),
followed by a lookup of one or more columns on the qualifying rows (the scan
and lookup operations of Sec. 2.2; the conjunction pipelines each scan's
result into the next as its incoming mask, Sec. 3.3).  Every column stays
resident in device memory.  The server runs in steps:

* admission: arrived queries enter in arrival order while the device bytes
  they reserve fit the budget: two result bitvectors of ceil(n/64) words, and
  the lookup outputs for its qualifying rows (4-byte values per lookup column
  and 4-byte row IDs; every row of the table by default, or up to
  ``lookup_cap_rows``).  These reservations may hold
  only a share of the budget (half by default), so a query whose rows exceed
  its reservation always finds room to finish, and a queue of new arrivals
  cannot starve it;
* scan step: admitted queries that still have predicates contribute their
  next one, with the previous result as the incoming mask, to ONE batch (the
  scans of small tables share persistent launches; a large scan runs as its
  own single-column launch).  The oldest queries go first, and a step stops
  adding queries once its scans cover ``step_rows`` rows (2^27 by default,
  about what fills the device): so a query advances one predicate per step,
  the scans of small tables share launches, and a query whose scan fills the
  device by itself does not wait for later queries' scans merged into its
  step (measured on a 500M-row column: steps of 2^30 rows raised the p99 at
  25 % load from 4.1 to 5.3 ms and the p50 at 80 % load from 1.1 to 1.35 ms);
* finish: right behind a query's last scan, on the same stream, the executor
  enqueues the compaction of its result (ascending row IDs and their count,
  kept on the device), the lookups of its columns into the reserved outputs,
  and an asynchronous copy of the count to the host.  No host round trip
  separates a query's scans from its lookups, and the device runs every
  query's work in arrival order, as one query at a time would, without the
  gaps.  A query with more rows than its reservation reserves the exact bytes
  once its count is known and looks up again.

The loop never waits for the device while it has work to enqueue: each step
and each finish is followed by an event, the host completes queries once
their events have passed, and keeps few scan steps in flight -- at most
``lookahead`` of them, covering at most ``lookahead_rows`` rows -- so that
new arrivals join soon.

Latency is completion time minus arrival time.  ``run_serial`` serves the
same queries one at a time with the plain per-query calls (one scan launch
per predicate, then the row count read back to size the lookup, then the
lookups), waiting for each query: the baseline that continuous batching is
measured against.

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
    __slots__ = ("q", "k", "cur", "nxt", "admitted", "reserved", "cap")

    def __init__(self, q, cur, nxt, admitted, reserved, cap):
        self.q, self.k, self.cur, self.nxt, self.admitted, self.reserved, self.cap = q, 0, cur, nxt, admitted, reserved, cap


class Server:
    """Continuous-batching server.

    executor: object with ``n_rows(table)``, ``bv_bytes(table)``, ``new_bv(table)``,
    ``scan_step(items)``, ``finish(table, bv, columns, cap)``, ``result(token)``,
    ``is_done(token)`` and ``wait(token)``.  ``scan_step`` takes a list of
    (table, column, op, lo, hi, in_bv or None, out_bv), enqueues the scans and
    returns a token that marks them; ``finish`` enqueues, behind every scan so
    far, the row count of bv and the values of `columns` for up to `cap` of its
    rows, and returns a token; once that token is done, ``result`` gives
    (count, {column: values}), or (count, None) when count > cap; ``is_done``
    tests a token without waiting and ``wait`` waits for it.
    budget_bytes: device bytes the admitted queries may hold at once.  A query
    that alone exceeds the budget is still served once nothing else is admitted.
    scan_share: fraction of the budget the admission reservations (bitvectors
    and lookup outputs) may hold; the rest is kept for queries whose rows
    exceed their reservation.  lookup_cap_rows: qualifying rows whose lookup
    outputs a query reserves at admission (None: all rows of its table, so no
    lookup ever waits for a count; 0: none, every lookup waits for the count).
    max_batch: most scans per step.  step_rows: a step takes no
    further query once its scans cover this many rows.  lookahead /
    lookahead_rows: most scan steps, and most rows scanned by them, in flight
    (one step always may be).
    """

    def __init__(self, executor, budget_bytes: int, max_batch: int = 256, scan_share: float = 0.5,
                 step_rows: int = 1 << 27, lookahead: int = 8, lookahead_rows: int = 1 << 30,
                 lookup_cap_rows: Optional[int] = None,
                 clock: Callable[[], float] = time.perf_counter, sleep: Callable[[float], None] = time.sleep):
        if (budget_bytes <= 0 or max_batch <= 0 or step_rows <= 0 or lookahead <= 0 or lookahead_rows <= 0
                or (lookup_cap_rows is not None and lookup_cap_rows < 0) or not 0.0 < scan_share <= 1.0):
            raise ValueError("budget_bytes, max_batch, step_rows, lookahead and lookahead_rows must be "
                             "positive, lookup_cap_rows non-negative, scan_share in (0, 1]")
        self.ex = executor
        self.budget = int(budget_bytes)
        self.scan_budget = max(1, int(budget_bytes * scan_share))
        self.max_batch = int(max_batch)
        self.step_rows = int(step_rows)
        self.lookahead = int(lookahead)
        self.lookahead_rows = int(lookahead_rows)
        self.lookup_cap_rows = None if lookup_cap_rows is None else int(lookup_cap_rows)
        self.clock = clock
        self.sleep = sleep
        self.in_use = 0
        self.scan_in_use = 0
        self.peak_in_use = 0
        self.steps = 0
        self.batch_sizes: List[int] = []
        self.relookups = 0

    def _reservation(self, q: Query) -> Tuple[int, int]:
        """(bytes, rows): two bitvectors, and lookup outputs for up to lookup_cap_rows rows."""
        n = self.ex.n_rows(q.table)
        cap = (n if self.lookup_cap_rows is None else min(n, self.lookup_cap_rows)) if q.lookups else 0
        return 2 * self.ex.bv_bytes(q.table) + 4 * cap * (len(q.lookups) + 1), cap

    def run(self, queries: Sequence[Query], keep_values: bool = True) -> Dict[int, Result]:
        order = sorted(queries, key=lambda q: (q.arrival, q.qid))
        for q in order:
            if not q.preds:
                raise ValueError("query %d has no predicate" % q.qid)
        ex = self.ex
        release = getattr(ex, "release", lambda tok: None)   # optional: a retired step token
        t0 = self.clock()
        nxt_arrival = 0
        waiting: collections.deque = collections.deque()
        scanning: List[_Active] = []          # admitted, predicates left, in admission order
        steps: collections.deque = collections.deque()      # (seq, token, rows) of scan steps in flight
        inflight_rows = 0
        finishing: collections.deque = collections.deque()  # (seq, token, _Active, extra bytes)
        blocked: collections.deque = collections.deque()    # (_Active, count): rows beyond the reservation
        seq = 0
        done: Dict[int, Result] = {}
        while len(done) < len(order):
            now = self.clock() - t0
            while nxt_arrival < len(order) and order[nxt_arrival].arrival <= now:
                waiting.append(order[nxt_arrival])
                nxt_arrival += 1
            # admission in arrival order (no overtaking: a large query blocks later ones)
            while waiting:
                need, cap = self._reservation(waiting[0])
                busy = scanning or finishing or blocked
                if busy and (self.in_use + need > self.budget or self.scan_in_use + need > self.scan_budget):
                    break
                q = waiting.popleft()
                self.in_use += need
                self.scan_in_use += need
                self.peak_in_use = max(self.peak_in_use, self.in_use)
                scanning.append(_Active(q, None, ex.new_bv(q.table), self.clock() - t0, need, cap))
            enqueued = False
            # one scan step: the next predicate of the oldest scanning queries, one launch
            while steps and ex.is_done(steps[0][1]):
                _, tok, r = steps.popleft()
                inflight_rows -= r
                release(tok)
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
                    for a in fin:   # counts and lookups right behind the last scans, no host wait
                        seq += 1
                        finishing.append((seq, ex.finish(a.q.table, a.cur, a.q.lookups, a.cap), a, 0))
                enqueued = True
            # finished work: complete the query, or look up again with the exact count
            progress = True
            while progress:
                progress = False
                while finishing and ex.is_done(finishing[0][1]):
                    _, tok, a, extra = finishing.popleft()
                    count, vals = ex.result(tok)
                    progress = True
                    if vals is None:
                        blocked.append((a, count))
                        continue
                    t = self.clock() - t0
                    self.in_use -= extra + a.reserved
                    self.scan_in_use -= a.reserved
                    done[a.q.qid] = Result(a.q.qid, count, vals if keep_values else {}, a.q.arrival, a.admitted, t)
                while blocked:
                    a, count = blocked[0]
                    extra = 4 * int(count) * (len(a.q.lookups) + 1)
                    if self.in_use + extra > self.budget and finishing:
                        break
                    blocked.popleft()
                    self.in_use += extra
                    self.peak_in_use = max(self.peak_in_use, self.in_use)
                    self.relookups += 1
                    seq += 1
                    finishing.append((seq, ex.finish(a.q.table, a.cur, a.q.lookups, int(count)), a, extra))
                    enqueued = progress = True
            if enqueued or len(done) == len(order):
                continue
            # nothing to enqueue: wait for the earliest outstanding token, else the next arrival
            fronts = [d[0][:2] for d in (steps, finishing) if d]
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
    """Serve the queries one at a time in arrival order with the plain per-query
    calls: one scan launch per predicate, the row count read back to size the
    lookup outputs, then the lookups; each query completes before the next starts."""
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
        tok = executor.finish(q.table, cur, [], 0)
        executor.wait(tok)
        count, _ = executor.result(tok)
        tok = executor.finish(q.table, cur, q.lookups, int(count))
        executor.wait(tok)
        _, vals = executor.result(tok)
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


class _Finish:
    __slots__ = ("ev", "slot", "vals", "cap")

    def __init__(self, ev, slot, vals, cap):
        self.ev, self.slot, self.vals, self.cap = ev, slot, vals, cap   # vals: column -> output[cap]


class GpuExecutor:
    """Executor over resident DeviceColumns: tables = {table: {column: DeviceColumn}}.

    Everything runs in order on one stream (the current stream at creation):
    scans, then each finished query's compaction and lookups, so the device
    serves queries in the order their work was enqueued and a lookup never
    competes with a later query's scan.  Row counts come back through a pool of
    pinned host slots filled by asynchronous copies.
    """

    def __init__(self, tables, grid: int = 0, tiles_per_grab: int = 0, slots: int = 1024):
        import torch

        from . import _lib
        from . import column as C

        self.torch = torch
        self.L = _lib
        self.C = C
        self.tables = tables
        self.grid = grid
        self.grab = tiles_per_grab
        self.main = torch.cuda.current_stream()
        self._n = {}
        for t, cols in tables.items():
            ns = {int(dc.n_rows) for dc in cols.values()}
            if len(ns) != 1:
                raise ValueError("table %s: columns of different lengths" % t)
            self._n[t] = ns.pop()
        n_max = max(self._n.values()) if self._n else 0
        self.ws = torch.empty(max(1, int(_lib.bst_compact_workspace_bytes(n_max))), dtype=torch.uint8, device="cuda")
        self.ids = torch.empty(1, dtype=torch.int32, device="cuda")
        self.dev_counts = torch.empty(slots, dtype=torch.int64, device="cuda")
        self.host_counts = torch.empty(slots, dtype=torch.int64, pin_memory=True)
        self.free = list(range(slots - 1, -1, -1))
        self.events = []   # recorded events whose tokens are done, for reuse

    def _event(self):
        ev = self.events.pop() if self.events else self.torch.cuda.Event()
        ev.record(self.main)
        return ev

    def _on_main(self):
        """The scan stream as the current stream (a no-op when it already is)."""
        import contextlib

        if self.torch.cuda.current_stream() == self.main:
            return contextlib.nullcontext()
        return self.torch.cuda.stream(self.main)

    def n_rows(self, table):
        return self._n[table]

    def bv_bytes(self, table):
        return 8 * self.C.nwords(self._n[table])

    def new_bv(self, table):
        return self.torch.empty(self.C.nwords(self._n[table]), dtype=self.torch.int64, device="cuda")

    def _stream(self):
        return self.main.cuda_stream

    def _slot(self):
        if not self.free:
            raise RuntimeError("all %d count slots are in use" % self.dev_counts.numel())
        return self.free.pop()

    def _ids(self, cap):
        # one staging array for the row IDs of every compaction: the work on the
        # stream is ordered, so a finish's lookups have read it before the next
        # compaction writes it
        if self.ids.numel() < cap:
            self.ids = self.torch.empty(cap, dtype=self.torch.int32, device="cuda")
        return self.ids

    def scan_step(self, items):
        # enqueued only: the launch copies the batch's work list through the
        # library's pinned staging ring, and the workspace goes back to torch's
        # stream-ordered allocator, so no later work on the stream can reuse it
        # before the scans have run
        from .batch import Batch

        specs = [(self.tables[t][c], op, lo, hi, inb) for t, c, op, lo, hi, inb, _ in items]
        outs = [it[6] for it in items]
        with self._on_main():
            if len(items) == 1:
                dc, op, lo, hi, inb = specs[0]
                dc.scan(op, lo, hi, in_mask=inb, out=outs[0], stream=self.main)
            else:
                b = Batch(specs, outs)
                b.launch(self.grid, self.grab, use_graph=False, stream=self.main)
                b.close()
            return self._event()

    def finish(self, table, bv, columns, cap):
        torch, L = self.torch, self.L
        n = self._n[table]
        slot = self._slot()
        cnt = self.dev_counts[slot:slot + 1]
        vals = {}
        with self._on_main():
            st = self._stream()
            if columns and cap > 0:
                ids = self._ids(cap)
                L.bst_bv_compact(bv, n, ids, cap, cnt, self.ws, None, st)
                for c in columns:
                    v = torch.empty(cap, dtype=torch.int32, device="cuda")
                    L.bst_lookup_counted(self.tables[table][c].h, ids, cnt, cap, v, None, st)
                    vals[c] = v
            else:
                L.bst_bv_popcount(bv, n, cnt, st)
                vals = {c: torch.empty(0, dtype=torch.int32, device="cuda") for c in columns}
            self.host_counts[slot:slot + 1].copy_(cnt, non_blocking=True)
            ev = self._event()
        return _Finish(ev, slot, vals, cap)

    def result(self, tok):
        tok.ev.synchronize()
        count = int(self.host_counts[tok.slot])
        self.free.append(tok.slot)
        self.events.append(tok.ev)
        if count > tok.cap and tok.vals:
            return count, None
        return count, {c: v[:count] for c, v in tok.vals.items()}

    def release(self, token):
        """A scan-step token the server no longer needs: its event is reused."""
        self.events.append(token)

    def is_done(self, token):
        return getattr(token, "ev", token).query()

    def wait(self, token):
        getattr(token, "ev", token).synchronize()

    def sync(self):
        """Make the current stream wait for the work enqueued so far."""
        self.torch.cuda.current_stream().wait_stream(self.main)
