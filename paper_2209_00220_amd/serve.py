"""Serving loop over resident columns: admission by output bytes and continuous
batching of predicate scans.

A query is a conjunction of predicates on one table (columns of equal length),
followed by a lookup of one or more columns on the qualifying rows (the scan
and lookup operations of Sec. 2.2; the conjunction pipelines each scan's
result into the next as its incoming mask, Sec. 3.3).  Every column stays
resident in device memory.  The server runs in steps:

* admission: arrived queries enter in arrival order while the device bytes
  they need fit the budget -- two result bitvectors of ceil(n/64) words, and
  later 8 bytes per qualifying row per lookup column (values plus row IDs);
* scan step: each admitted query that still has predicates contributes its
  next one, with its previous result as the incoming mask, to ONE batched
  launch (a persistent kernel over all their tiles); so a query advances one
  predicate per step, and queries join and leave between steps;
* lookup: a query whose predicates are done counts its rows, gathers the
  values of its lookup columns, and completes.

Latency is completion time minus arrival time.  ``run_serial`` serves the
same queries one at a time with single scans, the baseline continuous batching
is measured against.

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
    ``scan_step(items)``, ``counts(pairs)``, ``lookup(table, column, bv, count)``
    and ``finish(values_list)``.  ``scan_step`` takes a list of (table, column,
    op, lo, hi, in_bv or None, out_bv) and may return before the scans finish
    (work is ordered on one stream); ``counts`` takes (table, bv) pairs and
    returns their row counts once known; ``finish`` returns when the lookups
    that produced the given value dicts have finished.
    budget_bytes: device bytes the admitted queries may hold at once.  A query
    that alone exceeds the budget is still served once nothing else is admitted.
    max_batch: most scans per step.
    """

    def __init__(self, executor, budget_bytes: int, max_batch: int = 256,
                 clock: Callable[[], float] = time.perf_counter, sleep: Callable[[float], None] = time.sleep):
        if budget_bytes <= 0 or max_batch <= 0:
            raise ValueError("budget_bytes and max_batch must be positive")
        self.ex = executor
        self.budget = int(budget_bytes)
        self.max_batch = int(max_batch)
        self.clock = clock
        self.sleep = sleep
        self.in_use = 0
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
        t0 = self.clock()
        nxt_arrival = 0
        waiting: collections.deque = collections.deque()
        active: List[_Active] = []
        done: Dict[int, Result] = {}
        while len(done) < len(order):
            now = self.clock() - t0
            while nxt_arrival < len(order) and order[nxt_arrival].arrival <= now:
                waiting.append(order[nxt_arrival])
                nxt_arrival += 1
            # admission in arrival order (no overtaking: a large query blocks later ones)
            while waiting:
                need = self._scan_bytes(waiting[0])
                if active and self.in_use + need > self.budget:
                    break
                q = waiting.popleft()
                self.in_use += need
                self.peak_in_use = max(self.peak_in_use, self.in_use)
                active.append(_Active(q, None, self.ex.new_bv(q.table), self.clock() - t0, need))
            if not active:
                if nxt_arrival < len(order):
                    wait = order[nxt_arrival].arrival - (self.clock() - t0)
                    if wait > 0:
                        self.sleep(wait)
                continue
            # one scan step: the next predicate of every scanning query, one launch
            scanning = [a for a in active if a.k < len(a.q.preds)][: self.max_batch]
            if scanning:
                items = []
                for a in scanning:
                    col, op, lo, hi = a.q.preds[a.k]
                    if a.cur is None and a.k + 1 < len(a.q.preds):
                        a.cur = self.ex.new_bv(a.q.table)   # second buffer, needed from the next step on
                    items.append((a.q.table, col, op, lo, hi, a.cur if a.k > 0 else None, a.nxt))
                self.ex.scan_step(items)
                self.steps += 1
                self.batch_sizes.append(len(items))
                for a in scanning:
                    a.k += 1
                    a.cur, a.nxt = a.nxt, a.cur
            # finished queries: count their rows (one wait for all), reserve lookup
            # bytes, gather (one wait for all), complete; the oldest finished query
            # always proceeds, later ones wait for memory
            finished = [a for a in active if a.k >= len(a.q.preds)]
            still = [a for a in active if a.k < len(a.q.preds)]
            if finished:
                counts = self.ex.counts([(a.q.table, a.cur) for a in finished])
                gathered = []
                for i, (a, count) in enumerate(zip(finished, counts)):
                    extra = 8 * int(count) * len(a.q.lookups)
                    if i and extra and self.in_use + extra > self.budget:
                        still.append(a)
                        continue
                    self.in_use += extra
                    self.peak_in_use = max(self.peak_in_use, self.in_use)
                    vals = {c: self.ex.lookup(a.q.table, c, a.cur, int(count)) for c in a.q.lookups}
                    gathered.append((a, int(count), extra, vals))
                self.ex.finish([g[3] for g in gathered])
                t = self.clock() - t0
                for a, count, extra, vals in gathered:
                    self.in_use -= extra + a.reserved
                    done[a.q.qid] = Result(a.q.qid, count, vals if keep_values else {}, a.q.arrival, a.admitted, t)
                still.sort(key=lambda a: a.admitted)
            active = still
        return done


def run_serial(executor, queries: Sequence[Query], keep_values: bool = True,
               clock: Callable[[], float] = time.perf_counter,
               sleep: Callable[[float], None] = time.sleep) -> Dict[int, Result]:
    """Serve the queries one at a time in arrival order, one scan launch per predicate."""
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
        count = int(executor.counts([(q.table, cur)])[0])
        vals = {c: executor.lookup(q.table, c, cur, count) for c in q.lookups}
        executor.finish([vals])
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


class GpuExecutor:
    """Executor over resident DeviceColumns: tables = {table: {column: DeviceColumn}}."""

    def __init__(self, tables, grid: int = 0, tiles_per_grab: int = 0):
        import torch

        from . import column as C

        self.torch = torch
        self.C = C
        self.tables = tables
        self.grid = grid
        self.grab = tiles_per_grab
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
        # enqueued only: later work on the stream is ordered after it, and the
        # batch's host list lives until its upload (done inside the launch)
        from .batch import Batch

        specs = [(self.tables[t][c], op, lo, hi, inb) for t, c, op, lo, hi, inb, _ in items]
        outs = [it[6] for it in items]
        if len(items) == 1:
            dc, op, lo, hi, inb = specs[0]
            dc.scan(op, lo, hi, in_mask=inb, out=outs[0])
        else:
            b = Batch(specs, outs)
            b.launch(self.grid, self.grab, use_graph=False)
            b.close()

    def counts(self, pairs):
        cs = [self.C.bv_popcount(bv, self._n[t]) for t, bv in pairs]
        return [int(v) for v in self.torch.cat(cs).cpu().tolist()]

    def lookup(self, table, column, bv, count):
        vals, _ = self.tables[table][column].lookup_bv(bv, max(int(count), 1))
        return vals[: int(count)]

    def finish(self, values_list):
        self.torch.cuda.synchronize()
