"""Batched scans: many predicates over many resident columns in one persistent
launch (optionally replayed from a HIP graph), and the autotuner that picks its
launch shape.

The work list (item, tile) and the rewritten literals are prepared once on the
host (``bst_batch_prepare``); ``launch`` enqueues a counter reset and one
persistent kernel whose waves take ``tiles_per_grab`` tiles at a time from a
shared counter, so columns of very different lengths balance across the chip.
"""
from __future__ import annotations

import itertools
import time

import numpy as np
import torch

from . import _lib as L
from .column import make_pred, stream_handle


class Batch:
    """specs: sequence of (DeviceColumn, op, lo, hi, in_mask tensor or None); outs: bitvector tensors."""

    def __init__(self, specs, outs, device="cuda"):
        if len(specs) != len(outs) or not specs:
            raise ValueError("need one output per scan")
        self.specs = list(specs)
        self.outs = list(outs)
        n = len(specs)
        self.ws = torch.empty(int(L.bst_batch_workspace_bytes(n)), dtype=torch.uint8, device=device)
        cols = [s[0].h for s in specs]
        preds = [make_pred(s[1], s[2], s[3]) for s in specs]
        masks = [s[4] for s in specs]
        self.h = L.bst_batch_prepare(cols, preds, masks, outs, self.ws)
        self.rows = sum(int(s[0].n_rows) for s in specs)

    def launch(self, grid: int = 0, tiles_per_grab: int = 0, use_graph: bool = False, stream=None):
        L.bst_batch_launch(self.h, int(grid), int(tiles_per_grab), use_graph, stream_handle(stream))

    def close(self):
        if self.h:
            L.bst_batch_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def time_call(fn, repeats: int = 5, warmup: int = 1, stream=None) -> float:
    """Median wall time of fn() on the GPU in milliseconds (HIP events)."""
    s = stream if stream is not None else torch.cuda.current_stream()
    for _ in range(warmup):
        fn()
    samples = []
    for _ in range(repeats):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(s)
        fn()
        e1.record(s)
        e1.synchronize()
        samples.append(e0.elapsed_time(e1))
    return float(np.median(samples))


def autotune(batch: Batch, grids=None, grabs=(1, 2, 4, 8, 16), streams=(1,), repeats: int = 5,
             use_graph: bool = True):
    """Time every (grid, tiles_per_grab, streams) triple and return the fastest
    with all timings.  streams: how many streams the batch's groups are spread
    over (1..4).

    The chosen triple is also stored as the library's default batch shape.
    """
    if grids is None:
        cus = torch.cuda.get_device_properties(torch.cuda.current_device()).multi_processor_count
        grids = [cus * k for k in (2, 4, 8, 16)]
    results = {}
    saved = L.bst_tune_get(L.TUNE_BATCH_STREAMS)
    try:
        for s, g, t in itertools.product(streams, grids, grabs):
            L.bst_tune_set(L.TUNE_BATCH_STREAMS, s)
            results[(g, t, s)] = time_call(lambda: batch.launch(g, t, use_graph), repeats=repeats)
    finally:
        L.bst_tune_set(L.TUNE_BATCH_STREAMS, saved)
    best = min(results, key=results.get)
    L.bst_tune_set(L.TUNE_BATCH_GRID, best[0])
    L.bst_tune_set(L.TUNE_BATCH_GRAB, best[1])
    L.bst_tune_set(L.TUNE_BATCH_STREAMS, best[2])
    return best, results


def autotune_batch(specs, outs, solos=(1 << 12, 1 << 14, 1 << 62), **kw):
    """autotune() over the solo threshold as well: for every value of
    TUNE_BATCH_SOLO_TILES (items of at least that many tiles run as single-column
    scan launches; it is read when a batch is prepared) a Batch of `specs` is
    prepared and its launch shape tuned.  Returns (the fastest Batch, open;
    (solo, grid, tiles_per_grab, streams); {tuple: ms}).  The winning values
    stay the library's defaults."""
    saved = L.bst_tune_get(L.TUNE_BATCH_SOLO_TILES)
    best, best_b, table = None, None, {}
    try:
        for solo in solos:
            L.bst_tune_set(L.TUNE_BATCH_SOLO_TILES, solo)
            b = Batch(specs, outs)
            shape, res = autotune(b, **kw)
            table.update({(solo,) + k: v for k, v in res.items()})
            if best is None or res[shape] < table[best]:
                if best_b is not None:
                    best_b.close()
                best, best_b = (solo,) + shape, b
            else:
                b.close()
    finally:
        L.bst_tune_set(L.TUNE_BATCH_SOLO_TILES, saved)
    L.bst_tune_set(L.TUNE_BATCH_SOLO_TILES, best[0])
    L.bst_tune_set(L.TUNE_BATCH_GRID, best[1])
    L.bst_tune_set(L.TUNE_BATCH_GRAB, best[2])
    L.bst_tune_set(L.TUNE_BATCH_STREAMS, best[3])
    return best_b, best, table


def autotune_scan(scans, grids=None, gathers=(1, 2, 4), repeats: int = 3):
    """Pick the single-column scan launch shape by timing: every (grid, gather)
    pair runs all `scans` -- (DeviceColumn, op, lo, hi) -- and the pair with the
    smallest total time is stored as the library's default.  grid: workgroups
    per scan launch (0 keeps each layout's built-in default); gather: pending
    rows per 32-row lane that a later level gathers one by one before the tile
    stages the level's run in LDS instead.  Returns (best pair, {pair: ms})."""
    if grids is None:
        cus = torch.cuda.get_device_properties(torch.cuda.current_device()).multi_processor_count
        grids = [0] + [cus * k for k in (2, 3, 4, 6)]
    outs = [s[0].new_bv() for s in scans]

    def run():
        for (col, op, lo, hi), o in zip(scans, outs):
            col.scan(op, lo, hi, out=o)

    saved = (L.bst_tune_get(L.TUNE_SCAN_GRID), L.bst_tune_get(L.TUNE_GATHER_ROWS))
    results = {}
    try:
        for g, r in itertools.product(grids, gathers):
            L.bst_tune_set(L.TUNE_SCAN_GRID, g)
            L.bst_tune_set(L.TUNE_GATHER_ROWS, r)
            results[(g, r)] = time_call(run, repeats=repeats)
    finally:
        L.bst_tune_set(L.TUNE_SCAN_GRID, saved[0])
        L.bst_tune_set(L.TUNE_GATHER_ROWS, saved[1])
    best = min(results, key=results.get)
    L.bst_tune_set(L.TUNE_SCAN_GRID, best[0])
    L.bst_tune_set(L.TUNE_GATHER_ROWS, best[1])
    return best, results
