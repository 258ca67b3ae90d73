"""Batched scans (one persistent launch, optionally a HIP graph) equal per-query
scans; the advisor's timing loop feeds Algorithm 5's choice."""
import numpy as np
import pytest
import torch

import datagen
from helpers import close_columns, device_columns, flush
from oracle import advisor as oadv
from oracle.scan import scan_values_bv

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu(built_lib):
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    torch.cuda.set_device(0)
    yield
    torch.cuda.synchronize()


def _mixed_items(seed=0, n_cols=6):
    rng = np.random.default_rng(seed)
    cols, xs = [], []
    for i in range(n_cols):
        n = int(rng.integers(1, 400_000))
        w = int(rng.integers(8, 33))
        s = float(rng.uniform(0, 1.5))
        x = datagen.zipf_column(n, w, s, seed=1000 + i)
        xs.append((x, w))
        cols.append(device_columns(x, w))
    items = []
    ops = ["lt", "le", "gt", "ge", "eq", "ne", "between"]
    for k in range(40):
        ci = int(rng.integers(0, n_cols))
        lay = ["ppvbs", "byteslice", "bitpacked"][k % 3]
        x, w = xs[ci]
        op = ops[int(rng.integers(0, len(ops)))]
        a, b = sorted(int(v) for v in x[rng.integers(0, x.shape[0], size=2)])
        if rng.random() < 0.1:
            a = int(rng.integers(0, 2 ** 32))
        items.append((ci, lay, op, a, b))
    return cols, xs, items


RR = 0xFFFFFFFF   # tiles_per_grab: round-robin tiles, no counter


@pytest.mark.parametrize("use_graph,streams,grab,grid,solo", [
    (False, 1, 2, 0, 16384), (True, 1, RR, 0, 16384), (False, 4, RR, 0, 16384), (True, 2, 2, 0, 16384),
    (True, 4, RR, 3, 16384), (False, 1, RR, 3, 16384), (False, 2, 1, 5, 16384),
    (False, 1, RR, 0, 64), (False, 3, 2, 0, 64), (True, 4, RR, 7, 64), (True, 2, 1, 0, 1)])
def test_batch_equals_single(use_graph, streams, grab, grid, solo):
    """Every item of a mixed batch (three layouts, every operator) equals the plain
    definition, eager and replayed from a graph, with the groups on one stream or
    spread over several (helper streams forked off and joined back), tiles taken
    from a counter or assigned round robin; small grids give each wave many
    tiles per item. Items of at least `solo` tiles run as single-column launches
    (solo = 1: every item), side by side with the groups."""
    from paper_2209_00220_amd import _lib
    from paper_2209_00220_amd.batch import Batch
    from paper_2209_00220_amd.column import bv_to_numpy

    assert _lib.BATCH_ROUND_ROBIN == RR
    flush("batch equals single: graph=%s streams=%d grab=%d grid=%d solo=%d" % (use_graph, streams, grab, grid, solo))
    cols, xs, items = _mixed_items(seed=(1 if use_graph else 0) + 2 * streams + (grab == RR) + 8 * (solo < 100))
    saved = _lib.bst_tune_get(_lib.TUNE_BATCH_STREAMS), _lib.bst_tune_get(_lib.TUNE_BATCH_SOLO_TILES)
    _lib.bst_tune_set(_lib.TUNE_BATCH_STREAMS, streams)
    _lib.bst_tune_set(_lib.TUNE_BATCH_SOLO_TILES, solo)
    try:
        outs, specs = [], []
        for ci, lay, op, a, b in items:
            dc = cols[ci][lay][1]
            outs.append(dc.new_bv())
            specs.append((dc, op, a, b if op == "between" else None, None))
        # predicate pipelining across batches: item 5 takes as its incoming mask
        # the result of a scan on the same column that an earlier batch wrote
        ci5, lay5, op5, a5, b5 = items[5]
        x5, _ = xs[ci5]
        first_lit = int(np.median(x5))
        first_out = cols[ci5]["bitpacked"][1].new_bv()
        first = Batch([(cols[ci5]["bitpacked"][1], "ge", first_lit, None, None)], [first_out])
        specs[5] = (specs[5][0], op5, a5, b5 if op5 == "between" else None, first_out)
        batch = Batch(specs, outs)
        for rep in range(3):
            for o in outs:
                o.fill_(-1)
            first_out.fill_(0)
            first.launch(grid=0, tiles_per_grab=1, use_graph=use_graph)
            batch.launch(grid=grid, tiles_per_grab=grab, use_graph=use_graph)
            torch.cuda.synchronize()
            for k, ((ci, lay, op, a, b), o) in enumerate(zip(items, outs)):
                x, w = xs[ci]
                prior = (x >= np.uint32(first_lit)) if k == 5 else None
                want = scan_values_bv(x, op, a, b if op == "between" else None, prior)
                assert np.array_equal(bv_to_numpy(o), want), (rep, k, lay, op, a, b)
            # eager work between graph replays
            _ = cols[0]["ppvbs"][1].scan("lt", 5)
            torch.cuda.synchronize()
        batch.close()
        first.close()
    finally:
        _lib.bst_tune_set(_lib.TUNE_BATCH_STREAMS, saved[0])
        _lib.bst_tune_set(_lib.TUNE_BATCH_SOLO_TILES, saved[1])
        for c in cols:
            close_columns(c)


def test_batch_with_in_masks():
    from paper_2209_00220_amd.batch import Batch
    from paper_2209_00220_amd.column import bv_from_numpy, bv_to_numpy
    from oracle.layout import unpack_bits

    n = 250_001
    x = datagen.zipf_column(n, 20, 1.0, seed=8)
    cols = device_columns(x, 20)
    mask = datagen.random_mask_words(n, seed=9, density=0.05)
    mt = bv_from_numpy(mask)
    try:
        specs, outs = [], []
        for lay in ("ppvbs", "byteslice", "bitpacked"):
            for op, lo, hi in (("lt", 70_000, None), ("between", 5, 500_000), ("eq", int(x[10]), None)):
                specs.append((cols[lay][1], op, lo, hi, mt))
                outs.append(cols[lay][1].new_bv())
        b = Batch(specs, outs)
        b.launch(use_graph=True)
        torch.cuda.synchronize()
        rows = unpack_bits(mask, n)
        for (dc, op, lo, hi, _), o in zip(specs, outs):
            assert np.array_equal(bv_to_numpy(o), scan_values_bv(x, op, lo, hi, rows))
        b.close()
    finally:
        close_columns(cols)


def test_advisor_choice_consistent_with_oracle():
    from paper_2209_00220_amd.advisor import advise_column

    flush("advisor")
    n = 2_000_000
    x = datagen.zipf_column(n, 16, 1.5, seed=31)
    res = advise_column(x, numeric=True, width=16, repeats=3, count=20)
    # the product's area and choice are Algorithm 5's on its own measured times
    for lay, t in res.times.items():
        assert res.aucs[lay] == pytest.approx(oadv.auc(res.sels, t), rel=1e-9)
    want = oadv.choose({oadv.BITPACKED if k == "bitpacked" else oadv.BYTESLICE if k == "byteslice" else oadv.PPVBS: v
                        for k, v in res.aucs.items()})
    name = {oadv.BITPACKED: "bitpacked", oadv.BYTESLICE: "byteslice", oadv.PPVBS: "ppvbs"}[want]
    assert res.chosen == name
    assert all(np.all(t > 0) for t in res.times.values())


def test_advisor_equality_profile_on_categorical_columns():
    """Algorithm 5's '=' profile on a categorical column (codes of Algorithm 2):
    the profiling literals are the oracle's, each layout's area is the trapezoid
    sum of its own measured times, and the choice is the oracle's on those areas."""
    from paper_2209_00220_amd.advisor import advise_column
    from oracle.dictionary import build_dictionary

    flush("advisor, '=' profile")
    n = 1_500_000
    x = datagen.zipf_column(n, 16, 1.2, seed=41)
    count = 40
    res = advise_column(x, numeric=False, width=16, layouts=("byteslice", "ppvbs_categorical"), repeats=3,
                        count=count)
    A, Q, _ = build_dictionary(x)
    lits, sels = oadv.literals_eq(A, Q, count)
    assert np.array_equal(res.lits, lits)
    assert np.allclose(res.sels, sels, rtol=0, atol=1e-12)
    for lay, t in res.times.items():
        assert res.aucs[lay] == pytest.approx(oadv.auc(res.sels, t), rel=1e-9)
        assert np.all(np.asarray(t) > 0)
    want = oadv.choose({oadv.BYTESLICE: res.aucs["byteslice"], oadv.PPVBS: res.aucs["ppvbs_categorical"]})
    assert res.chosen == ("byteslice" if want == oadv.BYTESLICE else "ppvbs_categorical")
    for hc, dc in res.columns.values():
        dc.close()
        hc.close()


def test_batches_back_to_back_without_waits():
    """Batches launched one after another with no host wait in between (their
    work lists go through the library's pinned staging ring, wrapping it at
    least twice), each freed right after its launch: every result is still
    the plain scan."""
    from paper_2209_00220_amd import _lib as L
    from paper_2209_00220_amd.batch import Batch
    from paper_2209_00220_amd.column import bv_to_numpy

    rng = np.random.default_rng(21)
    cols, xs = [], []
    for i in range(4):
        n = int(rng.integers(5_000, 40_000))
        w = int(rng.integers(8, 25))
        x = datagen.zipf_column(n, w, 1.0, seed=2100 + i)
        xs.append(x)
        cols.append(device_columns(x, w))
    ops = ["lt", "le", "gt", "ge", "eq", "ne", "between"]
    specs = []
    for k in range(64):
        ci = int(rng.integers(0, 4))
        x = xs[ci]
        a, b = sorted(int(v) for v in x[rng.integers(0, x.shape[0], size=2)])
        op = ops[int(rng.integers(0, len(ops)))]
        specs.append((ci, ["ppvbs", "byteslice", "bitpacked"][k % 3], op, a, b if op == "between" else None))
    want = [scan_values_bv(xs[ci], op, a, b) for ci, lay, op, a, b in specs]
    per_batch = 32
    image = int(L.bst_batch_workspace_bytes(per_batch))
    n_batches = 2 * (8 << 20) // image + 8
    flush("%d batches of %d scans, %d-byte work lists" % (n_batches, per_batch, image))
    try:
        launched = []
        for bi in range(n_batches):
            pick = rng.integers(0, len(specs), size=per_batch)
            outs = []
            items = []
            for j in pick:
                ci, lay, op, a, b = specs[int(j)]
                dc = cols[ci][lay][1]
                outs.append(dc.new_bv())
                items.append((dc, op, a, b, None))
            bt = Batch(items, outs)
            bt.launch(grid=0, tiles_per_grab=1, use_graph=False)
            bt.close()
            del bt
            launched.append((pick, outs))
        torch.cuda.synchronize()
        for bi, (pick, outs) in enumerate(launched):
            for j, o in zip(pick, outs):
                assert np.array_equal(bv_to_numpy(o), want[int(j)]), (bi, specs[int(j)])
    finally:
        for c in cols:
            close_columns(c)


def test_batch_larger_than_staging_ring():
    """A work list larger than the pinned staging ring goes up by a synchronous
    copy instead; results are the plain scans, and a small batch launched right
    after still goes through the ring."""
    from paper_2209_00220_amd import _lib as L
    from paper_2209_00220_amd.batch import Batch
    from paper_2209_00220_amd.column import bv_to_numpy

    rng = np.random.default_rng(31)
    xs, cols = [], []
    for i in range(3):
        x = datagen.zipf_column(3000 + 777 * i, 16, 1.0, seed=3100 + i)
        xs.append(x)
        cols.append(device_columns(x, 16))
    ops = ["lt", "ge", "eq", "between"]
    specs = []
    for k in range(48):
        ci = k % 3
        x = xs[ci]
        a, b = sorted(int(v) for v in x[rng.integers(0, x.shape[0], size=2)])
        op = ops[k % len(ops)]
        specs.append((ci, ["ppvbs", "byteslice", "bitpacked"][(k // 3) % 3], op, a, b if op == "between" else None))
    want = [scan_values_bv(xs[ci], op, a, b) for ci, lay, op, a, b in specs]
    item_bytes = int(L.bst_batch_workspace_bytes(1) - L.bst_batch_workspace_bytes(0))
    n_items = (8 << 20) // item_bytes + 700
    flush("one batch of %d scans (%d-byte work list)" % (n_items, int(L.bst_batch_workspace_bytes(n_items))))
    try:
        pick = rng.integers(0, len(specs), size=n_items)
        items, outs = [], []
        for j in pick:
            ci, lay, op, a, b = specs[int(j)]
            dc = cols[ci][lay][1]
            items.append((dc, op, a, b, None))
            outs.append(dc.new_bv())
        big = Batch(items, outs)
        for rep in range(2):
            for o in outs[:: max(1, n_items // 50)]:
                o.fill_(-1)
            big.launch(grid=0, tiles_per_grab=0, use_graph=False)
            small_outs = [cols[0]["ppvbs"][1].new_bv() for _ in range(4)]
            small = Batch([(cols[0]["ppvbs"][1], "lt", int(xs[0][i]), None, None) for i in range(4)], small_outs)
            small.launch(grid=0, tiles_per_grab=1, use_graph=False)
            small.close()
            torch.cuda.synchronize()
            for i, o in enumerate(small_outs):
                assert np.array_equal(bv_to_numpy(o), scan_values_bv(xs[0], "lt", int(xs[0][i]), None))
            for j, o in zip(pick, outs):
                assert np.array_equal(bv_to_numpy(o), want[int(j)]), (rep, specs[int(j)])
        big.close()
    finally:
        for c in cols:
            close_columns(c)
