"""GPU lookups, compaction and bitvector helpers against the oracle (Sec. 2.2, 3.3)."""
import numpy as np
import pytest
import torch

import datagen
from helpers import close_columns, device_columns, flush
from oracle.layout import pack_bits, unpack_bits
from oracle.lookup import bv_row_ids, lookup_bv, lookup_ids

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu(built_lib):
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    torch.cuda.set_device(0)
    yield
    torch.cuda.synchronize()


def _np32(t):
    from paper_2209_00220_amd.column import u32_to_numpy

    torch.cuda.synchronize()
    return u32_to_numpy(t)


@pytest.mark.parametrize("dir_stride", [64, 128, 256, 512, 1024, 2048])
def test_lookup_every_directory_stride(dir_stride):
    """PP-VBS lookups of every row at each directory stride: one mask word per
    block (64), blocks read as 16-byte pairs (128..512), and the per-word walk
    (1024, 2048); codes of up to five bytes from the sorted mapping, a ragged
    tail, rows at every position of a block."""
    from paper_2209_00220_amd.column import u32_from_numpy

    n = 70_001
    flush("lookup every row, dir_stride=%d" % dir_stride)
    x = datagen.zipf_column(n, 16, 1.0, seed=11, mapping=datagen.SORTED)
    cols = device_columns(x, 16, layouts=("ppvbs",), dir_stride=dir_stride)
    try:
        hc, col = cols["ppvbs"]
        assert hc.info.k_max >= 3
        ids = np.arange(n, dtype=np.uint32)
        got = _np32(col.lookup(u32_from_numpy(ids)))
        assert np.array_equal(got, lookup_ids(x, ids))
    finally:
        close_columns(cols)


@pytest.mark.parametrize("n,w,s,mapping", [
    (1, 12, 1.0, datagen.SCATTER), (65, 12, 1.0, datagen.SCATTER), (4097, 20, 1.0, datagen.SORTED),
    (300_007, 20, 1.0, datagen.SCATTER), (2_000_003, 20, 0.5, datagen.SORTED), (200_000, 32, 0.0, datagen.SCATTER),
    (100_000, 8, 1.5, datagen.SCATTER),
])
def test_lookup_identity(n, w, s, mapping):
    flush("lookup n=%d w=%d s=%g" % (n, w, s))
    from paper_2209_00220_amd.column import u32_from_numpy

    x = datagen.zipf_column(n, w, s, seed=n ^ w, mapping=mapping)
    ids = np.concatenate([datagen.uniform_ids(20_000, n, seed=n), np.array([0, n - 1], dtype=np.uint32)])
    for domain in (True, False):
        cols = device_columns(x, w, domain=domain)
        try:
            for lay, (hc, col) in cols.items():
                got = _np32(col.lookup(u32_from_numpy(ids)))
                assert np.array_equal(got, lookup_ids(x, ids)), (lay, domain)
                # every row in order
                if n <= 300_007:
                    allv = _np32(col.lookup(u32_from_numpy(np.arange(n, dtype=np.uint32))))
                    assert np.array_equal(allv, x), (lay, domain)
        finally:
            close_columns(cols)


def test_bad_row_sets_status():
    from paper_2209_00220_amd.column import u32_from_numpy

    n = 1000
    x = datagen.zipf_column(n, 12, 1.0, seed=1)
    cols = device_columns(x, 12)
    try:
        for lay, (hc, col) in cols.items():
            status = torch.zeros(1, dtype=torch.int32, device="cuda")
            ids = np.array([3, n, 5, 0xFFFFFFFF], dtype=np.uint32)
            got = _np32(col.lookup(u32_from_numpy(ids), status=status))
            assert list(got) == [x[3], 0, x[5], 0]
            assert int(status.item()) & 1
    finally:
        close_columns(cols)


@pytest.mark.parametrize("n,density", [(1, 1.0), (64, 0.5), (2049, 0.01), (1_000_003, 0.2), (1_000_003, 0.0)])
def test_compact_and_lookup_bv(n, density):
    from paper_2209_00220_amd.column import bv_compact, bv_from_numpy

    x = datagen.zipf_column(n, 16, 1.0, seed=n)
    R = datagen.random_mask_words(n, seed=n + 3, density=density)
    Rt = bv_from_numpy(R)
    want_ids = bv_row_ids(R, n)
    cap = max(1, want_ids.shape[0])
    ids, count = bv_compact(Rt, n, cap)
    torch.cuda.synchronize()
    assert int(count.item()) == want_ids.shape[0]
    assert np.array_equal(_np32(ids)[: want_ids.shape[0]], want_ids)
    cols = device_columns(x, 16)
    try:
        for lay, (hc, col) in cols.items():
            vals, cnt = col.lookup_bv(Rt, cap)
            torch.cuda.synchronize()
            k = int(cnt.item())
            assert k == want_ids.shape[0]
            assert np.array_equal(_np32(vals)[:k], lookup_bv(x, R, n)), lay
    finally:
        close_columns(cols)


@pytest.mark.parametrize("n,density", [
    (2048 * 64, 0.3),            # exactly one chunk of 64 tiles
    (2048 * 64 + 1, 0.3),        # a second chunk holding one row (odd word count: a half quad at the end)
    (2048 * 64 * 3 - 5, 0.02),   # ragged last chunk and tile
    (2048 * 64 * 2 + 134, 0.97), # nearly every row, odd word count
    (97, 0.5),                   # one partial tile
])
def test_compact_and_popcount_ignore_tail_bits(n, density):
    """Compaction and popcount of bitvectors whose words past row n - 1 hold
    set bits: only rows < n count, at chunk and quad boundaries."""
    from paper_2209_00220_amd.column import bv_compact, bv_from_numpy, bv_popcount

    flush("compaction with tail bits, n=%d" % n)
    R = datagen.random_mask_words(n, seed=n + 11, density=density)
    want_ids = bv_row_ids(R, n)
    dirty = R.copy()
    if n % 64:
        dirty[-1] |= np.uint64(~((1 << (n % 64)) - 1) & 0xFFFFFFFFFFFFFFFF)   # garbage past the last row
    Rt = bv_from_numpy(dirty)
    assert int(bv_popcount(Rt, n).item()) == want_ids.shape[0]
    ids, count = bv_compact(Rt, n, max(1, want_ids.shape[0]))
    torch.cuda.synchronize()
    assert int(count.item()) == want_ids.shape[0]
    assert np.array_equal(_np32(ids)[: want_ids.shape[0]], want_ids)


def test_compact_and_popcount_random_sizes():
    """Compaction and popcount over 30 seeded (rows, density) pairs, from one
    row to several chunks, each bitvector with garbage past its last row."""
    from paper_2209_00220_amd.column import bv_compact, bv_from_numpy, bv_popcount

    rng = np.random.default_rng(2024)
    for i in range(30):
        n = int(rng.integers(1, 700_000)) if i % 3 else int(rng.integers(1, 5000))
        density = float(rng.choice([0.0, 0.001, 0.05, 0.5, 0.99, 1.0]))
        flush("random compaction %d: n=%d density=%g" % (i, n, density))
        R = datagen.random_mask_words(n, seed=1000 + i, density=density)
        want_ids = bv_row_ids(R, n)
        dirty = R.copy()
        if n % 64:
            dirty[-1] |= np.uint64(~((1 << (n % 64)) - 1) & 0xFFFFFFFFFFFFFFFF)
        Rt = bv_from_numpy(dirty)
        assert int(bv_popcount(Rt, n).item()) == want_ids.shape[0], (n, density)
        cap = int(want_ids.shape[0]) if i % 5 else max(0, int(want_ids.shape[0]) - 3)   # sometimes too small
        ids, count = bv_compact(Rt, n, cap)
        torch.cuda.synchronize()
        assert int(count.item()) == want_ids.shape[0], (n, density)
        k = min(cap, want_ids.shape[0])
        assert np.array_equal(_np32(ids)[:k], want_ids[:k]), (n, density)


def test_compact_overflow_flag():
    from paper_2209_00220_amd.column import bv_compact, bv_from_numpy

    n = 10_000
    R = datagen.random_mask_words(n, seed=5, density=0.5)
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    ids, count = bv_compact(bv_from_numpy(R), n, 100, status=status)
    torch.cuda.synchronize()
    want = bv_row_ids(R, n)
    assert int(count.item()) == want.shape[0]
    assert np.array_equal(_np32(ids)[:100], want[:100])
    assert int(status.item()) & 2


def test_bitvector_helpers():
    from paper_2209_00220_amd.column import bv_and, bv_andnot, bv_from_numpy, bv_not, bv_or, bv_popcount, bv_to_numpy

    n = 123_457
    a = datagen.random_mask_words(n, seed=1, density=0.3)
    b = datagen.random_mask_words(n, seed=2, density=0.6)
    ta, tb = bv_from_numpy(a), bv_from_numpy(b)
    ra, rb = unpack_bits(a, n), unpack_bits(b, n)
    assert np.array_equal(bv_to_numpy(bv_and(ta, tb, n)), pack_bits(ra & rb))
    assert np.array_equal(bv_to_numpy(bv_or(ta, tb, n)), pack_bits(ra | rb))
    assert np.array_equal(bv_to_numpy(bv_andnot(ta, tb, n)), pack_bits(ra & ~rb))
    assert np.array_equal(bv_to_numpy(bv_not(ta, n)), pack_bits(~ra))
    assert int(bv_popcount(ta, n).item()) == int(ra.sum())


def test_disjunction_and_negation_of_scans():
    # (x < a OR x > b) AND NOT (x = c) on every layout, against the plain definition
    from paper_2209_00220_amd.column import bv_andnot, bv_not, bv_or, bv_to_numpy

    n, w = 77_777, 16
    x = datagen.zipf_column(n, w, 1.2, seed=21)
    a, b, c = int(np.quantile(x, 0.2)), int(np.quantile(x, 0.7)), int(x[5])
    from oracle.scan import scan_values

    want = (scan_values(x, "lt", a) | scan_values(x, "gt", b)) & ~scan_values(x, "eq", c)
    cols = device_columns(x, w)
    try:
        for lay, (_, dc) in cols.items():
            r = bv_andnot(bv_or(dc.scan("lt", a), dc.scan("gt", b), n), dc.scan("eq", c), n)
            assert np.array_equal(bv_to_numpy(r), pack_bits(want)), lay
            assert np.array_equal(bv_to_numpy(bv_not(r, n)), pack_bits(~want)), lay
    finally:
        close_columns(cols)


def test_empty_column_every_entry_point():
    # n = 0: every call succeeds and produces nothing (tail rules with no rows)
    from paper_2209_00220_amd.batch import Batch
    from paper_2209_00220_amd.column import (DeviceColumn, Dictionary, HostColumn, bv_compact, bv_popcount,
                                             u32_from_numpy)

    x0 = np.zeros(0, dtype=np.uint32)
    x1 = datagen.zipf_column(5000, 12, 1.0, seed=3)
    d0, d1 = Dictionary(x0), Dictionary(x1)
    keep = []
    try:
        for lay in ("ppvbs", "byteslice", "bitpacked", "ppvbs_categorical"):
            w = 0 if lay.startswith("ppvbs") else 12
            h0, h1 = HostColumn.encode(d0, lay, width=w), HostColumn.encode(d1, lay, width=w)
            c0, c1 = DeviceColumn(h0), DeviceColumn(h1)
            keep += [h0, h1, c0, c1]
            op = "eq" if lay == "ppvbs_categorical" else "lt"
            bv = c0.scan(op, 7)
            assert bv.numel() == 0
            _, ctr = c0.scan_stats(op, 7)
            assert int(ctr.sum().item()) == 0
            assert c0.lookup(u32_from_numpy(np.zeros(0, dtype=np.uint32))).numel() == 0
            ids, count = bv_compact(bv, 0, 4)
            assert int(count.item()) == 0 and int(bv_popcount(bv, 0).item()) == 0
            vals, count = c0.lookup_bv(bv, 4)
            assert int(count.item()) == 0
            # a batch mixing the empty column with a real one
            o0, o1 = c0.new_bv(), c1.new_bv()
            b = Batch([(c0, op, 7, None, None), (c1, op, int(x1[0]), None, None)], [o0, o1])
            b.launch()
            torch.cuda.synchronize()
            from paper_2209_00220_amd.column import bv_to_numpy
            from oracle.scan import scan_values

            assert np.array_equal(bv_to_numpy(o1), pack_bits(scan_values(x1, op, int(x1[0]))))
            b.close()
    finally:
        for o in reversed(keep):
            o.close()
        d0.close()
        d1.close()


def test_lookup_counted_all_or_nothing():
    """bst_lookup_counted looks up the compacted row IDs whose count stays on the
    device: every value when the count fits the capacity, nothing (and the
    overflow flag) when it does not."""
    from paper_2209_00220_amd import _lib as L
    from paper_2209_00220_amd.column import bv_compact, u32_to_numpy

    n = 300_007
    x = datagen.zipf_column(n, 16, 1.0, seed=71)
    cols = device_columns(x, 16)
    try:
        for lay, (hc, col) in cols.items():
            bv = col.scan("lt", 4000)
            rows = np.nonzero(x < 4000)[0]
            ids, count = bv_compact(bv, n, n)
            for cap, fits in ((rows.shape[0], True), (rows.shape[0] + 17, True), (rows.shape[0] - 1, False)):
                vals = torch.full((max(cap, 1),), -1, dtype=torch.int32, device="cuda")
                status = torch.zeros(1, dtype=torch.int32, device="cuda")
                L.bst_lookup_counted(col.h, ids, count, cap, vals, status, 0)
                torch.cuda.synchronize()
                got = u32_to_numpy(vals)
                st = int(status.item())
                if fits:
                    assert st == 0 and np.array_equal(got[:rows.shape[0]], x[rows]), lay
                    assert np.all(got[rows.shape[0]:] == 0xFFFFFFFF), lay
                else:
                    assert st & L.BST_DEV_OVERFLOW and np.all(got == 0xFFFFFFFF), lay
    finally:
        close_columns(cols)
