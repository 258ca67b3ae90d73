"""GPU scans through the C ABI against the oracle, bit for bit (Sec. 2.2, 3.3)."""
import numpy as np
import pytest
import torch

import datagen
from helpers import close_columns, device_columns, flush, literal_set
from oracle.dictionary import build_dictionary
from oracle.layout import unpack_bits
from oracle.ppe import padded, ppe_numerical
from oracle.scan import OPS, classify_rows, scan_padded_codes, scan_values_bv

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu(built_lib):
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    torch.cuda.set_device(0)
    yield
    torch.cuda.synchronize()


def _bv(t):
    from paper_2209_00220_amd.column import bv_to_numpy

    torch.cuda.synchronize()
    return bv_to_numpy(t)


@pytest.mark.parametrize("key", ["scan_example", "scan_example_second_literal"])
def test_worked_examples(golden, key):
    from paper_2209_00220_amd.column import DeviceColumn, HostColumn

    g = golden[key]
    codes = np.array([int(h, 16) for h in g["codes"]], dtype=np.uint64)
    lens = np.array([len(h) // 2 for h in g["codes"]], dtype=np.uint8)
    hc = HostColumn.from_codes(codes, lens, 2)
    col = DeviceColumn(hc)
    lit, l = int(g["literal"], 16), len(g["literal"]) // 2
    got = _bv(col.scan_codes(g["op"], lit, l))
    assert int(got[0]) == g["result_word"]
    # every operator on these codes against plain padded-integer comparison
    P = padded(codes, lens.astype(np.int64), 2)
    pl = int(padded([lit], [l], 2)[0])
    for op in OPS:
        hi, lh = (0xC0, 1) if op == "between" else (0, 0)
        want = scan_padded_codes(P, op, pl, int(padded([hi], [1], 2)[0]) if op == "between" else None)
        from oracle.layout import pack_bits

        assert np.array_equal(_bv(col.scan_codes(op, lit, l, hi, lh)), pack_bits(want)), op
    col.close()
    hc.close()


CASES = [
    # n, w, s, mapping
    (1, 12, 1.0, datagen.SCATTER),
    (63, 12, 1.0, datagen.SCATTER),
    (64, 8, 0.0, datagen.SCATTER),
    (65, 12, 1.0, datagen.SCATTER),
    (2047, 12, 1.0, datagen.SCATTER),
    (2049, 16, 1.0, datagen.SORTED),
    (4097, 20, 1.0, datagen.SCATTER),
    (70_001, 12, 1.0, datagen.SCATTER),
    (100_000, 20, 1.0, datagen.SORTED),     # K = 4
    (150_000, 24, 0.0, datagen.SCATTER),    # uniform, K = 4
    (2_000_003, 20, 0.5, datagen.SORTED),   # K = 5
    (300_000, 32, 1.5, datagen.SCATTER),
    (200_003, 4, 1.0, datagen.SCATTER),     # the sensitivity sweep's smallest domain
]


@pytest.mark.parametrize("n,w,s,mapping", CASES)
def test_scan_parity(n, w, s, mapping):
    flush("scan parity n=%d w=%d s=%g mapping=%d" % (n, w, s, mapping))
    x = datagen.zipf_column(n, w, s, seed=n + w, mapping=mapping)
    A, _, _ = build_dictionary(x)
    cols = device_columns(x, w)
    mask_np = datagen.random_mask_words(n, seed=n + 1, density=0.4)
    from paper_2209_00220_amd.column import bv_from_numpy

    mask_t = bv_from_numpy(mask_np)
    mask_rows = unpack_bits(mask_np, n)
    lits = literal_set(A, w)
    try:
        for lay, (hc, col) in cols.items():
            if lay == "ppvbs":
                assert hc.info.k_max >= 1
            for op in OPS:
                for i, lo in enumerate(lits):
                    hi = lits[(i * 5 + 3) % len(lits)] if op == "between" else None
                    for msk in (None, mask_t):
                        got = _bv(col.scan(op, lo, hi, in_mask=msk))
                        want = scan_values_bv(x, op, lo, hi, None if msk is None else mask_rows)
                        assert np.array_equal(got, want), (lay, op, lo, hi, msk is not None)
    finally:
        close_columns(cols)


def test_k5_reached():
    x = datagen.zipf_column(2_000_003, 20, 0.5, seed=2_000_003 + 20, mapping=datagen.SORTED)
    from paper_2209_00220_amd.column import HostColumn

    hc = HostColumn.from_values(x, "ppvbs")
    assert hc.info.k_max == 5
    hc.close()


@pytest.mark.parametrize("dir_stride", [64, 512, 2048])
def test_directory_strides(dir_stride):
    n = 50_001
    x = datagen.zipf_column(n, 16, 1.0, seed=9, mapping=datagen.SORTED)
    A, _, _ = build_dictionary(x)
    cols = device_columns(x, 16, layouts=("ppvbs",), dir_stride=dir_stride)
    try:
        col = cols["ppvbs"][1]
        for lo in literal_set(A, 16):
            for op in ("lt", "eq", "gt"):
                assert np.array_equal(_bv(col.scan(op, lo)), scan_values_bv(x, op, lo)), (op, lo)
    finally:
        close_columns(cols)


def test_config1_scan_and_lookup():
    """1M rows, Zipf(1.0) over 4096 values, seed 0: '<' at about 10%, 10k random lookups."""
    from oracle import advisor as oadv
    from oracle.lookup import lookup_ids
    from paper_2209_00220_amd.column import u32_from_numpy, u32_to_numpy

    n = 1_000_000
    x = datagen.zipf_column(n, 12, 1.0, seed=0)
    A, Q, _ = build_dictionary(x)
    below = np.concatenate([[0], np.cumsum(Q)[:-1]]) / n
    lit = int(A[int(np.argmin(np.abs(below - 0.10)))])
    ids = datagen.uniform_ids(10_000, n, seed=0)
    cols = device_columns(x, 12)
    try:
        for lay, (hc, col) in cols.items():
            got = _bv(col.scan("lt", lit))
            want = scan_values_bv(x, "lt", lit)
            assert np.array_equal(got, want), lay
            sel = unpack_bits(want, n).mean()
            assert abs(sel - 0.10) < 0.06
            vals = col.lookup(u32_from_numpy(ids))
            torch.cuda.synchronize()
            assert np.array_equal(u32_to_numpy(vals), lookup_ids(x, ids)), lay
    finally:
        close_columns(cols)


def test_conjunction_pipeline():
    n = 333_333
    xs = [datagen.zipf_column(n, w, s, seed=50 + i) for i, (w, s) in enumerate(((12, 1.0), (16, 0.5), (20, 1.5)))]
    preds = [("lt", 2000, None), ("between", 1000, 40000), ("ne", int(xs[2][5]), None)]
    want = np.ones(n, dtype=bool)
    for x, (op, lo, hi) in zip(xs, preds):
        from oracle.scan import scan_values

        want &= scan_values(x, op, lo, hi)
    from oracle.layout import pack_bits

    for lay in ("ppvbs", "byteslice", "bitpacked"):
        cols = [device_columns(x, w, layouts=(lay,)) for x, w in zip(xs, (12, 16, 20))]
        try:
            bv = None
            for c, (op, lo, hi) in zip(cols, preds):
                bv = c[lay][1].scan(op, lo, hi, in_mask=bv)
            assert np.array_equal(_bv(bv), pack_bits(want)), lay
        finally:
            for c in cols:
                close_columns(c)


def test_early_stop_counters_lemma1():
    """Row bytes examined equal the byte-serial classifier's, within Lemma 1's bound."""
    n = 200_001
    x = datagen.zipf_column(n, 16, 1.0, seed=21, mapping=datagen.SORTED)
    A, Q, rank = build_dictionary(x)
    C, Lc = ppe_numerical(Q)
    cols = device_columns(x, 16, layouts=("ppvbs", "byteslice"))
    try:
        col = cols["ppvbs"][1]
        for k in (0, 3, 100, 1000, len(A) // 2, len(A) - 1):
            for op in ("lt", "gt", "eq"):
                if (op == "lt" and k == 0) or (op == "gt" and k == len(A) - 1):
                    continue   # always-false predicates become a fill: nothing is scanned
                bv, ctr = col.scan_stats(op, int(A[k]))
                torch.cuda.synchronize()
                ctr = ctr.cpu().numpy()
                _, m = classify_rows(C[rank], Lc[rank], int(C[k]), int(Lc[k]))
                assert int(ctr[1]) == int(m.sum()), (k, op)
                assert int(m.sum()) <= int(np.minimum(Lc[rank], Lc[k]).sum())
                assert 0 < int(ctr[0]) <= int(ctr[3])
                # the same bytes at 128-byte granularity: whole lines, at least the
                # bytes themselves, at most the lines an exhaustive read of each
                # tile's runs touches (its bytes plus one partial line per run)
                tiles = (n + 2047) // 2048
                assert int(ctr[4]) % 128 == 0 and int(ctr[0]) <= int(ctr[4])
                assert int(ctr[4]) <= int(ctr[3]) + 128 * tiles * (int(Lc.max()) - 1), (k, op)
                if op == "lt" and Lc[k] == 1:   # settled by byte 1 alone: BS_1 and the result
                    assert int(ctr[4]) == int(ctr[0]) == tiles * (2048 + 256)
                assert np.array_equal(_bv(bv), scan_values_bv(x, op, int(A[k])))
        # ByteSlice: fixed 2-byte codes, counters bounded by the full read
        bvb, cb = cols["byteslice"][1].scan_stats("lt", int(A[len(A) // 3]))
        torch.cuda.synchronize()
        cb = cb.cpu().numpy()
        assert 0 < int(cb[0]) <= int(cb[3])
        assert int(cb[4]) % 128 == 0 and int(cb[0]) <= int(cb[4]) <= int(cb[3])
    finally:
        close_columns(cols)


def _expected_touch(P, Lr, K, lit, l, op):
    """Counters 0 and 4 of an instrumented PP-VBS scan with one literal (code
    `lit` of l bytes), from their definitions on the rows' padded codes P and
    lengths Lr: per 2048-row tile, BS_1 and the result words; at each byte j of
    the literal, the BS_j bytes of every 64-row group holding a row that is
    equal to the literal over bytes 1..j-1 and has a j-th byte; after byte j,
    the M_{j+1} words of the groups holding rows equal over bytes 1..j, unless
    j is the last byte of a '<' literal (such rows are not below it).  Counter 0
    sums the bytes, counter 4 is 128 x the distinct 128-byte lines (by offset in
    the slice) that hold them, per tile and level."""
    n = P.shape[0]
    tiles = (n + 2047) // 2048
    exact, lines = tiles * (2048 + 256), tiles * 18
    rows = np.arange(n, dtype=np.int64)
    group, tile = rows // 64, rows // 2048
    eq = np.ones(n, dtype=bool)
    for j in range(1, l + 1):
        byte = (P >> np.uint64(8 * (K - j))) & np.uint64(0xFF)
        has = Lr >= j
        if j >= 2:
            pend_groups = np.unique(group[eq & has])
            touched = np.isin(group, pend_groups) & has
            pos = np.cumsum(has) - 1                      # position in BS_j
            exact += int(touched.sum())
            lines += np.unique(tile[touched] * (1 << 40) + pos[touched] // 128).shape[0]
        eq &= has & (byte == np.uint64((lit >> (8 * (l - j))) & 0xFF))
        if j < K and not (op == "lt" and j == l):
            tied_groups = np.unique(group[eq])
            exact += 8 * tied_groups.shape[0]
            lines += np.unique(tied_groups // 16).shape[0]
    return exact, 128 * lines


def test_touch_counters_exact():
    """The instrumented scan's algorithmic bytes, exact and at 128-byte
    granularity, equal their definitions computed from the oracle's codes, for
    literals of one, two and three bytes, over a column with a ragged tail."""
    n = 200_001
    x = datagen.zipf_column(n, 16, 1.0, seed=23, mapping=datagen.SORTED)
    A, Q, rank = build_dictionary(x)
    C, Lc = ppe_numerical(Q)
    K = int(Lc.max())
    assert K >= 3
    P = padded(C[rank], Lc[rank], K)
    Lr = Lc[rank]
    cols = device_columns(x, 16, layouts=("ppvbs",))
    try:
        col = cols["ppvbs"][1]
        picks = [int(np.flatnonzero(Lc == L)[i]) for L in (1, 2, 3) for i in (0, 5)]
        for k in picks:
            for op in ("lt", "gt", "eq"):
                if (op == "lt" and k == 0) or (op == "gt" and k == len(A) - 1):
                    continue
                _, ctr = col.scan_stats(op, int(A[k]))
                torch.cuda.synchronize()
                ctr = ctr.cpu().numpy()
                want = _expected_touch(P, Lr, K, int(C[k]), int(Lc[k]), op)
                assert (int(ctr[0]), int(ctr[4])) == want, (k, int(Lc[k]), op)
    finally:
        close_columns(cols)


def test_repeatable():
    n = 500_000
    x = datagen.zipf_column(n, 20, 1.0, seed=77)
    cols = device_columns(x, 20)
    try:
        for lay, (hc, col) in cols.items():
            a = _bv(col.scan("between", 1000, 900_000))
            for _ in range(3):
                assert np.array_equal(_bv(col.scan("between", 1000, 900_000)), a), lay
    finally:
        close_columns(cols)


@pytest.mark.parametrize("grid,gather", [(1, 0), (3, 1), (3, 4), (1, 2)])
def test_scan_parity_many_tiles_per_wave(grid, gather):
    """A tiny launch (grid workgroups of 4 waves) gives each wave from two to
    nine tiles, odd and even counts, so every prefetch slot of the tile
    rotation and of the deferred level-2 reads holds a tile at some point and
    the slots past a wave's last tile are exercised; the gather limit switches
    later levels between the run staged in LDS (0: whenever a row is pending)
    and per-row gathers (up to 1, 2 or 4 pending rows per lane)."""
    from paper_2209_00220_amd import _lib as L
    from paper_2209_00220_amd.column import bv_from_numpy

    flush("scan parity with grid=%d gather=%d" % (grid, gather))
    saved = (L.bst_tune_get(L.TUNE_SCAN_GRID), L.bst_tune_get(L.TUNE_GATHER_ROWS))
    L.bst_tune_set(L.TUNE_SCAN_GRID, grid)
    L.bst_tune_set(L.TUNE_GATHER_ROWS, gather)
    try:
        for n, w, s in ((2048 * 9 + 5, 20, 1.0), (2048 * 14, 16, 0.5), (70_001, 24, 1.2)):
            x = datagen.zipf_column(n, w, s, seed=3 * n + w)
            A, _, _ = build_dictionary(x)
            cols = device_columns(x, w)
            mask_np = datagen.random_mask_words(n, seed=n + 7, density=0.5)
            mask_t = bv_from_numpy(mask_np)
            mask_rows = unpack_bits(mask_np, n)
            lits = literal_set(A, w)[::2]
            try:
                for lay, (hc, col) in cols.items():
                    for op in ("lt", "gt", "eq", "ne", "between"):
                        for i, lo in enumerate(lits):
                            hi = lits[(i * 5 + 3) % len(lits)] if op == "between" else None
                            for msk in (None, mask_t):
                                got = _bv(col.scan(op, lo, hi, in_mask=msk))
                                want = scan_values_bv(x, op, lo, hi, None if msk is None else mask_rows)
                                assert np.array_equal(got, want), (n, lay, op, lo, hi, msk is not None)
            finally:
                close_columns(cols)
    finally:
        L.bst_tune_set(L.TUNE_SCAN_GRID, saved[0])
        L.bst_tune_set(L.TUNE_GATHER_ROWS, saved[1])


@pytest.mark.parametrize("w,sigma_exp", [(12, 0.25), (12, 0.5), (12, 0.75), (20, 0.25), (20, 0.5), (20, 0.75)])
def test_gaussian_columns(w, sigma_exp):
    """The sensitivity sweep's Gaussian inputs (mean at the domain's centre,
    sigma = 2^(w/4), 2^(w/2), 2^(3w/4), rounded and clipped): every layout and
    operator against the plain comparison, with and without an incoming mask."""
    from paper_2209_00220_amd.column import bv_from_numpy

    n = 150_001
    sigma = 2.0 ** (w * sigma_exp)
    flush("gaussian w=%d sigma=2^%.2f" % (w, w * sigma_exp))
    x = datagen.gaussian_column(n, w, sigma, seed=31 * w + int(4 * sigma_exp))
    A, _, _ = build_dictionary(x)
    cols = device_columns(x, w)
    mask_np = datagen.random_mask_words(n, seed=w + 5, density=0.5)
    mask_t = bv_from_numpy(mask_np)
    mask_rows = unpack_bits(mask_np, n)
    lits = literal_set(A, w)
    try:
        for lay, (hc, col) in cols.items():
            for op in OPS:
                for i, lo in enumerate(lits):
                    hi = lits[(i * 5 + 3) % len(lits)] if op == "between" else None
                    for msk in (None, mask_t):
                        got = _bv(col.scan(op, lo, hi, in_mask=msk))
                        want = scan_values_bv(x, op, lo, hi, None if msk is None else mask_rows)
                        assert np.array_equal(got, want), (lay, op, lo, hi, msk is not None)
    finally:
        close_columns(cols)
