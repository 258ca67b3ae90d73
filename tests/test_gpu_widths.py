"""Fixed-width layouts at every code width, rank-mode columns and six-byte codes,
through the C ABI against the plain definition (Sec. 2.2; Sec. 2.3, 2.5; Sec. 3.1).

* Bit-Packed and ByteSlice columns of every width w = 1..32 (domain mode: the
  code is the value), each scanned with every operator, with and without an
  incoming mask, by the single-column kernels and by one batched launch.
* ByteSlice and Bit-Packed in dictionary (rank) mode, whose literals go
  through the rank rewrite.
* PP-VBS columns built from explicit codes of up to six bytes (the longest a
  code gets), with literals of every length: the scan in code space must equal
  the comparison of the zero-padded codes as integers (Sec. 3.1's order).
"""
import numpy as np
import pytest
import torch

import datagen
from helpers import close_columns, device_columns, flush, literal_set
from oracle.dictionary import build_dictionary
from oracle.layout import pack_bits, unpack_bits
from oracle.ppe import padded
from oracle.scan import OPS, scan_padded_codes, scan_values_bv

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


def _width_column(n, w, seed):
    # Zipf(1.0) over the whole w-bit domain: every code width is exercised at its
    # extremes (values 0 and 2^w - 1 come in through the literal set)
    return datagen.zipf_column(n, w, 1.0 if w > 1 else 0.0, seed=seed)


@pytest.mark.parametrize("w", list(range(1, 33)))
def test_fixed_width_scans_every_width(w):
    from paper_2209_00220_amd.batch import Batch
    from paper_2209_00220_amd.column import bv_from_numpy

    n = 2048 * 3 + 77   # several tiles and a ragged tail
    flush("width sweep w=%d" % w)
    x = _width_column(n, w, seed=500 + w)
    A, _, _ = build_dictionary(x)
    cols = device_columns(x, w, layouts=("bitpacked", "byteslice"))
    mask_np = datagen.random_mask_words(n, seed=600 + w, density=0.5)
    mask_t = bv_from_numpy(mask_np)
    mask_rows = unpack_bits(mask_np, n)
    lits = literal_set(A, w)
    lits = lits[:: max(1, len(lits) // 8)] + [lits[-1]]
    try:
        specs, outs, wants = [], [], []
        for lay, (hc, col) in cols.items():
            assert hc.info.width_bits == w
            for op in OPS:
                for i, lo in enumerate(lits):
                    hi = lits[(i * 3 + 2) % len(lits)] if op == "between" else None
                    for msk in (None, mask_t):
                        want = scan_values_bv(x, op, lo, hi, None if msk is None else mask_rows)
                        got = _bv(col.scan(op, lo, hi, in_mask=msk))
                        assert np.array_equal(got, want), (lay, w, op, lo, hi, msk is not None)
                        specs.append((col, op, lo, hi, msk))
                        outs.append(col.new_bv())
                        wants.append(want)
        # the same scans as one batched launch (one persistent kernel per width group)
        b = Batch(specs, outs)
        b.launch(grid=0, tiles_per_grab=1, use_graph=False)
        torch.cuda.synchronize()
        for (col, op, lo, hi, msk), o, want in zip(specs, outs, wants):
            assert np.array_equal(_bv(o), want), ("batch", w, op, lo, hi, msk is not None)
        b.close()
    finally:
        close_columns(cols)


@pytest.mark.parametrize("n,w,s", [(70_001, 12, 1.0), (2049, 20, 0.5), (300_000, 24, 1.5), (5000, 32, 0.0)])
def test_rank_mode_scans(n, w, s):
    """ByteSlice and Bit-Packed over dictionary ranks (width = bits for the
    distinct count), every operator, literals present, absent and out of range."""
    from paper_2209_00220_amd.column import bv_from_numpy

    flush("rank mode n=%d w=%d s=%g" % (n, w, s))
    x = datagen.zipf_column(n, w, s, seed=7 * n + w)
    A, _, _ = build_dictionary(x)
    cols = device_columns(x, w, layouts=("byteslice", "bitpacked"), domain=False)
    mask_np = datagen.random_mask_words(n, seed=n + 3, density=0.3)
    mask_t = bv_from_numpy(mask_np)
    mask_rows = unpack_bits(mask_np, n)
    lits = literal_set(A, w)
    try:
        for lay, (hc, col) in cols.items():
            assert hc.info.domain_mode == 0 and (1 << hc.info.width_bits) >= len(A)
            for op in OPS:
                for i, lo in enumerate(lits):
                    hi = lits[(i * 5 + 3) % len(lits)] if op == "between" else None
                    for msk in (None, mask_t):
                        got = _bv(col.scan(op, lo, hi, in_mask=msk))
                        want = scan_values_bv(x, op, lo, hi, None if msk is None else mask_rows)
                        assert np.array_equal(got, want), (lay, op, lo, hi, msk is not None)
    finally:
        close_columns(cols)


def _six_byte_codes(n_codes, seed):
    """Distinct codes of 1..6 bytes whose last byte is non-zero (so a code that is
    a proper prefix of another leaves a non-zero remainder), over a four-letter
    alphabet for the inner bytes: long runs of rows share prefixes, and scans
    reach every level up to the sixth byte."""
    rng = np.random.default_rng(seed)
    alphabet = np.array([0, 1, 0x7F, 0xFF], dtype=np.uint64)
    seen, codes, lens = set(), [], []
    while len(codes) < n_codes:
        L = int(rng.integers(1, 7))
        body = alphabet[rng.integers(0, 4, size=L - 1)]
        last = int(rng.choice([1, 2, 0x80, 0xFF]))
        c = 0
        for b in body:
            c = (c << 8) | int(b)
        c = (c << 8) | last
        if (c, L) in seen:
            continue
        seen.add((c, L))
        codes.append(c)
        lens.append(L)
    return np.array(codes, dtype=np.uint64), np.array(lens, dtype=np.uint8)


def test_six_byte_codes_every_level():
    from paper_2209_00220_amd.column import DeviceColumn, HostColumn, bv_from_numpy

    n = 2048 * 7 + 333
    flush("six-byte codes, n=%d" % n)
    dc, dl = _six_byte_codes(400, seed=6)
    rng = np.random.default_rng(66)
    pick = rng.zipf(1.3, size=n) % dc.shape[0]
    codes, lens = dc[pick], dl[pick]
    hc = HostColumn.from_codes(codes, lens, 6)
    assert hc.info.k_max == 6
    col = DeviceColumn(hc)
    P = padded(codes, lens.astype(np.int64), 6)
    mask_np = datagen.random_mask_words(n, seed=67, density=0.5)
    mask_t = bv_from_numpy(mask_np)
    mask_rows = unpack_bits(mask_np, n)
    # literals: stored codes of every length plus codes absent from the column
    lit_codes, lit_lens = _six_byte_codes(60, seed=7)
    lits = list(zip(dc[:40].tolist(), dl[:40].tolist())) + list(zip(lit_codes.tolist(), lit_lens.tolist()))
    try:
        for op in OPS:
            for i, (c, l) in enumerate(lits):
                pc = int(padded([c], [l], 6)[0])
                hc2, hl2 = lits[(i * 7 + 3) % len(lits)]
                ph = int(padded([hc2], [hl2], 6)[0])
                for msk in (None, mask_t):
                    got = _bv(col.scan_codes(op, c, l, hc2, hl2, in_mask=msk))
                    want = pack_bits(scan_padded_codes(P, op, pc, ph if op == "between" else None,
                                                       None if msk is None else mask_rows))
                    assert np.array_equal(got, want), (op, hex(c), l, hex(hc2), hl2, msk is not None)
    finally:
        col.close()
        hc.close()
