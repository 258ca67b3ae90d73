"""A PP-VBS column of the largest size the ABI takes: 2^32 - 1 rows (row IDs are
uint32), 20-bit Zipf(1.0) values.  Row positions past 2^31 and up to the last
row exercise every 64-bit offset of the scan, lookup and compaction paths.

The plain definition is checked where it can be computed cheaply at this size:
every scan's popcount equals the count from the value histogram; the result
bits of the first, middle (around 2^31) and last 70,000 rows and of 2M random
rows equal the comparison on the raw values, and the tail bits past the last
row are zero; lookups of the extreme and 1M random IDs equal the raw values;
the compaction of a rare '=' result equals the positions of that value.
"""
import numpy as np
import pytest
import torch

import datagen
from helpers import flush
from oracle.scan import scan_values

pytestmark = pytest.mark.gpu

N = (1 << 32) - 1


@pytest.fixture(scope="module")
def big(built_lib):
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    torch.cuda.set_device(0)
    from datagen import workloads
    from paper_2209_00220_amd.column import DeviceColumn, Dictionary, HostColumn

    flush("max size: generating %d rows" % N)
    x = datagen.zipf_column(N, 20, 1.0, seed=77)
    flush("max size: value counts")
    v, c = workloads.value_counts(x, 20)
    flush("max size: dictionary and PP-VBS encoding")
    d = Dictionary(x)
    hc = HostColumn.encode(d, "ppvbs")
    d.close()
    flush("max size: upload (%.2f GB)" % (hc.info.total_bytes / 1e9))
    col = DeviceColumn(hc)
    torch.cuda.synchronize()
    rng = np.random.default_rng(78)
    sample = np.unique(np.concatenate([
        np.arange(0, 70_000), np.arange((1 << 31) - 70_000, (1 << 31) + 70_000), np.arange(N - 70_000, N),
        rng.integers(0, N, size=2_000_000)]).astype(np.uint64))
    yield {"x": x, "v": v, "c": c, "col": col, "sample": sample}
    col.close()
    hc.close()
    torch.cuda.synchronize()


def _bits(words, rows):
    return ((words[(rows >> 6).astype(np.int64)] >> (rows & 63)) & 1).astype(bool)


def _check(w, out, op, lo, hi, keep_values, prior=None):
    from paper_2209_00220_amd.column import bv_popcount, bv_to_numpy

    want_count = int(w["c"][keep_values].sum())
    assert int(bv_popcount(out, N).item()) == want_count, (op, lo, hi)
    words = bv_to_numpy(out)
    assert words.shape[0] == (N + 63) // 64
    assert int(words[-1]) >> (N % 64) == 0, "tail bits past the last row"
    rows = w["sample"]
    want = scan_values(w["x"][rows], op, lo, hi)
    if prior is not None:
        want &= prior
    assert np.array_equal(_bits(words, rows), want), (op, lo, hi)
    return words


def test_maxsize_scans_and_conjunction(big):
    from datagen import workloads

    w = big
    col = w["col"]
    v, c = w["v"], w["c"]
    lt, _ = workloads.lit_lt(v, c, 0.10)
    eq, _ = workloads.lit_eq(v, c, 0.01)
    blo, bhi, _ = workloads.lit_between(v, c, 0.5)
    flush("max size: '<' %d" % lt)
    out_lt = col.scan("lt", lt)
    words_lt = _check(w, out_lt, "lt", lt, None, v < lt)
    flush("max size: '=' %d" % eq)
    _check(w, col.scan("eq", eq), "eq", eq, None, v == eq)
    flush("max size: BETWEEN %d..%d" % (blo, bhi))
    _check(w, col.scan("between", blo, bhi), "between", blo, bhi, (v >= blo) & (v <= bhi))
    flush("max size: BETWEEN within '<' (incoming mask)")
    prior = _bits(words_lt, w["sample"])
    _check(w, col.scan("between", blo, bhi, in_mask=out_lt), "between", blo, bhi,
           (v < lt) & (v >= blo) & (v <= bhi), prior=prior)


def test_maxsize_lookups(big):
    from paper_2209_00220_amd.column import u32_from_numpy, u32_to_numpy

    w = big
    rng = np.random.default_rng(79)
    ids = np.concatenate([np.array([0, 1, (1 << 31) - 1, 1 << 31, (1 << 31) + 1, N - 2, N - 1], dtype=np.uint64),
                          rng.integers(0, N, size=1_000_000).astype(np.uint64)]).astype(np.uint32)
    flush("max size: %d lookups" % ids.shape[0])
    got = u32_to_numpy(w["col"].lookup(u32_from_numpy(ids)))
    assert np.array_equal(got, w["x"][ids.astype(np.int64)])


def test_maxsize_compaction_of_a_rare_value(big):
    from paper_2209_00220_amd.column import bv_compact

    w = big
    v, c = w["v"], w["c"]
    # a value with a few hundred thousand rows, spread over the whole column
    k = int(np.argmin(np.abs(c - 300_000)))
    lit, cnt = int(v[k]), int(c[k])
    flush("max size: '=' %d (%d rows), compaction and lookup of its rows" % (lit, cnt))
    out = w["col"].scan("eq", lit)
    ids, count = bv_compact(out, N, cnt)
    torch.cuda.synchronize()
    assert int(count.item()) == cnt
    got_ids = ids.cpu().numpy().view(np.uint32)[:cnt]
    want_ids = np.flatnonzero(w["x"] == lit).astype(np.uint32)
    assert np.array_equal(got_ids, want_ids)
    assert int(want_ids[-1]) > (1 << 31)
    vals, vcount = w["col"].lookup_bv(out, cnt)
    torch.cuda.synchronize()
    assert int(vcount.item()) == cnt
    assert np.all(vals.cpu().numpy().view(np.uint32)[:cnt] == lit)
