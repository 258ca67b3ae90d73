"""A PP-VBS column with more than 2^28 distinct values (Sec. 3.1, Algorithm 1;
Sec. 3.3's scan and lookup).

Every value occurs once, so Algorithm 1's 255 largest frequencies tie and the
smallest values take the slots: the 255 smallest get one-byte codes at the
root, the next 255 two-byte codes under the root's last pointer, and the rest
six-byte codes (a leaf past the depth cut with four-digit slot numbers).  With
this many distinct values the decode tables' leaf entries carry no length, so
every lookup of a code shorter than six bytes reads M_{L+1} to see it end (the
column info reports that), and the six-byte codes run the scan and the lookup
at the largest K.

Checked against the plain definition: every result bit of the scans, the
lookups of every short-code row, of the extremes and of 2M random rows.
"""
import numpy as np
import pytest
import torch

from helpers import flush
from oracle.scan import scan_values_bv

pytestmark = pytest.mark.gpu

N = (1 << 28) + (1 << 20)


@pytest.fixture(scope="module")
def col(built_lib):
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    torch.cuda.set_device(0)
    from paper_2209_00220_amd.column import DeviceColumn, Dictionary, HostColumn

    flush("many distinct: %d rows, every value distinct" % N)
    # r -> r * odd mod 2^32 is a bijection: N distinct values spread over 32 bits
    x = (np.arange(N, dtype=np.uint64) * np.uint64(2654435761) & np.uint64(0xFFFFFFFF)).astype(np.uint32)
    flush("many distinct: dictionary")
    d = Dictionary(x)
    flush("many distinct: PP-VBS encoding")
    hc = HostColumn.encode(d, "ppvbs")
    d.close()
    flush("many distinct: upload (%.2f GB)" % (hc.info.total_bytes / 1e9))
    dc = DeviceColumn(hc)
    torch.cuda.synchronize()
    sorted_vals = np.sort(x[np.argpartition(x, 520)[:521]])   # the 521 smallest values
    yield {"x": x, "hc": hc, "col": dc, "small": sorted_vals}
    dc.close()
    hc.close()
    torch.cuda.synchronize()


def test_many_distinct_code_shape(col):
    info = col["hc"].info
    assert info.n_distinct == N and info.n_distinct >= (1 << 28)
    assert info.k_max == 6
    assert [int(info.rows_by_len[j]) for j in range(7)] == [0, 255, 255, 0, 0, 0, N - 510]
    # no length-carrying leaves: every code shorter than K ends at a 0 of M_{L+1}
    assert [int(info.rows_end_by_mask[j]) for j in range(7)] == [0, 255, 255, 0, 0, 0, 0]


def test_many_distinct_lookups(col):
    from paper_2209_00220_amd.column import u32_from_numpy, u32_to_numpy

    x = col["x"]
    rng = np.random.default_rng(90)
    short_rows = np.flatnonzero(x <= col["small"][509]).astype(np.uint64)   # the 510 one- and two-byte codes
    assert short_rows.shape[0] == 510
    ids = np.concatenate([short_rows, np.array([0, 1, N - 2, N - 1], dtype=np.uint64),
                          rng.integers(0, N, size=2_000_000).astype(np.uint64)]).astype(np.uint32)
    flush("many distinct: %d lookups" % ids.shape[0])
    got = u32_to_numpy(col["col"].lookup(u32_from_numpy(ids)))
    assert np.array_equal(got, x[ids.astype(np.int64)])


@pytest.mark.parametrize("op,k_lo,k_hi", [
    ("lt", 200, None),        # a one-byte literal
    ("le", 300, None),        # a two-byte literal
    ("eq", 509, None),        # the last two-byte code
    ("eq", 520, None),        # a six-byte code
    ("between", 100, 400),    # one-byte to two-byte
    ("lt", None, None),       # the median value: every row tied on bytes 1 and 2
])
def test_many_distinct_scans(col, op, k_lo, k_hi):
    from paper_2209_00220_amd.column import bv_to_numpy

    x = col["x"]
    lo = int(col["small"][k_lo]) if k_lo is not None else int(np.partition(x[::4096], x[::4096].shape[0] // 2)[
        x[::4096].shape[0] // 2])
    hi = int(col["small"][k_hi]) if k_hi is not None else None
    flush("many distinct: %s %d %s" % (op, lo, hi))
    got = bv_to_numpy(col["col"].scan(op, lo, hi))
    torch.cuda.synchronize()
    assert np.array_equal(got, scan_values_bv(x, op, lo, hi)), (op, lo, hi)
