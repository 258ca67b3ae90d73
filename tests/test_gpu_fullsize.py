"""The benchmark workload at full size (500M rows, 20-bit Zipf(1.0) values), through
the same launch configuration the benchmark times.

The oracle cannot scan 500M rows one by one in test time, so each scan is checked
by properties that hold at any size plus sampled rows:
  * popcount of the result equals the plain count, sum over distinct values v of
    count(v) * [v op literal] (Sec. 2.2's predicate on the raw values);
  * 2M random rows, the first 64k rows and the last (ragged) tile agree bit for bit
    with the plain comparison on the raw values;
  * tail bits past row n are zero.
Lookups of the 5M row IDs are compared in full with the raw values.
"""
import numpy as np
import pytest
import torch

from helpers import flush
from oracle.lookup import lookup_ids
from oracle.scan import scan_values

pytestmark = pytest.mark.gpu

N = 500_000_000
LAYOUTS = ("ppvbs", "byteslice", "bitpacked")


@pytest.fixture(scope="module")
def workload(built_lib):
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    torch.cuda.set_device(0)
    from datagen import workloads
    from paper_2209_00220_amd.column import DeviceColumn, Dictionary, HostColumn, u32_from_numpy

    flush("full-size workload: generating %d rows" % N)
    wl = workloads.config2(N)
    x = wl["x"]
    v, c = workloads.value_counts(x, 20)
    d = Dictionary(x)
    cols = {}
    for lay in LAYOUTS:
        flush("full-size workload: encode + upload %s" % lay)
        hc = HostColumn.encode(d, lay, width=0 if lay == "ppvbs" else 20)
        cols[lay] = (hc, DeviceColumn(hc))
    d.close()
    rng = np.random.default_rng(7)
    sample = np.concatenate([np.arange(65536), np.arange(N - 3000, N), rng.integers(0, N, 2_000_000)])
    yield {"x": x, "v": v, "c": c, "preds": wl["preds"], "ids": wl["ids"], "ids_t": u32_from_numpy(wl["ids"]),
           "cols": cols, "sample": sample}
    for hc, dc in cols.values():
        dc.close()
        hc.close()
    torch.cuda.synchronize()


def _bits(words, rows):
    return ((words[rows >> 6] >> (rows & 63).astype(np.uint64)) & np.uint64(1)).astype(bool)


@pytest.mark.parametrize("layout", LAYOUTS)
def test_fullsize_scans(workload, layout):
    from paper_2209_00220_amd.column import bv_to_numpy

    w = workload
    col = w["cols"][layout][1]
    out = col.new_bv()
    xs = w["x"][w["sample"]]
    for i, (op, lo, hi, _) in enumerate(w["preds"]):
        flush("full-size %s pred %d: %s %s %s" % (layout, i, op, lo, hi))
        col.scan(op, lo, hi, out=out)
        got = bv_to_numpy(out)
        want_count = int(w["c"][scan_values(w["v"], op, lo, hi)].sum())
        assert int(np.bitwise_count(got).sum()) == want_count, (op, lo, hi)
        assert np.array_equal(_bits(got, w["sample"]), scan_values(xs, op, lo, hi)), (op, lo, hi)
        # conjunction: this predicate restricted by the previous one's complement
        if i == 7:
            col.scan("ge", lo, out=out)
            prev = out.clone()
            col.scan("lt", lo + 1000, in_mask=prev, out=out)
            got = bv_to_numpy(out)
            want = scan_values(xs, "ge", lo) & scan_values(xs, "lt", lo + 1000)
            assert np.array_equal(_bits(got, w["sample"]), want)
            keep = scan_values(w["v"], "ge", lo) & scan_values(w["v"], "lt", lo + 1000)
            assert int(np.bitwise_count(got).sum()) == int(w["c"][keep].sum())


@pytest.mark.parametrize("layout", LAYOUTS)
def test_fullsize_lookup(workload, layout):
    from paper_2209_00220_amd.column import u32_to_numpy

    w = workload
    flush("full-size %s lookup of %d ids" % (layout, w["ids"].shape[0]))
    got = u32_to_numpy(w["cols"][layout][1].lookup(w["ids_t"]))
    assert np.array_equal(got, lookup_ids(w["x"], w["ids"]))
