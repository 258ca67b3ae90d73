"""The benchmark workload at full size (500M rows, 20-bit Zipf(1.0) values), through
the same launch configuration the benchmark times.

Every result bitvector is compared in full, all 62.5 MB of it, with the plain
comparison on the raw values (Sec. 2.2's predicate), computed once per predicate
and shared by the three layouts; its popcount must also equal the count from
the value histogram, sum over distinct values v of count(v) * [v op literal].
Lookups of the 5M row IDs are compared in full with the raw values.
"""
import numpy as np
import pytest
import torch

from helpers import flush
from oracle.lookup import lookup_ids
from oracle.scan import scan_values, scan_values_bv

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
    yield {"x": x, "v": v, "c": c, "preds": wl["preds"], "ids": wl["ids"], "ids_t": u32_from_numpy(wl["ids"]),
           "cols": cols, "want": {}}
    for hc, dc in cols.values():
        dc.close()
        hc.close()
    torch.cuda.synchronize()


def _want(w, key, op, lo, hi, in_mask=None):
    """The plain result bitvector of a predicate on all N raw values (cached)."""
    if key not in w["want"]:
        w["want"][key] = scan_values_bv(w["x"], op, lo, hi, in_mask)
    return w["want"][key]


@pytest.mark.parametrize("layout", LAYOUTS)
def test_fullsize_scans(workload, layout):
    from paper_2209_00220_amd.column import bv_to_numpy

    w = workload
    col = w["cols"][layout][1]
    out = col.new_bv()
    for i, (op, lo, hi, _) in enumerate(w["preds"]):
        flush("full-size %s pred %d: %s %s %s" % (layout, i, op, lo, hi))
        col.scan(op, lo, hi, out=out)
        got = bv_to_numpy(out)
        want_count = int(w["c"][scan_values(w["v"], op, lo, hi)].sum())
        assert int(np.bitwise_count(got).sum()) == want_count, (op, lo, hi)
        assert np.array_equal(got, _want(w, i, op, lo, hi)), (op, lo, hi)
        # conjunction: x >= lo pipelined into x < lo + 1000
        if i == 7:
            col.scan("ge", lo, out=out)
            prev = out.clone()
            col.scan("lt", lo + 1000, in_mask=prev, out=out)
            got = bv_to_numpy(out)
            keep = scan_values(w["v"], "ge", lo) & scan_values(w["v"], "lt", lo + 1000)
            assert int(np.bitwise_count(got).sum()) == int(w["c"][keep].sum())
            assert np.array_equal(got, _want(w, "conj", "between", lo, lo + 999)), "conjunction"


@pytest.mark.parametrize("layout", LAYOUTS)
def test_fullsize_lookup(workload, layout):
    from paper_2209_00220_amd.column import u32_to_numpy

    w = workload
    flush("full-size %s lookup of %d ids" % (layout, w["ids"].shape[0]))
    got = u32_to_numpy(w["cols"][layout][1].lookup(w["ids_t"]))
    assert np.array_equal(got, lookup_ids(w["x"], w["ids"]))
