"""bst_lookup_bv_static (no caller-provided device memory) against bst_lookup_bv:
the same values and counts through the C ABI, on two calls in a row, the second
with a smaller column and a smaller capacity, for every layout."""
import numpy as np
import pytest
import torch

import datagen
from helpers import close_columns, device_columns, flush

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu(built_lib):
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    torch.cuda.set_device(0)
    yield
    torch.cuda.synchronize()


def _static_lookup(col, bv, cap):
    from paper_2209_00220_amd import _lib as L

    vals = torch.full((max(cap, 1),), -1, dtype=torch.int32, device="cuda")
    count = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    L.bst_lookup_bv_static(col.h, bv, vals, cap, count, status, 0)
    torch.cuda.synchronize()
    return vals.cpu().numpy().view(np.uint32), int(count.item()), int(status.item())


def test_static_lookup_matches_workspace_lookup():
    from paper_2209_00220_amd import _lib as L
    from paper_2209_00220_amd.column import u32_to_numpy

    assert L.bst_lookup_bv_static_max_rows() == 1 << 29
    assert L.bst_lookup_bv_static_max_ids() == 1 << 21
    # a large call first, then a smaller column with a smaller capacity: the
    # second must not see anything the first left in the shared array
    for n, w, lit, cap_extra in ((1_500_007, 20, 300_000, 5), (70_001, 12, 700, 0)):
        flush("static lookup n=%d" % n)
        x = datagen.zipf_column(n, w, 1.0, seed=n)
        cols = device_columns(x, w)
        try:
            for lay, (hc, col) in cols.items():
                bv = col.scan("lt", lit)
                want_rows = np.nonzero(x < lit)[0]
                cap = int(want_rows.shape[0]) + cap_extra
                ref_vals, ref_count = col.lookup_bv(bv, cap)
                torch.cuda.synchronize()
                got, count, status = _static_lookup(col, bv, cap)
                assert count == int(ref_count.item()) == want_rows.shape[0], lay
                assert status == 0
                assert np.array_equal(got[:count], u32_to_numpy(ref_vals)[:count]), lay
                assert np.array_equal(got[:count], x[want_rows]), lay
                # capacity below the count: the first cap values and the overflow flag
                small = max(1, count // 3)
                got2, count2, status2 = _static_lookup(col, bv, small)
                assert count2 == count and status2 & L.BST_DEV_OVERFLOW
                assert np.array_equal(got2[:small], x[want_rows[:small]]), lay
        finally:
            close_columns(cols)


def test_static_lookup_rejects_oversized_capacity():
    from paper_2209_00220_amd import _lib as L

    x = datagen.zipf_column(10_000, 12, 1.0, seed=5)
    cols = device_columns(x, 12, layouts=("ppvbs",))
    try:
        col = cols["ppvbs"][1]
        bv = col.scan("lt", 100)
        with pytest.raises(L.BstError):
            _static_lookup(col, bv, (1 << 21) + 1)
    finally:
        close_columns(cols)
