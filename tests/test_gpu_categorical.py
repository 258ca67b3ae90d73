"""PP-VBS over the categorical PPE (Algorithm 2): '=' and '!=' scans and lookups
through the C ABI against the plain definition; range operators are refused."""
import numpy as np
import pytest
import torch

import datagen
from helpers import flush, literal_set
from oracle.layout import pack_bits
from oracle.lookup import lookup_ids
from oracle.scan import scan_values

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu(built_lib):
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    torch.cuda.set_device(0)
    yield
    torch.cuda.synchronize()


CASES = [
    (1, 8, 1.0), (2047, 8, 0.0), (100_003, 12, 1.0), (250_000, 20, 1.0), (300_000, 24, 0.0), (70_001, 17, 0.7),
]


@pytest.mark.parametrize("n,w,s", CASES)
def test_categorical_eq_ne_and_lookup(n, w, s):
    from paper_2209_00220_amd import _lib as L
    from paper_2209_00220_amd.column import DeviceColumn, Dictionary, HostColumn, bv_from_numpy, bv_to_numpy, u32_from_numpy, u32_to_numpy

    x = datagen.zipf_column(n, w, s, seed=n + w)
    flush("categorical n=%d w=%d s=%.1f" % (n, w, s))
    d = Dictionary(x)
    hc = HostColumn.encode(d, "ppvbs_categorical")
    A, _ = d.values_counts()
    d.close()
    col = DeviceColumn(hc)
    try:
        assert int(hc.info.categorical) == 1
        rng = np.random.default_rng(n)
        in_np = rng.random(n) < 0.5
        in_t = bv_from_numpy(pack_bits(in_np))
        for lit in literal_set(A, w):
            for op in ("eq", "ne"):
                got = bv_to_numpy(col.scan(op, lit))
                assert np.array_equal(got, pack_bits(scan_values(x, op, lit))), (op, lit)
                got = bv_to_numpy(col.scan(op, lit, in_mask=in_t))
                assert np.array_equal(got, pack_bits(scan_values(x, op, lit, in_mask=in_np))), (op, lit, "in")
        ids = rng.integers(0, n, size=min(n, 50_000)).astype(np.uint32)
        assert np.array_equal(u32_to_numpy(col.lookup(u32_from_numpy(ids))), lookup_ids(x, ids))
        for op in ("lt", "le", "gt", "ge", "between"):
            with pytest.raises(L.BstError):
                col.scan(op, int(A[0]), int(A[-1]))
    finally:
        col.close()
        hc.close()
