"""Randomised parity: 40 seeded column configurations drawn across the input
space (length 1..40,000 rows; code width 1..32; Zipf skew 0..2; scattered or
sorted value mapping; domain or rank codes for the fixed-width layouts; PP-VBS
directory strides 64..2048), each scanned with random operators and literals,
with and without a random incoming mask, and looked up at random row IDs.
Every result is compared whole with the plain definition on the raw values."""
import numpy as np
import pytest
import torch

import datagen
from helpers import close_columns, flush
from oracle.layout import unpack_bits
from oracle.lookup import lookup_ids
from oracle.scan import OPS, scan_values_bv

pytestmark = pytest.mark.gpu

N_CASES = 40


@pytest.fixture(scope="module", autouse=True)
def _gpu(built_lib):
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    torch.cuda.set_device(0)
    yield
    torch.cuda.synchronize()


def _case(k):
    rng = np.random.default_rng(9000 + k)
    n = int(rng.integers(1, 40_001))
    w = int(rng.integers(1, 33))
    s = float(rng.choice([0.0, 0.5, 1.0, 1.5, 2.0]))
    mapping = int(rng.integers(0, 2))
    domain = bool(rng.integers(0, 2))
    stride = int(2 ** rng.integers(6, 12))
    return rng, n, w, s, mapping, domain, stride


@pytest.mark.parametrize("k", range(N_CASES))
def test_random_configuration(k):
    from paper_2209_00220_amd.column import (DeviceColumn, Dictionary, HostColumn, bv_from_numpy, bv_to_numpy,
                                             u32_from_numpy, u32_to_numpy)

    rng, n, w, s, mapping, domain, stride = _case(k)
    flush("random case %d: n=%d w=%d s=%g mapping=%d domain=%s stride=%d" % (k, n, w, s, mapping, domain, stride))
    x = datagen.zipf_column(n, w, s, seed=9100 + k, mapping=mapping)
    d = Dictionary(x)
    cols = {}
    for lay in ("ppvbs", "byteslice", "bitpacked"):
        width = w if (domain and lay != "ppvbs") else 0
        hc = HostColumn.encode(d, lay, width=width, dir_stride=stride if lay == "ppvbs" else 0)
        cols[lay] = (hc, DeviceColumn(hc))
    d.close()
    mask_np = datagen.random_mask_words(n, seed=9200 + k, density=float(rng.uniform(0.05, 0.95)))
    mask_t = bv_from_numpy(mask_np)
    mask_rows = unpack_bits(mask_np, n)
    ids = rng.integers(0, n, size=min(n, 3000)).astype(np.uint32)
    want_vals = lookup_ids(x, ids)
    try:
        for _ in range(6):
            op = OPS[int(rng.integers(0, len(OPS)))]
            # literals: present values, their neighbours, and the domain's edges
            pick = lambda: int(rng.choice([x[int(rng.integers(0, n))], x[int(rng.integers(0, n))] + 1,
                                           max(int(x[int(rng.integers(0, n))]) - 1, 0), 0, (1 << w) - 1,
                                           (1 << w), 2 ** 32 - 1])) & 0xFFFFFFFF
            lo, hi = pick(), pick()
            if op == "between" and lo > hi and rng.random() < 0.8:
                lo, hi = hi, lo
            for msk in (None, mask_t):
                want = scan_values_bv(x, op, lo, hi if op == "between" else None,
                                      None if msk is None else mask_rows)
                for lay, (hc, col) in cols.items():
                    got = bv_to_numpy(col.scan(op, lo, hi if op == "between" else None, in_mask=msk))
                    assert np.array_equal(got, want), (k, lay, op, lo, hi, msk is not None)
        for lay, (hc, col) in cols.items():
            got = u32_to_numpy(col.lookup(u32_from_numpy(ids)))
            assert np.array_equal(got, want_vals), (k, lay)
    finally:
        torch.cuda.synchronize()
        close_columns(cols)
