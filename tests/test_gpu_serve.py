"""The serving loop on the GPU: batched scan steps and lookups through the C ABI
give every query the plain result (Sec. 2.2) on the raw values, in a mix and alone."""
import numpy as np
import pytest
import torch

import datagen
from helpers import flush
from oracle.scan import scan_values

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def served(built_lib):
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    torch.cuda.set_device(0)
    from paper_2209_00220_amd.column import DeviceColumn, Dictionary, HostColumn

    raw, tables, keep = {}, {}, []
    spec = {"t0": (300_001, [(12, 1.0), (20, 0.5), (16, 1.5)]), "t1": (130_000, [(8, 0.0), (24, 1.0)])}
    layouts = ["ppvbs", "byteslice", "bitpacked"]
    for ti, (t, (n, cols)) in enumerate(spec.items()):
        raw[t], tables[t] = {}, {}
        for ci, (w, s) in enumerate(cols):
            x = datagen.zipf_column(n, w, s, seed=50 + 10 * ti + ci)
            lay = layouts[(ti + ci) % 3]
            d = Dictionary(x)
            hc = HostColumn.encode(d, lay, width=0 if lay == "ppvbs" else w)
            d.close()
            raw[t]["c%d" % ci] = x
            tables[t]["c%d" % ci] = DeviceColumn(hc)
            keep.append(hc)
    yield raw, tables
    for cols in tables.values():
        for dc in cols.values():
            dc.close()
    for hc in keep:
        hc.close()
    torch.cuda.synchronize()


def _queries(raw, n, seed):
    from paper_2209_00220_amd.serve import Query

    rng = np.random.default_rng(seed)
    ops = ["lt", "le", "gt", "ge", "eq", "ne", "between"]
    qs = []
    for i in range(n):
        t = ["t0", "t1"][int(rng.integers(0, 2))]
        cols = list(raw[t])
        preds = []
        for _ in range(int(rng.integers(1, 5))):
            c = cols[int(rng.integers(0, len(cols)))]
            x = raw[t][c]
            lo, hi = sorted(int(v) for v in x[rng.integers(0, x.shape[0], 2)])
            op = ops[int(rng.integers(0, len(ops)))]
            preds.append((c, op, lo, hi if op == "between" else None))
        look = [cols[int(j)] for j in rng.choice(len(cols), size=int(rng.integers(1, 3)), replace=False)]
        qs.append(Query(i, t, preds, look))
    return qs


def _check(raw, q, r):
    sel = None
    for c, op, lo, hi in q.preds:
        sel = scan_values(raw[q.table][c], op, lo, hi, in_mask=sel)
    assert r.count == int(sel.sum()), q
    for c in q.lookups:
        got = r.values[c].cpu().numpy().view(np.uint32)
        assert np.array_equal(got, raw[q.table][c][sel]), (q, c)


def test_served_mix_equals_plain(served):
    from paper_2209_00220_amd.serve import GpuExecutor, Server, run_serial

    raw, tables = served
    qs = _queries(raw, 48, seed=11)
    flush("serving %d queries" % len(qs))
    ex = GpuExecutor(tables)
    res = Server(ex, budget_bytes=1 << 30).run(qs)
    for q in qs:
        _check(raw, q, res[q.qid])
    flush("serving with a tight budget")
    budget = 5 * 2 * 8 * ((300_001 + 63) // 64)
    srv = Server(ex, budget_bytes=budget)
    res2 = srv.run(qs)
    # at most as many admitted queries as the smaller table's bitvector pairs fit
    assert max(srv.batch_sizes) <= budget // (2 * 8 * ((130_000 + 63) // 64))
    assert srv.in_use == 0
    for q in qs:
        _check(raw, q, res2[q.qid])
    flush("serial baseline")
    ser = run_serial(ex, qs)
    for q in qs:
        _check(raw, q, ser[q.qid])


def test_served_alone_equals_in_mix(served):
    from paper_2209_00220_amd.serve import GpuExecutor, Server

    raw, tables = served
    qs = _queries(raw, 16, seed=12)
    ex = GpuExecutor(tables)
    mix = Server(ex, budget_bytes=1 << 30).run(qs)
    for q in qs:
        alone = Server(ex, budget_bytes=1 << 30).run([q])[q.qid]
        assert alone.count == mix[q.qid].count
        for c in q.lookups:
            assert torch.equal(alone.values[c], mix[q.qid].values[c])
