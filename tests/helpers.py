"""Shared pieces of the GPU tests: columns on the device and literal sets."""
from __future__ import annotations

import numpy as np

import datagen

LAYOUTS = ("ppvbs", "byteslice", "bitpacked")


def literal_set(A, x_max_bits: int, extra=()):
    """Literals covering present values, absent neighbours and the extremes."""
    A = [int(a) for a in np.asarray(A)]
    cand = {0, 1, 2 ** 32 - 1, (1 << x_max_bits) - 1, 1 << x_max_bits, A[0], A[-1], A[len(A) // 2]}
    step = max(1, len(A) // 6)
    for a in A[::step]:
        cand |= {a, a + 1, max(a - 1, 0)}
    cand |= set(int(e) for e in extra)
    return sorted(c for c in cand if 0 <= c < 2 ** 32)


def device_columns(x, w, layouts=LAYOUTS, domain=True, dir_stride=0):
    """{layout: (HostColumn, DeviceColumn)} for one value column."""
    from paper_2209_00220_amd.column import DeviceColumn, Dictionary, HostColumn

    d = Dictionary(x)
    out = {}
    for lay in layouts:
        width = w if (domain and lay != "ppvbs") else 0
        hc = HostColumn.encode(d, lay, width=width, dir_stride=dir_stride)
        out[lay] = (hc, DeviceColumn(hc))
    d.close()
    return out


def close_columns(cols):
    for hc, dc in cols.values():
        dc.close()
        hc.close()


def flush(msg: str):
    print(msg, flush=True)
