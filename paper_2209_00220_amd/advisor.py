"""Experiment-driven column-layout advisor (Sec. 4, Algorithm 5) on the GPU.

For a column: build its dictionary once, encode it in every candidate layout,
choose the profiling literals ('<' for numerical columns, '=' for categorical
ones), time each literal's scan on the GPU (``bst_advise``: HIP events, median
of repeats), integrate time over selectivity and keep the layout with the
smallest area (ties keep ByteSlice, as the paper does).  The paper decides
between ByteSlice and PP-VBS; Bit-Packed can be added as a third candidate.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import torch

from . import _lib as L
from .column import DeviceColumn, Dictionary, HostColumn, nwords, stream_handle


@dataclass
class Advice:
    chosen: str
    aucs: dict
    times: dict
    lits: np.ndarray
    sels: np.ndarray
    columns: dict = field(default_factory=dict)   # layout -> (HostColumn, DeviceColumn) kept


def advise_column(x, numeric: bool = True, width: int = 0, layouts=("byteslice", "ppvbs"), count: int = 100,
                  repeats: int = 5, keep: str = "chosen", dictionary: Dictionary | None = None) -> Advice:
    """Run Algorithm 5 on one column of uint32 values.

    width: domain width for ByteSlice / Bit-Packed (0 = dictionary ranks).
    keep: "chosen" keeps only the winning layout resident, "all" keeps every one,
    "none" frees them all.
    """
    d = dictionary if dictionary is not None else Dictionary(x)
    op = L.LT if numeric else L.EQ
    lits, sels = d.profile_literals(op, count)
    cols = {}
    for lay in layouts:
        hc = HostColumn.encode(d, lay, width=width if not lay.startswith("ppvbs") else 0)
        cols[lay] = (hc, DeviceColumn(hc))
    scratch = torch.empty(nwords(d.n_rows), dtype=torch.int64, device="cuda")
    chosen_idx, aucs, times = L.bst_advise([cols[l][1].h for l in layouts], op, lits, sels, repeats, scratch,
                                           stream_handle())
    chosen = layouts[chosen_idx]
    kept = {}
    for lay in layouts:
        if keep == "all" or (keep == "chosen" and lay == chosen):
            kept[lay] = cols[lay]
        else:
            cols[lay][1].close()
            cols[lay][0].close()
    if dictionary is None:
        d.close()
    return Advice(chosen=chosen, aucs=dict(zip(layouts, aucs.tolist())), times=dict(zip(layouts, list(times))),
                  lits=lits, sels=sels, columns=kept)
