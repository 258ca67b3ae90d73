"""Column-layout advisor (Sec. 4, Algorithm 5).

Per column: profile scans with 100 literals taken from the column that span its
feasible selectivities ('<' for numerical columns, '=' for categorical ones),
fit a time-versus-selectivity curve per layout, and keep the layout with the
smaller area under the curve; on a tie the paper keeps ByteSlice.

Readings taken where the paper is silent:
* '<' literals: for i = 1..count, the distinct value A_k whose selectivity
  sum(Q_0..Q_{k-1}) / n is nearest to (i - 0.5) / count (ties: smaller k);
* '=' literals: the distinct values in descending-frequency order (ties:
  smaller value), taken at count evenly spaced positions, so their
  selectivities run from the largest frequency down to the smallest;
* the curve is piecewise linear through the points (times at an equal
  selectivity averaged) and its area is the trapezoid sum over the measured
  selectivity range; with fewer than two distinct selectivities the area is the
  mean time;
* with more than two candidate layouts the smallest area wins and ties go to
  ByteSlice first, then PP-VBS, then Bit-Packed.
"""
from __future__ import annotations

import numpy as np

BITPACKED, BYTESLICE, PPVBS = 0, 1, 2
TIE_ORDER = (BYTESLICE, PPVBS, BITPACKED)


def literals_lt(A, Q, count: int = 100):
    """(literals, selectivities) for the '<' profile."""
    A = np.asarray(A)
    Q = np.asarray(Q, dtype=np.int64)
    n = int(Q.sum())
    below = np.concatenate([[0], np.cumsum(Q)[:-1]])     # rows with value < A_k
    lits, sels = [], []
    for i in range(1, count + 1):
        target = (i - 0.5) / count
        k = int(np.argmin(np.abs(below / n - target)))     # first minimum: smaller k
        lits.append(int(A[k]))
        sels.append(below[k] / n)
    return np.asarray(lits, dtype=np.uint32), np.asarray(sels, dtype=np.float64)


def literals_eq(A, Q, count: int = 100):
    """(literals, selectivities) for the '=' profile."""
    A = np.asarray(A)
    Q = np.asarray(Q, dtype=np.int64)
    n = int(Q.sum())
    order = np.lexsort((A, -Q))                          # by -Q, then by value
    nd = order.shape[0]
    if count == 1:
        picks = [0]
    else:
        picks = [int(round(i * (nd - 1) / (count - 1))) for i in range(count)]
    idx = order[picks]
    return A[idx].astype(np.uint32), Q[idx] / n


def auc(sel, t) -> float:
    """Area under the piecewise-linear time-vs-selectivity curve."""
    sel = np.asarray(sel, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    xs = np.unique(sel)
    ys = np.asarray([t[sel == s].mean() for s in xs])
    if xs.shape[0] < 2:
        return float(ys.mean()) if ys.shape[0] else 0.0
    return float(np.sum((xs[1:] - xs[:-1]) * (ys[1:] + ys[:-1]) / 2.0))


def choose(aucs: dict) -> int:
    """The layout with the smallest area; ties in TIE_ORDER."""
    best = None
    for lay in TIE_ORDER:
        if lay not in aucs:
            continue
        if best is None or aucs[lay] < aucs[best]:
            best = lay
    return best
