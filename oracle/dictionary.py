"""Order-preserving dictionary (Sec. 2.2, scan-based OLAP framework).

A column's distinct values, sorted ascending, are the dictionary
A_0 < A_1 < ... < A_{n-1}; Q_i counts how often A_i occurs.  A fixed-length
dictionary code of a value is its rank i in A, so comparing codes compares
values.  The numerical PPE of Sec. 3.1 (Algorithm 1) takes exactly (A, Q) as its
input.
"""
from __future__ import annotations

import numpy as np


def build_dictionary(x: np.ndarray):
    """Return (A, Q, rank): sorted distinct values, their counts, and each row's rank."""
    x = np.asarray(x, dtype=np.uint32)
    A, rank, Q = np.unique(x, return_inverse=True, return_counts=True)
    return A.astype(np.uint32), Q.astype(np.int64), rank.astype(np.int64)


def rank_bits(n_distinct: int) -> int:
    """Width in bits of a rank code for n_distinct values (at least 1)."""
    w = 1
    while (1 << w) < n_distinct:
        w += 1
    return w
