"""Synthetic workloads: value columns, predicate literals at target selectivities,
and row-ID lists.  Literals are picked from the value counts of the generated
column (plain quantiles); nothing here encodes or scans.

Workloads
---------
config1: one column of 1M rows, Zipf(1.0) over 4096 values (12-bit), seed 0;
         '<' at about 10 %, 10k uniform row IDs.
config2: one column of 500M rows, Zipf(1.0) over 2^20 values (20-bit); '<', '='
         and BETWEEN at selectivities 0.1, 1, 10, 50, 90 % ('=' cannot exceed
         the largest value frequency, about 6.9 %, and takes the nearest one);
         5M uniform row IDs (1 %), seed 1.
"""
from __future__ import annotations

import numpy as np

from . import uniform_ids, zipf_column

SELECTIVITIES = (0.001, 0.01, 0.10, 0.50, 0.90)


def value_counts(x: np.ndarray, w: int):
    """(values, counts) of the distinct values, ascending."""
    if w <= 26:
        c = np.bincount(x, minlength=1 << w)
        v = np.nonzero(c)[0]
        return v.astype(np.uint32), c[v].astype(np.int64)
    v, c = np.unique(x, return_counts=True)
    return v.astype(np.uint32), c.astype(np.int64)


def lit_lt(values, counts, target: float):
    """Literal c with fraction of rows below c nearest target; returns (c, selectivity)."""
    n = counts.sum()
    below = np.concatenate([[0], np.cumsum(counts)[:-1]]) / n
    k = int(np.argmin(np.abs(below - target)))
    return int(values[k]), float(below[k])


def lit_eq(values, counts, target: float):
    """Value whose frequency is nearest target; returns (value, selectivity)."""
    n = counts.sum()
    f = counts / n
    k = int(np.argmin(np.abs(f - target)))
    return int(values[k]), float(f[k])


def lit_between(values, counts, target: float):
    """Centred range [q((1-s)/2), q((1+s)/2)]; returns (lo, hi, selectivity)."""
    n = counts.sum()
    cum = np.cumsum(counts) / n
    lo_k = int(np.searchsorted(cum, (1.0 - target) / 2.0, side="left"))
    hi_k = int(np.searchsorted(cum, (1.0 + target) / 2.0, side="left"))
    lo_k = min(lo_k, len(values) - 1)
    hi_k = min(max(hi_k, lo_k), len(values) - 1)
    sel = float(cum[hi_k] - (cum[lo_k - 1] if lo_k > 0 else 0.0))
    return int(values[lo_k]), int(values[hi_k]), sel


def predicate_set(x: np.ndarray, w: int, selectivities=SELECTIVITIES):
    """[(op, lo, hi, selectivity)] for '<', '=' and BETWEEN at each target."""
    v, c = value_counts(x, w)
    preds = []
    for s in selectivities:
        lo, sel = lit_lt(v, c, s)
        preds.append(("lt", lo, None, sel))
    for s in selectivities:
        lo, sel = lit_eq(v, c, s)
        preds.append(("eq", lo, None, sel))
    for s in selectivities:
        lo, hi, sel = lit_between(v, c, s)
        preds.append(("between", lo, hi, sel))
    return preds


def config1(threads=None):
    x = zipf_column(1_000_000, 12, 1.0, seed=0, threads=threads)
    v, c = value_counts(x, 12)
    lit, sel = lit_lt(v, c, 0.10)
    return {"x": x, "w": 12, "lt_literal": lit, "lt_selectivity": sel, "ids": uniform_ids(10_000, x.shape[0], seed=0)}


def config2(n: int = 500_000_000, threads=None, n_ids: int | None = None):
    x = zipf_column(n, 20, 1.0, seed=2, threads=threads)
    preds = predicate_set(x, 20)
    m = n_ids if n_ids is not None else max(1, n // 100)
    ids = uniform_ids(m, n, seed=1)
    return {"x": x, "w": 20, "preds": preds, "ids": ids}


def config2_predicates(n: int = 500_000_000, threads=None):
    """The predicates of config2 alone (the column is regenerated to pick them)."""
    return predicate_set(zipf_column(n, 20, 1.0, seed=2, threads=threads), 20)


# config3: a wide table -- 16 columns of n rows; column c has width
# [8, 12, 16, 20, 24, 32][c % 6] and Zipf exponent [0, 0.5, 1.0, 1.5][c % 4]
# (0 = uniform), seed c.  The query pipelines '<' on columns 2, 5, 7, 9, each at
# about 31.6 % selectivity (about 1 % together), and looks up columns 0, 10, 11
# on the qualifying rows.
WIDE_WIDTHS = (8, 12, 16, 20, 24, 32)
WIDE_SKEWS = (0.0, 0.5, 1.0, 1.5)
WIDE_FILTER = (2, 5, 7, 9)
WIDE_LOOKUP = (0, 10, 11)


def config3_column(c: int, n: int, threads=None):
    w = WIDE_WIDTHS[c % 6]
    return zipf_column(n, w, WIDE_SKEWS[c % 4], seed=c, threads=threads), w


# config4: 64 columns, n_c = exp(U[ln 1e6, ln 1e8]), w_c ~ U{8..32},
# s_c ~ U[0, 1.5]; 256 predicates: column ~ U, op ~ U{<, <=, =, BETWEEN},
# selectivity log-uniform in [0.01 %, 50 %] (the nearest reachable one).
def config4_columns(n_cols: int = 64, seed: int = 4, n_lo: float = 1e6, n_hi: float = 1e8):
    rng = np.random.default_rng(seed)
    specs = []
    for c in range(n_cols):
        n = int(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi))))
        w = int(rng.integers(8, 33))
        s = float(rng.uniform(0.0, 1.5))
        specs.append((n, w, s, 100 + c))
    return specs


def config4_predicates(counts, n_preds: int = 256, seed: int = 5):
    """counts: per column (values, counts); returns [(column, op, lo, hi, selectivity)]."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n_preds):
        c = int(rng.integers(0, len(counts)))
        v, k = counts[c]
        op = ("lt", "le", "eq", "between")[int(rng.integers(0, 4))]
        sel = float(np.exp(rng.uniform(np.log(1e-4), np.log(0.5))))
        if op in ("lt", "le"):
            lo, got = lit_lt(v, k, sel)
            out.append((c, op, lo, None, got))
        elif op == "eq":
            lo, got = lit_eq(v, k, sel)
            out.append((c, op, lo, None, got))
        else:
            lo, hi, got = lit_between(v, k, sel)
            out.append((c, op, lo, hi, got))
    return out


def config5_tables(n_tables: int = 8, n_cols: int = 4, n_lo: float = 4e8, n_hi: float = 1e9, seed: int = 55,
                   log_uniform: bool = False):
    """Tables for the serving workload: n_t uniform in [n_lo, n_hi] (log-uniform
    when asked; every column of a table has n_t rows), width w ~ U{8..32},
    Zipf s ~ U[0.5, 1.5].  Returns [(n_t, [(w, s, seed), ...])]."""
    rng = np.random.default_rng(seed)
    out = []
    for t in range(n_tables):
        u = rng.uniform(0.0, 1.0)
        n = int(np.exp(np.log(n_lo) + u * (np.log(n_hi) - np.log(n_lo)))) if log_uniform else int(n_lo + u * (n_hi - n_lo))
        cols = [(int(rng.integers(8, 33)), float(rng.uniform(0.5, 1.5)), 500 + 10 * t + c) for c in range(n_cols)]
        out.append((n, cols))
    return out


def config5_queries(counts, n_queries: int, seed: int):
    """Serving queries: counts[t][c] = (values, counts) of column c of table t.
    Each query: 1-4 predicates on one table (op in <, >=, BETWEEN; selectivity
    log-uniform in [0.01 %, 50 %]), then a lookup of 1-2 of its columns.
    Returns [(table, [(column, op, lo, hi)], [lookup columns])]."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n_queries):
        t = int(rng.integers(0, len(counts)))
        nc = len(counts[t])
        preds = []
        for _ in range(int(rng.integers(1, 5))):
            c = int(rng.integers(0, nc))
            v, k = counts[t][c]
            sel = float(np.exp(rng.uniform(np.log(1e-4), np.log(0.5))))
            kind = int(rng.integers(0, 3))
            if kind == 0:
                preds.append((c, "lt", lit_lt(v, k, sel)[0], None))
            elif kind == 1:
                preds.append((c, "ge", lit_lt(v, k, 1.0 - sel)[0], None))
            else:
                lo, hi, _ = lit_between(v, k, sel)
                preds.append((c, "between", lo, hi))
        look = sorted(int(j) for j in rng.choice(nc, size=int(rng.integers(1, 3)), replace=False))
        out.append((t, preds, look))
    return out

