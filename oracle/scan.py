"""Scan: predicate -> result bitvector (Sec. 2.2; PP-VBS scan of Sec. 3.3).

The plain definition: bit r of the result is 1 exactly when row r is selected by
the incoming row mask (when one is given) and its value satisfies the
predicate.  Operators are <, <=, >, >=, =, != and BETWEEN lo AND hi
(lo <= v <= hi, empty when lo > hi); values compare as unsigned 32-bit
integers.  An incoming mask models predicate pipelining (Sec. 3.3: the result
of one scan is handed to the next).

The oracle reaches a layout's result by decoding every stored code back to its
value and applying that definition.  ``classify`` / ``classify_rows`` restate the
byte-serial comparison of Sec. 3.3 (Algorithm 3 generalised to every operator)
for the early-stop checks of Lemma 1; they compare a code v against a literal
code c one byte at a time:

* byte j of v below / above byte j of c: v < c / v > c, decided;
* equal at byte j < l(c): if v has no byte j+1 then v is a proper prefix of c
  and c's remaining bytes are not all zero, so v < c; otherwise go on;
* equal at byte j = l(c): v > c if v has a byte j+1 (its remaining bytes are not
  all zero), else v = c.

Unsigned byte comparison is the reading the worked example of Sec. 3.3 needs
(0x77 < 0x81 there); Algorithm 3's listing writes Z_ep for Z_eq.
"""
from __future__ import annotations

import numpy as np

from .layout import bitpacked_decode, byteslice_decode, pack_bits, vbs_decode
from .ppe import code_digit, padded

OPS = ("lt", "le", "gt", "ge", "eq", "ne", "between")


def scan_values(x, op: str, lo: int, hi: int | None = None, in_mask=None) -> np.ndarray:
    """Boolean result of `x op lo` (or lo <= x <= hi for BETWEEN), AND the incoming mask."""
    x = np.asarray(x).astype(np.uint64)
    lo = np.uint64(lo)
    if op == "lt":
        r = x < lo
    elif op == "le":
        r = x <= lo
    elif op == "gt":
        r = x > lo
    elif op == "ge":
        r = x >= lo
    elif op == "eq":
        r = x == lo
    elif op == "ne":
        r = x != lo
    elif op == "between":
        r = (x >= lo) & (x <= np.uint64(hi))
    else:
        raise ValueError(op)
    if in_mask is not None:
        r = r & np.asarray(in_mask, dtype=bool)
    return r


def scan_values_bv(x, op, lo, hi=None, in_mask=None) -> np.ndarray:
    return pack_bits(scan_values(x, op, lo, hi, in_mask))


# ------------------------------------------------ byte-serial classification
def classify(Cv: int, Lv: int, Cc: int, lc: int):
    """Compare code v (Lv bytes) with literal c (lc bytes) byte by byte.

    Returns (sign, m): sign -1 / 0 / +1 for v < c / v = c / v > c under the
    as-if-padded order, and m the number of bytes examined (Lemma 1: m <= min(Lv, lc)).
    """
    j = 1
    while True:
        vj = code_digit(Cv, Lv, j)
        cj = code_digit(Cc, lc, j)
        if vj < cj:
            return -1, j
        if vj > cj:
            return 1, j
        v_has_next = Lv > j
        if j < lc:
            if not v_has_next:
                return -1, j
            j += 1
            continue
        return (1 if v_has_next else 0), j


def classify_rows(C, L, Cc: int, lc: int):
    """``classify`` for every row at once; returns (sign[], bytes_examined[])."""
    C = np.asarray(C, dtype=np.uint64)
    L = np.asarray(L, dtype=np.int64)
    n = C.shape[0]
    sign = np.zeros(n, dtype=np.int64)
    m = np.zeros(n, dtype=np.int64)
    pending = np.ones(n, dtype=bool)
    for j in range(1, lc + 1):
        if not pending.any():
            break
        m[pending] = j
        vj = np.where(L >= j, (C >> (np.maximum(L - j, 0) * 8).astype(np.uint64)) & np.uint64(0xFF), 0)
        cj = code_digit(Cc, lc, j)
        lt = pending & (vj < cj)
        gt = pending & (vj > cj)
        eq = pending & (vj == cj)
        sign[lt] = -1
        sign[gt] = 1
        has_next = L > j
        if j < lc:
            sign[eq & ~has_next] = -1
            pending = eq & has_next
        else:
            sign[eq & has_next] = 1
            sign[eq & ~has_next] = 0
            pending = np.zeros(n, dtype=bool)
    return sign, m


def select_by_sign(op: str, sign_lo, sign_hi=None) -> np.ndarray:
    """Turn per-row comparison signs against the literal(s) into the operator's result."""
    if op == "lt":
        return sign_lo < 0
    if op == "le":
        return sign_lo <= 0
    if op == "gt":
        return sign_lo > 0
    if op == "ge":
        return sign_lo >= 0
    if op == "eq":
        return sign_lo == 0
    if op == "ne":
        return sign_lo != 0
    if op == "between":
        return (sign_lo >= 0) & (sign_hi <= 0)
    raise ValueError(op)


def scan_padded_codes(P, op: str, c_lo: int, c_hi: int | None = None, in_mask=None) -> np.ndarray:
    """Scan on padded codes as plain integers (the as-if-padded order of Sec. 3.1)."""
    return scan_values(np.asarray(P, dtype=np.uint64), op, c_lo, c_hi, in_mask)


# ------------------------------------------------------ scans through layouts
class CodeTable:
    """Map from a padded PP-VBS code to its value (the decoding dictionary)."""

    def __init__(self, A, C, L, K: int):
        P = padded(C, L, K)
        order = np.argsort(P, kind="stable")
        self.P = P[order]
        self.V = np.asarray(A, dtype=np.uint32)[order]
        if self.P.shape[0] > 1:
            assert np.all(self.P[1:] != self.P[:-1]), "padded codes must be unique"

    def values(self, P) -> np.ndarray:
        P = np.asarray(P, dtype=np.uint64)
        idx = np.searchsorted(self.P, P)
        idx = np.minimum(idx, max(self.P.shape[0] - 1, 0))
        assert np.all(self.P[idx] == P), "a stored code is not in the dictionary"
        return self.V[idx]


def decode_vbs_values(BS, M, K: int, table: CodeTable) -> np.ndarray:
    C, L = vbs_decode(BS, M, K)
    return table.values(padded(C, L, K))


def decode_fixed_values(code, A=None) -> np.ndarray:
    """Fixed-length codes -> values: the rank's dictionary entry, or the code itself
    when the column stores values directly (domain mode)."""
    code = np.asarray(code, dtype=np.uint64)
    if A is None:
        return code.astype(np.uint32)
    return np.asarray(A, dtype=np.uint32)[code.astype(np.int64)]


def scan_vbs(BS, M, K, table, op, lo, hi=None, in_mask=None) -> np.ndarray:
    return scan_values_bv(decode_vbs_values(BS, M, K, table), op, lo, hi, in_mask)


def scan_byteslice(BS, w, A, op, lo, hi=None, in_mask=None) -> np.ndarray:
    return scan_values_bv(decode_fixed_values(byteslice_decode(BS, w), A), op, lo, hi, in_mask)


def scan_bitpacked(words, n, w, A, op, lo, hi=None, in_mask=None) -> np.ndarray:
    return scan_values_bv(decode_fixed_values(bitpacked_decode(words, n, w), A), op, lo, hi, in_mask)
