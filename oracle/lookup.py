"""Lookup: plain values of selected rows (Sec. 2.2; PP-VBS lookup of Sec. 3.3).

The plain definition: for a list of row IDs, out[i] is the value of row ids[i];
for a result bitvector R, the values of the rows whose bit is set, in ascending
row order.  The oracle decodes the stored codes (``scan.decode_*``) and indexes.

``lookup_vbs_alg4`` restates Algorithm 4, which rebuilds the selected rows'
codes block by block with the bit tricks E(x) = x & (x - 1) (erase the lowest
set bit) and P(x) = x xor -x (set every bit above the lowest set bit, clear the
rest), pext, and running cursors I_j.  Its listing mixes two bit orders (the
byte index POPCNT(P(x)) + 1 counts from the top of the word while pext packs
from the bottom); it is read here in the LSB-first order used everywhere else:
the popped row's offset in the block is (S/8 - 1) - POPCNT(P(x)), and its byte
in BS_j is found by popping the pext-packed word x_j in step with x.
"""
from __future__ import annotations

import numpy as np

from .layout import unpack_bits


def lookup_ids(values, ids) -> np.ndarray:
    values = np.asarray(values, dtype=np.uint32)
    ids = np.asarray(ids, dtype=np.int64)
    return values[ids]


def lookup_bv(values, words, n: int) -> np.ndarray:
    values = np.asarray(values, dtype=np.uint32)
    return values[unpack_bits(words, n)]


def bv_row_ids(words, n: int) -> np.ndarray:
    """Ascending row IDs of the set bits."""
    return np.nonzero(unpack_bits(words, n))[0].astype(np.uint32)


# -------------------------------------------------------------- bit tricks
def bit_E(x: int, width: int) -> int:
    """Erase the lowest set bit."""
    return (x & (x - 1)) & ((1 << width) - 1)


def bit_P(x: int, width: int) -> int:
    """x xor -x within `width` bits."""
    m = (1 << width) - 1
    return (x ^ ((-x) & m)) & m


def popcount(x: int) -> int:
    return bin(x).count("1")


def pext(src: int, mask: int, width: int) -> int:
    """Gather the bits of src at mask's set positions into the low bits, in order."""
    out = 0
    k = 0
    for b in range(width):
        if (mask >> b) & 1:
            out |= ((src >> b) & 1) << k
            k += 1
    return out


def lookup_vbs_alg4(BS, M, K: int, R_words, n: int, S8: int = 32):
    """Algorithm 4 on a row-order VBS layout.

    Returns the selected rows' codes padded to K bytes, in ascending row order.
    R, M_j are taken S8 rows (one block) at a time.
    """
    R = unpack_bits(R_words, n)
    Mb = {j: np.asarray(M[j], dtype=bool) for j in range(2, K + 1)}
    out = []
    I = [0] * (K + 1)                       # cursors I_1..I_K (0-based positions)
    for base in range(0, n, S8):
        rows = min(S8, n - base)
        x = 0
        B = {}
        for i in range(rows):
            if R[base + i]:
                x |= 1 << i
        for j in range(2, K + 1):
            B[j] = 0
            for i in range(rows):
                if Mb[j][base + i]:
                    B[j] |= 1 << i
        # local maximum length of the selected codes
        beta = 1
        for j in range(2, K + 1):
            if (x & B[j]) == 0:
                break
            beta += 1
        xj = {j: pext(x, B[j], S8) for j in range(2, beta + 1)}
        while x != 0:
            pos = (S8 - 1) - popcount(bit_P(x, S8))
            C = int(BS[1][I[1] + pos])
            x = bit_E(x, S8)
            width = 1
            for j in range(2, beta + 1):
                if (B[j] >> pos) & 1 == 0:
                    break
                t = (S8 - 1) - popcount(bit_P(xj[j], S8))
                C = (C << 8) + int(BS[j][I[j] + t])
                xj[j] = bit_E(xj[j], S8)
                width = j
            out.append(C << (8 * (K - width)))
        I[1] += rows
        for j in range(2, K + 1):
            I[j] += popcount(B[j])
    return np.asarray(out, dtype=np.uint64)
