"""Prefix-preserving encoding (PPE), Sec. 3.1.

Numerical columns: Algorithm 1 (PPE_NUMERICAL), an order-preserving M-way tree
built depth first.  Each call encodes the distinct values A_s..A_{e-1} in one
sub-tree whose parent sits at level b:

* if the range fits a leaf (e - s < M) or the depth cut is reached (b >= 2),
  the values get consecutive slot numbers 1..e-s written in beta digits, where
  beta is the smallest integer with M^beta >= e - s + 1, and length b + beta;
* otherwise the M-1 most frequent values of the range become this node's slots
  (sub-codes 1..M-1, length b + 1, in value order), the values strictly between
  slot t and slot t+1 go under pointer t+1, the values left of the first slot
  under pointer 0 and the values right of the last slot under pointer M-1, and
  each group recurses at level b + 1.

A code is the concatenation of the pointer digits on the root path and the
value's own slot number; with M = 256 a digit is one byte.

Readings taken where the paper is silent:
* ties among "the largest M-1 frequencies" go to the smaller index;
* the digit width and the depth cut are parameters (the paper fixes M = 256 and
  a cut of 2) so that small trees can be checked by hand with M = 4;
* a wide leaf (beta >= 2, reachable only at the depth cut) writes its slot
  numbers big-endian, so a last byte may be 0 (slot 256 is bytes 01 00).  What
  the scan needs still holds: when a code is a proper prefix of another, the
  longer code's remaining digits are not all zero (they spell a slot number of
  at least 1).

Categorical columns: Algorithm 2 fills a balanced tree breadth first in
descending frequency order.  Its listing writes c << 8 + i for (c << 8) + i,
c_alpha for C_alpha, and indexes L from 1; it is read here with the first
meaning, the upper-case C, and L_0..L_{n-1}.
"""
from __future__ import annotations

import numpy as np


def digits_needed(count: int, M: int) -> int:
    """Smallest beta with M**beta >= count (0 when count <= 1)."""
    beta = 0
    cap = 1
    while cap < count:
        cap *= M
        beta += 1
    return beta


def ppe_numerical(Q, digit_bits: int = 8, depth_cut: int = 2):
    """Algorithm 1.  Q[i] is the frequency of the i-th smallest distinct value.

    Returns (C, L): C[i] is the code as an unpadded integer of L[i] digits.
    """
    Q = np.asarray(Q, dtype=np.int64)
    n = int(Q.shape[0])
    M = 1 << digit_bits
    C = np.zeros(n, dtype=np.uint64)   # Alg. 1: C_i = 0
    L = np.zeros(n, dtype=np.int64)    # Alg. 1: L_i = 0

    def shift_in(lo, hi, digit):
        """C_i = (C_i << digit_bits) + digit for i in [lo, hi)."""
        if hi > lo:
            C[lo:hi] = (C[lo:hi] << np.uint64(digit_bits)) + np.uint64(digit)

    def encode(b, s, e):
        # two terminating conditions
        if e - s < M or b >= depth_cut:
            beta = digits_needed(e - s + 1, M)
            if e > s:
                slot = np.arange(1, e - s + 1, dtype=np.uint64)   # 1 + (i - s)
                C[s:e] = (C[s:e] << np.uint64(beta * digit_bits)) + slot
                L[s:e] = b + beta
            return
        # the M-1 largest frequencies in Q_s..Q_{e-1}, indices ascending
        order = np.argsort(-Q[s:e], kind="stable")[: M - 1]
        I = np.sort(order) + s
        for t in range(M - 1):
            L[I[t]] = b + 1
            C[I[t]] = (C[I[t]] << np.uint64(digit_bits)) + np.uint64(t + 1)
        for t in range(M - 2):
            shift_in(I[t] + 1, I[t + 1], t + 1)
            encode(b + 1, int(I[t]) + 1, int(I[t + 1]))
        # leftmost sub-tree: pointer 0
        shift_in(s, I[0], 0)
        encode(b + 1, s, int(I[0]))
        # rightmost sub-tree: pointer M-1
        shift_in(I[M - 2] + 1, e, M - 1)
        encode(b + 1, int(I[M - 2]) + 1, e)

    encode(0, 0, n)
    return C, L


def ppe_categorical(n: int, digit_bits: int = 8):
    """Algorithm 2 for n values already sorted by descending frequency.

    Level b (1-based) holds the codes (c << digit_bits) + i, i in 1..M-1, over all
    pointer paths c of b-1 digits; every level but the last is filled completely,
    and the last level is filled slot-major so the remaining values spread
    evenly over its nodes.  Returns (C, L) in the input order.
    """
    M = 1 << digit_bits
    C = np.zeros(n, dtype=np.uint64)
    L = np.zeros(n, dtype=np.int64)
    if n == 0:
        return C, L
    B = digits_needed(n + 1, M)        # levels of the balanced tree
    alpha = 0
    for b in range(1, B):
        for c in range(M ** (b - 1)):
            for i in range(1, M):
                C[alpha] = (c << digit_bits) + i
                L[alpha] = b
                alpha += 1
    for i in range(1, M):
        for j in range(M ** (B - 1)):
            if alpha == n:
                return C, L
            C[alpha] = (j << digit_bits) + i
            L[alpha] = B
            alpha += 1
    return C, L


def padded(C, L, K: int, digit_bits: int = 8):
    """Codes padded with zero digits on the right to K digits (Sec. 3.1, 'as if' padding)."""
    C = np.asarray(C, dtype=np.uint64)
    L = np.asarray(L, dtype=np.int64)
    return C << ((np.int64(K) - L) * digit_bits).astype(np.uint64)


def code_digit(C: int, L: int, j: int, digit_bits: int = 8) -> int:
    """The j-th digit (1-based, most significant first) of a code of L digits; 0 past its end."""
    if j > L:
        return 0
    return (int(C) >> (digit_bits * (L - j))) & ((1 << digit_bits) - 1)
