"""Storage layouts in the paper's row order, and their decoders.

* Bit-Packed (Sec. 2.3): k-bit codes back to back, ignoring byte boundaries;
  code r occupies stream bits [r*k, r*k + k), the stream read LSB first
  (bit b is bit b % 64 of 64-bit word b // 64).
* ByteSlice (Sec. 2.5): the j-th byte of every code in its own contiguous
  slice BS_j, ceil(k/8) slices.  A k-bit code is left-aligned in those bytes
  (its top 8 bits are byte 1), so byte 1 carries the most significant bits.
* VBS (Sec. 3.2): BS_1 holds byte 1 of every code; for j >= 2, BS_j packs, in
  row order, the j-th bytes of only those codes that have one, and the
  bitmask M_j marks which codes do (M_1 is omitted).

Bitmasks and result bitvectors are LSB-first: row r is bit r % 64 of 64-bit
word r // 64; bits past the last row are 0.
"""
from __future__ import annotations

import numpy as np


def pack_bits(bits: np.ndarray) -> np.ndarray:
    """Boolean row vector -> LSB-first uint64 words, tail bits zero."""
    bits = np.asarray(bits, dtype=bool)
    n = bits.shape[0]
    nw = (n + 63) // 64
    buf = np.zeros(nw * 64, dtype=np.uint8)
    buf[:n] = bits
    return np.packbits(buf, bitorder="little").view(np.uint64).copy()


def unpack_bits(words: np.ndarray, n: int) -> np.ndarray:
    """LSB-first uint64 words -> boolean vector of n rows."""
    words = np.ascontiguousarray(words, dtype=np.uint64)
    return np.unpackbits(words.view(np.uint8), bitorder="little")[:n].astype(bool)


# --------------------------------------------------------------------- VBS
def vbs_build(C, L, K: int):
    """VBS layout of per-row codes (C[r] an unpadded code of L[r] bytes).

    Returns (BS, M): BS[j] for j = 1..K (uint8 arrays), M[j] for j = 2..K
    (boolean row vectors).  Index 0 (and M[1]) is unused.
    """
    C = np.asarray(C, dtype=np.uint64)
    L = np.asarray(L, dtype=np.int64)
    n = C.shape[0]
    BS = [None] * (K + 1)
    M = [None] * (K + 1)
    for j in range(1, K + 1):
        has = L >= j
        if j >= 2:
            M[j] = has.copy()
        sh = ((L[has] - j) * 8).astype(np.uint64)
        BS[j] = ((C[has] >> sh) & np.uint64(0xFF)).astype(np.uint8)
    if n:
        assert BS[1].shape[0] == n
    return BS, M


def vbs_decode(BS, M, K: int):
    """Rebuild (C, L) of every row from a VBS layout.

    Follows the cursor reading of Sec. 3.3: a row's j-th byte is the next unread
    byte of BS_j exactly when its bit in M_j is set, so the byte's position is
    the number of earlier rows with that bit (a running count).
    """
    b1 = np.asarray(BS[1], dtype=np.uint8)
    n = b1.shape[0]
    C = b1.astype(np.uint64)
    L = np.ones(n, dtype=np.int64)
    prev = np.ones(n, dtype=bool)
    for j in range(2, K + 1):
        has = np.asarray(M[j], dtype=bool)
        assert not np.any(has & ~prev), "M_j must be a subset of M_{j-1}"
        pos = np.cumsum(has) - 1           # running cursor I_j
        assert np.asarray(BS[j]).shape[0] == int(has.sum())
        byte = np.zeros(n, dtype=np.uint64)
        byte[has] = np.asarray(BS[j], dtype=np.uint64)[pos[has]]
        C = np.where(has, (C << np.uint64(8)) | byte, C)
        L = np.where(has, j, L)
        prev = has
    return C, L


def vbs_block_bytes(L_block, K: int, block: int = 32) -> int:
    """Bytes one VBS block takes (Sec. 3.2): a block-bit word of each M_2..M_K,
    the block's BS_1 bytes, and one BS_j byte per code that has a j-th byte."""
    L_block = np.asarray(L_block, dtype=np.int64)
    mask_bytes = (K - 1) * (block // 8)
    return mask_bytes + block + int(sum(int((L_block >= j).sum()) for j in range(2, K + 1)))


# --------------------------------------------------------------- ByteSlice
def byteslice_width_bytes(w: int) -> int:
    return (w + 7) // 8


def byteslice_build(code, w: int):
    """ByteSlice slices BS_1..BS_K of fixed w-bit codes, left-aligned."""
    code = np.asarray(code, dtype=np.uint64)
    K = byteslice_width_bytes(w)
    v = code << np.uint64(8 * K - w)
    BS = [None] * (K + 1)
    for j in range(1, K + 1):
        BS[j] = ((v >> np.uint64(8 * (K - j))) & np.uint64(0xFF)).astype(np.uint8)
    return BS


def byteslice_decode(BS, w: int):
    K = byteslice_width_bytes(w)
    v = np.zeros(np.asarray(BS[1]).shape[0], dtype=np.uint64)
    for j in range(1, K + 1):
        v = (v << np.uint64(8)) | np.asarray(BS[j], dtype=np.uint64)
    return v >> np.uint64(8 * K - w)


# -------------------------------------------------------------- Bit-Packed
def bitpacked_build(code, w: int) -> np.ndarray:
    """LSB-first bit stream of w-bit codes as uint64 words."""
    code = np.asarray(code, dtype=np.uint64)
    n = code.shape[0]
    bits = ((code[:, None] >> np.arange(w, dtype=np.uint64)[None, :]) & np.uint64(1)).astype(bool)
    return pack_bits(bits.reshape(-1)) if n else np.zeros(0, dtype=np.uint64)


def bitpacked_decode(words: np.ndarray, n: int, w: int) -> np.ndarray:
    bits = unpack_bits(words, n * w).reshape(n, w).astype(np.uint64)
    return (bits << np.arange(w, dtype=np.uint64)[None, :]).sum(axis=1, dtype=np.uint64)
