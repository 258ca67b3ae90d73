"""Pins of the oracle's layouts (Sec. 2.3 Bit-Packed, Sec. 2.5 ByteSlice, Sec. 3.2 VBS)."""
import numpy as np
import pytest

import datagen
from oracle.dictionary import build_dictionary
from oracle.layout import (
    bitpacked_build, bitpacked_decode, byteslice_build, byteslice_decode, pack_bits,
    unpack_bits, vbs_block_bytes, vbs_build, vbs_decode,
)
from oracle.ppe import ppe_numerical


def test_vbs_fixture(golden):
    g = golden["vbs_fixture"]
    n = g["n"]
    # v1's first byte and v2's bytes are the printed ones; the other codes are 1-byte fillers
    C = [g["v1_first_byte"], (g["bs1_row1"] << 8) | g["bs2_first"], 0x10, 0x20, 0x30, 0x4455, 0x60, 0x70]
    L = [1, 2, 1, 1, 1, 2, 1, 1]
    BS, M = vbs_build(C, L, 2)
    assert BS[1][0] == g["v1_first_byte"]
    assert BS[1][1] == g["bs1_row1"]
    assert BS[2][0] == g["bs2_first"]
    assert list(np.nonzero(M[2])[0]) == g["rows_with_second_byte"]
    assert BS[2].shape[0] == 2 and BS[1].shape[0] == n
    C2, L2 = vbs_decode(BS, M, 2)
    assert [int(c) for c in C2] == C and list(L2) == L


def test_vbs_block_size_example(golden):
    g = golden["vbs_block_size"]
    L = np.ones(g["block"], dtype=np.int64)
    L[: g["with_byte2"]] = 2
    L[: g["with_byte3"]] = 3
    assert vbs_block_bytes(L, g["K"], g["block"]) == g["vbs_bytes"]
    assert g["block"] * g["K"] == g["byteslice_bytes"]


@pytest.mark.parametrize("n", [0, 1, 63, 64, 65, 1000, 4097])
def test_vbs_roundtrip_and_structure(n):
    x = datagen.zipf_column(n, 16, 1.0, seed=n + 1)
    if n == 0:
        return
    A, Q, rank = build_dictionary(x)
    C, L = ppe_numerical(Q)
    K = int(L.max())
    BS, M = vbs_build(C[rank], L[rank], K)
    for j in range(2, K + 1):
        assert BS[j].shape[0] == int(M[j].sum())
        if j >= 3:
            assert not np.any(M[j] & ~M[j - 1])
    C2, L2 = vbs_decode(BS, M, K)
    assert np.array_equal(C2, C[rank]) and np.array_equal(L2, L[rank])


def test_byteslice_left_aligned_and_roundtrip():
    code = np.array([0, 1, 0xABC, 0xFFF, 0x800], dtype=np.uint64)
    BS = byteslice_build(code, 12)
    # a 12-bit code's top 8 bits are byte 1, its low 4 bits the high nibble of byte 2
    assert list(BS[1]) == [0x00, 0x00, 0xAB, 0xFF, 0x80]
    assert list(BS[2]) == [0x00, 0x10, 0xC0, 0xF0, 0x00]
    assert np.array_equal(byteslice_decode(BS, 12), code)
    rng = np.random.default_rng(0)
    for w in (1, 7, 8, 9, 16, 20, 24, 31, 32):
        c = rng.integers(0, 2 ** w, size=333, dtype=np.uint64)
        assert np.array_equal(byteslice_decode(byteslice_build(c, w), w), c)


def test_bitpacked_positions(golden):
    g = golden["bitpacked_positions"]
    w = g["width"]
    words = bitpacked_build(np.array([(1 << w) - 1, 0, 0], dtype=np.uint64), w)
    bits = unpack_bits(words, 3 * w)
    lo, hi = g["v1_bits_0based"]
    assert bits[lo:hi + 1].all() and not bits[hi + 1:].any()
    words = bitpacked_build(np.array([0, (1 << w) - 1, 0], dtype=np.uint64), w)
    bits = unpack_bits(words, 3 * w)
    lo, hi = g["v2_bits_0based"]
    assert bits[lo:hi + 1].all() and not bits[:lo].any() and not bits[hi + 1:].any()
    rng = np.random.default_rng(1)
    for w in (1, 3, 11, 20, 32):
        c = rng.integers(0, 2 ** w, size=257, dtype=np.uint64)
        assert np.array_equal(bitpacked_decode(bitpacked_build(c, w), 257, w), c)


def test_pack_bits_lsb_first():
    b = np.zeros(130, dtype=bool)
    b[[0, 5, 64, 129]] = True
    w = pack_bits(b)
    assert w.shape[0] == 3
    assert int(w[0]) == (1 << 0) | (1 << 5)
    assert int(w[1]) == 1 and int(w[2]) == 2
    assert np.array_equal(unpack_bits(w, 130), b)
