"""Pins of the oracle's lookup (Sec. 3.3, Algorithm 4) and advisor (Sec. 4, Algorithm 5)."""
import numpy as np
import pytest

import datagen
from oracle import advisor
from oracle.dictionary import build_dictionary
from oracle.layout import pack_bits, unpack_bits, vbs_build
from oracle.lookup import bit_E, bit_P, bv_row_ids, lookup_bv, lookup_ids, lookup_vbs_alg4, pext, popcount
from oracle.ppe import padded, ppe_numerical
from oracle.scan import CodeTable, decode_vbs_values


def test_bit_trick_examples(golden):
    g = golden["bit_tricks"]
    x = int(g["x"], 2)
    assert bit_E(x, g["width"]) == int(g["E"], 2)
    assert bit_P(x, g["width"]) == int(g["P"], 2)
    # the lowest set bit's position follows from POPCNT(P(x)): 8 - 1 - 6 = 1
    assert (g["width"] - 1) - popcount(bit_P(x, g["width"])) == 1


def test_pext_by_hand():
    # mask bits 1,3,4,7 of src 0b1001_1010 are 1,1,1,1 -> 0b1111; of 0b0000_1010 -> 1,1,0,0
    assert pext(0b10011010, 0b10011010, 8) == 0b1111
    assert pext(0b00001010, 0b10011010, 8) == 0b0011
    assert pext(0, 0xFF, 8) == 0


@pytest.mark.parametrize("n,seed", [(1, 0), (64, 1), (200, 2), (1111, 3)])
def test_lookup_identity_and_alg4(n, seed):
    x = datagen.zipf_column(n, 16, 1.2, seed=seed, mapping=datagen.SORTED)
    A, Q, rank = build_dictionary(x)
    C, L = ppe_numerical(Q)
    K = int(L.max())
    BS, M = vbs_build(C[rank], L[rank], K)
    vals = decode_vbs_values(BS, M, K, CodeTable(A, C, L, K))
    assert np.array_equal(vals, x)                       # decode(encode(x)) = x
    ids = datagen.uniform_ids(3 * n, n, seed=seed)
    assert np.array_equal(lookup_ids(vals, ids), x[ids.astype(np.int64)])
    R = datagen.random_mask_words(n, seed=seed + 50, density=0.3)
    assert np.array_equal(lookup_bv(vals, R, n), x[unpack_bits(R, n)])
    # Algorithm 4's padded codes are the selected rows' padded codes, in row order
    got = lookup_vbs_alg4(BS, M, K, R, n)
    sel = unpack_bits(R, n)
    assert np.array_equal(got, padded(C[rank], L[rank], K)[sel])
    assert np.array_equal(bv_row_ids(R, n), np.nonzero(sel)[0])


def test_literals_lt_closed_form():
    # 200 distinct values, one row each: '< A_k' selects k/200 of the rows, so the
    # literal nearest (i - 0.5)/100 is A_{2i-1} exactly
    A = np.arange(200, dtype=np.uint32) * 3
    Q = np.ones(200, dtype=np.int64)
    lits, sels = advisor.literals_lt(A, Q)
    assert list(lits) == [3 * (2 * i - 1) for i in range(1, 101)]
    assert np.allclose(sels, [(2 * i - 1) / 200 for i in range(1, 101)])


def test_literals_eq_by_hand():
    A = np.array([10, 20, 30, 40], dtype=np.uint32)
    Q = np.array([1, 5, 5, 2], dtype=np.int64)
    lits, sels = advisor.literals_eq(A, Q, count=4)
    # descending frequency, ties by value: 20, 30, 40, 10
    assert list(lits) == [20, 30, 40, 10]
    assert np.allclose(sels, [5 / 13, 5 / 13, 2 / 13, 1 / 13])
    lits, _ = advisor.literals_eq(A, Q, count=2)
    assert list(lits) == [20, 10]


def test_auc_and_choice():
    # trapezoids: points (0,1),(0.5,3),(1,1) -> 0.5*(1+3)/2 + 0.5*(3+1)/2 = 2
    assert advisor.auc([0, 0.5, 1], [1, 3, 1]) == pytest.approx(2.0)
    # duplicate selectivities are averaged before integrating
    assert advisor.auc([0, 0, 1], [1, 3, 2]) == pytest.approx((2 + 2) / 2)
    assert advisor.auc([0.3, 0.3], [4, 6]) == pytest.approx(5.0)
    # Algorithm 5: ByteSlice when its area is not larger (ties keep ByteSlice)
    assert advisor.choose({advisor.BYTESLICE: 1.0, advisor.PPVBS: 1.0}) == advisor.BYTESLICE
    assert advisor.choose({advisor.BYTESLICE: 1.0, advisor.PPVBS: 0.9}) == advisor.PPVBS
    assert advisor.choose({advisor.BYTESLICE: 1.0, advisor.PPVBS: 2.0, advisor.BITPACKED: 0.5}) == advisor.BITPACKED
    assert advisor.choose({advisor.BITPACKED: 1.0, advisor.PPVBS: 1.0}) == advisor.PPVBS
