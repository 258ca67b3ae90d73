"""Pins of the oracle's scan (Sec. 2.2 result bitvector; Sec. 3.3 scan and Lemma 1)."""
import numpy as np
import pytest

import datagen
from oracle.dictionary import build_dictionary, rank_bits
from oracle.layout import bitpacked_build, byteslice_build, pack_bits, unpack_bits, vbs_build
from oracle.ppe import padded, ppe_numerical
from oracle.scan import (
    OPS, CodeTable, classify, classify_rows, scan_bitpacked, scan_byteslice, scan_padded_codes, scan_values,
    scan_vbs, select_by_sign,
)


def _hexcode(h):
    return int(h, 16), len(h) // 2


@pytest.mark.parametrize("key", ["scan_example", "scan_example_second_literal"])
def test_worked_scan_examples(golden, key):
    g = golden[key]
    codes = [_hexcode(h) for h in g["codes"]]
    c, l = _hexcode(g["literal"])
    signs, examined = zip(*(classify(cv, lv, c, l) for cv, lv in codes))
    res = select_by_sign(g["op"], np.array(signs))
    assert list(np.nonzero(res)[0]) == g["passing_rows"]
    assert int(pack_bits(res)[0]) == g["result_word"]
    assert list(examined) == g["bytes_examined"]
    # the same rows through plain integer comparison of the padded codes
    K = max(lv for _, lv in codes + [(c, l)])
    P = padded([cv for cv, _ in codes], [lv for _, lv in codes], K)
    pc = int(padded([c], [l], K)[0])
    assert list(np.nonzero(P > np.uint64(pc))[0]) == g["passing_rows"]


def test_signed_compare_would_fail_example(golden):
    # 0x77 < 0x81 only as unsigned bytes; a signed byte compare flips v3's outcome
    g = golden["scan_example"]
    assert np.int8(np.uint8(0x77)) > np.int8(np.uint8(0x81))
    s, _ = classify(0x77A9, 2, 0x81, 1)
    assert s == -1


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_lemma1_and_padded_order(seed):
    # the byte-serial classifier agrees with the padded integer order, and stops
    # after at most min(l(v), l(c)) bytes (Lemma 1)
    x = datagen.zipf_column(20_000, 16, 1.0, seed=seed, mapping=datagen.SORTED if seed == 2 else datagen.SCATTER)
    A, Q, rank = build_dictionary(x)
    C, L = ppe_numerical(Q)
    K = int(L.max())
    P = padded(C, L, K)
    rng = np.random.default_rng(seed)
    for k in rng.integers(0, A.shape[0], size=40):
        sign, m = classify_rows(C, L, int(C[k]), int(L[k]))
        truth = np.sign(P.astype(np.float64) - float(P[k])).astype(np.int64)
        assert np.array_equal(sign, truth)
        assert np.all(m >= 1) and np.all(m <= np.minimum(L, L[k]))
    # scalar and vector classifiers agree
    for k in rng.integers(0, A.shape[0], size=5):
        sv, mv = classify_rows(C[:300], L[:300], int(C[k]), int(L[k]))
        for i in range(300):
            assert classify(int(C[i]), int(L[i]), int(C[k]), int(L[k])) == (sv[i], mv[i])


def _literals(A):
    A = [int(a) for a in A]
    cand = {0, 1, 2 ** 32 - 1, 2 ** 31, A[0], A[-1], A[len(A) // 2]}
    for a in A[:: max(1, len(A) // 7)]:
        cand |= {a, a + 1, max(a - 1, 0)}
    return sorted(c for c in cand if c < 2 ** 32)


@pytest.mark.parametrize("n", [1, 63, 64, 65, 300, 2049])
def test_layout_scans_equal_raw_comparisons(n):
    x = datagen.zipf_column(n, 12, 1.0, seed=100 + n)
    A, Q, rank = build_dictionary(x)
    C, L = ppe_numerical(Q)
    K = int(L.max())
    BS, M = vbs_build(C[rank], L[rank], K)
    table = CodeTable(A, C, L, K)
    w_dict = rank_bits(A.shape[0])
    bs_dict = byteslice_build(rank, w_dict)
    bp_dom = bitpacked_build(x, 12)
    bs_dom = byteslice_build(x, 12)
    in_mask = unpack_bits(datagen.random_mask_words(n, seed=7), n)
    lits = _literals(A)
    for op in OPS:
        for i, lo in enumerate(lits):
            hi = lits[(i * 5 + 3) % len(lits)] if op == "between" else None
            for msk in (None, in_mask):
                want = pack_bits(scan_values(x, op, lo, hi, msk))
                assert np.array_equal(scan_vbs(BS, M, K, table, op, lo, hi, msk), want)
                assert np.array_equal(scan_byteslice(bs_dict, w_dict, A, op, lo, hi, msk), want)
                assert np.array_equal(scan_byteslice(bs_dom, 12, None, op, lo, hi, msk), want)
                assert np.array_equal(scan_bitpacked(bp_dom, n, 12, None, op, lo, hi, msk), want)


def test_scan_values_definitions():
    x = np.array([0, 5, 5, 7, 2 ** 32 - 1], dtype=np.uint32)
    assert list(scan_values(x, "lt", 5)) == [1, 0, 0, 0, 0]
    assert list(scan_values(x, "le", 5)) == [1, 1, 1, 0, 0]
    assert list(scan_values(x, "gt", 5)) == [0, 0, 0, 1, 1]
    assert list(scan_values(x, "ge", 5)) == [0, 1, 1, 1, 1]
    assert list(scan_values(x, "eq", 5)) == [0, 1, 1, 0, 0]
    assert list(scan_values(x, "ne", 5)) == [1, 0, 0, 1, 1]
    assert list(scan_values(x, "between", 5, 7)) == [0, 1, 1, 1, 0]
    assert list(scan_values(x, "between", 7, 5)) == [0, 0, 0, 0, 0]
    assert list(scan_values(x, "gt", 0, in_mask=[1, 1, 0, 1, 0])) == [0, 1, 0, 1, 0]


@pytest.mark.parametrize("seed", [3, 4])
def test_select_by_sign_every_operator(seed):
    """Each operator's selection from the byte-serial signs (the classifier of
    Sec. 3.3) equals the comparison of the zero-padded codes as plain integers
    (Sec. 3.1's order), for one and two literals, present and absent: a wrong
    branch (say '<=' taken as '<', or BETWEEN's bounds swapped) fails here."""
    x = datagen.zipf_column(30_000, 16, 1.0, seed=seed, mapping=datagen.SORTED if seed == 4 else datagen.SCATTER)
    A, Q, rank = build_dictionary(x)
    C, L = ppe_numerical(Q)
    K = int(L.max())
    P = padded(C, L, K)
    Cr, Lr, Pr = C[rank], L[rank], P[rank]
    rng = np.random.default_rng(seed)
    ks = list(rng.integers(0, A.shape[0], size=12)) + [0, A.shape[0] - 1]
    for k in ks:
        s_lo, _ = classify_rows(Cr, Lr, int(C[k]), int(L[k]))
        k2 = int(rng.integers(0, A.shape[0]))
        s_hi, _ = classify_rows(Cr, Lr, int(C[k2]), int(L[k2]))
        for op in OPS:
            got = select_by_sign(op, s_lo, s_hi if op == "between" else None)
            want = scan_padded_codes(Pr, op, int(P[k]), int(P[k2]) if op == "between" else None)
            assert np.array_equal(got, want), (op, k, k2)
    # literals that are not codes of the column: a proper prefix of a stored
    # code, and a code past the last one
    long = int(np.argmax(L))
    if L[long] >= 2:
        c1, l1 = int(C[long]) >> 8 * (int(L[long]) - 1), 1
        s, _ = classify_rows(Cr, Lr, c1, l1)
        for op in OPS[:-1]:
            assert np.array_equal(select_by_sign(op, s), scan_padded_codes(Pr, op, int(padded([c1], [l1], K)[0])))
    with pytest.raises(ValueError):
        select_by_sign("like", s_lo)
