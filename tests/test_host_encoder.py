"""Host half of the library (dictionary, Algorithm 1, layouts, advisor arithmetic)
against the oracle, bit for bit.  Runs without a GPU: no kernel is launched."""
import numpy as np
import pytest

import datagen
from oracle import advisor as oadv
from oracle.dictionary import build_dictionary, rank_bits
from oracle.layout import bitpacked_build, byteslice_build, pack_bits, vbs_build
from oracle.ppe import ppe_numerical


@pytest.fixture(scope="module")
def L(built_lib):
    from paper_2209_00220_amd import _lib

    return _lib


def _columns():
    yield "tiny", np.array([5], dtype=np.uint32)
    yield "n255", (np.arange(255, dtype=np.uint32) * 7)
    yield "n256", np.repeat(np.arange(256, dtype=np.uint32), 3)
    yield "n257", np.arange(257, dtype=np.uint32)[::-1].copy()
    yield "zipf12", datagen.zipf_column(100_003, 12, 1.0, seed=0)
    yield "zipf16s", datagen.zipf_column(200_000, 16, 1.0, seed=3, mapping=datagen.SORTED)
    yield "zipf20", datagen.zipf_column(300_000, 20, 1.0, seed=5)
    yield "unif24", datagen.zipf_column(150_000, 24, 0.0, seed=6)
    yield "zipf32", datagen.zipf_column(120_000, 32, 1.5, seed=7)   # sort-based dictionary
    yield "wide65791", np.arange(255 + 256 * 255 + 1, dtype=np.uint32)
    yield "gauss20", datagen.gaussian_column(200_000, 20, 2.0 ** 10, seed=8)


def _rows_end_by_mask(C, Lc, Q):
    """Rows whose code ends in a slot of an internal node of Algorithm 1's tree,
    per code length below K, read off the codes alone: the root is internal once
    a code is longer than one byte, so every 1-byte code is then a root slot; the
    values under root pointer t (codes longer than one byte with first digit t)
    get an internal node of their own when there are 256 or more of them, and its
    slots are exactly their 2-byte codes (fewer take 2-byte slot numbers of a
    leaf); past the depth cut every code ends in a leaf."""
    K = int(Lc.max())
    out = [0] * 7
    if K == 1:
        return out
    out[1] = int(Q[Lc == 1].sum())
    if K > 2:
        first = (C >> ((Lc - 1) * 8).astype(np.uint64)).astype(np.int64)
        under = np.bincount(first[Lc >= 2], minlength=256)
        two = Lc == 2
        out[2] = int(Q[two & (under[first] >= 256)].sum())
    return out


@pytest.mark.parametrize("name,x", list(_columns()), ids=[c[0] for c in _columns()])
def test_dictionary_and_ppe_codes(L, name, x):
    A, Q, rank = build_dictionary(x)
    d = L.bst_dict_build(x)
    try:
        A2, Q2 = L.bst_dict_values(d)
        assert np.array_equal(A2, A) and np.array_equal(Q2.astype(np.int64), Q)
        C, Lc = ppe_numerical(Q)
        h = L.bst_encode(d, L.PPVBS)
        try:
            info = L.bst_host_info(h)
            codes, lens = L.bst_host_code_table(h, A.shape[0])
            assert np.array_equal(codes, C), name
            assert np.array_equal(lens.astype(np.int64), Lc), name
            K = int(Lc.max())
            assert info.k_max == K and info.n_rows == x.shape[0]
            # paper-order view of the layout equals the oracle's VBS
            BS, M = vbs_build(C[rank], Lc[rank], K)
            for j in range(1, K + 1):
                assert np.array_equal(L.bst_host_paper_view(h, 0, j), BS[j]), (name, j)
            for j in range(2, K + 1):
                assert np.array_equal(L.bst_host_paper_view(h, 1, j).view(np.uint64), pack_bits(M[j])), (name, j)
            by_len = np.bincount(Lc[rank], minlength=7)
            assert [int(info.rows_by_len[j]) for j in range(1, 7)] == [int(v) for v in by_len[1:7]]
            assert [int(info.rows_end_by_mask[j]) for j in range(7)] == _rows_end_by_mask(C, Lc, Q)
        finally:
            L.bst_free_host(h)
    finally:
        L.bst_dict_free(d)


@pytest.mark.parametrize("w,s", [(8, 0.0), (12, 1.0), (20, 1.0), (32, 0.5)])
def test_fixed_layouts(L, w, s):
    n = 70_001
    x = datagen.zipf_column(n, w, s, seed=w)
    A, Q, rank = build_dictionary(x)
    d = L.bst_dict_build(x)
    try:
        for width, codes, cw in ((0, rank, rank_bits(A.shape[0])), (w, x, w)):
            hb = L.bst_encode(d, L.BYTESLICE, width)
            hp = L.bst_encode(d, L.BITPACKED, width)
            try:
                ib = L.bst_host_info(hb)
                assert ib.width_bits == cw and ib.domain_mode == (1 if width else 0)
                BS = byteslice_build(codes, cw)
                for j in range(1, (cw + 7) // 8 + 1):
                    assert np.array_equal(L.bst_host_paper_view(hb, 0, j), BS[j]), (width, j)
                stream = L.bst_host_paper_view(hp, 2, 0).view(np.uint64)
                assert np.array_equal(stream, bitpacked_build(codes, cw))
                ct, cl = L.bst_host_code_table(hb, A.shape[0])
                assert np.array_equal(ct, A.astype(np.uint64) if width else np.arange(A.shape[0], dtype=np.uint64))
            finally:
                L.bst_free_host(hb)
                L.bst_free_host(hp)
    finally:
        L.bst_dict_free(d)


def test_encode_errors(L):
    x = np.array([0, 300], dtype=np.uint32)
    d = L.bst_dict_build(x)
    try:
        with pytest.raises(L.BstError, match="domain width"):
            L.bst_encode(d, L.BYTESLICE, 8)
        with pytest.raises(L.BstError):
            L.bst_encode(d, 7)
        with pytest.raises(L.BstError):
            L.bst_encode(d, L.PPVBS, 0, 100)
    finally:
        L.bst_dict_free(d)
    with pytest.raises(L.BstError, match="prefix"):
        L.bst_encode_codes(np.array([0x81, 0x8100], dtype=np.uint64), np.array([1, 2], dtype=np.uint8), 2)


def test_encode_codes_worked_example(L, golden):
    g = golden["scan_example"]
    codes = np.array([int(h, 16) for h in g["codes"]], dtype=np.uint64)
    lens = np.array([len(h) // 2 for h in g["codes"]], dtype=np.uint8)
    h = L.bst_encode_codes(codes, lens, 2)
    try:
        assert list(L.bst_host_paper_view(h, 0, 1)) == [0x81, 0xC0, 0x77, 0x81]
        assert list(L.bst_host_paper_view(h, 0, 2)) == [0xA9, 0x89]
        assert int(L.bst_host_paper_view(h, 1, 2).view(np.uint64)[0]) == 0b1100
    finally:
        L.bst_free_host(h)


@pytest.mark.parametrize("seed,w,s", [(0, 12, 1.0), (1, 20, 1.0), (2, 16, 0.0), (3, 12, 1.5)])
def test_profile_literals_match_oracle(L, seed, w, s):
    x = datagen.zipf_column(50_000, w, s, seed=seed)
    A, Q, _ = build_dictionary(x)
    d = L.bst_dict_build(x)
    try:
        lits, sels = L.bst_profile_literals(d, L.LT, 100)
        ol, os_ = oadv.literals_lt(A, Q, 100)
        assert np.array_equal(lits, ol) and np.allclose(sels, os_)
        lits, sels = L.bst_profile_literals(d, L.EQ, 100)
        ol, os_ = oadv.literals_eq(A, Q, 100)
        assert np.array_equal(lits, ol) and np.allclose(sels, os_)
    finally:
        L.bst_dict_free(d)


def test_auc_and_choose_match_oracle(L):
    rng = np.random.default_rng(0)
    for _ in range(50):
        k = int(rng.integers(1, 30))
        s = np.round(rng.random(k), 2)
        t = rng.random(k) * 10
        assert L.bst_auc(s, t) == pytest.approx(oadv.auc(s, t), rel=1e-12, abs=1e-12)
    for aucs in ([1.0, 1.0, 1.0], [2.0, 1.0, 1.0], [0.5, 1.0, 0.5], [3.0, 2.0, 1.0]):
        layouts = [L.BITPACKED, L.BYTESLICE, L.PPVBS]
        want = oadv.choose(dict(zip(layouts, aucs)))
        assert layouts[L.bst_choose(layouts, aucs)] == want


@pytest.mark.parametrize("name,x", [c for c in _columns() if c[0] != "zipf32"], ids=[c[0] for c in _columns() if c[0] != "zipf32"])
def test_categorical_codes(L, name, x):
    # Algorithm 2: codes in descending-frequency order (ties: smaller value), bit-exact
    from oracle.ppe import ppe_categorical

    A, Q, rank = build_dictionary(x)
    order = np.argsort(-Q, kind="stable")
    C, Lc = ppe_categorical(A.shape[0])
    want_c = np.empty_like(C)
    want_l = np.empty_like(Lc)
    want_c[order] = C
    want_l[order] = Lc
    d = L.bst_dict_build(x)
    try:
        h = L.bst_encode(d, L.PPVBS_CATEGORICAL, 0, 0, 0)
        try:
            info = L.bst_host_info(h)
            assert info.layout == L.PPVBS and info.categorical == 1
            codes, lens = L.bst_host_code_table(h, A.shape[0])
            assert np.array_equal(codes, want_c)
            assert np.array_equal(lens.astype(np.int64), want_l)
            K = int(want_l.max())
            assert info.k_max == K
            BS, M = vbs_build(want_c[rank], want_l[rank], K)
            for j in range(1, K + 1):
                assert np.array_equal(L.bst_host_paper_view(h, 0, j), BS[j]), j
            for j in range(2, K + 1):
                assert np.array_equal(L.bst_host_paper_view(h, 1, j).view(np.uint64), pack_bits(M[j])), j
        finally:
            L.bst_free_host(h)
    finally:
        L.bst_dict_free(d)


def test_gaussian_column_generator():
    """Seeded, inside the domain, and spread by sigma (the sweep's input)."""
    a = datagen.gaussian_column(400_000, 12, 64.0, seed=3)
    b = datagen.gaussian_column(400_000, 12, 64.0, seed=3)
    c = datagen.gaussian_column(400_000, 12, 64.0, seed=4)
    assert a.dtype == np.uint32 and np.array_equal(a, b) and not np.array_equal(a, c)
    assert a.max() < 4096 and abs(float(a.mean()) - 2048.0) < 1.0 and abs(float(a.std()) - 64.0) < 1.0
    wide = datagen.gaussian_column(100_000, 8, 1e6, seed=5)   # clipped to [0, 255]
    assert wide.min() == 0 and wide.max() == 255

