"""Pins of the oracle's prefix-preserving encoding (Sec. 3.1, Algorithms 1 and 2).

Each case is derived by hand from the algorithm's definition or is a property
the paper states (Property 1, Property 2, order preservation, the top-255
rule), so a dropped term, a wrong digit or a wrong index fails one of them.
"""
import numpy as np
import pytest

import datagen
from oracle.dictionary import build_dictionary
from oracle.ppe import digits_needed, padded, ppe_categorical, ppe_numerical


def test_small_domain_closed_form():
    # e - s < 256 at the root: slot numbers 1..n, one byte each
    for n in (0, 1, 2, 17, 255):
        Q = np.arange(n, 0, -1)
        C, L = ppe_numerical(Q)
        assert list(C) == list(range(1, n + 1))
        assert list(L) == [1] * n


def test_rightmost_subtree_by_hand():
    # frequencies put the 255 largest at indices 0..254, so 255..299 sit right of
    # the last slot: pointer 255, then a leaf with slots 1..45
    Q = np.concatenate([np.full(255, 10), np.full(45, 1)])
    C, L = ppe_numerical(Q)
    assert list(C[:255]) == list(range(1, 256)) and set(L[:255]) == {1}
    assert list(C[255:]) == [(255 << 8) + k for k in range(1, 46)]
    assert set(L[255:]) == {2}


def test_leftmost_subtree_and_ties_by_hand():
    # all 256 frequencies equal: ties go to the smaller index, so 0..254 are slots
    C, L = ppe_numerical(np.ones(256))
    assert list(C[:255]) == list(range(1, 256))
    assert C[255] == (255 << 8) + 1 and L[255] == 2
    # the rarest value first: it goes under pointer 0 with slot 1 -> bytes 00 01
    Q = np.ones(256, dtype=np.int64) * 5
    Q[0] = 1
    C, L = ppe_numerical(Q)
    assert C[0] == 0x0001 and L[0] == 2
    assert list(C[1:]) == list(range(1, 256))


def test_interior_subtree_by_hand():
    # 300 values; the rare ones are indices 100..144 (45 of them), between slot
    # 100 (index 99) and slot 101 (index 145): pointer 100, slots 1..45
    Q = np.full(300, 9)
    Q[100:145] = 1
    Q[255 + 45:] = 9
    C, L = ppe_numerical(Q)
    assert list(C[100:145]) == [(100 << 8) + k for k in range(1, 46)]
    assert set(L[100:145]) == {2}
    assert C[99] == 100 and C[145] == 101


def test_four_way_toy_by_hand(golden):
    # M = 4 (two-bit digits).  Q = [1, 5, 1, 5, 5]: slots are indices 1, 3, 4
    # (digits 01, 10, 11); index 2 sits between slots 1 and 2 (pointer 01,
    # slot 01); index 0 sits left of slot 1 (pointer 00, slot 01).
    C, L = ppe_numerical([1, 5, 1, 5, 5], digit_bits=2)
    assert list(L) == [2, 1, 2, 1, 1]
    assert [int(c) for c in C] == [0b0001, 0b01, 0b0101, 0b10, 0b11]
    g = golden["prefix_preserving_toy"]
    # the paper's A = 0001 < C = 01 under as-if padding, and E = 0110 shares C's prefix
    a, c, e = int(g["A"], 2), int(g["C"], 2), int(g["E"], 2)
    pa, pc, pe = padded([a, c, e], [2, 1, 2], 2, digit_bits=2)
    assert pa < pc < pe


def test_depth_cut_wide_leaf_by_hand():
    # M = 4, 40 equally frequent values.  Root slots: indices 0,1,2.  Right of
    # them (3..39, 37 values) a level-1 node: slots 3,4,5 under pointer 11.
    # Right of those (6..39, 34 values) the depth cut makes one leaf of
    # beta = 3 digits (4^3 = 64 >= 35), slot numbers 1..34.
    C, L = ppe_numerical(np.ones(40), digit_bits=2)
    assert [int(c) for c in C[:3]] == [1, 2, 3] and set(L[:3]) == {1}
    assert [int(c) for c in C[3:6]] == [0b1101, 0b1110, 0b1111] and set(L[3:6]) == {2}
    prefix = 0b1111
    assert [int(c) for c in C[6:]] == [(prefix << 6) + k for k in range(1, 35)]
    assert set(L[6:]) == {5}
    # slot 4 is digits 010 base 4... i.e. 0,1,0: a zero last digit, as in the paper's
    # wide leaves; it still differs from every other code once padded
    assert int(C[6 + 3]) & 0b11 == 0
    P = padded(C, L, 5, digit_bits=2)
    assert np.all(np.diff(P.astype(np.float64)) > 0)


def _nodes(C, L, digit_bits=8):
    """Map pointer path (prefix value, prefix length) -> (slot count, has children)."""
    nodes = {}
    for c, l in zip(C.tolist(), L.tolist()):
        for p in range(0, l):
            key = (c >> (digit_bits * (l - p)), p)
            ent = nodes.setdefault(key, [0, False])
            if p == l - 1:
                ent[0] += 1
            else:
                ent[1] = True
    return nodes


@pytest.mark.parametrize("s,w,n", [(1.0, 12, 200_000), (0.5, 16, 300_000), (1.5, 12, 100_000), (1.0, 20, 400_000)])
def test_properties_on_zipf_columns(s, w, n):
    x = datagen.zipf_column(n, w, s, seed=11)
    A, Q, _ = build_dictionary(x)
    C, L = ppe_numerical(Q)
    nd = A.shape[0]
    K = int(L.max())
    # max length: two internal levels, then a leaf of ceil(log256(n+1)) bytes
    assert K <= 2 + digits_needed(nd + 1, 256)
    # order preserving and unique under as-if padding
    P = padded(C, L, K)
    assert np.all(P[1:] > P[:-1])
    # the 255 most frequent values (ties: smaller index) are exactly the 1-byte codes
    if nd >= 256:
        top = np.sort(np.argsort(-Q, kind="stable")[:255])
        assert np.array_equal(np.nonzero(L == 1)[0], top)
    # Property 1: every node with children is full (255 slots)
    for (prefix, plen), (slots, has_children) in _nodes(C, L).items():
        if has_children:
            assert slots == 255, (prefix, plen, slots)
    # when a code is a proper prefix of another, the longer one's rest is not zero
    codes = set(zip(C.tolist(), L.tolist()))
    for c, l in zip(C.tolist(), L.tolist()):
        for p in range(1, l):
            if (c >> (8 * (l - p)), p) in codes:
                assert c & ((1 << (8 * (l - p))) - 1) != 0


def test_sorted_mapping_reaches_wide_leaf():
    # hot values are the smallest ones: the tail past the last level-1 slot is
    # larger than 255 values, so the depth cut makes a 2-byte-slot leaf (K = 4)
    x = datagen.zipf_column(300_000, 16, 1.0, seed=3, mapping=datagen.SORTED)
    A, Q, _ = build_dictionary(x)
    C, L = ppe_numerical(Q)
    assert int(L.max()) == 4
    P = padded(C, L, 4)
    assert np.all(P[1:] > P[:-1])
    assert np.any((L == 4) & ((C & np.uint64(0xFF)) == 0))   # a zero last byte exists


def test_categorical_closed_forms():
    # Algorithm 2: B = ceil(log256(n+1)) levels; all but the last are full
    C, L = ppe_categorical(255)
    assert list(C) == list(range(1, 256)) and set(L) == {1}
    C, L = ppe_categorical(300)
    assert list(C[:255]) == list(range(1, 256))
    # last level slot-major: slot 1 under pointers 0..44
    assert [int(c) for c in C[255:]] == [(j << 8) + 1 for j in range(45)]
    assert set(L[255:]) == {2}
    n = 255 + 256 * 255 + 10
    C, L = ppe_categorical(n)
    assert (L == 1).sum() == 255 and (L == 2).sum() == 256 * 255 and (L == 3).sum() == 10
    # Property 2: balanced (lengths differ by at most... all leaves on the last level)
    assert set(L.tolist()) == {1, 2, 3}
    P = padded(C, L, 3)
    assert np.unique(P).shape[0] == n
