"""Table 1 of the paper (compression factors modulo 3, 53-bit mantissa, Q = 2^t)
against the selection rule of oracle.bounds, from the golden transcription."""
import os

import numpy as np

from oracle import bounds
from oracle import reference as ref

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table1_mod3.txt")


def load_table1():
    cols = []
    with open(GOLDEN) as f:
        lines = [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]
    for t, dim, comp, deg in lines[1:]:
        lo, _, hi = comp.partition("-")
        cols.append(dict(t=int(t), dim=int(dim), comp=(int(lo), int(hi or lo)),
                         degree=None if deg == "-" else int(deg)))
    return cols


def test_table1_transcription_shape():
    cols = load_table1()
    assert [c["t"] for c in cols] == [3, 4, 5, 6, 7, 8, 10, 13, 17]
    # each printed dimension limit is Q/(p-1)^2 = 2^t / 4
    assert all(c["dim"] == (1 << c["t"]) // 4 for c in cols)


def test_table1_reproduced_by_non_strict_reading():
    # Read eq. (3) as k (p-1)^2 <= Q: the rule then gives every printed column, over
    # the whole dimension range the column covers (the first column is printed for
    # the single dimension 2, the others for "<= dim").  A column prints the largest
    # Q with its compression factor: t = 9, 11, 12, 14, 15, 16 give the same e as the
    # next printed column and are folded into it.
    cols = load_table1()
    prev = cols[0]["dim"] - 1
    for c in cols:
        for k in range(prev + 1, c["dim"] + 1):
            t, d = bounds.paper_choice(3, k, 53, strict=False)
            assert t <= c["t"] and 53 // t == 53 // c["t"], (k, t, c)
            e = 53 // t
            assert min(e, k) == d + 1
            if c["comp"][0] == c["comp"][1] and k >= e:
                assert d + 1 == c["comp"][0]
            if c["degree"] is not None and k >= e:
                assert d == c["degree"]
        lo, hi = c["comp"]
        assert lo <= min(53 // c["t"], c["dim"]) <= hi
        prev = c["dim"]


def test_table1_strict_reading_differs_only_at_range_tops():
    # With the strict eq. (3) every k strictly inside a column keeps the printed t;
    # the printed top end k = Q/(p-1)^2 needs the next power of two.
    prev = 0
    for c in load_table1():
        for k in range(prev + 1, c["dim"]):
            t = bounds.paper_choice(3, k, 53)[0]
            assert t <= c["t"] and 53 // t == 53 // c["t"]
        assert bounds.paper_choice(3, c["dim"], 53)[0] > c["t"]
        prev = c["dim"]


def test_table1_top_end_is_wrong_on_all_p_minus_one():
    # At k = Q/(p-1)^2 the printed (Q, d) returns a wrong residue (exact integers),
    # which is why the strict reading is the one the library enforces.
    for c in load_table1()[3:6]:          # t = 6, 7, 8 keep the exact model small
        k, t, d = c["dim"], c["t"], c["degree"]
        A = np.full((1, k), 2, np.uint8)
        B = np.full((k, 1), 2, np.uint8)
        assert ref.qadic_product_mod_p(A, B, 3, t, d)[0, 0] != ref.modmul(A, B, 3)[0, 0]
        A1, B1 = A[:, :k - 1], B[:k - 1]
        assert ref.qadic_product_mod_p(A1, B1, 3, t, d)[0, 0] == ref.modmul(A1, B1, 3)[0, 0]


def test_compression_factor_section5():
    assert [bounds.compression_factor(t, 53) for t in (3, 5, 6, 10, 17, 26, 27)] == [17, 10, 8, 5, 3, 2, 1]
    assert [bounds.compression_factor(t, 24) for t in (11, 12, 13)] == [2, 2, 1]
