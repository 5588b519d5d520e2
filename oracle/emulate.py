"""Bit-exact emulation of the method's floating-point accumulation (test infrastructure only).

Floating-point numbers are modelled as integers rounded to beta significant bits
(round to nearest, ties to even), which is exact for the integer-valued words of
the method.  A fused multiply-add rounds once; a "group" of g products is summed
exactly and added with one rounding.  With these the tests show each bound of
oracle.bounds tight.
"""
from __future__ import annotations

from . import reference


def round_to_beta(x: int, beta: int) -> int:
    """Nearest integer with at most beta significant bits (ties to even)."""
    if x == 0:
        return 0
    s = -1 if x < 0 else 1
    a = -x if x < 0 else x
    drop = a.bit_length() - beta
    if drop <= 0:
        return x
    q, r = divmod(a, 1 << drop)
    half = 1 << (drop - 1)
    if r > half or (r == half and (q & 1)):
        q += 1
    return s * (q << drop)


def accumulate(words_a, words_b, beta: int, start: int = 0, g: int = 1) -> int:
    """acc = start; for each group of g products: acc = round(acc + exact group sum)."""
    acc = start
    n = len(words_a)
    for l0 in range(0, n, g):
        grp = sum(int(words_a[l]) * int(words_b[l]) for l in range(l0, min(n, l0 + g)))
        acc = round_to_beta(acc + grp, beta)
    return acc


def qadic_entry(a_row, b_col, p: int, t: int, d: int, beta: int, regime: str, g: int = 1) -> int:
    """One entry of procedure (2) through the emulated accumulation.

    regime 'exact' : accumulator starts at 0, digit d of the final word (the paper's
                     init routine: scale by Q^-d, floor, keep t bits, reduce).
    regime 'offset': accumulator starts at M = 2^(beta-1) Q^d, digit d of T - M.
    """
    import numpy as np

    ca = reference.compress_rows_rev(np.asarray(a_row, dtype=np.uint8)[None, :], t, d)[0]
    cb = reference.compress_cols_fwd(np.asarray(b_col, dtype=np.uint8)[:, None], t, d)[:, 0]
    M = (1 << (beta - 1)) << (t * d) if regime == "offset" else 0
    T = accumulate(ca, cb, beta, start=M, g=g)
    return (((T - M) >> (t * d)) % (1 << t)) % p


def int32_dot_wrapped(a, b) -> int:
    """Dot product of centred residues accumulated in two's-complement int32."""
    acc = 0
    for x, y in zip(a, b):
        acc = (acc + int(x) * int(y)) & 0xFFFFFFFF
    return acc - (1 << 32) if acc >= (1 << 31) else acc
