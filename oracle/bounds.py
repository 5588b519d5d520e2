"""The paper's bounds on Q = 2^t and d, and the regimes where the floating-point
accumulation of packed words is provably exact (test infrastructure only).

All arithmetic is on Python integers / fractions: no rounding.

Pins: tests/test_bounds_tight.py shows each bound tight with the bit-exact
emulation in oracle.emulate (a concrete wrong result just outside, the
worst-case input correct just inside); tests/test_choose_qd.py checks the
paper's selection rule against Table 1 (tests/golden/table1_mod3.txt).
"""
from __future__ import annotations

from fractions import Fraction


def ceil_div(a: int, b: int) -> int:
    return -(-a // b)


# -- eq. (3), section 2.4 ----------------------------------------------------
def eq3_lower_ok(p: int, k: int, t: int) -> bool:
    """Delayed reduction: k (p-1)^2 < Q, so the degree-d coefficient never reaches Q."""
    return k * (p - 1) ** 2 < (1 << t)


def smallest_t(p: int, k: int, strict: bool = True) -> int:
    """Smallest t with k (p-1)^2 < 2^t (eq. (3)); strict=False uses <= instead."""
    t = 1
    while not (eq3_lower_ok(p, k, t) if strict else k * (p - 1) ** 2 <= (1 << t)):
        t += 1
    return t


# -- eq. (4) and its sum form, section 2.5 ----------------------------------
def eq4_upper_ok(t: int, d: int, beta: int) -> bool:
    """Q^(d+1) < 2^beta."""
    return t * (d + 1) < beta


def eq4_sum_form(p: int, k, t: int, d: int) -> Fraction:
    """Left side of the sharper form: sum_{i=0..d} (k/(d+1)) (i+1) (p-1)^2 Q^(d-i).

    This is the largest possible high part c_H = floor(S / Q^d) when every residue
    equals p-1 and k is a multiple of d+1.
    """
    Q = 1 << t
    return sum(Fraction(k, d + 1) * (i + 1) * (p - 1) ** 2 * Q ** (d - i) for i in range(d + 1))


def compression_factor(t: int, beta: int) -> int:
    """e = floor(beta / log2 Q) (section 5)."""
    return beta // t


def paper_choice(p: int, k: int, beta: int = 53, strict: bool = True):
    """The paper's rule (sections 2.4-2.6, 5): smallest t allowed by eq. (3), then
    d = min(e, k) - 1 with e = floor(beta / t).  Returns (t, d).

    strict=False reads eq. (3) as k (p-1)^2 <= Q, the reading under which Table 1
    was printed (its dimension ranges end at Q/(p-1)^2)."""
    t = smallest_t(p, k, strict)
    return t, min(compression_factor(t, beta), k) - 1


# -- exactness regimes of the floating-point accumulation --------------------
def coeff_max(p: int, N: int, d: int, j: int) -> int:
    """Largest value of coefficient j of a sum of N products of chunk polynomials of
    degree d with entries in [0, p-1]: N (p-1)^2 times the number of index pairs."""
    pairs = j + 1 if j <= d else 2 * d + 1 - j
    return N * (p - 1) ** 2 * max(pairs, 0)


def s_max(p: int, kb: int, t: int, d: int) -> int:
    """Largest exact sum S = sum_l abar_l bbar_l over N = ceil(kb/(d+1)) chunks."""
    N = ceil_div(kb, d + 1)
    Q = 1 << t
    return sum(coeff_max(p, N, d, j) * Q ** j for j in range(2 * d + 1))


def high_max(p: int, kb: int, t: int, d: int) -> int:
    """Largest high part c_H = sum_{j>=d} c_j Q^(j-d)."""
    N = ceil_div(kb, d + 1)
    Q = 1 << t
    return sum(coeff_max(p, N, d, j) * Q ** (j - d) for j in range(d, 2 * d + 1))


def word_max(p: int, t: int, d: int) -> int:
    """Largest packed word (p-1)(1 + Q + ... + Q^d)."""
    return (p - 1) * sum(1 << (t * j) for j in range(d + 1))


def low_max(p: int, t: int, d: int) -> int:
    """Largest low part sum_{j<d} c_j Q^j of ONE product of two chunk words."""
    Q = 1 << t
    return sum((j + 1) * (p - 1) ** 2 * Q ** j for j in range(d))


def exact_ok(p: int, kb: int, t: int, d: int, beta: int) -> bool:
    """Exact regime: eq. (3) and S_max < 2^beta.  Every product and partial sum is an
    integer below 2^beta, so any summation order is exact and the word holds S."""
    return (d >= 0 and t >= 1 and eq3_lower_ok(p, kb, t) and word_max(p, t, d) < (1 << beta)
            and s_max(p, kb, t, d) < (1 << beta))


def offset_ok(p: int, kb: int, t: int, d: int, beta: int, g: int = 1) -> bool:
    """Offset regime: the accumulator starts at M = 2^(beta-1) Q^d (the Q^(2d+1)
    addition of section 2.5, moved to the start).  Conditions:
      (i)   eq. (3);
      (ii)  the sum form of eq. (4) with one bit less, high_max < 2^(beta-1), so every
            partial sum stays in [M, 2M) where the spacing of floats is exactly Q^d;
      (iii) g * low_max < Q^d / 2, so each rounding step (g products per step) lands
            on the multiple of Q^d just below.
    The word then holds M + floor(S / Q^d) Q^d, whatever the order of the steps.
    The packed words themselves must be exact floats: word_max < 2^beta.
    """
    return (d >= 0 and t >= 1 and eq3_lower_ok(p, kb, t) and word_max(p, t, d) < (1 << beta)
            and high_max(p, kb, t, d) < (1 << (beta - 1))
            and 2 * g * low_max(p, t, d) < (1 << (t * d)))


def qadic_regime(p: int, kb: int, t: int, d: int, beta: int, g: int = 1):
    """'exact' if exact_ok, else 'offset' if offset_ok, else None."""
    if exact_ok(p, kb, t, d, beta):
        return "exact"
    if offset_ok(p, kb, t, d, beta, g):
        return "offset"
    return None


def redq_ok(p: int, k: int, t: int, d: int, beta: int) -> bool:
    """Right-compressed product (section 3): eqs. (3) and (4).  Every coefficient stays
    below Q and every word below Q^(d+1) < 2^beta, so the accumulation is exact."""
    return eq3_lower_ok(p, k, t) and eq4_upper_ok(t, d, beta)


def centred_max(p: int) -> int:
    """max |x - p [x > (p-1)//2]| over x in [0, p-1]."""
    return p // 2


def int32_ok(p: int, kb: int) -> bool:
    """kb products of centred residues never leave the int32 range."""
    return kb * centred_max(p) ** 2 <= (1 << 31) - 1


# --- FP4 (e2m1) operands with FP32 accumulation --------------------------------------
# The FP4 path multiplies centred residues on the FP4 matrix cores.  It is exact when
# every centred residue is an e2m1 value and every partial sum is an integer of at
# most 2^24 in magnitude (the range where FP32 holds every integer).

def e2m1_value(code: int) -> Fraction:
    """Value of a 4-bit e2m1 code: sign bit 3, exponent bits 2..1 with bias 1, mantissa
    bit 0; exponent 0 is subnormal (0 or 1/2 before the sign)."""
    sign = -1 if code & 8 else 1
    e, mant = (code >> 1) & 3, code & 1
    if e == 0:
        return sign * Fraction(mant, 2)
    return sign * Fraction(2 + mant, 2) * (2 ** (e - 1))


def e2m1_values() -> set:
    return {e2m1_value(c) for c in range(16)}


def fp4_representable(p: int) -> bool:
    """Every centred residue x - p [x > (p-1)//2], 0 <= x < p, is an e2m1 value."""
    vals = e2m1_values()
    return all(Fraction(x - p if x > (p - 1) // 2 else x) in vals for x in range(p))


def fp4_block_ok(p: int, kb: int) -> bool:
    """A block of kb products, started from the previous block's residue (< p), keeps
    every partial sum an integer of magnitude at most 2^24."""
    return kb * centred_max(p) ** 2 + (p - 1) <= 1 << 24



# -- left and full compression (sections 4 and 5) ---------------------------
def left_ok(p: int, k: int, t: int, d: int, beta: int) -> bool:
    """Left compression (Table 2): the same words as section 3 along m instead of n,
    so the same bounds, eqs. (3) and (4)."""
    return redq_ok(p, k, t, d, beta)


def full_ok(p: int, k: int, t: int, dq: int, dth: int, beta: int) -> bool:
    """Full compression (section 4): eq. (3) for every coefficient, Theta = Q^(d_q+1)
    (eq. (6) with equality) and eq. (7), Q^((d_q+1)(d_theta+1)) < 2^beta, so every
    product word and every partial sum is an integer below 2^beta."""
    return (dq >= 0 and dth >= 0 and eq3_lower_ok(p, k, t)
            and t * (dq + 1) * (dth + 1) < beta)


def full_word_max(p: int, k: int, t: int, dq: int, dth: int) -> int:
    """Largest product word: every coefficient of Q^i Theta^j at its largest, k (p-1)^2."""
    D = (dq + 1) * (dth + 1)
    return sum(k * (p - 1) ** 2 << (t * q) for q in range(D))


def table2_word_products(algorithm: str, m: int, n: int, k: int, d: int, d2: int = 0) -> int:
    """Multiply-adds of packed words of each algorithm of Table 2 with classical
    matrix multiplication (omega = 3), for degree d (and d_theta = d2 for 'full'):
      'qadic' procedure (2): m n ceil(k/(d+1));  'right' procedure (5): m ceil(n/(d+1)) k;
      'left': ceil(m/(d+1)) n k;  'full' (section 4): ceil(m/(d+1)) ceil(n/(d2+1)) k."""
    if algorithm == "qadic":
        return m * n * ceil_div(k, d + 1)
    if algorithm == "right":
        return m * ceil_div(n, d + 1) * k
    if algorithm == "left":
        return ceil_div(m, d + 1) * n * k
    if algorithm == "full":
        return ceil_div(m, d + 1) * ceil_div(n, d2 + 1) * k
    raise ValueError(algorithm)
