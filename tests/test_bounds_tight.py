"""The bounds of oracle.bounds are tight: just outside each one a concrete input
gives a wrong residue (exact integers or the bit-exact float emulation), just
inside the worst-case input (and random ones) give the right residue."""
import numpy as np
import pytest

from oracle import bounds, emulate
from oracle import reference as ref


def test_t1_eq3_lower_bound_tight():
    # k (p-1)^2 = Q: the degree-d coefficient equals Q and its digit reads 0.
    p, t, d = 3, 8, 5
    k = (1 << t) // (p - 1) ** 2          # 64: eq. (3) fails by equality
    assert not bounds.eq3_lower_ok(p, k, t)
    A = np.full((1, k), p - 1, np.uint8)
    B = np.full((k, 1), p - 1, np.uint8)
    assert ref.qadic_product_mod_p(A, B, p, t, d)[0, 0] != ref.modmul(A, B, p)[0, 0]
    # one less: eq. (3) holds, worst case and random inputs are exact
    k -= 1
    assert bounds.eq3_lower_ok(p, k, t)
    A = np.full((1, k), p - 1, np.uint8)
    B = np.full((k, 1), p - 1, np.uint8)
    assert ref.qadic_product_mod_p(A, B, p, t, d)[0, 0] == ref.modmul(A, B, p)[0, 0]
    rng = np.random.default_rng(1)
    A, B = rng.integers(0, p, (8, k), np.uint8), rng.integers(0, p, (k, 8), np.uint8)
    np.testing.assert_array_equal(ref.qadic_product_mod_p(A, B, p, t, d), ref.modmul(A, B, p))
    # the same at the next t (what the strict reading of eq. (3) picks for k = 64)
    A = np.full((1, 64), p - 1, np.uint8)
    B = np.full((64, 1), p - 1, np.uint8)
    assert ref.qadic_product_mod_p(A, B, p, 9, 4)[0, 0] == ref.modmul(A, B, p)[0, 0]


def test_t2_high_part_bound_tight():
    # Offset regime, 24-bit mantissa, p = 2, Q = 2^13, d = 1.  The high part may reach
    # 2^(beta-1) once N = 1025 chunks: then the accumulator leaves [M, 2M), the float
    # spacing doubles and a chunk with odd high part rounds up.
    p, beta, t, d = 2, 24, 13, 1
    assert bounds.offset_ok(p, 2046, t, d, beta) and not bounds.offset_ok(p, 2050, t, d, beta)
    assert bounds.eq3_lower_ok(p, 2050, t) and 2 * bounds.low_max(p, t, d) < (1 << t)
    bad_a = np.array([1] * 2048 + [0, 1], np.uint8)
    bad_b = np.array([1] * 2048 + [1, 1], np.uint8)
    want = int(bad_a.astype(int) @ bad_b.astype(int)) % p
    assert emulate.qadic_entry(bad_a, bad_b, p, t, d, beta, "offset") != want
    ok_a = np.array([1] * 2044 + [0, 1], np.uint8)
    ok_b = np.array([1] * 2044 + [1, 1], np.uint8)
    assert emulate.qadic_entry(ok_a, ok_b, p, t, d, beta, "offset") == int(ok_a.astype(int) @ ok_b.astype(int)) % p
    ones = np.ones(2046, np.uint8)
    assert emulate.qadic_entry(ones, ones, p, t, d, beta, "offset") == 2046 % p


def test_t3_low_part_rounding_bound_tight():
    # Offset regime, one product per rounding: a product whose low part reaches Q^d/2
    # rounds up and adds one to the extracted digit.
    p, beta, t = 3, 53, 5
    d, k = 4, 5
    assert 2 * bounds.low_max(p, t, d) >= (1 << (t * d))
    assert not bounds.offset_ok(p, k, t, d, beta)
    a = np.full(k, p - 1, np.uint8)
    assert emulate.qadic_entry(a, a, p, t, d, beta, "offset") != (k * (p - 1) ** 2) % p
    d = 3
    for k in (4, 7):
        assert bounds.offset_ok(p, k, t, d, beta)
        a = np.full(k, p - 1, np.uint8)
        assert emulate.qadic_entry(a, a, p, t, d, beta, "offset") == (k * (p - 1) ** 2) % p
    rng = np.random.default_rng(5)
    for _ in range(50):
        a, b = rng.integers(0, p, 7, np.uint8), rng.integers(0, p, 7, np.uint8)
        assert emulate.qadic_entry(a, b, p, t, 3, beta, "offset") == int(a.astype(int) @ b.astype(int)) % p


def test_t3_grouped_summation_needs_the_g_factor():
    # If g products were summed exactly before one rounding, g * low_max must stay
    # below Q^d/2; p=3, t=7, d=5 is fine one product at a time but not four at a time.
    p, beta, t, d = 3, 53, 7, 5
    k = 24
    assert bounds.offset_ok(p, k, t, d, beta, g=1) and not bounds.offset_ok(p, k, t, d, beta, g=4)
    a = np.full(k, p - 1, np.uint8)
    want = (k * (p - 1) ** 2) % p
    assert emulate.qadic_entry(a, a, p, t, d, beta, "offset", g=1) == want
    assert emulate.qadic_entry(a, a, p, t, d, beta, "offset", g=4) != want


def test_t4_int32_bound_tight():
    # Centred residues of p = 251 lie in [-125, 125]; k products of 125*125 overflow
    # int32 exactly from k = 137439 on.
    p = 251
    assert bounds.int32_ok(p, 137438) and not bounds.int32_ok(p, 137439)
    assert ref.centre(np.array([125, 126, 250, 0]), p).tolist() == [125, -125, -1, 0]
    for k, fits in ((137438, True), (137439, False)):
        exact = k * 125 * 125
        got = emulate.int32_dot_wrapped(np.full(k, 125), np.full(k, 125))
        assert (got == exact) == fits


def test_exact_regime_is_exact_for_any_order():
    # Inside the exact regime the emulated accumulation equals S for any grouping.
    p, beta = 7, 53
    k = 4096
    t = bounds.smallest_t(p, k)
    d = 1
    assert (t, bounds.exact_ok(p, k, t, d, beta)) == (18, True)
    a = np.full(k, p - 1, np.uint8)
    for g in (1, 4, 2048):
        assert emulate.qadic_entry(a, a, p, t, d, beta, "exact", g=g) == (k * (p - 1) ** 2) % p


@pytest.mark.parametrize("p,k", [(3, 64), (3, 16384), (7, 4096), (101, 6688)])
def test_offset_regime_worst_case_and_random(p, k):
    # The regimes that the large workloads use give exact residues on the worst case.
    beta = 53
    t = bounds.smallest_t(p, k)
    d = max(dd for dd in range(0, 60) if bounds.qadic_regime(p, k, t, dd, beta) and dd <= k - 1)
    a = np.full(k, p - 1, np.uint8)
    regime = bounds.qadic_regime(p, k, t, d, beta)
    assert emulate.qadic_entry(a, a, p, t, d, beta, regime) == (k * (p - 1) ** 2) % p
    rng = np.random.default_rng(k)
    for _ in range(3):
        x, y = rng.integers(0, p, k, np.uint8), rng.integers(0, p, k, np.uint8)
        assert emulate.qadic_entry(x, y, p, t, d, beta, regime) == int(x.astype(int) @ y.astype(int)) % p


def test_redq_one_division_identity():
    # REDQ reads every digit mod p from one quotient by p: floor(floor(r/p)/Q^i)
    # equals floor(floor(r/Q^i)/p), so floor(r/Q^i) mod p = (r >> ti) - p (s >> ti).
    rng = np.random.default_rng(2)
    for _ in range(2000):
        t = int(rng.integers(1, 27))
        d = int(rng.integers(0, 52 // t))
        p = int(rng.integers(2, 300))
        r = int(rng.integers(0, 1 << (t * (d + 1))))
        s = r // p
        for i in range(d + 1):
            assert (r >> (t * i)) - p * (s >> (t * i)) == (r >> (t * i)) % p


def test_e2m1_table_and_which_primes_fit():
    # the e2m1 format's sixteen codes decode to the published magnitudes
    mags = sorted({abs(bounds.e2m1_value(c)) for c in range(16)})
    assert [float(v) for v in mags] == [0, 0.5, 1, 1.5, 2, 3, 4, 6]
    assert bounds.e2m1_value(0b0101) == 3 and bounds.e2m1_value(0b1110) == -4 and bounds.e2m1_value(0b1000) == 0
    # centred residues are exact e2m1 values up to p = 9 (|x| <= 4); from p = 10 on
    # some |x| = 5 appears, which e2m1 cannot hold
    assert all(bounds.fp4_representable(p) for p in range(2, 10))
    assert not any(bounds.fp4_representable(p) for p in range(10, 40))


@pytest.mark.parametrize("p", (7, 8))
def test_fp32_accumulation_bound_is_tight(p):
    # Worst case: every product is h^2 (h = floor(p/2)) and the block starts from the
    # residue p - 1.  Summed in 64-product groups (one MFMA) with one rounding to
    # 24 significant bits per group: exact at the largest admissible block, wrong
    # one product later, where the sum is an odd integer above 2^24.
    h = bounds.centred_max(p)
    kb = ((1 << 24) - (p - 1)) // (h * h)
    assert bounds.fp4_block_ok(p, kb) and not bounds.fp4_block_ok(p, kb + 1)
    inside = emulate.accumulate([h] * kb, [h] * kb, 24, start=p - 1, g=64)
    assert inside == kb * h * h + (p - 1)
    exact = (kb + 1) * h * h + (p - 1)
    outside = emulate.accumulate([h] * (kb + 1), [h] * (kb + 1), 24, start=p - 1, g=64)
    assert exact % 2 and exact > 1 << 24           # odd above 2^24: not a float32
    assert outside != exact and outside % p != exact % p



# --- full compression (section 4): eqs. (6) and (7) -------------------------
@pytest.mark.parametrize("beta,outside,inside", [(24, (5, 5), (2, 11)), (53, (6, 9), (4, 13))])
def test_eq7_full_word_bound_tight(beta, outside, inside):
    # p = 2, k = 1, Q = 2 (eq. (3): 1 < 2).  All-ones operands make the product word
    # sum_{i,j} Q^i Theta^j = 2^D - 1 with D = (d_q+1)(d_theta+1) digits.  With D one
    # past the mantissa the single rounded product lands on 2^D: every digit reads 0.
    p, k, t = 2, 1, 1
    for (eq_, eth), ok in ((outside, False), (inside, True)):
        dq, dth = eq_ - 1, eth - 1
        assert bounds.full_ok(p, k, t, dq, dth, beta) == ok
        A = np.ones((eq_, k), np.uint8)
        B = np.ones((k, eth), np.uint8)
        a = int(ref.compress_left(A, t, dq)[0, 0])
        b = int(ref.compress_full_right(B, t, dq, dth)[0, 0])
        w = emulate.accumulate([a], [b], beta)
        got = ref.redq_full(np.array([[w]], dtype=object), t, dq, dth, p, eq_, eth)
        want = ref.modmul(A, B, p)
        assert np.array_equal(got, want) == ok
    # (the strict form of eq. (7) also leaves out t D = beta, where the largest word
    # 2^beta - 1 is still exact; t D = beta + 1 is the first failure)
    assert outside[0] * outside[1] == beta + 1


def test_eq6_theta_bound_tight():
    # Theta = Q^(d_q+1) / 2 lets coefficient (d_q, 0) run into coefficient (0, 1):
    # the worst-case input is wrong; Theta = Q^(d_q+1) is exact.
    p, k, t, dq, dth = 3, 2, 4, 1, 1        # k (p-1)^2 = 8 < Q = 16
    A = np.full((2, k), p - 1, np.uint8)
    B = np.full((k, 2), p - 1, np.uint8)
    want = ref.modmul(A, B, p)
    np.testing.assert_array_equal(ref.full_compressed_product_mod_p(A, B, p, t, dq, dth), want)
    bad = ref.full_compressed_product_mod_p(A, B, p, t, dq, dth, theta_t=t * (dq + 1) - 1)
    assert not np.array_equal(bad, want)


def test_eq3_bound_tight_for_full_compression():
    # k (p-1)^2 = Q: a coefficient of Q^i Theta^j reaches Q and reads 0.
    p, t, dq, dth = 3, 6, 1, 1
    k = (1 << t) // (p - 1) ** 2
    A = np.full((2, k), p - 1, np.uint8)
    B = np.full((k, 2), p - 1, np.uint8)
    assert not bounds.full_ok(p, k, t, dq, dth, 53)
    assert not np.array_equal(ref.full_compressed_product_mod_p(A, B, p, t, dq, dth), ref.modmul(A, B, p))
    k -= 1
    A, B = A[:, :k], B[:k]
    assert bounds.full_ok(p, k, t, dq, dth, 53)
    np.testing.assert_array_equal(ref.full_compressed_product_mod_p(A, B, p, t, dq, dth), ref.modmul(A, B, p))
