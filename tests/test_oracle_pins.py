"""Pins of the CPU oracle against facts fixed by the paper and by the mathematics.

Each test would fail for a plausible slip in the oracle: a transposed operand, a
dropped term, a reversed word, a wrong padding side, a missing reduction.
"""
import itertools

import numpy as np
import pytest

from oracle import reference as ref

PRIMES = (2, 3, 5, 7, 11, 13, 31, 101, 251)


def rnd(rng, shape, p):
    return rng.integers(0, p, size=shape, dtype=np.uint8)


# --- the product: brute force and invariants ------------------------------
@pytest.mark.parametrize("p", PRIMES)
def test_modmul_matches_bruteforce(p):
    rng = np.random.default_rng(p)
    for m, n, k in [(1, 1, 1), (2, 3, 4), (5, 1, 7), (8, 8, 8), (3, 7, 1), (7, 2, 5)]:
        A, B = rnd(rng, (m, k), p), rnd(rng, (k, n), p)
        np.testing.assert_array_equal(ref.modmul(A, B, p), ref.modmul_bruteforce(A, B, p))


def test_modmul_degenerate_shapes():
    A = np.zeros((3, 0), np.uint8)
    B = np.zeros((0, 4), np.uint8)
    np.testing.assert_array_equal(ref.modmul(A, B, 5), np.zeros((3, 4), np.uint8))
    assert ref.modmul(np.zeros((0, 3), np.uint8), np.zeros((3, 2), np.uint8), 5).shape == (0, 2)


def test_modmul_reduces_bytes_beyond_p():
    # The definition reduces the exact integer dot product: inputs >= p are allowed.
    rng = np.random.default_rng(0)
    A = rng.integers(0, 256, (6, 9), dtype=np.uint8)
    B = rng.integers(0, 256, (9, 5), dtype=np.uint8)
    exact = A.astype(np.int64) @ B.astype(np.int64)
    np.testing.assert_array_equal(ref.modmul(A, B, 7), (exact % 7).astype(np.uint8))


@pytest.mark.parametrize("p", (3, 7, 101))
def test_modmul_invariants(p):
    rng = np.random.default_rng(10 + p)
    m, k, n, r = 37, 53, 41, 29
    A, B, B2 = rnd(rng, (m, k), p), rnd(rng, (k, n), p), rnd(rng, (k, n), p)
    Cm = rnd(rng, (n, r), p)
    I = np.eye(k, dtype=np.uint8)
    # identity and zero
    np.testing.assert_array_equal(ref.modmul(A, I, p), A % p)
    np.testing.assert_array_equal(ref.modmul(A, np.zeros((k, n), np.uint8), p), 0)
    # associativity (AB)C = A(BC)
    AB = ref.modmul(A, B, p)
    np.testing.assert_array_equal(ref.modmul(AB, Cm, p), ref.modmul(A, ref.modmul(B, Cm, p), p))
    # distributivity A(B + B2) = AB + AB2
    s = ((B.astype(np.int64) + B2) % p).astype(np.uint8)
    rhs = (ref.modmul(A, B, p).astype(np.int64) + ref.modmul(A, B2, p)) % p
    np.testing.assert_array_equal(ref.modmul(A, s, p), rhs)
    # linearity (alpha A) B = alpha (A B)
    alpha = 2 if p > 2 else 1
    aA = ((alpha * A.astype(np.int64)) % p).astype(np.uint8)
    np.testing.assert_array_equal(ref.modmul(aA, B, p), (alpha * AB.astype(np.int64)) % p)
    # transpose (AB)^T = B^T A^T
    np.testing.assert_array_equal(ref.modmul(np.ascontiguousarray(B.T), np.ascontiguousarray(A.T), p), AB.T)


@pytest.mark.parametrize("p,k", [(3, 1), (3, 64), (7, 4096), (101, 777), (251, 1000)])
def test_all_p_minus_one_closed_form(p, k):
    # every entry p-1: each C_ij = k (p-1)^2 = k (mod p)
    A = np.full((5, k), p - 1, np.uint8)
    B = np.full((k, 6), p - 1, np.uint8)
    np.testing.assert_array_equal(ref.modmul(A, B, p), k % p)


def _tuples(p, n=8, cap=3000):
    """All of GF(p)^n when that is small, else a seeded sample of it."""
    if p ** n <= 20000:
        return itertools.product(range(p), repeat=n)
    rng = np.random.default_rng(p)
    return (tuple(int(v) for v in rng.integers(0, p, n)) for _ in range(cap))


def _paley(q):
    squares = {(x * x) % q for x in range(1, q)}
    idx = np.arange(q)
    diff = (idx[:, None] - idx[None, :]) % q
    return np.isin(diff, list(squares)).astype(np.uint8)


@pytest.mark.parametrize("q", (5, 13, 17, 29, 101, 401, 1009))
@pytest.mark.parametrize("p", (3, 5, 7))
def test_paley_graph_closed_form(q, p):
    # The Paley graph on a prime q = 1 (mod 4) is strongly regular with parameters
    # (q, (q-1)/2, (q-5)/4, (q-1)/4):  A^2 = (q-1)/2 I + (q-5)/4 A + (q-1)/4 (J - I - A).
    A = _paley(q)
    assert (A == A.T).all() and A.diagonal().sum() == 0
    I = np.eye(q, dtype=np.int64)
    J = np.ones((q, q), np.int64)
    want = ((q - 1) // 2 * I + (q - 5) // 4 * A + (q - 1) // 4 * (J - I - A)) % p
    np.testing.assert_array_equal(ref.modmul(A, A, p), want)


def test_modmul_entries_match_full():
    rng = np.random.default_rng(3)
    A, B = rnd(rng, (50, 70), 11), rnd(rng, (70, 40), 11)
    C = ref.modmul(A, B, 11)
    rows = rng.integers(0, 50, 200)
    cols = rng.integers(0, 40, 200)
    np.testing.assert_array_equal(ref.modmul_entries(A, B, 11, rows, cols), C[rows, cols])


# --- Q-adic words (section 2.1) --------------------------------------------
def test_init3_horner_order():
    # init3(r, u, v, w) computes ((u Q) + v) Q + w: the first residue gets the top power.
    t = 6
    Q = 1 << t
    u, v, w = 5, 17, 33
    word = ref.compress_rows_rev(np.array([[u, v, w]], np.uint8), t, 2)[0, 0]
    assert int(word) == (u * Q + v) * Q + w
    # the forward word of a column puts its first residue at Q^0
    fwd = ref.compress_cols_fwd(np.array([[u], [v], [w]], np.uint8), t, 2)[0, 0]
    assert int(fwd) == u + v * Q + w * Q * Q


def test_partial_compression_padding():
    # Section 2.3: a short last chunk is zero-padded at its end; on the reversed word
    # that multiplies by Q once per missing slot, on the forward word it changes nothing.
    t, d = 5, 3
    Q = 1 << t
    a = np.array([[1, 2, 3, 4, 5, 6]], np.uint8)    # chunks [1,2,3,4] and [5,6,_,_]
    CA = ref.compress_rows_rev(a, t, d)
    assert CA.shape == (1, 2)
    assert int(CA[0, 1]) == (5 * Q + 6) * Q * Q
    b = a.T.copy()
    CB = ref.compress_cols_fwd(b, t, d)
    assert int(CB[1, 0]) == 5 + 6 * Q


@pytest.mark.parametrize("t,d,k", [(4, 1, 5), (9, 4, 64), (7, 6, 31), (13, 3, 100), (3, 0, 9)])
def test_uncompress_roundtrip(t, d, k):
    rng = np.random.default_rng(t * 100 + d)
    A = rng.integers(0, 1 << min(t, 8), (7, k), dtype=np.uint8)
    np.testing.assert_array_equal(ref.uncompress_rows_rev(ref.compress_rows_rev(A, t, d), t, d, k), A)
    B = rng.integers(0, 1 << min(t, 8), (k, 9), dtype=np.uint8)
    np.testing.assert_array_equal(ref.uncompress_cols_fwd(ref.compress_cols_fwd(B, t, d), t, d, k), B)
    np.testing.assert_array_equal(ref.uncompress_rows_fwd(ref.compress_rows_fwd(B, t, d), t, d, 9), B)


# --- the 2x2 worked examples, enumerated exhaustively -----------------------
@pytest.mark.parametrize("p", (2, 3, 5, 7))
def test_worked_example_k_compressed(p):
    # Section 2.2: [Qa+b; Qc+d] x [e+Qg, f+Qh] = [* + (ae+bg)Q + *Q^2, ...].
    # Exhaustive over GF(p)^8 for p = 2, 3; a seeded sample of it for p = 5, 7.
    t = 7                      # Q = 128 > 2 (p-1)^2 for p <= 7
    Q = 1 << t
    for a, b, c, d_, e, f, g, h in _tuples(p):
        A = np.array([[a, b], [c, d_]], np.uint8)
        B = np.array([[e, f], [g, h]], np.uint8)
        CA = ref.compress_rows_rev(A, t, 1)
        CB = ref.compress_cols_fwd(B, t, 1)
        assert [int(x) for x in CA[:, 0]] == [Q * a + b, Q * c + d_]
        assert [int(x) for x in CB[0]] == [e + Q * g, f + Q * h]
        S = ref.packed_product_exact(CA, CB)
        assert (int(S[0, 0]) >> t) % Q == a * e + b * g
        assert (int(S[0, 1]) >> t) % Q == a * f + b * h
        assert (int(S[1, 0]) >> t) % Q == c * e + d_ * g
        assert (int(S[1, 1]) >> t) % Q == c * f + d_ * h
        np.testing.assert_array_equal(ref.coefficient_mod_p(S, t, 1, p),
                                      ref.modmul_bruteforce(A, B, p))


@pytest.mark.parametrize("p", (2, 3, 5, 7))
def test_worked_example_right_compressed(p):
    # Section 3: [a b; c d] x [e+Qf; g+Qh] = [(ae+bg) + Q(af+bh); (ce+dg) + Q(cf+dh)].
    t = 7
    Q = 1 << t
    for a, b, c, d_, e, f, g, h in _tuples(p):
        A = np.array([[a, b], [c, d_]], np.uint8)
        B = np.array([[e, f], [g, h]], np.uint8)
        CBr = ref.compress_rows_fwd(B, t, 1)
        assert [int(x) for x in CBr[:, 0]] == [e + Q * f, g + Q * h]
        CC = A.astype(object).dot(CBr.astype(object))
        assert int(CC[0, 0]) == (a * e + b * g) + Q * (a * f + b * h)
        assert int(CC[1, 0]) == (c * e + d_ * g) + Q * (c * f + d_ * h)
        np.testing.assert_array_equal(ref.redq(CC, t, 1, p, 2), ref.modmul_bruteforce(A, B, p))


# --- the exact-integer method equals the definition inside eq. (3) ----------
@pytest.mark.parametrize("p,k,d", [(3, 64, 4), (3, 15, 7), (7, 100, 1), (101, 50, 0),
                                   (2, 33, 9), (5, 17, 5), (13, 40, 3)])
def test_qadic_exact_model_equals_definition(p, k, d):
    from oracle import bounds
    t = bounds.smallest_t(p, k)
    rng = np.random.default_rng(k + p)
    A, B = rnd(rng, (6, k), p), rnd(rng, (k, 5), p)
    want = ref.modmul(A, B, p)
    np.testing.assert_array_equal(ref.qadic_product_mod_p(A, B, p, t, d), want)
    np.testing.assert_array_equal(ref.right_compressed_product_mod_p(A, B, p, t, d), want)


def test_extract_offset_word():
    # An accumulator started at M = 2^(beta-1) Q^d holds M + floor(S/Q^d) Q^d:
    # extract() with that offset returns digit d of S, reduced.
    t, d, p, beta = 9, 4, 3, 53
    M = (1 << (beta - 1)) << (t * d)
    S = 123456789012345678901234
    T = M + (S >> (t * d) << (t * d))
    got = ref.extract(np.array([[T]], dtype=object), t, d, p, offset=M)[0, 0]
    assert got == ((S >> (t * d)) % (1 << t)) % p


# --- left and full compression (sections 4 and 5), ReduceAndCompress (procedure (1)) --
@pytest.mark.parametrize("p", (2, 3, 5, 7))
def test_worked_example_full_compressed(p):
    # Section 4: [a+Qc, b+Qd] x [e+Theta f; g+Theta h]
    #          = (ae+bg) + Q(ce+dg) + Theta(af+bh) + Q Theta(cf+dh),
    # with A = [a b; c d] packed along m and B = [e f; g h] packed along n.
    t = 7
    Q, Th = 1 << t, 1 << (2 * t)   # Theta = Q^(d_q+1), d_q = 1 (eq. (6))
    for a, b, c, d_, e, f, g, h in _tuples(p):
        A = np.array([[a, b], [c, d_]], np.uint8)
        B = np.array([[e, f], [g, h]], np.uint8)
        CA = ref.compress_left(A, t, 1)
        CB = ref.compress_full_right(B, t, 1, 1)
        assert [int(x) for x in CA[0]] == [a + Q * c, b + Q * d_]
        assert [int(x) for x in CB[:, 0]] == [e + Th * f, g + Th * h]
        w = int(CA.astype(object).dot(CB)[0, 0])
        assert w == (a * e + b * g) + Q * (c * e + d_ * g) + Th * (a * f + b * h) + Q * Th * (c * f + d_ * h)
        np.testing.assert_array_equal(ref.full_compressed_product_mod_p(A, B, p, t, 1, 1),
                                      ref.modmul_bruteforce(A, B, p))


@pytest.mark.parametrize("p", (2, 3, 5, 7))
def test_worked_example_left_compressed(p):
    # Left compression (Table 2), the transpose of section 3's example:
    # [a+Qc, b+Qd] x [e f; g h] = [(ae+bg) + Q(ce+dg), (af+bh) + Q(cf+dh)].
    t = 7
    Q = 1 << t
    for a, b, c, d_, e, f, g, h in _tuples(p):
        A = np.array([[a, b], [c, d_]], np.uint8)
        B = np.array([[e, f], [g, h]], np.uint8)
        CA = ref.compress_left(A, t, 1)
        CC = CA.astype(object).dot(B.astype(object))
        assert int(CC[0, 0]) == (a * e + b * g) + Q * (c * e + d_ * g)
        assert int(CC[0, 1]) == (a * f + b * h) + Q * (c * f + d_ * h)
        np.testing.assert_array_equal(ref.redq_left(CC, t, 1, p, 2), ref.modmul_bruteforce(A, B, p))


def test_compress_left_is_the_transposed_row_compression():
    # Packing A along m equals packing A^T along n (section 3's row compression).
    rng = np.random.default_rng(5)
    A = rng.integers(0, 7, (11, 6), np.uint8)
    for t, d in [(5, 2), (9, 4), (17, 1)]:
        np.testing.assert_array_equal(ref.compress_left(A, t, d), ref.compress_rows_fwd(A.T.copy(), t, d).T)
        np.testing.assert_array_equal(ref.uncompress_rows_fwd(ref.compress_left(A, t, d).T, t, d, 11), A.T)


@pytest.mark.parametrize("p,k,dq,dth", [(2, 5, 3, 3), (3, 64, 1, 1), (3, 31, 2, 1), (7, 40, 1, 2),
                                        (5, 9, 2, 2), (101, 3, 0, 0), (13, 11, 1, 0), (3, 1, 4, 5)])
def test_left_and_full_models_equal_definition(p, k, dq, dth):
    t = bounds_smallest_t(p, k)
    rng = np.random.default_rng(k * p + dq)
    for m, n in [(1, 1), (7, 5), (9, 13), (4, 4)]:
        A, B = rnd(rng, (m, k), p), rnd(rng, (k, n), p)
        want = ref.modmul(A, B, p)
        np.testing.assert_array_equal(ref.full_compressed_product_mod_p(A, B, p, t, dq, dth), want)
        np.testing.assert_array_equal(ref.left_compressed_product_mod_p(A, B, p, t, dq), want)
    # worst case: every residue p-1, so every coefficient is k (p-1)^2 < Q
    A, B = np.full((5, k), p - 1, np.uint8), np.full((k, 7), p - 1, np.uint8)
    np.testing.assert_array_equal(ref.full_compressed_product_mod_p(A, B, p, t, dq, dth),
                                  np.full((5, 7), (k * (p - 1) ** 2) % p, np.uint8))


def bounds_smallest_t(p, k):
    from oracle import bounds
    return bounds.smallest_t(p, k)


@pytest.mark.parametrize("p,k,d", [(3, 64, 4), (7, 100, 1), (2, 33, 9), (5, 17, 3)])
def test_reduce_and_compress_chains_products(p, k, d):
    # Procedure (1) hands C back compressed (rows reversed, as CompressRows packs a
    # left operand), so a chain of products stays packed: A^3 = (A A) A mod p.
    t = bounds_smallest_t(p, k)
    rng = np.random.default_rng(p + k)
    A = rnd(rng, (k, k), p)
    CA = ref.compress_rows_rev(A, t, d)
    CB = ref.compress_cols_fwd(A, t, d)
    CC = ref.reduce_and_compress(ref.packed_product_exact(CA, CB), t, d, p)
    A2 = ref.modmul(A, A, p)
    np.testing.assert_array_equal(CC, ref.compress_rows_rev(A2, t, d))
    np.testing.assert_array_equal(ref.uncompress_rows_rev(CC, t, d, k), A2)
    A3 = ref.coefficient_mod_p(ref.packed_product_exact(CC, CB), t, d, p)
    np.testing.assert_array_equal(A3, ref.modmul_bruteforce(A2, A, p))
    np.testing.assert_array_equal(A3, ref.modmul(A, A2, p))   # associativity
    # the offset form of the accumulated word gives the same compressed output
    beta = 53
    M = (1 << (beta - 1)) << (t * d)
    S = ref.packed_product_exact(CA, CB)
    T = np.vectorize(lambda s: M + (int(s) >> (t * d) << (t * d)), otypes=[object])(S)
    np.testing.assert_array_equal(ref.reduce_and_compress(T, t, d, p, offset=M), CC)
