"""Plain definitions of what the compressed product computes (test infrastructure only).

Paper: Dumas, Fousse, Salvy, "Compressed Modular Matrix Multiplication".
Notation: Q = 2^t, d+1 residues per word, N = ceil(k/(d+1)) words along k.

Parity status: every function here is pinned by tests/test_oracle_pins.py
(brute force, algebraic invariants, the paper's worked examples enumerated
exhaustively, closed forms); none is "parity unpinned".
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "_oracle_modmul.so")
_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        i64, u32, vp = ctypes.c_int64, ctypes.c_uint32, ctypes.c_void_p
        lib.qmm_oracle_modmul.argtypes = [i64, i64, i64, u32, vp, i64, vp, i64, vp, i64]
        lib.qmm_oracle_modmul.restype = ctypes.c_int
        lib.qmm_oracle_modmul_entries.argtypes = [i64, vp, vp, i64, u32, vp, i64, vp, i64, vp]
        lib.qmm_oracle_modmul_entries.restype = ctypes.c_int
        lib.qmm_oracle_threads.argtypes = []
        lib.qmm_oracle_threads.restype = ctypes.c_int
        lib.qmm_oracle_set_threads.argtypes = [ctypes.c_int]
        lib.qmm_oracle_set_threads.restype = None
        _lib = lib
    return _lib


def _as_u8(x: np.ndarray) -> np.ndarray:
    x = np.ascontiguousarray(x)
    if x.dtype != np.uint8:
        raise TypeError("residue matrices are uint8")
    return x


# --------------------------------------------------------------------------
# The product itself (section 2: a dot product of residues, one reduction mod p)
# --------------------------------------------------------------------------
def modmul(A: np.ndarray, B: np.ndarray, p: int) -> np.ndarray:
    """C = (A B) mod p with 64-bit accumulation and one reduction per entry (C library)."""
    A, B = _as_u8(A), _as_u8(B)
    m, k = A.shape
    k2, n = B.shape
    if k != k2:
        raise ValueError("inner dimensions differ")
    C = np.empty((m, n), dtype=np.uint8)
    rc = _load().qmm_oracle_modmul(m, n, k, p, A.ctypes.data, k, B.ctypes.data, n,
                                   C.ctypes.data, n)
    if rc:
        raise RuntimeError(f"oracle modmul failed ({rc})")
    return C


def modmul_entries(A: np.ndarray, B: np.ndarray, p: int, rows, cols) -> np.ndarray:
    """Selected entries C[rows[e], cols[e]] of (A B) mod p, each a plain dot product."""
    A, B = _as_u8(A), _as_u8(B)
    m, k = A.shape
    _, n = B.shape
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    cols = np.ascontiguousarray(cols, dtype=np.int64)
    if rows.shape != cols.shape:
        raise ValueError("rows/cols length mismatch")
    if rows.size and (rows.min() < 0 or rows.max() >= m or cols.min() < 0 or cols.max() >= n):
        raise ValueError("entry index out of range")
    out = np.empty(rows.shape, dtype=np.uint8)
    rc = _load().qmm_oracle_modmul_entries(rows.size, rows.ctypes.data, cols.ctypes.data, k, p,
                                           A.ctypes.data, k, B.ctypes.data, n, out.ctypes.data)
    if rc:
        raise RuntimeError(f"oracle modmul_entries failed ({rc})")
    return out


def oracle_threads() -> int:
    """Number of OpenMP threads the C oracle runs with."""
    return int(_load().qmm_oracle_threads())


def set_oracle_threads(n: int) -> None:
    """Run the following C oracle products on n threads."""
    _load().qmm_oracle_set_threads(int(n))


def modmul_bruteforce(A, B, p: int):
    """Pure-Python triple loop over exact integers (tiny inputs only)."""
    A = [[int(x) for x in row] for row in np.asarray(A)]
    B = [[int(x) for x in row] for row in np.asarray(B)]
    m, k = len(A), (len(A[0]) if A else 0)
    n = len(B[0]) if B else 0
    C = [[0] * n for _ in range(m)]
    for i in range(m):
        for j in range(n):
            s = 0
            for l in range(k):
                s += A[i][l] * B[l][j]
            C[i][j] = s % p
    return np.array(C, dtype=np.uint8).reshape(m, n)


# --------------------------------------------------------------------------
# Q-adic packings (section 2.1 words, section 2.2 CA/CB, section 2.3 padding,
# section 3 row-compressed right operand)
# --------------------------------------------------------------------------
def _check_word_width(t: int, d: int) -> None:
    if t < 1 or d < 0 or t * (d + 1) > 63:
        raise ValueError("word does not fit 63 bits; use the big-integer helpers")


def compress_rows_rev(A: np.ndarray, t: int, d: int) -> np.ndarray:
    """CA[i, l] = sum_{s=0..d} A[i, l(d+1)+s] * Q^(d-s)  (the reversed word, section 2.1).

    The row is cut into chunks of d+1 residues; a short last chunk is padded with
    zeros at its end (section 2.3), which on the reversed word amounts to extra
    factors of Q.  Returns uint64 words of shape (m, ceil(k/(d+1))).
    """
    _check_word_width(t, d)
    A = np.asarray(A)
    m, k = A.shape
    e = d + 1
    N = -(-k // e)
    pad = np.zeros((m, N * e), dtype=np.uint64)
    pad[:, :k] = A
    CA = np.zeros((m, N), dtype=np.uint64)
    for s in range(e):
        CA += pad[:, s::e] << np.uint64(t * (d - s))
    return CA


def compress_cols_fwd(B: np.ndarray, t: int, d: int) -> np.ndarray:
    """CB[l, j] = sum_{s=0..d} B[l(d+1)+s, j] * Q^s  (the forward word, section 2.1).

    Zero padding at the end of a short last chunk changes nothing (section 2.3).
    Returns uint64 words of shape (ceil(k/(d+1)), n).
    """
    _check_word_width(t, d)
    B = np.asarray(B)
    k, n = B.shape
    e = d + 1
    N = -(-k // e)
    pad = np.zeros((N * e, n), dtype=np.uint64)
    pad[:k] = B
    CB = np.zeros((N, n), dtype=np.uint64)
    for s in range(e):
        CB += pad[s::e, :] << np.uint64(t * s)
    return CB


def compress_rows_fwd(B: np.ndarray, t: int, d: int) -> np.ndarray:
    """Row-compressed right operand of section 3: CBr[i, J] = sum_j B[i, J(d+1)+j] * Q^j.

    Columns past n are zero.  Returns uint64 words of shape (k, ceil(n/(d+1))).
    """
    _check_word_width(t, d)
    B = np.asarray(B)
    k, n = B.shape
    e = d + 1
    nw = -(-n // e)
    pad = np.zeros((k, nw * e), dtype=np.uint64)
    pad[:, :n] = B
    out = np.zeros((k, nw), dtype=np.uint64)
    for j in range(e):
        out += pad[:, j::e] << np.uint64(t * j)
    return out


def digit(words, t: int, j: int):
    """Coefficient of Q^j of non-negative integer words: floor(w / Q^j) mod Q."""
    w = np.asarray(words, dtype=np.uint64)
    return (w >> np.uint64(t * j)) & np.uint64((1 << t) - 1)


def uncompress_rows_rev(CA: np.ndarray, t: int, d: int, k: int) -> np.ndarray:
    """Inverse of compress_rows_rev: residue (i, l(d+1)+s) is digit d-s of CA[i, l]."""
    CA = np.asarray(CA, dtype=np.uint64)
    m, N = CA.shape
    e = d + 1
    out = np.zeros((m, N * e), dtype=np.uint64)
    for s in range(e):
        out[:, s::e] = digit(CA, t, d - s)
    return out[:, :k].astype(np.uint8)


def uncompress_cols_fwd(CB: np.ndarray, t: int, d: int, k: int) -> np.ndarray:
    """Inverse of compress_cols_fwd: residue (l(d+1)+s, j) is digit s of CB[l, j]."""
    CB = np.asarray(CB, dtype=np.uint64)
    N, n = CB.shape
    e = d + 1
    out = np.zeros((N * e, n), dtype=np.uint64)
    for s in range(e):
        out[s::e, :] = digit(CB, t, s)
    return out[:k].astype(np.uint8)


def uncompress_rows_fwd(CBr: np.ndarray, t: int, d: int, n: int) -> np.ndarray:
    """Inverse of compress_rows_fwd (the Uncompress step of the right-compressed procedure)."""
    CBr = np.asarray(CBr, dtype=np.uint64)
    k, nw = CBr.shape
    e = d + 1
    out = np.zeros((k, nw * e), dtype=np.uint64)
    for j in range(e):
        out[:, j::e] = digit(CBr, t, j)
    return out[:, :n].astype(np.uint8)


# --------------------------------------------------------------------------
# Products of packed words over exact integers (sections 2.2 and 3)
# --------------------------------------------------------------------------
def _to_pyint(x: np.ndarray) -> np.ndarray:
    return np.asarray(x).astype(object)


def packed_product_exact(CA: np.ndarray, CB: np.ndarray) -> np.ndarray:
    """S = CA x CB over the integers (Python ints, no rounding anywhere)."""
    return _to_pyint(CA).dot(_to_pyint(CB))


def coefficient_mod_p(S, t: int, d: int, p: int) -> np.ndarray:
    """Degree-d coefficient of the accumulated words, reduced mod p (section 2.2)."""
    Q = 1 << t
    f = np.vectorize(lambda s: ((int(s) >> (t * d)) % Q) % p, otypes=[object])
    return f(S).astype(np.uint8)


def qadic_product_mod_p(A: np.ndarray, B: np.ndarray, p: int, t: int, d: int) -> np.ndarray:
    """Procedure (2) carried out in exact integers: compress A by reversed rows, B by
    forward columns, multiply the packed matrices, keep coefficient d, reduce mod p.

    Equals modmul(A, B, p) exactly when k (p-1)^2 < Q (eq. (3)); see the pins.
    """
    S = packed_product_exact(compress_rows_rev(A, t, d), compress_cols_fwd(B, t, d))
    return coefficient_mod_p(S, t, d, p)


def extract(T, t: int, d: int, p: int, offset: int = 0) -> np.ndarray:
    """The per-entry REDC step (the paper's init routine, section 2.5) on integer words T:
    floor((T - offset) / Q^d) mod Q, then mod p.  offset = 0 for words that hold the
    exact sum, offset = 2^(beta-1) Q^d for an accumulator started at that value.
    """
    Q = 1 << t
    f = np.vectorize(lambda w: (((int(w) - offset) >> (t * d)) % Q) % p, otypes=[object])
    return f(T).astype(np.uint8)


def redq(CC, t: int, d: int, p: int, n: int) -> np.ndarray:
    """REDQ by its output (section 3): a word r = sum_j c_j Q^j (0 <= c_j < Q) yields
    c_j mod p for every j; the d+1 residues of word (i, J) go to C[i, J(d+1)+j]."""
    CC = np.asarray(CC)
    m, nw = CC.shape
    e = d + 1
    Q = 1 << t
    out = np.zeros((m, nw * e), dtype=np.uint8)
    for i in range(m):
        for J in range(nw):
            r = int(CC[i, J])
            for j in range(e):
                out[i, J * e + j] = ((r >> (t * j)) % Q) % p
    return out[:, :n]


def right_compressed_product_mod_p(A: np.ndarray, B: np.ndarray, p: int, t: int, d: int) -> np.ndarray:
    """Procedure (5) in exact integers: A (uncompressed) times the row-compressed B,
    then REDQ of every word (section 3)."""
    CBr = compress_rows_fwd(B, t, d)
    CC = _to_pyint(np.asarray(A)).dot(_to_pyint(CBr))
    return redq(CC, t, d, p, np.asarray(B).shape[1])


def centre(x: np.ndarray, p: int) -> np.ndarray:
    """Centred representative: x - p if x > (p-1)//2, as int64 (the INT8 path's operands)."""
    x = np.asarray(x, dtype=np.int64)
    return np.where(x > (p - 1) // 2, x - p, x)


# --------------------------------------------------------------------------
# Left compression (section 5, Table 2): the transpose of section 3's form.
# A is packed along m, d+1 consecutive rows per word, forward in Q; B stays as
# residues; every word of CC = CAl x B holds d+1 entries of one column of C.
# --------------------------------------------------------------------------
def compress_left(A: np.ndarray, t: int, d: int) -> np.ndarray:
    """CAl[I, l] = sum_{i=0..d} A[I(d+1)+i, l] * Q^i; rows past m read as 0.

    Returns uint64 words of shape (ceil(m/(d+1)), k).
    """
    _check_word_width(t, d)
    A = np.asarray(A)
    m, k = A.shape
    e = d + 1
    mw = -(-m // e)
    pad = np.zeros((mw * e, k), dtype=np.uint64)
    pad[:m] = A
    out = np.zeros((mw, k), dtype=np.uint64)
    for i in range(e):
        out += pad[i::e, :] << np.uint64(t * i)
    return out


def redq_left(CC, t: int, d: int, p: int, m: int) -> np.ndarray:
    """REDQ by its output for left-compressed words: digit i of word (I, j) is the
    dot product of row I(d+1)+i of A with column j of B; it goes, reduced mod p,
    to C[I(d+1)+i, j]."""
    CC = np.asarray(CC)
    mw, n = CC.shape
    e = d + 1
    Q = 1 << t
    out = np.zeros((mw * e, n), dtype=np.uint8)
    for I in range(mw):
        for j in range(n):
            r = int(CC[I, j])
            for i in range(e):
                out[I * e + i, j] = ((r >> (t * i)) % Q) % p
    return out[:m]


def left_compressed_product_mod_p(A: np.ndarray, B: np.ndarray, p: int, t: int, d: int) -> np.ndarray:
    """Left compression in exact integers: CAl x B (B uncompressed), then REDQ of
    every word into d+1 entries of a column of C."""
    CAl = compress_left(A, t, d)
    CC = _to_pyint(CAl).dot(_to_pyint(np.asarray(B)))
    return redq_left(CC, t, d, p, np.asarray(A).shape[0])


# --------------------------------------------------------------------------
# Full compression (section 4): A packed along m in Q (degree d_q), B packed
# along n in Theta (degree d_theta), Theta = Q^(d_q+1) (eq. (6) with equality).
# Entry (i, j) of a block of C is the coefficient of Q^i Theta^j of one word.
# --------------------------------------------------------------------------
def compress_full_right(B: np.ndarray, t: int, dq: int, dth: int, theta_t: int | None = None) -> np.ndarray:
    """CBt[l, J] = sum_{j=0..d_theta} B[l, J(d_theta+1)+j] * Theta^j with
    Theta = 2^theta_t (default 2^(t (d_q+1)) = Q^(d_q+1)); columns past n read as 0.

    Returns Python-int words of shape (k, ceil(n/(d_theta+1))) (object array: a
    word may exceed 64 bits when the bounds are deliberately broken)."""
    if theta_t is None:
        theta_t = t * (dq + 1)
    B = np.asarray(B)
    k, n = B.shape
    e = dth + 1
    nw = -(-n // e)
    out = np.zeros((k, nw), dtype=object)
    for l in range(k):
        for J in range(nw):
            w = 0
            for j in range(e):
                c = J * e + j
                if c < n:
                    w += int(B[l, c]) << (theta_t * j)
            out[l, J] = w
    return out


def full_word_digit(r: int, t: int, dq: int, i: int, j: int, theta_t: int | None = None) -> int:
    """Coefficient of Q^i Theta^j of a word whose coefficients are all below Q:
    floor(r / (Q^i Theta^j)) mod Q."""
    if theta_t is None:
        theta_t = t * (dq + 1)
    return (r >> (t * i + theta_t * j)) % (1 << t)


def redq_full(CC, t: int, dq: int, dth: int, p: int, m: int, n: int, theta_t: int | None = None) -> np.ndarray:
    """Two-variable REDQ by its output: word (I, J) yields C[I(d_q+1)+i, J(d_theta+1)+j]
    = (coefficient of Q^i Theta^j) mod p for every i <= d_q, j <= d_theta."""
    CC = np.asarray(CC)
    mw, nw = CC.shape
    eq, eth = dq + 1, dth + 1
    out = np.zeros((mw * eq, nw * eth), dtype=np.uint8)
    for I in range(mw):
        for J in range(nw):
            r = int(CC[I, J])
            for i in range(eq):
                for j in range(eth):
                    out[I * eq + i, J * eth + j] = full_word_digit(r, t, dq, i, j, theta_t) % p
    return out[:m, :n]


def full_compressed_product_mod_p(A: np.ndarray, B: np.ndarray, p: int, t: int, dq: int, dth: int,
                                  theta_t: int | None = None) -> np.ndarray:
    """Full compression in exact integers: pack A along m (base Q, degree d_q) and B
    along n (base Theta, degree d_theta), multiply the packed matrices, read every
    coefficient of the two-variable polynomial words and reduce it mod p.

    Equals modmul(A, B, p) when k (p-1)^2 < Q (eq. (3)) and Theta >= Q^(d_q+1)
    (eq. (6)); eq. (7) is what keeps the words exact in floating point."""
    CAl = compress_left(A, t, dq) if t * (dq + 1) <= 63 else None
    if CAl is None:
        raise ValueError("A word does not fit 63 bits")
    CBt = compress_full_right(B, t, dq, dth, theta_t)
    CC = _to_pyint(CAl).dot(CBt)
    return redq_full(CC, t, dq, dth, p, np.asarray(A).shape[0], np.asarray(B).shape[1], theta_t)


# --------------------------------------------------------------------------
# ReduceAndCompress (procedure (1)): the product of compressed matrices handed
# back compressed, so that products can be chained without leaving the packing.
# --------------------------------------------------------------------------
def reduce_and_compress(S, t: int, d: int, p: int, offset: int = 0) -> np.ndarray:
    """Procedure (1)'s second step on accumulated words S (m x n): reduce every entry
    (digit d mod p, as extract) and compress the rows of the result, reversed, as
    CompressRows does: out[i, L] = sum_s C[i, L(d+1)+s] Q^(d-s)."""
    C = extract(S, t, d, p, offset)
    return compress_rows_rev(C, t, d)
