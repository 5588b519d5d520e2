"""Parity of the HIP library against the CPU oracle, through the C ABI (needs an MI355X).

Integer results must match bit for bit.  Small shapes are checked entry by entry
against the full oracle product; the workload-size products are checked on
sampled entries (each a plain dot product in the oracle), on whole rows, and on
closed forms that hold at any size.
"""
import sys

import numpy as np
import pytest

from oracle import reference as ref
from oracle import bounds
from paper_0803_1975_amd import qmm
import synth

pytestmark = pytest.mark.gpu

PATHS = (qmm.PATH_FP64_QADIC, qmm.PATH_FP64_REDQ, qmm.PATH_FP32_QADIC, qmm.PATH_FP32_REDQ, qmm.PATH_INT8,
         qmm.PATH_FP4, qmm.PATH_FP64_LEFT, qmm.PATH_FP32_LEFT, qmm.PATH_FP64_FULL, qmm.PATH_FP32_FULL)


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    if not _t.cuda.is_available():
        pytest.fail("these tests need a GPU")
    return _t


def note(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def dev(torch, x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def host(t):
    return t.cpu().numpy()


def run_gemm(torch, A, B, p, path, flags=0):
    m, k = A.shape
    n = B.shape[1]
    st, plan = qmm.try_choose_Qd(p, m, n, k, path=path, flags=flags)
    if st != qmm.OK:
        return None, None
    C = qmm.gemm_mod_p(dev(torch, A), dev(torch, B), p, plan=plan)
    torch.cuda.synchronize()
    return host(C), plan


def test_native_library_is_loaded(torch):
    qmm.lib()
    maps = open("/proc/self/maps").read()
    assert "libqmm.so" in maps


# --- conversions --------------------------------------------------------------
@pytest.mark.parametrize("p,t,d,beta", [(3, 9, 4, 53), (7, 18, 1, 53), (2, 5, 9, 53), (101, 27, 0, 53),
                                        (3, 11, 1, 24), (5, 7, 2, 24)])
def test_pack_and_unpack_match_oracle(torch, p, t, d, beta):
    note("pack", p, t, d, beta)
    rng = np.random.default_rng(t * 7 + d)
    plan = qmm.Plan(p=p, t=t, d=d, beta=beta, k_block=1 << 40,
                    path=qmm.PATH_FP64_QADIC if beta == 53 else qmm.PATH_FP32_QADIC)
    A = rng.integers(0, p, (37, 101), dtype=np.uint8)
    B = rng.integers(0, p, (101, 45), dtype=np.uint8)
    CA = qmm.pack_rows_rev(plan, dev(torch, A))
    CB = qmm.pack_cols_fwd(plan, dev(torch, B))
    CBr = qmm.pack_rows_fwd(plan, dev(torch, B))
    torch.cuda.synchronize()
    np.testing.assert_array_equal(host(CA).astype(np.uint64), ref.compress_rows_rev(A, t, d))
    np.testing.assert_array_equal(host(CB).astype(np.uint64), ref.compress_cols_fwd(B, t, d))
    np.testing.assert_array_equal(host(CBr).astype(np.uint64), ref.compress_rows_fwd(B, t, d))
    np.testing.assert_array_equal(host(qmm.unpack(plan, qmm.ROWS_REV, 37, 101, CA)), A)
    np.testing.assert_array_equal(host(qmm.unpack(plan, qmm.COLS_FWD, 101, 45, CB)), B)
    np.testing.assert_array_equal(host(qmm.unpack(plan, qmm.ROWS_FWD, 101, 45, CBr)), B)


def test_extract_matches_oracle_in_both_regimes(torch):
    rng = np.random.default_rng(11)
    # exact regime: p = 7, k = 4096, t = 18, d = 1; T is the exact sum S
    p, t, d, k = 7, 18, 1, 4096
    A = rng.integers(0, p, (20, k), dtype=np.uint8)
    B = rng.integers(0, p, (k, 24), dtype=np.uint8)
    S = ref.packed_product_exact(ref.compress_rows_rev(A, t, d), ref.compress_cols_fwd(B, t, d))
    assert max(int(x) for x in S.ravel()) < 2 ** 53
    T = np.array([[float(int(x)) for x in row] for row in S])
    plan = qmm.choose_Qd(p, 20, 24, k, path=qmm.PATH_FP64_QADIC, flags=qmm.PLAN_UNBLOCKED | qmm.BOUND_EQ4)
    assert (plan.t, plan.d, plan.regime) == (t, d, qmm.REGIME_EXACT)
    got = host(qmm.extract(plan, dev(torch, T)))
    np.testing.assert_array_equal(got, ref.extract(S, t, d, p))
    np.testing.assert_array_equal(got, ref.modmul(A, B, p))
    # offset regime: p = 3, k = 64, t = 9, d = 4; T = M + floor(S / Q^d) Q^d
    p, t, d, k = 3, 9, 4, 64
    A = rng.integers(0, p, (20, k), dtype=np.uint8)
    B = rng.integers(0, p, (k, 24), dtype=np.uint8)
    S = ref.packed_product_exact(ref.compress_rows_rev(A, t, d), ref.compress_cols_fwd(B, t, d))
    M = (1 << 52) << (t * d)
    Tint = [[M + ((int(x) >> (t * d)) << (t * d)) for x in row] for row in S]
    T = np.array([[float(v) for v in row] for row in Tint])
    assert all(int(T[i, j]) == Tint[i][j] for i in range(20) for j in range(24))
    plan = qmm.choose_Qd(p, 20, 24, k, path=qmm.PATH_FP64_QADIC, flags=qmm.BOUND_EQ4)
    assert plan.regime == qmm.REGIME_OFFSET and (plan.t, plan.d) == (t, d)
    got = host(qmm.extract(plan, dev(torch, T)))
    np.testing.assert_array_equal(got, ref.extract(np.array(Tint, dtype=object), t, d, p, offset=M))
    np.testing.assert_array_equal(got, ref.modmul(A, B, p))


@pytest.mark.parametrize("p,k,n", [(7, 4096, 50), (3, 64, 33), (101, 1000, 7), (2, 5, 100)])
def test_redq_matches_oracle(torch, p, k, n):
    note("redq", p, k, n)
    rng = np.random.default_rng(p + k)
    A = rng.integers(0, p, (9, k), dtype=np.uint8)
    B = rng.integers(0, p, (k, n), dtype=np.uint8)
    plan = qmm.choose_Qd(p, 9, n, k, path=qmm.PATH_FP64_REDQ)
    CBr = ref.compress_rows_fwd(B, plan.t, plan.d)
    CC = A.astype(object).dot(CBr.astype(object))
    T = np.array([[float(int(x)) for x in row] for row in CC])
    got = host(qmm.redq(plan, dev(torch, T), n))
    np.testing.assert_array_equal(got, ref.redq(CC, plan.t, plan.d, p, n))
    np.testing.assert_array_equal(got, ref.modmul(A, B, p))


# --- full products at oracle-sized shapes ----------------------------------------
SHAPES = [(1, 1, 1), (64, 64, 64), (17, 33, 5), (130, 257, 300), (300, 129, 1000), (128, 128, 16),
          (129, 127, 4097), (5, 200, 3)]


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("p", (2, 3, 7, 101, 251))
def test_gemm_matches_oracle(torch, path, p):
    rng = np.random.default_rng(path * 1000 + p)
    for m, n, k in SHAPES:
        note("gemm", qmm.PATH_NAMES[path], p, m, n, k)
        A = rng.integers(0, p, (m, k), dtype=np.uint8)
        B = rng.integers(0, p, (k, n), dtype=np.uint8)
        got, plan = run_gemm(torch, A, B, p, path)
        if got is None:
            continue
        np.testing.assert_array_equal(got, ref.modmul(A, B, p), err_msg=f"{plan} {m}x{n}x{k}")


@pytest.mark.parametrize("path", (qmm.PATH_FP64_QADIC, qmm.PATH_FP32_QADIC))
def test_unblocked_and_eq4_plans(torch, path):
    rng = np.random.default_rng(5)
    for p, (m, n, k) in ((3, (70, 90, 2047)), (7, (64, 64, 4096)), (101, (33, 65, 800))):
        A = rng.integers(0, p, (m, k), dtype=np.uint8)
        B = rng.integers(0, p, (k, n), dtype=np.uint8)
        for flags in (qmm.PLAN_UNBLOCKED, qmm.BOUND_EQ4, qmm.PLAN_UNBLOCKED | qmm.BOUND_EQ4):
            got, plan = run_gemm(torch, A, B, p, path, flags)
            if got is None:
                continue
            note("flags", flags, plan)
            np.testing.assert_array_equal(got, ref.modmul(A, B, p), err_msg=str(plan))


def test_gemm_packed_procedure_1(torch):
    rng = np.random.default_rng(9)
    for p, (m, n, k) in ((3, (64, 64, 64)), (7, (100, 70, 4096)), (3, (33, 31, 16384))):
        A = rng.integers(0, p, (m, k), dtype=np.uint8)
        B = rng.integers(0, p, (k, n), dtype=np.uint8)
        plan = qmm.choose_Qd(p, m, n, k, path=qmm.PATH_FP64_QADIC)
        note("packed", plan)
        CA = qmm.pack_rows_rev(plan, dev(torch, A))
        CB = qmm.pack_cols_fwd(plan, dev(torch, B))
        got = host(qmm.gemm_packed(plan, k, CA, CB))
        np.testing.assert_array_equal(got, ref.modmul(A, B, p))


# --- edge cases --------------------------------------------------------------------
@pytest.mark.parametrize("path", PATHS)
def test_degenerate_shapes(torch, path):
    p = 7
    A = np.zeros((5, 0), np.uint8)
    B = np.zeros((0, 6), np.uint8)
    plan = qmm.choose_Qd(p, 5, 6, 0, path=path)
    C = torch.full((5, 6), 99, dtype=torch.uint8, device="cuda")
    qmm.gemm_mod_p(dev(torch, A), dev(torch, B), p, plan=plan, C=C)
    assert int(C.max()) == 0
    C0 = qmm.gemm_mod_p(torch.zeros((0, 4), dtype=torch.uint8, device="cuda"),
                        torch.zeros((4, 3), dtype=torch.uint8, device="cuda"), p,
                        plan=qmm.choose_Qd(p, 0, 3, 4, path=path))
    assert C0.shape == (0, 3)


@pytest.mark.parametrize("path,p,k", [(qmm.PATH_FP64_QADIC, 3, 16384), (qmm.PATH_FP64_QADIC, 7, 4096),
                                      (qmm.PATH_FP64_QADIC, 101, 8192), (qmm.PATH_FP64_QADIC, 2, 100000),
                                      (qmm.PATH_FP64_REDQ, 7, 4096), (qmm.PATH_FP64_REDQ, 101, 8192),
                                      (qmm.PATH_FP32_QADIC, 3, 5000), (qmm.PATH_FP32_QADIC, 101, 4000),
                                      (qmm.PATH_FP32_REDQ, 3, 511), (qmm.PATH_INT8, 251, 1000),
                                      (qmm.PATH_INT8, 101, 8192), (qmm.PATH_FP64_LEFT, 7, 4096),
                                      (qmm.PATH_FP64_FULL, 3, 2047), (qmm.PATH_FP64_FULL, 101, 8192),
                                      (qmm.PATH_FP32_FULL, 2, 63)])
def test_worst_case_all_p_minus_one(torch, path, p, k):
    # every residue p-1: C = k (p-1)^2 = k (mod p); the largest digits, words and low parts
    st, plan = qmm.try_choose_Qd(p, 48, 40, k, path=path)
    assert st == qmm.OK, qmm.last_error()
    note("worst", plan, k)
    A = torch.full((48, k), p - 1, dtype=torch.uint8, device="cuda")
    B = torch.full((k, 40), p - 1, dtype=torch.uint8, device="cuda")
    C = host(qmm.gemm_mod_p(A, B, p, plan=plan))
    assert (C == (k * (p - 1) ** 2) % p).all(), (plan, np.unique(C))


# Blocked Q-adic plans with t <= 15 sum the digits of finished blocks in 16-bit
# fields and reduce them mod p every F = floor((2^16 - p) / (Q - 1)) blocks.  The
# k below put the block count just under, at and past a multiple of F (p = 5 at
# t = 13: F = 8, blocks of 448), and run several folds (FP32 p = 7 and 11, t = 12:
# F = 16, 53 and 157 blocks; FP64 p = 3, t = 10: F = 64, 417 blocks).
FOLD_CASES = [(qmm.PATH_FP64_QADIC, 5, 3584), (qmm.PATH_FP64_QADIC, 5, 3585), (qmm.PATH_FP64_QADIC, 5, 4032),
              (qmm.PATH_FP64_QADIC, 5, 20000), (qmm.PATH_FP64_QADIC, 3, 100000), (qmm.PATH_FP32_QADIC, 7, 5000),
              (qmm.PATH_FP32_QADIC, 11, 5000)]


@pytest.mark.parametrize("path,p,k", FOLD_CASES)
def test_blocked_digit_sums_across_folds(torch, path, p, k):
    plan = qmm.choose_Qd(p, 48, 40, k, path=path)
    assert plan.k_block < k and plan.t <= 15, plan
    note("folds", plan, k)
    A = torch.full((48, k), p - 1, dtype=torch.uint8, device="cuda")
    B = torch.full((k, 40), p - 1, dtype=torch.uint8, device="cuda")
    C = host(qmm.gemm_mod_p(A, B, p, plan=plan))
    assert (C == (k * (p - 1) ** 2) % p).all(), (plan, np.unique(C))
    rng = np.random.default_rng(k + p)
    A = rng.integers(0, p, (48, k), dtype=np.uint8)
    B = rng.integers(0, p, (k, 40), dtype=np.uint8)
    got = host(qmm.gemm_mod_p(dev(torch, A), dev(torch, B), p, plan=plan))
    np.testing.assert_array_equal(got, ref.modmul(A, B, p))


def test_int8_blocked_accumulation(torch):
    # centred residue 125 of p = 251: products 15625 overflow int32 after 137438 terms
    p, k = 251, 140000
    plan = qmm.choose_Qd(p, 16, 16, k, path=qmm.PATH_INT8)
    assert plan.k_block < k
    A = torch.full((16, k), 125, dtype=torch.uint8, device="cuda")
    B = torch.full((k, 16), 125, dtype=torch.uint8, device="cuda")
    C = host(qmm.gemm_mod_p(A, B, p, plan=plan))
    assert (C == (k * 125 * 125) % p).all()
    rng = np.random.default_rng(3)
    A = rng.integers(0, p, (20, k), dtype=np.uint8)
    B = rng.integers(0, p, (k, 9), dtype=np.uint8)
    got, _ = run_gemm(torch, A, B, p, qmm.PATH_INT8)
    want = ref.modmul(A, B, p)
    np.testing.assert_array_equal(got, want)
    dA, dB = dev(torch, A), dev(torch, B)
    for tile in (1, 2, 3, 4):
        plan = qmm.choose_Qd(p, 20, 9, k, path=qmm.PATH_INT8)
        plan.tile = tile
        np.testing.assert_array_equal(host(qmm.gemm_mod_p(dA, dB, p, plan=plan)), want, err_msg=f"tile {tile}")


@pytest.mark.parametrize("p,k", [(2, 20), (2, 12), (3, 15), (5, 13), (7, 7)])
def test_fp32_offset_plans_rely_on_one_rounding_per_product(torch, p, k):
    # The planner's FP32 Q-adic plans for these (p, k) are in the offset regime with a
    # low part that only a correctly rounded step per product floors away: the oracle's
    # 24-bit emulation gives the right digit with one rounding per product and a wrong
    # one with four products summed before a rounding.  On all-(p-1) operands every
    # low part is maximal, so the GPU result shows which the FP32 matrix cores do.
    from oracle import emulate
    plan = qmm.choose_Qd(p, 48, 40, k, path=qmm.PATH_FP32_QADIC)
    note("fp32 rounding", plan)
    assert plan.regime == qmm.REGIME_OFFSET and plan.g == 1 and plan.k_block == k
    assert bounds.offset_ok(p, k, plan.t, plan.d, 24, g=1) and not bounds.offset_ok(p, k, plan.t, plan.d, 24, g=4)
    a = np.full(k, p - 1, dtype=np.uint8)
    want = (k * (p - 1) ** 2) % p
    assert emulate.qadic_entry(a, a, p, plan.t, plan.d, 24, "offset", g=1) == want
    assert emulate.qadic_entry(a, a, p, plan.t, plan.d, 24, "offset", g=4) != want
    A = torch.full((48, k), p - 1, dtype=torch.uint8, device="cuda")
    B = torch.full((k, 40), p - 1, dtype=torch.uint8, device="cuda")
    C = host(qmm.gemm_mod_p(A, B, p, plan=plan))
    assert (C == want).all(), (plan, np.unique(C))
    # the same plan through the stage calls (pack, then procedure (1) on the words)
    C1 = host(qmm.gemm_packed(plan, k, qmm.pack_rows_rev(plan, A), qmm.pack_cols_fwd(plan, B)))
    assert (C1 == want).all()


def test_offset_regime_relies_on_one_rounding_per_product(torch):
    # p = 3, t = 7, d = 5, k = 24: every product's low part sits just below Q^d/2.
    # One correctly rounded step per product (what the matrix cores do) floors each
    # product; four products summed before one rounding would not (see the oracle's
    # emulation).  All-(p-1) operands make every low part maximal.
    p, t, d, k = 3, 7, 5, 24
    assert bounds.offset_ok(p, k, t, d, 53, g=1) and not bounds.offset_ok(p, k, t, d, 53, g=4)
    plan = qmm.Plan(p=p, t=t, d=d, beta=53, k_block=k, path=qmm.PATH_FP64_QADIC, regime=qmm.REGIME_OFFSET, g=1)
    assert qmm.validate_plan(plan, 64, 64, k) == qmm.OK
    A = torch.full((64, k), p - 1, dtype=torch.uint8, device="cuda")
    B = torch.full((k, 64), p - 1, dtype=torch.uint8, device="cuda")
    C = host(qmm.gemm_mod_p(A, B, p, plan=plan))
    assert (C == (k * (p - 1) ** 2) % p).all()


@pytest.mark.parametrize("path", PATHS)
def test_repeat_launches_are_bit_identical(torch, path):
    p = 7
    rng = np.random.default_rng(1)
    A = dev(torch, rng.integers(0, p, (300, 700), dtype=np.uint8))
    B = dev(torch, rng.integers(0, p, (700, 260), dtype=np.uint8))
    plan = qmm.choose_Qd(p, 300, 260, 700, path=path)
    ws = qmm.workspace(plan, 300, 260, 700)
    first = qmm.gemm_mod_p(A, B, p, plan=plan, ws=ws).clone()
    for _ in range(9):
        assert torch.equal(qmm.gemm_mod_p(A, B, p, plan=plan, ws=ws), first)


def test_strided_operands(torch):
    p = 5
    rng = np.random.default_rng(2)
    Abig = rng.integers(0, p, (90, 300), dtype=np.uint8)
    Bbig = rng.integers(0, p, (250, 180), dtype=np.uint8)
    A, B = Abig[:, 7:207], Bbig[:200, 3:163]
    dA, dB = dev(torch, Abig)[:, 7:207], dev(torch, Bbig)[:200, 3:163]
    Cbig = torch.zeros((90, 400), dtype=torch.uint8, device="cuda")
    for path in PATHS:
        plan = qmm.choose_Qd(p, 90, 160, 200, path=path)
        C = Cbig[:, 10:170]
        qmm.gemm_mod_p(dA, dB, p, plan=plan, C=C)
        np.testing.assert_array_equal(host(C), ref.modmul(np.ascontiguousarray(A), np.ascontiguousarray(B), p))
        assert int(Cbig[:, :10].max()) == 0 and int(Cbig[:, 170:].max()) == 0


@pytest.mark.parametrize("path,tile", [(qmm.PATH_INT8, t) for t in (1, 2, 3, 4)] + [(qmm.PATH_FP4, t) for t in (1, 2, 3)])
@pytest.mark.parametrize("col0", (4, 3))
def test_output_views_for_every_tile(torch, path, tile, col0):
    # C is a view into a larger zeroed buffer: at a 4-byte aligned column offset with
    # ldc a multiple of 4, whole tiles are stored as dwords; at an odd offset they are
    # stored as bytes.  Either way exactly the view's bytes change.
    p, m, n, k = 7, 520, 530, 700
    note("views", qmm.PATH_NAMES[path], "tile", tile, "col0", col0)
    rng = np.random.default_rng(100 * tile + col0)
    A = rng.integers(0, p, (m, k), dtype=np.uint8)
    B = rng.integers(0, p, (k, n), dtype=np.uint8)
    plan = qmm.choose_Qd(p, m, n, k, path=path)
    plan.tile = tile
    Cbig = torch.full((m + 3, 600), 0xEE, dtype=torch.uint8, device="cuda")
    C = Cbig[1:m + 1, col0:col0 + n]
    qmm.gemm_mod_p(dev(torch, A), dev(torch, B), p, plan=plan, C=C)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(host(C), ref.modmul(A, B, p))
    big = host(Cbig)
    outside = np.ones(big.shape, dtype=bool)
    outside[1:m + 1, col0:col0 + n] = False
    assert (big[outside] == 0xEE).all()


# --- workload sizes -------------------------------------------------------------------
def sampled_check(torch, A, B, p, C, nsamp=20000, rows=4, seed=0):
    rng = np.random.default_rng(seed)
    m, n = C.shape
    ri = rng.integers(0, m, nsamp)
    ci = rng.integers(0, n, nsamp)
    np.testing.assert_array_equal(C[ri, ci], ref.modmul_entries(A, B, p, ri, ci))
    for i in rng.integers(0, m, rows):
        np.testing.assert_array_equal(C[i], ref.modmul(A[i:i + 1], B, p)[0])
    # the last row and column cross the ragged tile edges when there are any
    np.testing.assert_array_equal(C[m - 1], ref.modmul(A[m - 1:m], B, p)[0])


@pytest.mark.parametrize("name", ("small", "square", "large", "thin"))
def test_workloads_all_paths(torch, name):
    p, A, B = synth.workload(name)
    m, k = A.shape
    n = B.shape[1]
    dA, dB = dev(torch, A), dev(torch, B)
    for path in PATHS:
        for flags in (0, qmm.PLAN_UNBLOCKED | qmm.BOUND_EQ4):
            st, plan = qmm.try_choose_Qd(p, m, n, k, path=path, flags=flags)
            if st != qmm.OK:
                note(name, "no plan", qmm.PATH_NAMES[path], flags, qmm.last_error())
                continue
            note(name, plan)
            C = host(qmm.gemm_mod_p(dA, dB, p, plan=plan))
            if m * n * k <= 64 ** 3:
                np.testing.assert_array_equal(C, ref.modmul(A, B, p))
            else:
                sampled_check(torch, A, B, p, C)


def test_graph_workload_and_paley_closed_form(torch):
    # Paley graph on q = 16381 (prime, q = 1 mod 4): strongly regular, so
    # A^2 = (q-1)/2 I + (q-5)/4 A + (q-1)/4 (J - I - A) holds entry by entry.
    q = 16381
    assert all(q % f for f in range(2, 128))
    x = torch.arange(q, device="cuda", dtype=torch.int64)
    is_sq = torch.zeros(q, dtype=torch.bool, device="cuda")
    is_sq[(x[1:] * x[1:]) % q] = True
    diff = (x[:, None] - x[None, :]) % q
    Ad = is_sq[diff].to(torch.uint8)
    del diff
    for path in (qmm.PATH_FP4, qmm.PATH_INT8, qmm.PATH_FP64_QADIC):
        for flags in (0, qmm.PLAN_UNBLOCKED | qmm.BOUND_EQ4):
            if path in (qmm.PATH_INT8, qmm.PATH_FP4) and flags:
                continue
            plan = qmm.choose_Qd(3, q, q, q, path=path, flags=flags)
            note("paley", plan)
            C = qmm.gemm_mod_p(Ad, Ad, 3, plan=plan)
            a, b, c = ((q - 5) // 4) % 3, ((q - 1) // 4) % 3, ((q - 1) // 2) % 3
            want = ((b + (a - b + 3) * Ad.to(torch.int16)) % 3).to(torch.uint8)
            want.fill_diagonal_(c)
            assert torch.equal(C, want)
            del C, want
    # the random graph of the workload itself, on sampled entries
    p, A, B = synth.workload("graph")
    dA = dev(torch, A)
    for path in (qmm.PATH_INT8, qmm.PATH_FP64_QADIC):
        plan = qmm.choose_Qd(p, A.shape[0], A.shape[0], A.shape[0], path=path)
        note("graph", plan)
        C = host(qmm.gemm_mod_p(dA, dA, p, plan=plan))
        sampled_check(torch, A, A, p, C, nsamp=5000, rows=2)
        assert (C == C.T).all()



@pytest.mark.parametrize("p,m,n,k", [(7, 300, 272, 1040), (2, 1, 16, 16), (251, 257, 512, 4096), (3, 640, 48, 130048),
                                     (101, 33, 1024, 16), (256, 96, 64, 1984), (101, 300, 260, 1001),
                                     (7, 257, 130, 4097), (13, 70, 300, 333)])
def test_int8_stages_match_one_call_and_oracle(torch, p, m, n, k):
    # The two INT8 stage calls (centring transpose, product) give what qmm_gemm_mod_p
    # gives; every tile variant (128 x 128, 256 x 256 with 8 or 16 wavefronts); k past
    # a 128-byte stage boundary.
    note("int8 stages", p, m, n, k)
    rng = np.random.default_rng(m + n + k)
    A = rng.integers(0, p, (m, k), dtype=np.uint8)
    B = rng.integers(0, p, (k, n), dtype=np.uint8)
    dA, dB = dev(torch, A), dev(torch, B)
    plan = qmm.choose_Qd(p, m, n, k, path=qmm.PATH_INT8)
    one = qmm.gemm_mod_p(dA, dB, p, plan=plan)
    Bt = qmm.pack_centred_cols(plan, dB)
    for tile in (1, 2, 3, 4):
        plan.tile = tile
        assert torch.equal(qmm.gemm_centred(plan, dA, Bt, n), one)
    if m * n * k <= 2 ** 28:
        np.testing.assert_array_equal(host(one), ref.modmul(A, B, p))
    else:
        sampled_check(torch, A, B, p, host(one), nsamp=4000, rows=2)
    plan.tile = 0
    worst = torch.full((m, k), p - 1, dtype=torch.uint8, device="cuda")
    worstB = torch.full((k, n), p - 1, dtype=torch.uint8, device="cuda")
    assert (host(qmm.gemm_mod_p(worst, worstB, p, plan=plan)) == (k * (p - 1) ** 2) % p).all()


def test_count_nonresidues_and_validated_product(torch):
    # Residues must lie in [0, p); validation counts the other bytes exactly and
    # gemm_mod_p(validate=True) refuses such input with EVALUE.
    rng = np.random.default_rng(21)
    for p, rows, cols, ld in ((7, 300, 257, 257), (101, 1, 1, 1), (2, 65, 4000, 4096), (256, 9, 9, 9)):
        X = rng.integers(0, p, (rows, ld), dtype=np.uint16)
        nbad = min(17, rows * cols)
        ri = rng.integers(0, rows, nbad)
        ci = rng.integers(0, cols, nbad)
        if p < 256:
            X[ri, ci] = rng.integers(p, 256, nbad)
        X[:, cols:] = 255                               # bytes past cols are not looked at
        X = X.astype(np.uint8)
        want = int((X[:, :cols] >= p).sum())
        dX = dev(torch, X)[:, :cols]
        got = int(qmm.count_nonresidues(p, dX).item())
        note("count", p, rows, cols, want, got)
        assert got == want
    empty = torch.zeros((0, 5), dtype=torch.uint8, device="cuda")
    assert int(qmm.count_nonresidues(3, empty).item()) == 0
    p = 5
    A = rng.integers(0, p, (64, 80), dtype=np.uint8)
    B = rng.integers(0, p, (80, 48), dtype=np.uint8)
    dA, dB = dev(torch, A), dev(torch, B)
    np.testing.assert_array_equal(host(qmm.gemm_mod_p(dA, dB, p, validate=True)), ref.modmul(A, B, p))
    dB[3, 7] = 9
    with pytest.raises(qmm.QmmError) as ei:
        qmm.gemm_mod_p(dA, dB, p, validate=True)
    assert ei.value.status == qmm.EVALUE and "1 of B" in str(ei.value)


@pytest.mark.parametrize("p,m,n,k", [(7, 300, 272, 1040), (2, 1, 16, 16), (3, 257, 512, 4096), (5, 640, 48, 12000),
                                     (8, 33, 1024, 16), (7, 96, 64, 1984), (3, 130, 70, 257)])
def test_fp4_stages_match_one_call_and_oracle(torch, p, m, n, k):
    # The FP4 stage calls (both conversions, product) give what qmm_gemm_mod_p gives,
    # on every tile variant; k across 256-value stage edges and ragged tiles.
    note("fp4 stages", p, m, n, k)
    rng = np.random.default_rng(m + n + k + p)
    A = rng.integers(0, p, (m, k), dtype=np.uint8)
    B = rng.integers(0, p, (k, n), dtype=np.uint8)
    dA, dB = dev(torch, A), dev(torch, B)
    plan = qmm.choose_Qd(p, m, n, k, path=qmm.PATH_FP4)
    one = qmm.gemm_mod_p(dA, dB, p, plan=plan)
    A4 = qmm.pack_fp4_rows(plan, dA)
    Bt4 = qmm.pack_fp4_cols(plan, dB)
    A4b, Bt4b = qmm.pack_fp4(plan, dA, dB)          # both conversions in one launch
    assert torch.equal(A4b, A4) and torch.equal(Bt4b, Bt4)
    for tile in (1, 2, 3):
        plan.tile = tile
        assert torch.equal(qmm.gemm_fp4(plan, A4, Bt4, k), one), tile
    if m * n * k <= 2 ** 28:
        np.testing.assert_array_equal(host(one), ref.modmul(A, B, p))
    else:
        sampled_check(torch, A, B, p, host(one), nsamp=4000, rows=2)


def test_fp4_codes_match_the_oracle_encoding(torch):
    # the packed operands decode (by the oracle's e2m1 table) to the centred residues
    from oracle import bounds
    for p in (2, 3, 5, 7, 8):
        rng = np.random.default_rng(p)
        A = rng.integers(0, p, (5, 77), dtype=np.uint8)
        plan = qmm.choose_Qd(p, 5, 5, 77, path=qmm.PATH_FP4)
        A4 = host(qmm.pack_fp4_rows(plan, dev(torch, A)))
        codes = np.stack([A4 & 15, A4 >> 4], axis=-1).reshape(5, -1)     # even k in the low nibble
        vals = np.vectorize(lambda c: float(bounds.e2m1_value(int(c))))(codes)
        np.testing.assert_array_equal(vals[:, :77], ref.centre(A, p))
        assert (codes[:, 77:] == 0).all()                                # zero past k
        Bt4 = host(qmm.pack_fp4_cols(plan, dev(torch, A.T.copy())))
        np.testing.assert_array_equal(Bt4[:, :A4.shape[1]], A4[:, :Bt4.shape[1]])


def test_fp4_worst_case_and_blocked_accumulation(torch):
    # all operands at the largest centred magnitude: sums of k h^2, blocked once k h^2
    # leaves the exact FP32 integers (p = 7: past 1 864 134 products)
    for p, v, k in ((7, 3, 70000), (7, 4, 2000000), (8, 4, 1100000), (3, 2, 40000)):
        plan = qmm.choose_Qd(p, 16, 24, k, path=qmm.PATH_FP4)
        note("fp4 worst", plan, v, k)
        assert (plan.k_block < k) == (k * (p // 2) ** 2 + p - 1 > 2 ** 24)
        A = torch.full((16, k), v, dtype=torch.uint8, device="cuda")
        B = torch.full((k, 24), v, dtype=torch.uint8, device="cuda")
        C = host(qmm.gemm_mod_p(A, B, p, plan=plan))
        assert (C == (k * v * v) % p).all(), (plan, np.unique(C))
        del A, B
    # forced short blocks on random data, every tile
    rng = np.random.default_rng(9)
    p, k = 5, 3000
    A = rng.integers(0, p, (50, k), dtype=np.uint8)
    B = rng.integers(0, p, (k, 40), dtype=np.uint8)
    want = ref.modmul(A, B, p)
    dA, dB = dev(torch, A), dev(torch, B)
    for tile in (1, 2, 3):
        plan = qmm.choose_Qd(p, 50, 40, k, path=qmm.PATH_FP4)
        plan.k_block, plan.tile = 512, tile
        np.testing.assert_array_equal(host(qmm.gemm_mod_p(dA, dB, p, plan=plan)), want, err_msg=f"tile {tile}")


@pytest.mark.parametrize("p,m,n,k", [(3, 64, 64, 64), (7, 1, 1, 1), (2, 65, 130, 33), (101, 100, 70, 50),
                                     (3, 128, 128, 128), (5, 100, 90, 200), (13, 129, 3, 700)])
def test_fused_small_qadic_matches_staged_calls_and_oracle(torch, p, m, n, k):
    # qmm_gemm_mod_p runs small unblocked FP64 Q-adic products in one launch that
    # packs in LDS (no workspace); the staged calls pack in HBM first
    rng = np.random.default_rng(p * m + n + k)
    A = rng.integers(0, p, (m, k), dtype=np.uint8)
    B = rng.integers(0, p, (k, n), dtype=np.uint8)
    want = ref.modmul(A, B, p)
    dA, dB = dev(torch, A), dev(torch, B)
    for flags in (0, qmm.PLAN_UNBLOCKED | qmm.BOUND_EQ4):
        st, plan = qmm.try_choose_Qd(p, m, n, k, path=qmm.PATH_FP64_QADIC, flags=flags)
        if st != qmm.OK or plan.k_block < k:
            continue
        note("fused", p, m, n, k, plan)
        assert qmm.gemm_workspace_size(plan, m, n, k) == 0
        C = torch.full((m, n), 0xCD, dtype=torch.uint8, device="cuda")
        qmm.gemm_mod_p(dA, dB, p, plan=plan, C=C, ws=torch.empty(0, dtype=torch.uint8, device="cuda"))
        np.testing.assert_array_equal(host(C), want)
        staged = qmm.gemm_packed(plan, k, qmm.pack_rows_rev(plan, dA), qmm.pack_cols_fwd(plan, dB))
        np.testing.assert_array_equal(host(staged), want)


@pytest.mark.parametrize("p,m,n,k", [(3, 64, 64, 64), (2, 1, 1, 1), (251, 65, 130, 33), (101, 100, 70, 70),
                                     (7, 50, 45, 200), (13, 129, 3, 700), (251, 8, 8, 4096),
                                     (101, 300, 260, 700), (31, 777, 65, 1000)])
def test_small_int8_one_launch_matches_staged_calls_and_oracle(torch, p, m, n, k):
    # qmm_gemm_mod_p runs small unblocked INT8 products in one launch that centres A
    # and B and transposes B in LDS (no workspace); the staged calls convert B in HBM
    rng = np.random.default_rng(p * m + n + k)
    A = rng.integers(0, p, (m, k), dtype=np.uint8)
    B = rng.integers(0, p, (k, n), dtype=np.uint8)
    if k == 4096:   # the largest centred magnitude everywhere: k (p/2)^2 = 64 000 000
        A[:] = p // 2
        B[:] = p // 2
    want = ref.modmul(A, B, p)
    plan = qmm.choose_Qd(p, m, n, k, path=qmm.PATH_INT8)
    assert plan.k_block >= k and qmm.gemm_workspace_size(plan, m, n, k) == 0
    note("small int8", p, m, n, k, plan)
    dA, dB = dev(torch, A), dev(torch, B)
    C = torch.full((m, n), 0xCD, dtype=torch.uint8, device="cuda")
    qmm.gemm_mod_p(dA, dB, p, plan=plan, C=C, ws=torch.empty(0, dtype=torch.uint8, device="cuda"))
    np.testing.assert_array_equal(host(C), want)
    staged = qmm.gemm_centred(plan, dA, qmm.pack_centred_cols(plan, dB), n)
    np.testing.assert_array_equal(host(staged), want)


# The direct-load INT8 tile (4) reads A's rows whole, as int8: the residues
# themselves when p <= 128, k is a multiple of 128 and the int32 sums stay in range
# with A uncentred, A's centred copy otherwise (qmm_gemm_mod_p), and tile 3's kernel
# where neither is possible (qmm_gemm_centred on rows it cannot read whole).  Output
# 300 x 520: two rows of 256 x 256 tiles, both ragged.
@pytest.mark.parametrize("p,k,k_block", [(101, 1024, 0), (101, 1024, 256), (127, 640, 0), (2, 384, 0),
                                         (251, 1024, 0), (251, 1024, 384), (101, 1000, 0), (13, 200, 0)])
def test_int8_direct_tile_on_raw_and_centred_rows(torch, p, k, k_block):
    m, n = 300, 520
    rng = np.random.default_rng(p + k + k_block)
    A = rng.integers(0, p, (m, k), dtype=np.uint8)
    B = rng.integers(0, p, (k, n), dtype=np.uint8)
    want = ref.modmul(A, B, p)
    dA, dB = dev(torch, A), dev(torch, B)
    plan = qmm.choose_Qd(p, m, n, k, path=qmm.PATH_INT8)
    if k_block:
        plan.k_block = k_block
    plan.tile = 4
    note("int8 direct", plan, k)
    np.testing.assert_array_equal(host(qmm.gemm_mod_p(dA, dB, p, plan=plan)), want)
    Bt = qmm.pack_centred_cols(plan, dB)
    np.testing.assert_array_equal(host(qmm.gemm_centred(plan, dA, Bt, n)), want)
    # A as a view whose rows start 3 bytes in: read whole only after centring
    big = torch.zeros((m, k + 8), dtype=torch.uint8, device="cuda")
    big[:, 3:3 + k] = dA
    np.testing.assert_array_equal(host(qmm.gemm_mod_p(big[:, 3:3 + k], dB, p, plan=plan)), want)
    np.testing.assert_array_equal(host(qmm.gemm_centred(plan, big[:, 3:3 + k], Bt, n)), want)


# A grid of 256 x 256 tiles just past whole rounds over the CUs (17 x 16 = 272 or
# 17 x 17 = 289 tiles on 256 CUs) keeps the block of whole tiles on the large tiles
# and runs the ragged edge strips (the last row, and the last column) as split-K
# products on 128 x 128 tiles whose chunks are summed mod p.  Raw and centred A, a
# blocked plan, the register-staged tile and FP4, one or both strips.
@pytest.mark.parametrize("p,k,k_block,tile,path,n", [
    (101, 1024, 0, 0, qmm.PATH_INT8, 4096), (101, 1000, 0, 0, qmm.PATH_INT8, 4097),
    (251, 1024, 384, 0, qmm.PATH_INT8, 4097), (101, 1024, 0, 3, qmm.PATH_INT8, 4097),
    (7, 700, 0, 0, qmm.PATH_FP4, 4096), (7, 3000, 0, 0, qmm.PATH_FP4, 4097),
    # a thin bottom strip (1 row) beside a split-K right strip (20 columns)
    (101, 1024, 0, 0, qmm.PATH_INT8, 4116), (7, 700, 0, 0, qmm.PATH_FP4, 4116)])
def test_tail_of_a_partial_round_on_small_tiles(torch, p, k, k_block, tile, path, n):
    m = 4097
    rng = np.random.default_rng(p + k + tile + n)
    A = rng.integers(0, p, (m, k), dtype=np.uint8)
    B = rng.integers(0, p, (k, n), dtype=np.uint8)
    plan = qmm.choose_Qd(p, m, n, k, path=path)
    if k_block:
        plan.k_block = k_block
    plan.tile = tile
    note("tail split", plan, m, n, k)
    got = host(qmm.gemm_mod_p(dev(torch, A), dev(torch, B), p, plan=plan))
    np.testing.assert_array_equal(got, ref.modmul(A, B, p))


# Edge strips of at most 16 rows (columns) past whole rounds of 256 x 256 tiles run
# as int8 dot products of whole rows (thin strips); 17 rows take the split-K strips.
# Raw residues (p <= 128, k a multiple of 128) and centred rows, bottom and right;
# FP4 strips decode their e2m1 codes to int8 first.
@pytest.mark.parametrize("p,k,r,side,path", [
    (101, 256, 1, "bottom", qmm.PATH_INT8), (101, 250, 16, "bottom", qmm.PATH_INT8),
    (7, 256, 5, "bottom", qmm.PATH_INT8), (251, 256, 9, "right", qmm.PATH_INT8), (101, 250, 3, "right", qmm.PATH_INT8),
    (101, 256, 17, "right", qmm.PATH_INT8), (7, 301, 1, "bottom", qmm.PATH_FP4), (5, 256, 16, "right", qmm.PATH_FP4),
    (3, 999, 7, "bottom", qmm.PATH_FP4)])
def test_thin_edge_strips(torch, p, k, r, side, path):
    m, n = (512 + r, 32768) if side == "bottom" else (32768, 512 + r)
    rng = np.random.default_rng(p * 1000 + k + r)
    A = rng.integers(0, p, (m, k), dtype=np.uint8)
    B = rng.integers(0, p, (k, n), dtype=np.uint8)
    plan = qmm.choose_Qd(p, m, n, k, path=path)
    note("thin strip", side, r, plan, m, n, k)
    got = host(qmm.gemm_mod_p(dev(torch, A), dev(torch, B), p, plan=plan))
    np.testing.assert_array_equal(got, ref.modmul(A, B, p))


# More than one round of 256 x 256 tiles on the direct-load tile: 18 x 18 tiles
# (ragged last row and column, too many whole tiles for the edge split), raw and
# centred rows, one blocked plan.
@pytest.mark.parametrize("p,k,k_block", [(101, 1024, 0), (101, 1000, 0), (251, 640, 384), (7, 256, 0)])
def test_int8_direct_tile_over_two_rounds(torch, p, k, k_block):
    m = n = 4600
    rng = np.random.default_rng(p + k)
    A = rng.integers(0, p, (m, k), dtype=np.uint8)
    B = rng.integers(0, p, (k, n), dtype=np.uint8)
    plan = qmm.choose_Qd(p, m, n, k, path=qmm.PATH_INT8)
    if k_block:
        plan.k_block = k_block
    note("direct tile, two rounds", plan, m, n, k)
    np.testing.assert_array_equal(host(qmm.gemm_mod_p(dev(torch, A), dev(torch, B), p, plan=plan)), ref.modmul(A, B, p))


def test_edge_strips_of_unaligned_rows_take_split_k(torch):
    # A view whose rows are not 16-byte aligned, with k a multiple of 16 and p <= 128,
    # is read in place (no centred copy) on the register-staged tile, and the thin
    # dot-product strips need aligned rows: the 5-row bottom strip then runs as split-K
    # products on small tiles.  Every entry against the oracle.
    p, m, n, k = 101, 517, 32768, 256
    rng = np.random.default_rng(517)
    Ab = rng.integers(0, p, (m, k + 3), dtype=np.uint8)
    B = rng.integers(0, p, (k, n), dtype=np.uint8)
    A = np.ascontiguousarray(Ab[:, 1:1 + k])
    dA = torch.from_numpy(Ab).cuda()[:, 1:1 + k]
    plan = qmm.choose_Qd(p, m, n, k, path=qmm.PATH_INT8)
    note("unaligned A view, split-K strips", plan, m, n, k)
    np.testing.assert_array_equal(host(qmm.gemm_mod_p(dA, dev(torch, B), p, plan=plan)), ref.modmul(A, B, p))


@pytest.mark.parametrize("k", (1001, 4097, 2049))
def test_int8_unaligned_rows_on_every_tile(torch, k):
    # k odd: rows of A start at every byte offset within a dword, so the product
    # kernel's windowed loads of A take each byte shift on every tile variant; one case
    # is also cut into blocks.
    p = 101
    m, n = 300, 260
    rng = np.random.default_rng(k)
    A = rng.integers(0, p, (m, k), dtype=np.uint8)
    B = rng.integers(0, p, (k, n), dtype=np.uint8)
    want = ref.modmul(A, B, p)
    dA, dB = dev(torch, A), dev(torch, B)
    plan = qmm.choose_Qd(p, m, n, k, path=qmm.PATH_INT8)
    Bt = qmm.pack_centred_cols(plan, dB)
    for tile in (1, 2, 3, 4):
        for k_block in ((plan.k_block, 512) if k == 4097 else (plan.k_block,)):
            plan.tile, plan.k_block = tile, k_block
            note("int8 unaligned", k, "tile", tile, "k_block", k_block)
            np.testing.assert_array_equal(host(qmm.gemm_centred(plan, dA, Bt, n)), want,
                                          err_msg=f"tile {tile} k_block {k_block}")
            np.testing.assert_array_equal(host(qmm.gemm_mod_p(dA, dB, p, plan=plan)), want)
        plan = qmm.choose_Qd(p, m, n, k, path=qmm.PATH_INT8)


@pytest.mark.parametrize("validate", (False, True))
def test_products_on_a_side_stream(torch, validate):
    # gemm_mod_p on a stream that is not torch's current one: the binding's own
    # workspace and output stay allocated until that stream's kernels are done, and
    # validation reads its counts after them.
    p = 7
    rng = np.random.default_rng(31)
    A = rng.integers(0, p, (700, 900), dtype=np.uint8)
    B = rng.integers(0, p, (900, 500), dtype=np.uint8)
    want = ref.modmul(A, B, p)
    dA, dB = dev(torch, A), dev(torch, B)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    outs = []
    for path in (qmm.PATH_FP64_QADIC, qmm.PATH_INT8, qmm.PATH_FP4, qmm.PATH_FP64_REDQ):
        plan = qmm.choose_Qd(p, 700, 500, 900, path=path)
        plan.tile = 1 if path in (qmm.PATH_INT8, qmm.PATH_FP4) else 0   # the two-kernel form, with a workspace
        outs.append((plan, qmm.gemm_mod_p(dA, dB, p, plan=plan, stream=side, validate=validate)))
        # churn the allocator on the current stream while the side stream may still run
        junk = [torch.empty(1 << 20, dtype=torch.uint8, device="cuda").fill_(0xAB) for _ in range(8)]
        del junk
    side.synchronize()
    for plan, C in outs:
        np.testing.assert_array_equal(host(C), want, err_msg=str(plan))
    if validate:
        dB[5, 5] = 200
        torch.cuda.current_stream().synchronize()
        with pytest.raises(qmm.QmmError) as ei:
            qmm.gemm_mod_p(dA, dB, p, stream=side, validate=True)
        assert ei.value.status == qmm.EVALUE
