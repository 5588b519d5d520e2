"""Left and full compression (sections 4 and 5) and ReduceAndCompress (procedure (1))
on the GPU against the CPU oracle, through the C ABI (needs an MI355X).

Every result is compared bit for bit: packed words with the oracle's packings,
products with the oracle's modular product, on shapes that span several 128 x 128
tiles of words and end in ragged tails.
"""
import sys

import numpy as np
import pytest

from oracle import bounds
from oracle import reference as ref
from paper_0803_1975_amd import qmm

pytestmark = pytest.mark.gpu


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


def words(x):
    return np.asarray(x).astype(np.uint64)


def full_plan(p, t, d, d2, k, beta=53):
    return qmm.Plan(p=p, t=t, d=d, beta=beta, k_block=max(k, 1),
                    path=qmm.PATH_FP64_FULL if beta == 53 else qmm.PATH_FP32_FULL, regime=qmm.REGIME_EXACT, d2=d2)


# --- packings -------------------------------------------------------------------
@pytest.mark.parametrize("p,t,d,d2,beta", [(3, 9, 1, 1, 53), (2, 3, 3, 3, 53), (7, 12, 1, 1, 53), (3, 4, 2, 1, 24),
                                           (101, 17, 0, 2, 53), (5, 6, 7, 0, 53)])
def test_left_and_theta_packings_match_oracle(torch, p, t, d, d2, beta):
    note("pack left/theta", p, t, d, d2, beta)
    rng = np.random.default_rng(t * 11 + d)
    A = rng.integers(0, p, (301, 37), dtype=np.uint8)
    B = rng.integers(0, p, (37, 299), dtype=np.uint8)
    pl = full_plan(p, t, d, d2, 37, beta)
    CAl = qmm.pack_left(pl, dev(torch, A))
    CBt = qmm.pack_full_right(pl, dev(torch, B))
    torch.cuda.synchronize()
    np.testing.assert_array_equal(words(host(CAl)), ref.compress_left(A, t, d))
    np.testing.assert_array_equal(words(host(CBt)), words(ref.compress_full_right(B, t, d, d2)))


# --- products -------------------------------------------------------------------
SHAPES = [(1, 1, 1), (3, 5, 7), (130, 257, 33), (389, 300, 61), (700, 517, 19)]


@pytest.mark.parametrize("path", [qmm.PATH_FP64_LEFT, qmm.PATH_FP32_LEFT, qmm.PATH_FP64_FULL, qmm.PATH_FP32_FULL])
@pytest.mark.parametrize("p", [2, 3, 7, 31, 101])
def test_left_and_full_gemm_match_oracle(torch, path, p):
    rng = np.random.default_rng(p * 13 + path)
    for m, n, k in SHAPES:
        st, pl = qmm.try_choose_Qd(p, m, n, k, path=path)
        if st != qmm.OK:
            assert st == qmm.EBOUND and bounds.smallest_t(p, k) >= (53 if path in (7, 9) else 24)
            continue
        note("gemm", qmm.PATH_NAMES[path], p, m, n, k, pl)
        A = rng.integers(0, p, (m, k), dtype=np.uint8)
        B = rng.integers(0, p, (k, n), dtype=np.uint8)
        C = host(qmm.gemm_mod_p(dev(torch, A), dev(torch, B), p, plan=pl))
        np.testing.assert_array_equal(C, ref.modmul(A, B, p))


@pytest.mark.parametrize("p,t,d,d2,k", [(3, 9, 1, 1, 64), (3, 9, 4, 0, 64), (3, 9, 0, 4, 64), (2, 3, 3, 3, 7),
                                        (2, 1, 6, 6, 1), (7, 12, 1, 1, 100), (5, 8, 1, 2, 15)])
def test_full_stages_every_degree_pair(torch, p, t, d, d2, k):
    # explicit plans (not only the planner's), including the degenerate pairs that
    # are left (d2 = 0) and right (d = 0) compression, at the largest word t(d+1)(d2+1)
    note("full stages", p, t, d, d2, k)
    pl = full_plan(p, t, d, d2, k)
    assert qmm.validate_plan(pl, 300, 290, k) == qmm.OK
    rng = np.random.default_rng(k + d * 10 + d2)
    A = rng.integers(0, p, (300, k), dtype=np.uint8)
    B = rng.integers(0, p, (k, 290), dtype=np.uint8)
    CAl = qmm.pack_left(pl, dev(torch, A))
    CBt = qmm.pack_full_right(pl, dev(torch, B))
    C = host(qmm.gemm_full_packed(pl, CAl, CBt, 300, 290))
    np.testing.assert_array_equal(C, ref.modmul(A, B, p))
    # the oracle's step-by-step model on a corner of the same inputs
    np.testing.assert_array_equal(C[:24, :20], ref.full_compressed_product_mod_p(A[:24], B[:, :20], p, t, d, d2))


@pytest.mark.parametrize("path", [qmm.PATH_FP64_LEFT, qmm.PATH_FP64_FULL, qmm.PATH_FP32_FULL])
@pytest.mark.parametrize("p", [2, 3, 7])
def test_worst_case_at_the_eq3_edge(torch, path, p):
    # every residue p-1 at the largest k with k (p-1)^2 < Q: every coefficient of
    # every word is Q - 1 or close, the largest words the bounds allow
    t = 9
    k = ((1 << t) - 1) // (p - 1) ** 2
    st, pl = qmm.try_choose_Qd(p, 257, 259, k, path=path)
    assert st == qmm.OK and pl.t <= t
    note("worst", qmm.PATH_NAMES[path], p, k, pl)
    A = np.full((257, k), p - 1, np.uint8)
    B = np.full((k, 259), p - 1, np.uint8)
    C = host(qmm.gemm_mod_p(dev(torch, A), dev(torch, B), p, plan=pl))
    np.testing.assert_array_equal(C, np.full((257, 259), (k * (p - 1) ** 2) % p, np.uint8))


@pytest.mark.parametrize("p,m,n,k", [(3, 8, 8, 4096), (3, 8, 4096, 2), (3, 4096, 8, 2), (3, 6, 6, 4),
                                     (7, 300, 200, 64)])
def test_any_compression_results(torch, p, m, n, k):
    pl = qmm.choose_Qd(p, m, n, k, path=qmm.PATH_FP64_QADIC, flags=qmm.PLAN_ANY_COMPRESSION)
    note("any compression", p, m, n, k, pl)
    rng = np.random.default_rng(m + n + k)
    A = rng.integers(0, p, (m, k), dtype=np.uint8)
    B = rng.integers(0, p, (k, n), dtype=np.uint8)
    C = host(qmm.gemm_mod_p(dev(torch, A), dev(torch, B), p, plan=pl))
    np.testing.assert_array_equal(C, ref.modmul(A, B, p))


@pytest.mark.parametrize("path", [qmm.PATH_FP64_LEFT, qmm.PATH_FP64_FULL])
def test_degenerate_shapes_and_guard_bytes(torch, path):
    p = 5
    for m, n, k in [(0, 5, 3), (5, 0, 3), (1, 1, 1), (2, 129, 3), (129, 2, 3)]:
        note("degenerate", qmm.PATH_NAMES[path], m, n, k)
        rng = np.random.default_rng(m * 7 + n)
        A = rng.integers(0, p, (m, k), dtype=np.uint8)
        B = rng.integers(0, p, (k, n), dtype=np.uint8)
        pl = qmm.choose_Qd(p, m, n, k, path=path)
        big = torch.full((m + 2, n + 9), 0xAB, dtype=torch.uint8, device="cuda")
        C = big[1:m + 1, 3:n + 3]
        qmm.gemm_mod_p(dev(torch, A), dev(torch, B), p, plan=pl, C=C)
        out = host(big)
        np.testing.assert_array_equal(out[1:m + 1, 3:n + 3], ref.modmul(A, B, p))
        mask = np.ones_like(out, dtype=bool)
        mask[1:m + 1, 3:n + 3] = False
        assert (out[mask] == 0xAB).all()
    # k = 0: the empty sum
    pl = qmm.choose_Qd(p, 4, 4, 0, path=path)
    C = qmm.gemm_mod_p(torch.empty((4, 0), dtype=torch.uint8, device="cuda"),
                       torch.empty((0, 4), dtype=torch.uint8, device="cuda"), p, plan=pl)
    assert (host(C) == 0).all()


# The word products store C through LDS as whole dwords when C and its leading
# dimension are 4-byte aligned and a wavefront's block of residues fits the staging
# buffers (E = residues per word up to 17 for doubles, 8 for floats), and byte by
# byte otherwise.  Each case runs both: an aligned view with a ragged right edge
# (ldc = 260, n = 257) and a view one byte in; E spans 1 to 52.
EPI_CASES = [(qmm.PATH_FP64_QADIC, 7, 70), (qmm.PATH_FP64_QADIC, 2, 7), (qmm.PATH_FP64_QADIC, 3, 3000),
             (qmm.PATH_FP32_QADIC, 7, 300),
             (qmm.PATH_FP64_REDQ, 7, 70), (qmm.PATH_FP64_REDQ, 3, 3), (qmm.PATH_FP64_REDQ, 2, 7),
             (qmm.PATH_FP64_REDQ, 2, 3), (qmm.PATH_FP64_LEFT, 3, 20), (qmm.PATH_FP64_LEFT, 2, 1),
             (qmm.PATH_FP64_FULL, 7, 50), (qmm.PATH_FP64_FULL, 3, 3), (qmm.PATH_FP64_FULL, 2, 7),
             (qmm.PATH_FP64_FULL, 2, 1), (qmm.PATH_FP32_REDQ, 2, 7), (qmm.PATH_FP32_REDQ, 3, 3),
             (qmm.PATH_FP32_LEFT, 2, 3), (qmm.PATH_FP32_FULL, 2, 1), (qmm.PATH_FP32_FULL, 7, 50)]


@pytest.mark.parametrize("path,p,k", EPI_CASES)
def test_dword_epilogue_and_byte_fallback(torch, path, p, k):
    m, n = 300, 257
    pl = qmm.choose_Qd(p, m, n, k, path=path)
    note("epilogue", pl, k)
    rng = np.random.default_rng(p * 100 + k + path)
    A = rng.integers(0, p, (m, k), dtype=np.uint8)
    B = rng.integers(0, p, (k, n), dtype=np.uint8)
    want = ref.modmul(A, B, p)
    dA, dB = dev(torch, A), dev(torch, B)
    for c0, width in ((0, 260), (1, 261)):
        big = torch.full((m + 2, width), 0xAB, dtype=torch.uint8, device="cuda")
        C = big[1:m + 1, c0:c0 + n]
        qmm.gemm_mod_p(dA, dB, p, plan=pl, C=C)
        out = host(big)
        np.testing.assert_array_equal(out[1:m + 1, c0:c0 + n], want, err_msg=f"view at column {c0}")
        mask = np.ones_like(out, dtype=bool)
        mask[1:m + 1, c0:c0 + n] = False
        assert (out[mask] == 0xAB).all(), f"view at column {c0}: bytes outside C written"


# Whole tiles of left compression (one residue per word along a row) store each
# output row's residues as dwords after a quad transpose; whole tiles of right or full
# compression with 2 or 4 residues along a row store each word's run of residues as
# one 2- or 4-byte store.  With m = 300 and n = 520 the first tile (128 x 128 words)
# is whole for up to 2 residues down and 4 across, the others take the general
# stores.  Each case names the (dq+1, dth+1) shape it is meant to reach.
DIRECT_CASES = [(qmm.PATH_FP64_REDQ, 31, 500, 1, 2), (qmm.PATH_FP64_REDQ, 7, 70, 1, 4),
                (qmm.PATH_FP64_FULL, 7, 50, 2, 2), (qmm.PATH_FP64_LEFT, 31, 500, 2, 1),
                (qmm.PATH_FP32_REDQ, 3, 256, 1, 2), (qmm.PATH_FP32_LEFT, 3, 256, 2, 1),
                (qmm.PATH_FP64_REDQ, 3, 256, 1, 4), (qmm.PATH_FP64_FULL, 3, 256, 2, 2)]


@pytest.mark.parametrize("path,p,k,dq1,dt1", DIRECT_CASES)
def test_direct_word_stores(torch, path, p, k, dq1, dt1):
    m, n = 300, 520
    pl = qmm.choose_Qd(p, m, n, k, path=path)
    if path in (qmm.PATH_FP64_REDQ, qmm.PATH_FP32_REDQ):
        shape = (1, pl.d + 1)
    elif path in (qmm.PATH_FP64_LEFT, qmm.PATH_FP32_LEFT):
        shape = (pl.d + 1, 1)
    else:
        shape = (pl.d + 1, pl.d2 + 1)
    assert shape == (dq1, dt1), pl
    note("direct stores", pl, k)
    rng = np.random.default_rng(p * 7 + k + 31 * path)
    A = rng.integers(0, p, (m, k), dtype=np.uint8)
    B = rng.integers(0, p, (k, n), dtype=np.uint8)
    want = ref.modmul(A, B, p)
    dA, dB = dev(torch, A), dev(torch, B)
    big = torch.full((m + 2, 528), 0xAB, dtype=torch.uint8, device="cuda")
    C = big[1:m + 1, 4:4 + n]
    qmm.gemm_mod_p(dA, dB, p, plan=pl, C=C)
    out = host(big)
    np.testing.assert_array_equal(out[1:m + 1, 4:4 + n], want)
    mask = np.ones_like(out, dtype=bool)
    mask[1:m + 1, 4:4 + n] = False
    assert (out[mask] == 0xAB).all(), "bytes outside C written"


# --- ReduceAndCompress ------------------------------------------------------------
def compress_case(torch, p, m, n, k, path=qmm.PATH_FP64_QADIC, flags=0):
    pl = qmm.choose_Qd(p, m, n, k, path=path, flags=flags)
    rng = np.random.default_rng(p * 1000 + m + n + k)
    A = rng.integers(0, p, (m, k), dtype=np.uint8)
    B = rng.integers(0, p, (k, n), dtype=np.uint8)
    CA = qmm.pack_rows_rev(pl, dev(torch, A))
    CB = qmm.pack_cols_fwd(pl, dev(torch, B))
    CC = qmm.gemm_packed_compress(pl, k, CA, CB)
    C = qmm.gemm_packed(pl, k, CA, CB)
    torch.cuda.synchronize()
    return pl, A, B, host(CC), host(C)


@pytest.mark.parametrize("p,m,n,k,path", [
    (3, 300, 389, 64, qmm.PATH_FP64_QADIC),      # offset regime, t = 9, d = 4: 5 columns per word
    (7, 260, 257, 200, qmm.PATH_FP64_QADIC),
    (3, 129, 700, 3000, qmm.PATH_FP64_QADIC),    # blocked plan
    (101, 130, 131, 50, qmm.PATH_FP64_QADIC),    # d small
    (2, 140, 333, 77, qmm.PATH_FP32_QADIC),      # 3 residues per float: tiles cut words
    (2, 150, 301, 15, qmm.PATH_FP32_QADIC),      # 6 residues per float: tiles of whole words
    (2, 150, 301, 15, qmm.PATH_FP64_QADIC),      # 8 residues per double: the most the slots take
    (2, 150, 256, 2, qmm.PATH_FP64_QADIC),       # n a multiple of 128
    (5, 99, 385, 9, qmm.PATH_FP32_QADIC),
    (3, 1, 1, 1, qmm.PATH_FP64_QADIC)])
def test_reduce_and_compress_matches_oracle(torch, p, m, n, k, path):
    pl, A, B, CC, C = compress_case(torch, p, m, n, k, path)
    note("compress", p, m, n, k, pl)
    want = ref.modmul(A, B, p)
    np.testing.assert_array_equal(C, want)
    np.testing.assert_array_equal(words(CC), ref.compress_rows_rev(want, pl.t, pl.d))


def test_reduce_and_compress_chains_a_power(torch):
    # A^3 mod p with the intermediate A^2 kept packed: (A A) comes out as CompressRows
    # words and is the left operand of the next product as it stands
    p, n = 3, 517
    pl = qmm.choose_Qd(p, n, n, n, path=qmm.PATH_FP64_QADIC)
    note("chain", pl)
    rng = np.random.default_rng(9)
    A = rng.integers(0, p, (n, n), dtype=np.uint8)
    Ad = dev(torch, A)
    CA = qmm.pack_rows_rev(pl, Ad)
    CB = qmm.pack_cols_fwd(pl, Ad)
    CC = qmm.gemm_packed_compress(pl, n, CA, CB)
    C3 = host(qmm.gemm_packed(pl, n, CC, CB))
    A2 = ref.modmul(A, A, p)
    np.testing.assert_array_equal(C3, ref.modmul(A2, A, p))
    # and once more: A^4 from the packed A^3
    CC3 = qmm.gemm_packed_compress(pl, n, CC, CB)
    np.testing.assert_array_equal(host(qmm.unpack(pl, qmm.ROWS_REV, n, n, CC3)), C3)
    C4 = host(qmm.gemm_packed(pl, n, CC3, CB))
    np.testing.assert_array_equal(C4, ref.modmul(C3, A, p))


def test_reduce_and_compress_output_view_and_guard_words(torch):
    p, m, n, k = 7, 200, 301, 90
    pl = qmm.choose_Qd(p, m, n, k, path=qmm.PATH_FP64_QADIC)
    rng = np.random.default_rng(3)
    A = rng.integers(0, p, (m, k), dtype=np.uint8)
    B = rng.integers(0, p, (k, n), dtype=np.uint8)
    CA = qmm.pack_rows_rev(pl, dev(torch, A))
    CB = qmm.pack_cols_fwd(pl, dev(torch, B))
    nw = -(-n // (pl.d + 1))
    big = torch.full((m + 2, nw + 5), -1.0, dtype=torch.float64, device="cuda")
    qmm.gemm_packed_compress(pl, k, CA, CB, CC=big[1:m + 1, 2:nw + 2])
    out = host(big)
    np.testing.assert_array_equal(words(out[1:m + 1, 2:nw + 2]), ref.compress_rows_rev(ref.modmul(A, B, p), pl.t, pl.d))
    mask = np.ones_like(out, dtype=bool)
    mask[1:m + 1, 2:nw + 2] = False
    assert (out[mask] == -1.0).all()


def test_reduce_and_compress_words_wider_than_their_bytes(torch):
    # nine residues per double (more than its 8 bytes): tiles of whole words, 126 columns
    p, m, n, k = 2, 150, 301, 15
    pl = qmm.Plan(p=p, t=5, d=8, beta=53, k_block=k, path=qmm.PATH_FP64_QADIC, regime=qmm.REGIME_OFFSET, g=1)
    assert qmm.validate_plan(pl, m, n, k) == qmm.OK
    note("compress whole words", pl)
    rng = np.random.default_rng(11)
    A = rng.integers(0, p, (m, k), dtype=np.uint8)
    B = rng.integers(0, p, (k, n), dtype=np.uint8)
    CC = qmm.gemm_packed_compress(pl, k, qmm.pack_rows_rev(pl, dev(torch, A)), qmm.pack_cols_fwd(pl, dev(torch, B)))
    np.testing.assert_array_equal(words(host(CC)), ref.compress_rows_rev(ref.modmul(A, B, p), pl.t, pl.d))


@pytest.mark.parametrize("beta", [53, 24])
@pytest.mark.parametrize("p,m,n,k", [(3, 389, 300, 61), (7, 130, 257, 33), (101, 200, 131, 20), (2, 1, 1, 1)])
def test_stage_calls_convert_residues_in_the_load_path(torch, beta, p, m, n, k):
    # qmm_gemm_right_packed / qmm_gemm_left_packed take the residue operand as bytes
    # and convert it on its way into LDS (qmm_gemm_mod_p converts it by a pass)
    rng = np.random.default_rng(m + n + k + beta)
    A = rng.integers(0, p, (m, k), dtype=np.uint8)
    B = rng.integers(0, p, (k, n), dtype=np.uint8)
    want = ref.modmul(A, B, p)
    dA, dB = dev(torch, A), dev(torch, B)
    for path in ((qmm.PATH_FP64_REDQ, qmm.PATH_FP64_LEFT) if beta == 53 else (qmm.PATH_FP32_REDQ, qmm.PATH_FP32_LEFT)):
        st, pl = qmm.try_choose_Qd(p, m, n, k, path=path)
        if st != qmm.OK:
            continue
        note("stage", qmm.PATH_NAMES[path], p, m, n, k, pl)
        if path in (qmm.PATH_FP64_REDQ, qmm.PATH_FP32_REDQ):
            C = qmm.gemm_right_packed(pl, dA, qmm.pack_rows_fwd(pl, dB), n)
        else:
            C = qmm.gemm_left_packed(pl, qmm.pack_left(pl, dA), dB, m)
        np.testing.assert_array_equal(host(C), want)
        np.testing.assert_array_equal(host(qmm.gemm_mod_p(dA, dB, p, plan=pl)), want)
