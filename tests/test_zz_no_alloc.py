"""qmm_gemm_mod_p_noalloc against qmm_gemm_mod_p (needs an MI355X).

The allocation-free entry point runs the same plan and kernels as qmm_gemm_mod_p
with the library's per-GPU scratch as workspace, so its output must equal that
entry point's byte for byte, on consecutive calls that reuse the scratch (the
second with a smaller input, so stale bytes of the first call sit past what the
second writes), and both must equal the CPU oracle.
"""
import sys

import numpy as np
import pytest

from oracle import reference as ref
from paper_0803_1975_amd import qmm

pytestmark = pytest.mark.gpu


def note(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    if not _t.cuda.is_available():
        pytest.fail("these tests need a GPU")
    return _t


# (p, path, flags): every kind of workspace the product uses -- packed words (Q-adic,
# right, left, full), centred transposed B (INT8), FP4 codes -- and the library's
# automatic plan (plan = NULL).
PATHS = [
    (7, qmm.PATH_FP64_QADIC, 0), (3, qmm.PATH_FP64_QADIC, qmm.PLAN_UNBLOCKED | qmm.BOUND_EQ4),
    (5, qmm.PATH_FP64_REDQ, 0), (3, qmm.PATH_FP64_LEFT, 0), (2, qmm.PATH_FP64_FULL, 0),
    (7, qmm.PATH_FP32_QADIC, 0), (101, qmm.PATH_INT8, 0), (251, qmm.PATH_INT8, 0), (7, qmm.PATH_FP4, 0),
    (13, None, 0), (3, None, 0),
]
# first a larger product, then a smaller one with ragged edges
SHAPES = [(1000, 900, 1100), (300, 200, 257)]


@pytest.mark.parametrize("case", PATHS, ids=[f"p{c[0]}-{qmm.PATH_NAMES[c[1]] if c[1] else 'auto'}"
                                            + ("-paper" if c[2] else "") for c in PATHS])
def test_noalloc_matches_gemm_mod_p_on_two_calls(torch, case):
    p, path, flags = case
    rng = np.random.default_rng(1000 + p)
    for m, n, k in SHAPES:
        A = rng.integers(0, p, (m, k), dtype=np.uint8)
        B = rng.integers(0, p, (k, n), dtype=np.uint8)
        want = ref.modmul(A, B, p)
        dA = torch.from_numpy(A).cuda()
        dB = torch.from_numpy(B).cuda()
        plan = None if path is None else qmm.choose_Qd(p, m, n, k, path=path, flags=flags)
        note(p, m, n, k, plan if plan is not None else "automatic plan")
        assert qmm.gemm_workspace_size(plan if plan is not None else qmm.choose_Qd(p, m, n, k), m, n, k) \
            <= qmm.NOALLOC_SCRATCH_BYTES
        C_ws = qmm.gemm_mod_p(dA, dB, p, plan=plan)
        C_na = torch.full((m, n), 255, dtype=torch.uint8, device="cuda")
        qmm.gemm_mod_p_noalloc(dA, dB, p, plan=plan, C=C_na)
        torch.cuda.synchronize()
        got_ws, got_na = C_ws.cpu().numpy(), C_na.cpu().numpy()
        assert np.array_equal(got_na, got_ws), f"{m}x{n}x{k}: noalloc differs from gemm_mod_p"
        assert np.array_equal(got_na, want), f"{m}x{n}x{k}: noalloc differs from the oracle"


def test_noalloc_strided_output_view(torch):
    # C as a column window of a wider matrix: only the window is written
    p, m, n, k = 31, 257, 130, 515
    rng = np.random.default_rng(7)
    A = rng.integers(0, p, (m, k), dtype=np.uint8)
    B = rng.integers(0, p, (k, n), dtype=np.uint8)
    big = torch.full((m, n + 40), 77, dtype=torch.uint8, device="cuda")
    qmm.gemm_mod_p_noalloc(torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda(), p, C=big[:, 20:20 + n])
    out = big.cpu().numpy()
    assert np.array_equal(out[:, 20:20 + n], ref.modmul(A, B, p))
    assert (out[:, :20] == 77).all() and (out[:, 20 + n:] == 77).all()


def test_noalloc_refuses_products_beyond_the_scratch(torch):
    # FP64 Q-adic with d = 1 at 4096 x 4096 x 4096: CA alone is 4096 x 2048 doubles
    # (64 MiB), so the workspace exceeds the scratch and nothing may be launched.
    p, m, n, k = 7, 4096, 16, 4096
    A = torch.zeros((m, k), dtype=torch.uint8, device="cuda")
    B = torch.zeros((k, n), dtype=torch.uint8, device="cuda")
    plan = qmm.choose_Qd(p, m, n, k, path=qmm.PATH_FP64_QADIC, flags=qmm.PLAN_UNBLOCKED | qmm.BOUND_EQ4)
    assert qmm.gemm_workspace_size(plan, m, n, k) > qmm.NOALLOC_SCRATCH_BYTES
    C = torch.full((m, n), 9, dtype=torch.uint8, device="cuda")
    with pytest.raises(qmm.QmmError) as e:
        qmm.gemm_mod_p_noalloc(A, B, p, plan=plan, C=C)
    assert e.value.status == qmm.ENOSPACE
    assert "scratch" in qmm.last_error()
    torch.cuda.synchronize()
    assert (C.cpu().numpy() == 9).all()
    # the entry point still works after the refusal
    small = torch.ones((64, 64), dtype=torch.uint8, device="cuda")
    got = qmm.gemm_mod_p_noalloc(small, small, p).cpu().numpy()
    assert (got == 64 % p).all()
