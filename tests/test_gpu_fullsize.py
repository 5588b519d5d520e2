"""Every entry of the full-size products against the CPU oracle (needs an MI355X).

The method recovers each dot product exactly (section 2.2, procedure (2): entry
(i, j) of C is the degree-d coefficient, reduced mod p), so every path must equal
the plain modular product bit for bit.  These tests compute the oracle once per
workload at its full size on all host threads -- GF(7) 4096^3, p = 101 8192^3, and
A x A for the n = 16384 random symmetric 0/1 matrix modulo 3 -- and compare every
entry of every path's result with it.  (The 2000-product batch is compared product
by product in test_gpu_batched.py; the 64^3 workload in test_gpu_parity.py.)
"""
import functools
import sys
import time

import numpy as np
import pytest

from oracle import reference as ref
from paper_0803_1975_amd import qmm
import synth

pytestmark = pytest.mark.gpu

UNBLOCKED_EQ4 = qmm.PLAN_UNBLOCKED | qmm.BOUND_EQ4

# (path, flags, tile) run at every workload that has a plan for them.  Q-adic paths
# run with the planner's plan and with the paper's (unblocked, eq. (4) as printed);
# the right, left and full compressions are unblocked by construction.  INT8 and
# FP4 run on the automatic tile and on each explicit tile variant.
COMMON = [
    (qmm.PATH_FP64_QADIC, 0, 0), (qmm.PATH_FP64_QADIC, UNBLOCKED_EQ4, 0),
    (qmm.PATH_FP64_REDQ, 0, 0), (qmm.PATH_FP64_LEFT, 0, 0), (qmm.PATH_FP64_FULL, 0, 0),
    (qmm.PATH_FP32_QADIC, 0, 0),
    (qmm.PATH_INT8, 0, 0), (qmm.PATH_INT8, 0, 1), (qmm.PATH_INT8, 0, 2), (qmm.PATH_INT8, 0, 3),
    (qmm.PATH_INT8, 0, 4),
    (qmm.PATH_AUTO, 0, 0),
]
SMALL_P = [  # p <= 8 (FP4 codes) and short enough k for every FP32 form
    (qmm.PATH_FP32_QADIC, UNBLOCKED_EQ4, 0), (qmm.PATH_FP32_REDQ, 0, 0), (qmm.PATH_FP32_LEFT, 0, 0),
    (qmm.PATH_FP32_FULL, 0, 0),
    (qmm.PATH_FP4, 0, 0), (qmm.PATH_FP4, 0, 1), (qmm.PATH_FP4, 0, 2), (qmm.PATH_FP4, 0, 3),
]
CASES = ([("square",) + c for c in COMMON + SMALL_P] + [("large",) + c for c in COMMON] +
         [("graph",) + c for c in COMMON + SMALL_P])


def note(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    if not _t.cuda.is_available():
        pytest.fail("these tests need a GPU")
    return _t


@functools.lru_cache(maxsize=1)
def workload_and_oracle(name):
    """(p, A, B, C) with C the oracle's full product; one workload cached at a time."""
    p, A, B = synth.workload(name)
    m, k = A.shape
    n = B.shape[1]
    note(f"oracle {name}: {m}x{k} times {k}x{n} mod {p} on {ref.oracle_threads()} threads")
    t0 = time.perf_counter()
    C = ref.modmul(A, B, p)
    note(f"oracle {name}: {time.perf_counter() - t0:.1f} s")
    return p, A, B, C


def case_id(c):
    name, path, flags, tile = c
    return f"{name}-{qmm.PATH_NAMES[path]}" + ("-paper" if flags else "") + (f"-tile{tile}" if tile else "")


@pytest.mark.timeout(600)
@pytest.mark.parametrize("case", CASES, ids=[case_id(c) for c in CASES])
def test_every_entry_matches_the_oracle(torch, case):
    name, path, flags, tile = case
    p, A, B, want = workload_and_oracle(name)
    m, k = A.shape
    n = B.shape[1]
    dA = torch.from_numpy(A).cuda()
    dB = dA if name == "graph" else torch.from_numpy(B).cuda()
    if path == qmm.PATH_AUTO:
        plan = None                                  # the library chooses inside qmm_gemm_mod_p
        note(name, "automatic plan", qmm.choose_Qd(p, m, n, k))
    else:
        st, plan = qmm.try_choose_Qd(p, m, n, k, path=path, flags=flags)
        assert st == qmm.OK, f"{case_id(case)}: no plan ({qmm.last_error()})"
        plan.tile = tile
        note(name, plan)
    C = qmm.gemm_mod_p(dA, dB, p, plan=plan)
    torch.cuda.synchronize()
    got = C.cpu().numpy()
    del C
    if not np.array_equal(got, want):
        bad = np.argwhere(got != want)
        raise AssertionError(f"{case_id(case)}: {len(bad)} of {got.size} entries differ, first at "
                             f"{tuple(bad[0])}: got {got[tuple(bad[0])]}, want {want[tuple(bad[0])]}")


def test_fp32_forms_are_refused_where_no_bound_holds(torch):
    # p = 101, k = 8192: k (p-1)^2 = 8.2e7 > 2^23, so no FP32 word holds even one
    # unblocked residue product sum (eq. (3) with a 24-bit mantissa); the FP32 Q-adic
    # path needs k-blocks, and the unblocked forms are refused rather than run.
    w = synth.WORKLOADS["large"]
    for path in (qmm.PATH_FP32_REDQ, qmm.PATH_FP32_LEFT, qmm.PATH_FP32_FULL, qmm.PATH_FP4):
        st, _ = qmm.try_choose_Qd(w["p"], w["m"], w["n"], w["k"], path=path)
        assert st != qmm.OK, qmm.PATH_NAMES[path]
    st, _ = qmm.try_choose_Qd(w["p"], w["m"], w["n"], w["k"], path=qmm.PATH_FP32_QADIC, flags=UNBLOCKED_EQ4)
    assert st == qmm.EBOUND
