"""The library's planner (qmm_choose_Qd) against the oracle's bound predicates.

Every plan it returns must satisfy the oracle's regime test, and no plan that the
oracle accepts may be cheaper under the planner's stated objective (packed words
per output plus 8 words per extra block, blocks a multiple of 16 words)."""
import pytest

from oracle import bounds
from paper_0803_1975_amd import qmm

KT_WORDS = 16
BLOCK_COST = 8


def brute_force_best(p, k, beta, g=1, unblocked=False, eq4=False):
    best = None
    for t in range(1, beta):
        kbmax = ((1 << t) - 1) // ((p - 1) ** 2)
        if kbmax < 1:
            continue
        for d in range(0, beta // t + 1):
            if k <= kbmax:
                kb = k
            elif unblocked:
                continue
            else:
                unit = (d + 1) * KT_WORDS
                kb = (kbmax // unit) * unit
                if kb < 1:
                    continue
            if d > 0 and d + 1 > kb:
                continue
            if eq4 and not bounds.eq4_upper_ok(t, d, beta):
                continue
            if bounds.qadic_regime(p, kb, t, d, beta, g) is None:
                continue
            blocks = -(-k // kb)
            cost = -(-k // (d + 1)) + (blocks - 1) * BLOCK_COST
            if best is None or cost < best[0] or (cost == best[0] and blocks < best[1]):
                best = (cost, blocks)
    return best


CASES = [(p, k) for p in (2, 3, 5, 7, 11, 13, 31, 101, 251)
         for k in (1, 2, 5, 15, 16, 63, 64, 100, 255, 256, 511, 1000, 4096, 8192, 16384, 100000)]


@pytest.mark.parametrize("p,k", CASES)
def test_fp64_qadic_plan_is_valid_and_optimal(p, k):
    for unblocked in (False, True):
      for eq4 in (False, True):
        flags = (qmm.PLAN_UNBLOCKED if unblocked else 0) | (qmm.BOUND_EQ4 if eq4 else 0)
        st, pl = qmm.try_choose_Qd(p, 32, 32, k, path=qmm.PATH_FP64_QADIC, flags=flags)
        best = brute_force_best(p, k, 53, unblocked=unblocked, eq4=eq4)
        if best is None:
            assert st == qmm.EBOUND
            continue
        assert st == qmm.OK, qmm.last_error()
        kb = min(pl.k_block, k)
        reg = bounds.qadic_regime(p, kb, pl.t, pl.d, 53, pl.g)
        assert reg == ("exact" if pl.regime == qmm.REGIME_EXACT else "offset")
        blocks = -(-k // pl.k_block)
        if pl.k_block < k:
            assert pl.k_block % ((pl.d + 1) * KT_WORDS) == 0
        cost = -(-k // (pl.d + 1)) + (blocks - 1) * BLOCK_COST
        assert (cost, blocks) == best
        assert qmm.validate_plan(pl, 32, 32, k) == qmm.OK


@pytest.mark.parametrize("p,k", [(3, 15), (3, 255), (7, 56), (2, 300), (101, 1000), (3, 511)])
def test_fp32_qadic_plans(p, k):
    st, pl = qmm.try_choose_Qd(p, 8, 8, k, path=qmm.PATH_FP32_QADIC)
    best = brute_force_best(p, k, 24)
    assert (st == qmm.OK) == (best is not None)
    if st == qmm.OK:
        assert bounds.qadic_regime(p, min(pl.k_block, k), pl.t, pl.d, 24, pl.g) is not None


def test_fp32_compression_for_p101_is_d0():
    # Q > 10^4 for p = 101 already, so Q^2 > 2^24: only d = 0 is possible in 24 bits.
    pl = qmm.choose_Qd(101, 8, 8, 8192, path=qmm.PATH_FP32_QADIC)
    assert pl.d == 0 and pl.k_block < 8192


def test_paper_rule_flag_matches_oracle():
    for p in (2, 3, 7, 101):
        for k in (1, 2, 7, 15, 64, 257, 4096, 32767, 32768):
            pl = qmm.choose_Qd(p, 1, 1, k, path=qmm.PATH_FP64_QADIC, flags=qmm.BOUND_PAPER)
            assert (pl.t, pl.d) == bounds.paper_choice(p, k, 53)


def test_proven_unblocked_plans_reproduce_table1_interior():
    # Strictly inside each printed range from Q = 2^6 on, the proven unblocked plan is
    # the paper's (t, d): the offset regime admits Table 1 there.
    for k, t, d in [(15, 6, 7), (31, 7, 6), (63, 8, 5), (255, 10, 4), (2047, 13, 3), (32767, 17, 2)]:
        pl = qmm.choose_Qd(3, 8, 8, k, path=qmm.PATH_FP64_QADIC, flags=qmm.PLAN_UNBLOCKED | qmm.BOUND_EQ4)
        assert (pl.t, pl.d) == (t, d), (k, pl)


def test_workload_plans():
    # small: eq. (4) as printed gives t = 9, d = 4 (offset regime); its sharper sum
    # form admits d = 5 at the same Q (words stay below 2^46, high part below 2^51)
    pl = qmm.choose_Qd(3, 64, 64, 64, path=qmm.PATH_FP64_QADIC, flags=qmm.BOUND_EQ4)
    assert (pl.t, pl.d, pl.k_block, pl.regime) == (9, 4, 64, qmm.REGIME_OFFSET)
    pl = qmm.choose_Qd(3, 64, 64, 64, path=qmm.PATH_FP64_QADIC)
    assert (pl.t, pl.d, pl.k_block, pl.regime) == (9, 5, 64, qmm.REGIME_OFFSET)
    # square, unblocked: t = 18, d = 1, exact regime (S_max < 2^53)
    pl = qmm.choose_Qd(7, 4096, 4096, 4096, path=qmm.PATH_FP64_QADIC, flags=qmm.PLAN_UNBLOCKED | qmm.BOUND_EQ4)
    assert (pl.t, pl.d, pl.regime) == (18, 1, qmm.REGIME_EXACT)
    # large, p = 101: unblocked only d = 0; blocked d = 1
    pl = qmm.choose_Qd(101, 8192, 8192, 8192, path=qmm.PATH_FP64_QADIC, flags=qmm.PLAN_UNBLOCKED | qmm.BOUND_EQ4)
    assert (pl.t, pl.d) == (27, 0)
    pl = qmm.choose_Qd(101, 8192, 8192, 8192, path=qmm.PATH_FP64_QADIC)
    assert pl.d == 1 and pl.k_block < 8192
    # graph: unblocked t = 17, d = 2
    pl = qmm.choose_Qd(3, 16384, 16384, 16384, path=qmm.PATH_FP64_QADIC, flags=qmm.PLAN_UNBLOCKED | qmm.BOUND_EQ4)
    assert (pl.t, pl.d, pl.regime) == (17, 2, qmm.REGIME_OFFSET)
    # no blocking needed at these sizes; AUTO picks FP4 where every centred residue is
    # an e2m1 value (p <= 8 on this path) and INT8 for other byte residues
    for p, k in ((7, 4096), (101, 8192), (3, 16384)):
        pl = qmm.choose_Qd(p, k, k, k)
        assert pl.path == (qmm.PATH_FP4 if p <= 8 else qmm.PATH_INT8) and pl.k_block == k
    for p in range(2, 257):
        want = qmm.PATH_FP4 if p <= 8 else qmm.PATH_INT8
        assert qmm.choose_Qd(p, 1024, 1024, 512).path == want, p       # 2^29 multiply-adds
        assert qmm.choose_Qd(p, 1024, 1024, 256).path == qmm.PATH_INT8, p  # 2^28: INT8's one launch wins
        assert qmm.choose_Qd(p, 64, 64, 64).path == qmm.PATH_INT8, p   # too small to repay a launch
        assert p > 8 or bounds.fp4_representable(p)


def test_redq_plans():
    pl = qmm.choose_Qd(7, 4096, 4096, 4096, path=qmm.PATH_FP64_REDQ)
    assert (pl.t, pl.d) == (18, 1)
    assert bounds.redq_ok(7, 4096, pl.t, pl.d, 53)
    pl = qmm.choose_Qd(3, 64, 64, 64, path=qmm.PATH_FP64_REDQ)
    assert bounds.redq_ok(3, 64, pl.t, pl.d, 53) and not bounds.redq_ok(3, 64, pl.t, pl.d + 1, 53)
    pl = qmm.choose_Qd(3, 64, 64, 300, path=qmm.PATH_FP32_REDQ)
    assert bounds.redq_ok(3, 300, pl.t, pl.d, 24)
    pl = qmm.choose_Qd(3, 64, 2, 64, path=qmm.PATH_FP64_REDQ)
    assert pl.d == 1                           # never more residues per word than columns


def test_fp4_blocks():
    for p in (2, 3, 5, 7, 8):
        k = 10 ** 8                                # past the bound for every p
        pl = qmm.choose_Qd(p, 4, 4, k, path=qmm.PATH_FP4)
        assert pl.k_block < k
        assert pl.path == qmm.PATH_FP4 and pl.beta == 24 and pl.regime == qmm.REGIME_INT
        assert bounds.fp4_block_ok(p, pl.k_block) and pl.k_block % 256 == 0
        assert not bounds.fp4_block_ok(p, pl.k_block + 256)      # the largest whole-stage block
        assert qmm.validate_plan(pl, 4, 4, k) == qmm.OK
        big = qmm.Plan.from_buffer_copy(pl)
        big.k_block += 256
        assert qmm.validate_plan(big, 4, 4, k) == qmm.EBOUND
    assert qmm.choose_Qd(7, 4, 4, 1000, path=qmm.PATH_FP4).k_block == 1000
    for p in (9, 11, 101):
        st, _ = qmm.try_choose_Qd(p, 4, 4, 16, path=qmm.PATH_FP4)
        assert st == qmm.EVALUE


def test_int8_blocks():
    for p in (2, 101, 251, 256):
        k = 10 ** 6
        pl = qmm.choose_Qd(p, 4, 4, k, path=qmm.PATH_INT8)
        h = p // 2
        assert pl.k_block * h * h + (p - 1) <= 2 ** 31 - 1
        if pl.k_block < k:
            assert pl.k_block % 128 == 0 and (pl.k_block + 128) * h * h + (p - 1) > 2 ** 31 - 1


# --- left and full compression, and the choice of the compressed dimension ----
@pytest.mark.parametrize("beta,path", [(53, qmm.PATH_FP64_LEFT), (24, qmm.PATH_FP32_LEFT)])
@pytest.mark.parametrize("p,m,k", [(3, 64, 64), (3, 5, 64), (7, 4096, 4096), (101, 100, 1000), (2, 1, 7),
                                   (13, 9, 1)])
def test_left_plans(beta, path, p, m, k):
    st, pl = qmm.try_choose_Qd(p, m, 16, k, path=path)
    t = bounds.smallest_t(p, k)
    if t >= beta:
        assert st == qmm.EBOUND
        return
    assert st == qmm.OK and pl.path == path and pl.beta == beta and pl.d2 == 0
    assert pl.t == t and bounds.left_ok(p, k, pl.t, pl.d, beta)
    # the largest d the bounds allow, unless m itself is smaller
    assert pl.d + 1 == m or not bounds.left_ok(p, k, pl.t, pl.d + 1, beta)
    assert qmm.validate_plan(pl, m, 16, k) == qmm.OK


def best_full_pair(p, m, n, k, t, beta):
    best = None
    for eq_ in range(1, min(m, beta) + 1):
        for eth in range(1, min(n, beta) + 1):
            if not bounds.full_ok(p, k, t, eq_ - 1, eth - 1, beta):
                continue
            key = (bounds.table2_word_products("full", m, n, k, eq_ - 1, eth - 1), eq_ * eth, abs(eq_ - eth))
            if best is None or key < best[0]:
                best = (key, (eq_ - 1, eth - 1))
    return best


@pytest.mark.parametrize("beta,path", [(53, qmm.PATH_FP64_FULL), (24, qmm.PATH_FP32_FULL)])
@pytest.mark.parametrize("p,m,n,k", [(3, 64, 64, 64), (2, 1000, 1000, 5), (3, 6, 6, 4), (7, 300, 7, 9),
                                     (5, 1, 1, 3), (3, 8192, 8192, 256), (101, 64, 64, 64)])
def test_full_plans_are_valid_and_optimal(beta, path, p, m, n, k):
    st, pl = qmm.try_choose_Qd(p, m, n, k, path=path)
    t = bounds.smallest_t(p, k)
    if t >= beta:
        assert st == qmm.EBOUND
        return
    assert st == qmm.OK and pl.t == t
    assert bounds.full_ok(p, k, pl.t, pl.d, pl.d2, beta)
    key = (bounds.table2_word_products("full", m, n, k, pl.d, pl.d2), (pl.d + 1) * (pl.d2 + 1), abs(pl.d - pl.d2))
    assert key == best_full_pair(p, m, n, k, t, beta)[0]
    assert qmm.validate_plan(pl, m, n, k) == qmm.OK


def table2_count(pl, m, n, k):
    algo = {qmm.PATH_FP64_QADIC: "qadic", qmm.PATH_FP64_REDQ: "right", qmm.PATH_FP64_LEFT: "left",
            qmm.PATH_FP64_FULL: "full"}[pl.path]
    c = bounds.table2_word_products(algo, m, n, k, pl.d, pl.d2)
    if algo == "qadic":
        c += m * n * (-(-k // pl.k_block) - 1) * BLOCK_COST
    return c


@pytest.mark.parametrize("p,m,n,k,want", [
    (3, 8, 8, 4096, qmm.PATH_FP64_QADIC),     # k largest: procedure (2)
    (3, 8, 4096, 2, qmm.PATH_FP64_REDQ),      # n largest: procedure (5)
    (3, 4096, 8, 2, qmm.PATH_FP64_LEFT),      # m largest: left compression
    (3, 8, 4096, 8, qmm.PATH_FP64_QADIC),     # all of k fits one word: a tie, which goes to k
    (3, 6, 6, 4, qmm.PATH_FP64_FULL),         # full compression wins on the rounding of m/2, n/2
    (7, 512, 512, 512, None), (101, 200, 3000, 100, None), (2, 33, 65, 129, None), (3, 4096, 4096, 8, None)])
def test_any_compression_picks_the_fewest_word_products(p, m, n, k, want):
    pl = qmm.choose_Qd(p, m, n, k, path=qmm.PATH_FP64_QADIC, flags=qmm.PLAN_ANY_COMPRESSION)
    if want is not None:
        assert pl.path == want
    assert qmm.validate_plan(pl, m, n, k) == qmm.OK
    got = table2_count(pl, m, n, k)
    # every alternative, planned by the library for its own path
    for path in (qmm.PATH_FP64_QADIC, qmm.PATH_FP64_REDQ, qmm.PATH_FP64_LEFT, qmm.PATH_FP64_FULL):
        st, alt = qmm.try_choose_Qd(p, m, n, k, path=path)
        if st == qmm.OK:
            assert got <= table2_count(alt, m, n, k)
    # and the oracle's own degrees for the three exact compressions
    t = bounds.smallest_t(p, k)
    for algo, dim in (("right", n), ("left", m)):
        d = max(d for d in range(0, 53) if bounds.redq_ok(p, k, t, d, 53) or d == 0)
        d = min(d, dim - 1)
        assert got <= bounds.table2_word_products(algo, m, n, k, d)
    bf = best_full_pair(p, m, n, k, t, 53)
    if bf is not None:
        assert got <= bf[0][0]
