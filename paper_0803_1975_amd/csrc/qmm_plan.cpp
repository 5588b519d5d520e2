// Choice of Q = 2^t, d and the k-block from p, the sizes and the mantissa
// (sections 1, 2.4, 2.5 and 5 of the paper), with exact integer arithmetic.
//
// Q-adic paths (procedure (2)).  A plan (t, d, kb) is accepted in one of two
// regimes; both make the floating-point accumulation deliver the exact digit:
//   EXACT : eq. (3) kb (p-1)^2 < Q, and S_max < 2^beta where S_max is the largest
//           accumulated sum over ceil(kb/(d+1)) chunk products.  No rounding occurs.
//   OFFSET: the paper's Q^(2d+1) addition (section 2.5) moved into the start value
//           of the accumulator, M = 2^(beta-1) Q^d, so every partial sum sits in
//           [M, 2M) where floats are spaced exactly Q^d apart.  Needs eq. (3); the
//           sum form of eq. (4) with one bit less (largest high part < 2^(beta-1));
//           and g * (largest low part of one chunk product) < Q^d / 2, so that each
//           rounding (one fused multiply-add per product on the matrix cores, g = 1)
//           drops the low part.  The word then holds M + floor(S/Q^d) Q^d.
// Among accepted plans the planner minimises the packed words per output plus a
// per-block extraction cost; k is split into blocks (each a whole number of
// K-tiles of words) when a smaller block admits a larger d.
#include <cstring>
#include <string>

#include "qmm_internal.h"

namespace qmm {

namespace {
thread_local std::string g_last_error;

using u128 = unsigned __int128;
constexpr u128 kHuge = ~(u128)0 >> 1;

u128 sat_mul(u128 a, u128 b) {
    if (a == 0 || b == 0) return 0;
    if (a > kHuge / b) return kHuge;
    return a * b;
}
u128 sat_add(u128 a, u128 b) { return (a > kHuge - b) ? kHuge : a + b; }
u128 pow2(uint32_t e) { return e >= 126 ? kHuge : ((u128)1 << e); }

// Largest value of coefficient j of a sum of N products of two degree-d chunk
// polynomials with entries in [0, p-1].
u128 coeff_max(uint64_t p, int64_t N, uint32_t d, uint32_t j) {
    const uint64_t pairs = (j <= d) ? j + 1 : 2 * d + 1 - j;
    return sat_mul(sat_mul((u128)N, (u128)(p - 1) * (p - 1)), pairs);
}

u128 s_max(uint64_t p, int64_t kb, uint32_t t, uint32_t d) {
    const int64_t N = ceil_div(kb, d + 1);
    u128 s = 0;
    for (uint32_t j = 0; j <= 2 * d; ++j) s = sat_add(s, sat_mul(coeff_max(p, N, d, j), pow2(t * j)));
    return s;
}

u128 high_max(uint64_t p, int64_t kb, uint32_t t, uint32_t d) {
    const int64_t N = ceil_div(kb, d + 1);
    u128 s = 0;
    for (uint32_t j = d; j <= 2 * d; ++j) s = sat_add(s, sat_mul(coeff_max(p, N, d, j), pow2(t * (j - d))));
    return s;
}

// Largest packed word (p-1)(1 + Q + ... + Q^d); it must be an exact float.
u128 word_max(uint64_t p, uint32_t t, uint32_t d) {
    u128 s = 0;
    for (uint32_t j = 0; j <= d; ++j) s = sat_add(s, pow2(t * j));
    return sat_mul(s, (u128)(p - 1));
}

u128 low_max(uint64_t p, uint32_t t, uint32_t d) {
    u128 s = 0;
    for (uint32_t j = 0; j < d; ++j)
        s = sat_add(s, sat_mul((u128)(j + 1) * (p - 1) * (p - 1), pow2(t * j)));
    return s;
}

bool eq3_ok(uint64_t p, int64_t kb, uint32_t t) {
    return sat_mul((u128)kb, (u128)(p - 1) * (p - 1)) < pow2(t);
}

// Regime of a Q-adic plan, or -1.
int qadic_regime(uint64_t p, int64_t kb, uint32_t t, uint32_t d, uint32_t beta, uint32_t g) {
    if (t < 1 || kb < 1 || !eq3_ok(p, kb, t)) return -1;
    if (word_max(p, t, d) >= pow2(beta)) return -1;
    if (s_max(p, kb, t, d) < pow2(beta)) return QMM_REGIME_EXACT;
    if (high_max(p, kb, t, d) < pow2(beta - 1) && sat_mul(2 * (u128)g, low_max(p, t, d)) < pow2(t * d))
        return QMM_REGIME_OFFSET;
    return -1;
}

uint32_t default_beta(uint32_t path) {
    if (path_is_fp64(path)) return 53;
    if (path_is_fp32(path)) return 24;
    return 31;
}

void base_plan(qmm_plan *pl, uint32_t p, uint32_t path) {
    std::memset(pl, 0, sizeof(*pl));
    pl->p = p;
    pl->path = path;
    pl->g = 1;
}

qmm_status choose_qadic(uint32_t p, int64_t k, uint32_t beta, uint32_t path, uint32_t flags,
                        qmm_plan *out) {
    const uint32_t g = (flags & QMM_BOUND_G4) ? 4 : 1;
    const u128 pm = (u128)(p - 1) * (p - 1);
    bool found = false;
    int64_t best_cost = 0, best_blocks = 0;
    qmm_plan best;
    base_plan(&best, p, path);
    for (uint32_t t = 1; t + 1 <= beta; ++t) {
        const u128 lim = pow2(t) - 1;  // kb (p-1)^2 <= 2^t - 1
        const u128 kbmax128 = pm ? lim / pm : lim;
        const int64_t kbmax = kbmax128 > (u128)INT64_MAX ? INT64_MAX : (int64_t)kbmax128;
        if (kbmax < 1) continue;
        const int64_t dmax = (int64_t)beta / t;  // t d > beta leaves no exact word
        for (int64_t d = dmax; d >= 0; --d) {
            int64_t kb;
            if (k <= kbmax) {
                kb = k;
            } else {
                if (flags & QMM_PLAN_UNBLOCKED) continue;
                const int64_t unit = (d + 1) * kQadicKT;
                kb = (kbmax / unit) * unit;
                if (kb < 1) continue;
            }
            if (d > 0 && d + 1 > kb) continue;  // more slots than residues: a smaller d does as well
            if ((flags & QMM_BOUND_EQ4) && (int64_t)t * (d + 1) >= (int64_t)beta) continue;
            const int reg = qadic_regime(p, kb, t, (uint32_t)d, beta, g);
            if (reg < 0) continue;
            const int64_t blocks = ceil_div(k, kb);
            const int64_t cost = ceil_div(k, d + 1) + (blocks - 1) * kBlockCostWords;
            const bool better = !found || cost < best_cost ||
                                (cost == best_cost && blocks < best_blocks) ||
                                (cost == best_cost && blocks == best_blocks &&
                                 reg == QMM_REGIME_EXACT && best.regime != QMM_REGIME_EXACT);
            if (better) {
                found = true;
                best_cost = cost;
                best_blocks = blocks;
                best.t = t;
                best.d = (uint32_t)d;
                best.beta = beta;
                best.k_block = kb;
                best.regime = (uint32_t)reg;
                best.g = g;
            }
        }
    }
    if (!found) return fail(QMM_EBOUND, "no (Q, d, k_block) satisfies the bounds for this p, k and mantissa");
    *out = best;
    return QMM_OK;
}

qmm_status choose_redq(uint32_t p, int64_t n, int64_t k, uint32_t beta, uint32_t path, qmm_plan *out) {
    base_plan(out, p, path);
    uint32_t t = 1;
    while (t + 1 <= beta && !eq3_ok(p, k, t)) ++t;
    if (!eq3_ok(p, k, t) || t > beta - 1)
        return fail(QMM_EBOUND, "REDQ path: k (p-1)^2 must stay below 2^(beta-1)");
    int64_t d = (int64_t)(beta - 1) / t - 1;  // t(d+1) < beta (eq. (4))
    if (n >= 1 && d > n - 1) d = n - 1;
    if (d < 0) d = 0;
    out->t = t;
    out->d = (uint32_t)d;
    out->beta = beta;
    out->k_block = k;
    out->regime = QMM_REGIME_EXACT;
    return QMM_OK;
}

// Left compression (Table 2): the words of section 3 along m, so the same bounds:
// eq. (3) over the whole k and t(d+1) < beta (eq. (4)); d+1 <= m.
qmm_status choose_left(uint32_t p, int64_t m, int64_t k, uint32_t beta, uint32_t path, qmm_plan *out) {
    const qmm_status st = choose_redq(p, m, k, beta, path, out);
    if (st != QMM_OK) return fail(st, "left compression: k (p-1)^2 must stay below 2^(beta-1)");
    return QMM_OK;
}

// Full compression (section 4): eq. (3) fixes t; Theta = Q^(d+1) (eq. (6) with
// equality) and eq. (7), t (d+1)(d2+1) < beta, bound the two degrees.  Among the
// admissible pairs the plan takes the one with the fewest packed-word products,
// ceil(m/(d+1)) ceil(n/(d2+1)) per unit of k; ties go to fewer digits per word,
// then to the more balanced pair (the paper's d = sqrt(e) - 1 for equal degrees).
qmm_status choose_full(uint32_t p, int64_t m, int64_t n, int64_t k, uint32_t beta, uint32_t path,
                       qmm_plan *out) {
    base_plan(out, p, path);
    uint32_t t = 1;
    while (t + 1 <= beta && !eq3_ok(p, k, t)) ++t;
    if (!eq3_ok(p, k, t) || t > beta - 1)
        return fail(QMM_EBOUND, "full compression: k (p-1)^2 must stay below 2^(beta-1)");
    const int64_t D = (int64_t)(beta - 1) / t;  // digits per word, eq. (7)
    const int64_t mm = m < 1 ? 1 : m, nn = n < 1 ? 1 : n;
    bool found = false;
    u128 best_cost = 0;
    int64_t best_q = 0, best_th = 0;
    for (int64_t eq_ = 1; eq_ <= D && eq_ <= mm; ++eq_) {
        for (int64_t eth = 1; eq_ * eth <= D && eth <= nn; ++eth) {
            const u128 cost = (u128)ceil_div(mm, eq_) * (u128)ceil_div(nn, eth);
            const int64_t digits = eq_ * eth, bdigits = best_q * best_th;
            const int64_t skew = eq_ > eth ? eq_ - eth : eth - eq_;
            const int64_t bskew = best_q > best_th ? best_q - best_th : best_th - best_q;
            const bool better = !found || cost < best_cost || (cost == best_cost && digits < bdigits) ||
                                (cost == best_cost && digits == bdigits && skew < bskew);
            if (better) {
                found = true;
                best_cost = cost;
                best_q = eq_;
                best_th = eth;
            }
        }
    }
    out->t = t;
    out->d = (uint32_t)(best_q - 1);
    out->d2 = (uint32_t)(best_th - 1);
    out->beta = beta;
    out->k_block = k;
    out->regime = QMM_REGIME_EXACT;
    return QMM_OK;
}

// Multiply-adds of packed words of a plan for an m x k by k x n product (Table 2,
// classical product), plus the planner's per-block extraction cost for blocked
// k-compressed plans.
u128 plan_work(const qmm_plan &pl, int64_t m, int64_t n, int64_t k) {
    const u128 M = (u128)(m < 1 ? 1 : m), N = (u128)(n < 1 ? 1 : n), K = (u128)(k < 1 ? 1 : k);
    if (path_is_qadic(pl.path)) {
        const int64_t blocks = ceil_div(k < 1 ? 1 : k, pl.k_block);
        return M * N * (u128)(ceil_div(k < 1 ? 1 : k, pl.d + 1) + (blocks - 1) * kBlockCostWords);
    }
    if (path_is_redq(pl.path)) return M * (u128)ceil_div((int64_t)N, pl.d + 1) * K;
    if (path_is_left(pl.path)) return (u128)ceil_div((int64_t)M, pl.d + 1) * N * K;
    return (u128)ceil_div((int64_t)M, pl.d + 1) * (u128)ceil_div((int64_t)N, pl.d2 + 1) * K;
}

qmm_status choose_int8(uint32_t p, int64_t k, qmm_plan *out) {
    base_plan(out, p, QMM_PATH_INT8);
    if (p > 256) return fail(QMM_EVALUE, "INT8 path needs p <= 256");
    const int64_t h = p / 2;  // largest |centred residue|
    // A block starts from the previous block's residue (< p) and adds kb products.
    const int64_t lim = (((int64_t)1 << 31) - 1 - (int64_t)(p - 1)) / (h * h);
    int64_t kb = k;
    if (k > lim) kb = (lim / kInt8KT) * kInt8KT;
    out->beta = 31;
    out->k_block = kb < 1 ? 1 : kb;
    out->regime = QMM_REGIME_INT;
    return QMM_OK;
}

// FP4: centred residues are exact e2m1 values for p <= 8 (|x| <= 4); a block
// starts from the previous block's residue (< p) and adds kb products of at most
// floor(p/2)^2 each, and every partial sum must stay an integer the FP32
// accumulator holds exactly (|s| <= 2^24).  Blocks are whole 256-value K stages.
qmm_status choose_fp4(uint32_t p, int64_t k, qmm_plan *out) {
    base_plan(out, p, QMM_PATH_FP4);
    if (p > 8) return fail(QMM_EVALUE, "FP4 path needs p <= 8");
    const int64_t h = p / 2;
    const int64_t lim = (((int64_t)1 << 24) - (int64_t)(p - 1)) / (h * h);
    int64_t kb = k;
    if (k > lim) kb = (lim / kFp4KB) * kFp4KB;
    out->beta = 24;
    out->k_block = kb < 1 ? 1 : kb;
    out->regime = QMM_REGIME_INT;
    return QMM_OK;
}

}  // namespace

void set_error(const std::string &msg) { g_last_error = msg; }
qmm_status fail(qmm_status st, const std::string &msg) {
    g_last_error = msg;
    return st;
}

bool words_exact(const qmm_plan &pl) {
    if (pl.p < 2 || pl.t < 1 || pl.t > 63 || pl.d > 63 || (uint64_t)pl.t * (pl.d + 1) > 64) return false;
    return word_max(pl.p, pl.t, pl.d) < pow2(pl.beta);
}

bool path_is_fp64(uint32_t path) {
    return path == QMM_PATH_FP64_QADIC || path == QMM_PATH_FP64_REDQ || path == QMM_PATH_FP64_LEFT ||
           path == QMM_PATH_FP64_FULL;
}
bool path_is_fp32(uint32_t path) {
    return path == QMM_PATH_FP32_QADIC || path == QMM_PATH_FP32_REDQ || path == QMM_PATH_FP32_LEFT ||
           path == QMM_PATH_FP32_FULL;
}
bool path_is_left(uint32_t path) { return path == QMM_PATH_FP64_LEFT || path == QMM_PATH_FP32_LEFT; }
bool path_is_full(uint32_t path) { return path == QMM_PATH_FP64_FULL || path == QMM_PATH_FP32_FULL; }
qmm_plan theta_plan(const qmm_plan &pl) {
    qmm_plan q = pl;
    q.t = pl.t * (pl.d + 1);
    q.d = pl.d2;
    q.d2 = 0;
    return q;
}
bool path_is_qadic(uint32_t path) { return path == QMM_PATH_FP64_QADIC || path == QMM_PATH_FP32_QADIC; }
bool path_is_redq(uint32_t path) { return path == QMM_PATH_FP64_REDQ || path == QMM_PATH_FP32_REDQ; }
int word_bytes(const qmm_plan &pl) { return pl.beta == 24 ? 4 : 8; }

}  // namespace qmm

using namespace qmm;

extern "C" const char *qmm_last_error(void) { return g_last_error.c_str(); }
extern "C" const char *qmm_version(void) { return "0.1.0"; }

extern "C" qmm_status qmm_choose_Qd(uint32_t p, int64_t m, int64_t n, int64_t k, uint32_t beta,
                                    qmm_path path, uint32_t flags, qmm_plan *out) {
    if (!out) return fail(QMM_EINVAL, "out is NULL");
    if (p < 2) return fail(QMM_EINVAL, "p must be >= 2");
    if (m < 0 || n < 0 || k < 0) return fail(QMM_EINVAL, "negative size");
    const int64_t kk = k < 1 ? 1 : k;
    uint32_t pth = (uint32_t)path;
    // Automatic choice: FP4 matrix cores (twice the INT8 rate, half the operand bytes)
    // when every centred residue is an e2m1 value and the product is large enough to
    // repay FP4's conversion launch against INT8's one-launch kernel (measured
    // crossover between 640^3 and 768^3 multiply-adds), INT8 for other byte residues.
    if (pth == QMM_PATH_AUTO) {
        const bool fp4 = p <= 8 && (double)m * (double)n * (double)kk >= 3.8e8;
        pth = fp4 ? QMM_PATH_FP4 : (p <= 256 ? QMM_PATH_INT8 : QMM_PATH_FP64_QADIC);
    }
    if (pth > QMM_PATH_FP32_FULL) return fail(QMM_EINVAL, "unknown path");
    if (beta == 0) beta = default_beta(pth);
    if (pth != QMM_PATH_INT8 && pth != QMM_PATH_FP4 && ((path_is_fp64(pth) && beta != 53) || (path_is_fp32(pth) && beta != 24)) &&
        !(flags & QMM_BOUND_PAPER))
        return fail(QMM_EINVAL, "beta must match the path (53 for FP64, 24 for FP32)");
    if (flags & QMM_BOUND_PAPER) {
        // The paper's rule, for reference: smallest t with k (p-1)^2 < 2^t (eq. (3)),
        // e = floor(beta / t), d = min(e, k) - 1 (section 5).
        base_plan(out, p, pth);
        uint32_t t = 1;
        while (t < 127 && !eq3_ok(p, kk, t)) ++t;
        const int64_t e = beta / t;
        const int64_t d = (e < kk ? e : kk) - 1;
        out->t = t;
        out->d = d < 0 ? 0 : (uint32_t)d;
        out->beta = beta;
        out->k_block = kk;
        out->regime = QMM_REGIME_PAPER;
        return (e >= 1) ? QMM_OK : fail(QMM_EBOUND, "no d >= 0 under the paper's rule");
    }
    if (pth == QMM_PATH_INT8) return choose_int8(p, kk, out);
    if (pth == QMM_PATH_FP4) return choose_fp4(p, kk, out);
    if (flags & QMM_PLAN_ANY_COMPRESSION) {
        // The four compressions of this mantissa; the fewest packed-word products wins
        // (Table 2: compressing the largest dimension, up to the rounding of each count).
        const bool fp64 = path_is_fp64(pth);
        const uint32_t cands[4] = {fp64 ? (uint32_t)QMM_PATH_FP64_QADIC : (uint32_t)QMM_PATH_FP32_QADIC,
                                   fp64 ? (uint32_t)QMM_PATH_FP64_REDQ : (uint32_t)QMM_PATH_FP32_REDQ,
                                   fp64 ? (uint32_t)QMM_PATH_FP64_LEFT : (uint32_t)QMM_PATH_FP32_LEFT,
                                   fp64 ? (uint32_t)QMM_PATH_FP64_FULL : (uint32_t)QMM_PATH_FP32_FULL};
        bool found = false;
        u128 best_work = 0;
        qmm_plan best{};
        for (uint32_t c : cands) {
            qmm_plan pl;
            qmm_status st;
            if (path_is_qadic(c)) st = choose_qadic(p, kk, beta, c, flags & ~QMM_PLAN_ANY_COMPRESSION, &pl);
            else if (path_is_redq(c)) st = choose_redq(p, n, kk, beta, c, &pl);
            else if (path_is_left(c)) st = choose_left(p, m, kk, beta, c, &pl);
            else st = choose_full(p, m, n, kk, beta, c, &pl);
            if (st != QMM_OK) continue;
            const u128 w = plan_work(pl, m, n, kk);
            if (!found || w < best_work) {
                found = true;
                best_work = w;
                best = pl;
            }
        }
        if (!found) return fail(QMM_EBOUND, "no compression satisfies the bounds for this p, k and mantissa");
        *out = best;
        return QMM_OK;
    }
    if (path_is_redq(pth)) return choose_redq(p, n, kk, beta, pth, out);
    if (path_is_left(pth)) return choose_left(p, m, kk, beta, pth, out);
    if (path_is_full(pth)) return choose_full(p, m, n, kk, beta, pth, out);
    return choose_qadic(p, kk, beta, pth, flags, out);
}

extern "C" qmm_status qmm_validate_plan(const qmm_plan *pl, int64_t m, int64_t n, int64_t k) {
    if (!pl) return fail(QMM_EINVAL, "plan is NULL");
    if (m < 0 || n < 0 || k < 0) return fail(QMM_EINVAL, "negative size");
    if (pl->p < 2) return fail(QMM_EINVAL, "p must be >= 2");
    const int64_t kk = k < 1 ? 1 : k;
    if (pl->d2 != 0 && !path_is_full(pl->path)) return fail(QMM_EINVAL, "d2 must be 0 off the FULL paths");
    switch (pl->path) {
    case QMM_PATH_INT8: {
        if (pl->p > 256) return fail(QMM_EVALUE, "INT8 path needs p <= 256");
        const int64_t h = pl->p / 2;
        const int64_t kb = pl->k_block;
        if (kb < 1) return fail(QMM_EBOUND, "k_block < 1");
        if (kb < kk && kb % kInt8KT) return fail(QMM_EBOUND, "INT8 k_block must be a multiple of 128");
        if (pl->tile > 4) return fail(QMM_EINVAL, "INT8 tile must be 0 (auto) or 1..4");
        if ((__int128)kb * h * h + (pl->p - 1) > (((__int128)1 << 31) - 1))
            return fail(QMM_EBOUND, "INT8 k_block overflows int32");
        return QMM_OK;
    }
    case QMM_PATH_FP4: {
        if (pl->p > 8) return fail(QMM_EVALUE, "FP4 path needs p <= 8");
        const int64_t h = pl->p / 2;
        const int64_t kb = pl->k_block;
        if (kb < 1) return fail(QMM_EBOUND, "k_block < 1");
        if (kb < kk && kb % kFp4KB) return fail(QMM_EBOUND, "FP4 k_block must be a multiple of 256");
        if (pl->tile > 3) return fail(QMM_EINVAL, "FP4 tile must be 0 (auto) or 1..3");
        if ((__int128)kb * h * h + (pl->p - 1) > ((__int128)1 << 24))
            return fail(QMM_EBOUND, "FP4 k_block leaves the exact FP32 integers");
        return QMM_OK;
    }
    case QMM_PATH_FP64_QADIC:
    case QMM_PATH_FP32_QADIC: {
        const uint32_t beta = path_is_fp64(pl->path) ? 53 : 24;
        if (pl->beta != beta) return fail(QMM_EBOUND, "plan beta does not match the path");
        if (pl->t < 1 || pl->t > 63 || pl->d > 63) return fail(QMM_EBOUND, "t or d out of range");
        const int64_t kb = pl->k_block;
        if (kb < 1) return fail(QMM_EBOUND, "k_block < 1");
        if (kb < kk && kb % (((int64_t)pl->d + 1) * kQadicKT))
            return fail(QMM_EBOUND, "k_block must be a multiple of (d+1) * 16 when k is blocked");
        const int64_t kb_eff = kb < kk ? kb : kk;
        const uint32_t g = pl->g < 1 ? 1 : pl->g;
        const int reg = qadic_regime(pl->p, kb_eff, pl->t, pl->d, beta, g);
        if (reg < 0) return fail(QMM_EBOUND, "plan violates the bounds (eq. (3), eq. (4) sum form or the rounding condition)");
        if (pl->regime == QMM_REGIME_EXACT && reg != QMM_REGIME_EXACT)
            return fail(QMM_EBOUND, "plan claims the exact regime but S_max >= 2^beta");
        if (pl->regime != QMM_REGIME_EXACT && pl->regime != QMM_REGIME_OFFSET)
            return fail(QMM_EBOUND, "plan regime is not executable");
        if (pl->regime == QMM_REGIME_OFFSET && pl->t > 32)
            return fail(QMM_EBOUND, "offset regime reads digit d from 32 mantissa bits: t must be <= 32");
        if (pl->regime == QMM_REGIME_OFFSET &&
            !(high_max(pl->p, kb_eff, pl->t, pl->d) < pow2(beta - 1) &&
              sat_mul(2 * (u128)g, low_max(pl->p, pl->t, pl->d)) < pow2(pl->t * pl->d)))
            return fail(QMM_EBOUND, "plan violates the offset-regime conditions");
        return QMM_OK;
    }
    case QMM_PATH_FP64_REDQ:
    case QMM_PATH_FP32_REDQ: {
        const uint32_t beta = path_is_fp64(pl->path) ? 53 : 24;
        if (pl->beta != beta) return fail(QMM_EBOUND, "plan beta does not match the path");
        if (pl->t < 1 || !eq3_ok(pl->p, kk, pl->t)) return fail(QMM_EBOUND, "eq. (3) violated: k (p-1)^2 >= Q");
        if ((uint64_t)pl->t * (pl->d + 1) >= beta) return fail(QMM_EBOUND, "eq. (4) violated: Q^(d+1) >= 2^beta");
        if (pl->k_block < kk) return fail(QMM_EUNSUPPORTED, "the REDQ path does not split k");
        if (pl->regime != QMM_REGIME_EXACT) return fail(QMM_EBOUND, "REDQ plans are exact");
        return QMM_OK;
    }
    case QMM_PATH_FP64_LEFT:
    case QMM_PATH_FP32_LEFT: {
        const uint32_t beta = path_is_fp64(pl->path) ? 53 : 24;
        if (pl->beta != beta) return fail(QMM_EBOUND, "plan beta does not match the path");
        if (pl->t < 1 || !eq3_ok(pl->p, kk, pl->t)) return fail(QMM_EBOUND, "eq. (3) violated: k (p-1)^2 >= Q");
        if ((uint64_t)pl->t * (pl->d + 1) >= beta) return fail(QMM_EBOUND, "eq. (4) violated: Q^(d+1) >= 2^beta");
        if (pl->k_block < kk) return fail(QMM_EUNSUPPORTED, "left compression does not split k");
        if (pl->regime != QMM_REGIME_EXACT) return fail(QMM_EBOUND, "left-compression plans are exact");
        return QMM_OK;
    }
    case QMM_PATH_FP64_FULL:
    case QMM_PATH_FP32_FULL: {
        const uint32_t beta = path_is_fp64(pl->path) ? 53 : 24;
        if (pl->beta != beta) return fail(QMM_EBOUND, "plan beta does not match the path");
        if (pl->t < 1 || !eq3_ok(pl->p, kk, pl->t)) return fail(QMM_EBOUND, "eq. (3) violated: k (p-1)^2 >= Q");
        if (pl->d > 63 || pl->d2 > 63 ||
            (uint64_t)pl->t * (pl->d + 1) * (pl->d2 + 1) >= beta)
            return fail(QMM_EBOUND, "eq. (7) violated: Q^((d+1)(d2+1)) >= 2^beta");
        if (pl->k_block < kk) return fail(QMM_EUNSUPPORTED, "full compression does not split k");
        if (pl->regime != QMM_REGIME_EXACT) return fail(QMM_EBOUND, "full-compression plans are exact");
        return QMM_OK;
    }
    default:
        return fail(QMM_EINVAL, "plan path must be a concrete path");
    }
}
