// The C ABI: argument checking, plan selection and validation, workspace
// layout, and the sequence of kernels for each procedure.
#include <hip/hip_runtime.h>

#include <cstring>
#include <string>

#include "qmm_internal.h"

using namespace qmm;

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

qmm_status check_plan_for_words(const qmm_plan *pl) {
    if (!pl) return fail(QMM_EINVAL, "plan is NULL");
    if (pl->p < 2) return fail(QMM_EINVAL, "plan p must be >= 2");
    if (pl->beta != 53 && pl->beta != 24) return fail(QMM_EINVAL, "packed words need beta 53 (double) or 24 (float)");
    if (!words_exact(*pl))
        return fail(QMM_EINVAL, "packed words (p-1)(1 + Q + ... + Q^d) must be exact floats of the plan's mantissa");
    return QMM_OK;
}

bool bad_matrix(int64_t rows, int64_t cols, const void *ptr, int64_t ld) {
    if (rows < 0 || cols < 0) return true;
    if (rows == 0 || cols == 0) return false;
    return ptr == nullptr || ld < cols;
}

struct Layout {
    size_t bytes = 0;
    size_t off_b = 0;  // second buffer offset
    int64_t ld_a = 0, ld_b = 0;
    size_t off_tail = 0, tail = 0;  // INT8 / FP4: partial outputs of a split-K strip
};

// Small unblocked FP64 Q-adic products run in one launch that packs in LDS.
bool fused_qadic(const qmm_plan &pl, int64_t m, int64_t n, int64_t k) {
    return path_is_qadic(pl.path) && pl.beta == 53 && pl.k_block >= k &&
           (double)m * (double)n * (double)k <= kFusedQadicMaxMacs;
}

// Small unblocked INT8 products run in one launch that centres and transposes in LDS
// (unless the plan asks for a tile of the two-kernel path).
bool small_int8(const qmm_plan &pl, int64_t m, int64_t n, int64_t k) {
    return pl.path == QMM_PATH_INT8 && pl.tile == 0 && pl.k_block >= k &&
           (double)m * (double)n * (double)k <= kSmallInt8MaxMacs;
}

Layout workspace_layout(const qmm_plan &pl, int64_t m, int64_t n, int64_t k) {
    Layout L;
    const int64_t kk = k < 1 ? 1 : k;
    if (fused_qadic(pl, m, n, k) || small_int8(pl, m, n, k)) return L;  // no packed operands in HBM
    if (path_is_qadic(pl.path)) {
        const int64_t nw = words_for(kk, pl.d);
        const size_t wb = (size_t)word_bytes(pl);
        L.ld_a = nw;
        L.ld_b = n;
        L.off_b = align_up((size_t)m * nw * wb);
        L.bytes = L.off_b + align_up((size_t)nw * n * wb);
    } else if (path_is_redq(pl.path)) {
        // CBr, then A as words (the Uncompress of procedure (5))
        const int64_t nw = words_for(n, pl.d);
        L.ld_b = nw;
        L.ld_a = kk;
        L.off_b = align_up((size_t)kk * nw * word_bytes(pl));
        L.bytes = L.off_b + align_up((size_t)m * kk * word_bytes(pl));
    } else if (path_is_left(pl.path)) {
        // CAl, then B as words
        L.ld_a = kk;
        L.ld_b = n;
        L.off_b = align_up((size_t)words_for(m, pl.d) * kk * word_bytes(pl));
        L.bytes = L.off_b + align_up((size_t)kk * n * word_bytes(pl));
    } else if (path_is_full(pl.path)) {
        L.ld_a = kk;
        L.ld_b = words_for(n, pl.d2);
        L.off_b = align_up((size_t)words_for(m, pl.d) * kk * word_bytes(pl));
        L.bytes = L.off_b + align_up((size_t)kk * L.ld_b * word_bytes(pl));
    } else if (pl.path == QMM_PATH_INT8) {
        // Bt, then (k not a multiple of 16) A centred into rows of the same length
        L.ld_b = int8_bt_ld(kk);
        L.bytes = align_up((size_t)n * L.ld_b);
        if (int8_centres_a(pl, m, n, kk)) {
            L.ld_a = L.ld_b;
            L.off_b = L.bytes;
            L.bytes += align_up((size_t)m * L.ld_a);
        }
    } else if (pl.path == QMM_PATH_FP4) {
        L.ld_a = L.ld_b = fp4_ld(kk);
        L.off_b = align_up((size_t)m * L.ld_a);
        L.bytes = L.off_b + align_up((size_t)n * L.ld_b);
    }
    if (pl.path == QMM_PATH_INT8 || pl.path == QMM_PATH_FP4) {
        L.tail = lowp_tail_bytes(pl, m, n, k);
        if (L.tail > 0) {
            L.off_tail = L.bytes;
            L.bytes += align_up(L.tail);
        }
    }
    return L;
}

qmm_plan with_degrees(const qmm_plan &pl, uint32_t d, uint32_t d2) {
    qmm_plan q = pl;
    q.d = d;
    q.d2 = d2;
    return q;
}

// The full-compression plan (degree d in Q along m, d2 along n) with pl's t and
// mantissa: the kernel of every word-times-word REDQ product.
qmm_plan full_plan_of(const qmm_plan &pl, uint32_t d, uint32_t d2) {
    qmm_plan q = with_degrees(pl, d, d2);
    q.path = pl.beta == 24 ? QMM_PATH_FP32_FULL : QMM_PATH_FP64_FULL;
    return q;
}

qmm_status resolve_plan(const qmm_plan *plan, uint32_t p, int64_t m, int64_t n, int64_t k, qmm_plan *out) {
    if (plan) {
        if (plan->p != p) return fail(QMM_EINVAL, "plan->p differs from p");
        const qmm_status st = qmm_validate_plan(plan, m, n, k);
        if (st != QMM_OK) return st;
        *out = *plan;
        return QMM_OK;
    }
    return qmm_choose_Qd(p, m, n, k, 0, QMM_PATH_AUTO, 0, out);
}

}  // namespace

extern "C" qmm_status qmm_pack_rows_rev(const qmm_plan *plan, int64_t m, int64_t k, const uint8_t *A, int64_t lda,
                                        void *CA, int64_t ldca, void *stream) {
    qmm_status st = check_plan_for_words(plan);
    if (st != QMM_OK) return st;
    if (bad_matrix(m, k, A, lda)) return fail(QMM_EINVAL, "A: bad size, pointer or lda");
    if (bad_matrix(m, words_for(k, plan->d), CA, ldca)) return fail(QMM_EINVAL, "CA: bad pointer or ldca");
    return launch_pack_rows_rev(*plan, m, k, A, lda, CA, ldca, stream);
}

extern "C" qmm_status qmm_pack_cols_fwd(const qmm_plan *plan, int64_t k, int64_t n, const uint8_t *B, int64_t ldb,
                                        void *CB, int64_t ldcb, void *stream) {
    qmm_status st = check_plan_for_words(plan);
    if (st != QMM_OK) return st;
    if (bad_matrix(k, n, B, ldb)) return fail(QMM_EINVAL, "B: bad size, pointer or ldb");
    if (bad_matrix(words_for(k, plan->d), n, CB, ldcb)) return fail(QMM_EINVAL, "CB: bad pointer or ldcb");
    return launch_pack_cols_fwd(*plan, k, n, B, ldb, CB, ldcb, stream);
}

extern "C" qmm_status qmm_pack_rows_fwd(const qmm_plan *plan, int64_t k, int64_t n, const uint8_t *B, int64_t ldb,
                                        void *CBr, int64_t ldcbr, void *stream) {
    qmm_status st = check_plan_for_words(plan);
    if (st != QMM_OK) return st;
    if (bad_matrix(k, n, B, ldb)) return fail(QMM_EINVAL, "B: bad size, pointer or ldb");
    if (bad_matrix(k, words_for(n, plan->d), CBr, ldcbr)) return fail(QMM_EINVAL, "CBr: bad pointer or ldcbr");
    return launch_pack_rows_fwd(*plan, k, n, B, ldb, CBr, ldcbr, stream);
}

extern "C" qmm_status qmm_unpack(const qmm_plan *plan, int which, int64_t rows, int64_t cols, const void *packed,
                                 int64_t ldp, uint8_t *out, int64_t ldo, void *stream) {
    qmm_status st = check_plan_for_words(plan);
    if (st != QMM_OK) return st;
    if (which < 0 || which > 2) return fail(QMM_EINVAL, "which must be 0, 1 or 2");
    if (bad_matrix(rows, cols, out, ldo)) return fail(QMM_EINVAL, "out: bad size, pointer or ldo");
    const int64_t prow = which == 1 ? words_for(rows, plan->d) : rows;
    const int64_t pcol = which == 1 ? cols : words_for(cols, plan->d);
    if (bad_matrix(prow, pcol, packed, ldp)) return fail(QMM_EINVAL, "packed: bad pointer or ldp");
    return launch_unpack(*plan, which, rows, cols, packed, ldp, out, ldo, stream);
}

extern "C" qmm_status qmm_count_nonresidues(uint32_t p, int64_t rows, int64_t cols, const uint8_t *X, int64_t ldx,
                                            uint32_t *count, void *stream) {
    if (p < 2 || p > 256) return fail(QMM_EINVAL, "p must be in [2, 256] for byte residues");
    if (bad_matrix(rows, cols, X, ldx)) return fail(QMM_EINVAL, "X: bad size, pointer or ldx");
    if (!count || (uintptr_t)count % 4 != 0) return fail(QMM_EINVAL, "count: needs a 4-byte aligned device pointer");
    return launch_count_nonresidues(p, rows, cols, X, ldx, count, stream);
}

extern "C" qmm_status qmm_extract(const qmm_plan *plan, int64_t m, int64_t n, const void *T, int64_t ldt,
                                  uint8_t *C, int64_t ldc, void *stream) {
    qmm_status st = check_plan_for_words(plan);
    if (st != QMM_OK) return st;
    if (plan->regime != QMM_REGIME_EXACT && plan->regime != QMM_REGIME_OFFSET)
        return fail(QMM_EINVAL, "extract needs an EXACT or OFFSET plan");
    if (plan->regime == QMM_REGIME_OFFSET && plan->t > 32)
        return fail(QMM_EINVAL, "offset extraction needs t <= 32");
    if (plan->p > 256) return fail(QMM_EINVAL, "byte results need p <= 256");
    if (bad_matrix(m, n, T, ldt) || bad_matrix(m, n, C, ldc)) return fail(QMM_EINVAL, "bad size, pointer or ld");
    return launch_extract(*plan, m, n, T, ldt, C, ldc, stream);
}

extern "C" qmm_status qmm_redq(const qmm_plan *plan, int64_t m, int64_t n, const void *CC, int64_t ldcc, uint8_t *C,
                               int64_t ldc, void *stream) {
    qmm_status st = check_plan_for_words(plan);
    if (st != QMM_OK) return st;
    if ((uint64_t)plan->t * (plan->d + 1) > 52) return fail(QMM_EINVAL, "REDQ words need t (d+1) <= 52");
    if (plan->p > 256) return fail(QMM_EINVAL, "byte results need p <= 256");
    if (bad_matrix(m, words_for(n, plan->d), CC, ldcc) || bad_matrix(m, n, C, ldc))
        return fail(QMM_EINVAL, "bad size, pointer or ld");
    return launch_redq(*plan, m, n, CC, ldcc, C, ldc, stream);
}

extern "C" qmm_status qmm_gemm_workspace_size(const qmm_plan *plan, int64_t m, int64_t n, int64_t k, size_t *bytes) {
    if (!bytes) return fail(QMM_EINVAL, "bytes is NULL");
    if (!plan) return fail(QMM_EINVAL, "plan is NULL (choose one with qmm_choose_Qd first)");
    if (m < 0 || n < 0 || k < 0) return fail(QMM_EINVAL, "negative size");
    *bytes = workspace_layout(*plan, m, n, k).bytes;
    return QMM_OK;
}

extern "C" qmm_status qmm_gemm_mod_p(const qmm_plan *plan, int64_t m, int64_t n, int64_t k, uint32_t p,
                                     const uint8_t *A, int64_t lda, const uint8_t *B, int64_t ldb, uint8_t *C,
                                     int64_t ldc, void *ws, size_t ws_bytes, void *stream) {
    if (p < 2 || p > 256) return fail(QMM_EINVAL, "byte residues need 2 <= p <= 256");
    if (m < 0 || n < 0 || k < 0) return fail(QMM_EINVAL, "negative size");
    if (bad_matrix(m, k, A, lda)) return fail(QMM_EINVAL, "A: bad pointer or lda");
    if (bad_matrix(k, n, B, ldb)) return fail(QMM_EINVAL, "B: bad pointer or ldb");
    if (bad_matrix(m, n, C, ldc)) return fail(QMM_EINVAL, "C: bad pointer or ldc");
    qmm_plan pl;
    qmm_status st = resolve_plan(plan, p, m, n, k, &pl);
    if (st != QMM_OK) return st;
    if (m == 0 || n == 0) return QMM_OK;
    if (k == 0) return launch_fill_u8(C, m, n, ldc, 0, stream);
    const Layout L = workspace_layout(pl, m, n, k);
    if (L.bytes > 0 && (ws == nullptr || ws_bytes < L.bytes))
        return fail(QMM_ENOSPACE, "workspace needs " + std::to_string(L.bytes) + " bytes");
    // the packed operands sit at ws and ws + off_b and are read with 16-byte loads
    if (L.bytes > 0 && (uintptr_t)ws % kAlign != 0) return fail(QMM_EINVAL, "ws must be 256-byte aligned");
    uint8_t *w = (uint8_t *)ws;
    if (fused_qadic(pl, m, n, k)) return launch_gemm_qadic_fused(pl, m, n, k, A, lda, B, ldb, C, ldc, stream);
    if (small_int8(pl, m, n, k)) return launch_gemm_int8_small(pl, m, n, k, A, lda, B, ldb, C, ldc, stream);
    if (path_is_qadic(pl.path)) {
        void *CA = w, *CB = w + L.off_b;
        if ((st = launch_pack_rows_rev(pl, m, k, A, lda, CA, L.ld_a, stream)) != QMM_OK) return st;
        if ((st = launch_pack_cols_fwd(pl, k, n, B, ldb, CB, L.ld_b, stream)) != QMM_OK) return st;
        return launch_gemm_qadic(pl, m, n, k, CA, L.ld_a, CB, L.ld_b, C, ldc, stream);
    }
    // Right and left compression convert their residue operand to words in a pass
    // of its own (procedure (5)'s Uncompress), then run the product of two word
    // matrices: converting in the product's load path measured slower.  A word of
    // one residue is the residue (degree 0), and the product is full compression
    // with one degree zero.
    if (path_is_redq(pl.path)) {
        void *CBr = w, *Aw = w + L.off_b;
        const qmm_plan one = with_degrees(pl, 0, 0), fp = full_plan_of(pl, 0, pl.d);
        if ((st = launch_pack_rows_fwd(pl, k, n, B, ldb, CBr, L.ld_b, stream)) != QMM_OK) return st;
        if ((st = launch_pack_cols_fwd(one, m, k, A, lda, Aw, L.ld_a, stream)) != QMM_OK) return st;
        return launch_gemm_full(fp, m, n, k, Aw, L.ld_a, CBr, L.ld_b, C, ldc, stream);
    }
    if (path_is_left(pl.path)) {
        void *CAl = w, *Bw = w + L.off_b;
        const qmm_plan one = with_degrees(pl, 0, 0), fp = full_plan_of(pl, pl.d, 0);
        if ((st = launch_pack_cols_fwd(pl, m, k, A, lda, CAl, L.ld_a, stream)) != QMM_OK) return st;
        if ((st = launch_pack_rows_fwd(one, k, n, B, ldb, Bw, L.ld_b, stream)) != QMM_OK) return st;
        return launch_gemm_full(fp, m, n, k, CAl, L.ld_a, Bw, L.ld_b, C, ldc, stream);
    }
    if (path_is_full(pl.path)) {
        void *CAl = w, *CBt = w + L.off_b;
        if ((st = launch_pack_cols_fwd(pl, m, k, A, lda, CAl, L.ld_a, stream)) != QMM_OK) return st;
        if ((st = launch_pack_rows_fwd(theta_plan(pl), k, n, B, ldb, CBt, L.ld_b, stream)) != QMM_OK) return st;
        return launch_gemm_full(pl, m, n, k, CAl, L.ld_a, CBt, L.ld_b, C, ldc, stream);
    }
    if (pl.path == QMM_PATH_INT8) {
        int8_t *Bt = (int8_t *)w;
        if ((st = launch_centre_transpose(pl, k, n, B, ldb, Bt, L.ld_b, stream)) != QMM_OK) return st;
        if (L.ld_a > 0) {
            // rows of A that cannot be whole 16-byte loads: centre them into aligned rows first
            int8_t *Ac = (int8_t *)(w + L.off_b);
            if ((st = launch_centre_rows(pl, m, k, A, lda, Ac, L.ld_a, stream)) != QMM_OK) return st;
            return launch_gemm_int8_centred_a(pl, m, n, k, Ac, L.ld_a, Bt, L.ld_b, C, ldc, stream, w + L.off_tail,
                                              L.tail);
        }
        return launch_gemm_int8(pl, m, n, k, A, lda, Bt, L.ld_b, C, ldc, stream, w + L.off_tail, L.tail);
    }
    if (pl.path == QMM_PATH_FP4) {
        uint8_t *A4 = w, *Bt4 = w + L.off_b;
        if ((st = launch_pack_fp4_both(pl, m, n, k, A, lda, B, ldb, A4, L.ld_a, Bt4, L.ld_b, stream)) != QMM_OK) return st;
        return launch_gemm_fp4(pl, m, n, k, A4, L.ld_a, Bt4, L.ld_b, C, ldc, stream, w + L.off_tail, L.tail);
    }
    return fail(QMM_EINVAL, "unknown path");
}

extern "C" qmm_status qmm_operand_ld(const qmm_plan *plan, int64_t k, int64_t *ld) {
    if (!plan || !ld) return fail(QMM_EINVAL, "plan and ld must not be NULL");
    if (k < 0) return fail(QMM_EINVAL, "negative k");
    const int64_t kk = k < 1 ? 1 : k;
    if (plan->path == QMM_PATH_INT8) *ld = int8_bt_ld(kk);
    else if (plan->path == QMM_PATH_FP4) *ld = fp4_ld(kk);
    else return fail(QMM_EINVAL, "qmm_operand_ld takes an INT8 or FP4 plan");
    return QMM_OK;
}

extern "C" qmm_status qmm_gemm_packed(const qmm_plan *plan, int64_t m, int64_t n, int64_t k, const void *CA,
                                      int64_t ldca, const void *CB, int64_t ldcb, uint8_t *C, int64_t ldc,
                                      void *stream) {
    if (!plan) return fail(QMM_EINVAL, "plan is NULL");
    if (!path_is_qadic(plan->path)) return fail(QMM_EINVAL, "qmm_gemm_packed takes a QADIC plan");
    if (plan->p > 256) return fail(QMM_EINVAL, "byte results need p <= 256");
    qmm_status st = qmm_validate_plan(plan, m, n, k);
    if (st != QMM_OK) return st;
    if (m < 0 || n < 0 || k < 0) return fail(QMM_EINVAL, "negative size");
    const int64_t nw = words_for(k < 1 ? 1 : k, plan->d);
    if (bad_matrix(m, nw, CA, ldca) || bad_matrix(nw, n, CB, ldcb) || bad_matrix(m, n, C, ldc))
        return fail(QMM_EINVAL, "bad pointer or leading dimension");
    if (m == 0 || n == 0) return QMM_OK;
    if (k == 0) return launch_fill_u8(C, m, n, ldc, 0, stream);
    return launch_gemm_qadic(*plan, m, n, k, CA, ldca, CB, ldcb, C, ldc, stream);
}

extern "C" qmm_status qmm_pack_centred_cols(const qmm_plan *plan, int64_t k, int64_t n, const uint8_t *B, int64_t ldb,
                                            int8_t *Bt, int64_t ldbt, void *stream) {
    if (!plan || plan->path != QMM_PATH_INT8) return fail(QMM_EINVAL, "an INT8 plan is required");
    if (plan->p < 2 || plan->p > 256) return fail(QMM_EINVAL, "INT8 needs 2 <= p <= 256");
    if (bad_matrix(k, n, B, ldb)) return fail(QMM_EINVAL, "B: bad size, pointer or ldb");
    if (n > 0 && (Bt == nullptr || ldbt % 128 != 0 || ldbt < k || ((uintptr_t)Bt % 16) != 0))
        return fail(QMM_EINVAL, "Bt: needs a 16-byte aligned pointer and ldbt a multiple of 128, >= k");
    return launch_centre_transpose(*plan, k, n, B, ldb, Bt, ldbt, stream);
}

extern "C" qmm_status qmm_gemm_centred(const qmm_plan *plan, int64_t m, int64_t n, int64_t k, const uint8_t *A,
                                       int64_t lda, const int8_t *Bt, int64_t ldbt, uint8_t *C, int64_t ldc,
                                       void *stream) {
    if (!plan || plan->path != QMM_PATH_INT8) return fail(QMM_EINVAL, "an INT8 plan is required");
    qmm_status st = qmm_validate_plan(plan, m, n, k);
    if (st != QMM_OK) return st;
    if (bad_matrix(m, k, A, lda) || bad_matrix(m, n, C, ldc)) return fail(QMM_EINVAL, "bad pointer or leading dimension");
    if (n > 0 && k > 0 && (Bt == nullptr || ldbt % 128 != 0 || ldbt < k || ((uintptr_t)Bt % 16) != 0))
        return fail(QMM_EINVAL, "Bt: needs a 16-byte aligned pointer and ldbt a multiple of 128, >= k");
    if (m == 0 || n == 0) return QMM_OK;
    if (k == 0) return launch_fill_u8(C, m, n, ldc, 0, stream);
    return launch_gemm_int8(*plan, m, n, k, A, lda, Bt, ldbt, C, ldc, stream);
}

namespace {
bool bad_fp4_operand(int64_t rows, int64_t k, const uint8_t *P, int64_t ld4) {
    if (rows == 0 || k == 0) return false;
    return P == nullptr || ld4 % 128 != 0 || 2 * ld4 < k || ((uintptr_t)P % 16) != 0;
}
}  // namespace

extern "C" qmm_status qmm_pack_fp4_rows(const qmm_plan *plan, int64_t m, int64_t k, const uint8_t *A, int64_t lda,
                                        uint8_t *A4, int64_t lda4, void *stream) {
    if (!plan || plan->path != QMM_PATH_FP4) return fail(QMM_EINVAL, "an FP4 plan is required");
    if (plan->p < 2 || plan->p > 8) return fail(QMM_EINVAL, "FP4 needs 2 <= p <= 8");
    if (bad_matrix(m, k, A, lda)) return fail(QMM_EINVAL, "A: bad size, pointer or lda");
    if (bad_fp4_operand(m, k < 1 ? 1 : k, A4, lda4))
        return fail(QMM_EINVAL, "A4: needs a 16-byte aligned pointer and lda4 a multiple of 128, >= k/2");
    return launch_pack_fp4_rows(*plan, m, k, A, lda, A4, lda4, stream);
}

extern "C" qmm_status qmm_pack_fp4_cols(const qmm_plan *plan, int64_t k, int64_t n, const uint8_t *B, int64_t ldb,
                                        uint8_t *Bt4, int64_t ldbt4, void *stream) {
    if (!plan || plan->path != QMM_PATH_FP4) return fail(QMM_EINVAL, "an FP4 plan is required");
    if (plan->p < 2 || plan->p > 8) return fail(QMM_EINVAL, "FP4 needs 2 <= p <= 8");
    if (bad_matrix(k, n, B, ldb)) return fail(QMM_EINVAL, "B: bad size, pointer or ldb");
    if (bad_fp4_operand(n, k < 1 ? 1 : k, Bt4, ldbt4))
        return fail(QMM_EINVAL, "Bt4: needs a 16-byte aligned pointer and ldbt4 a multiple of 128, >= k/2");
    return launch_pack_fp4_cols(*plan, k, n, B, ldb, Bt4, ldbt4, stream);
}

extern "C" qmm_status qmm_pack_fp4(const qmm_plan *plan, int64_t m, int64_t n, int64_t k, const uint8_t *A,
                                   int64_t lda, const uint8_t *B, int64_t ldb, uint8_t *A4, int64_t lda4, uint8_t *Bt4,
                                   int64_t ldbt4, void *stream) {
    if (!plan || plan->path != QMM_PATH_FP4) return fail(QMM_EINVAL, "an FP4 plan is required");
    if (plan->p < 2 || plan->p > 8) return fail(QMM_EINVAL, "FP4 needs 2 <= p <= 8");
    if (bad_matrix(m, k, A, lda)) return fail(QMM_EINVAL, "A: bad size, pointer or lda");
    if (bad_matrix(k, n, B, ldb)) return fail(QMM_EINVAL, "B: bad size, pointer or ldb");
    if (bad_fp4_operand(m, k < 1 ? 1 : k, A4, lda4) || bad_fp4_operand(n, k < 1 ? 1 : k, Bt4, ldbt4))
        return fail(QMM_EINVAL, "A4, Bt4: need 16-byte aligned pointers and leading dimensions that are "
                                "multiples of 128, >= k/2");
    return launch_pack_fp4_both(*plan, m, n, k, A, lda, B, ldb, A4, lda4, Bt4, ldbt4, stream);
}

extern "C" qmm_status qmm_gemm_fp4(const qmm_plan *plan, int64_t m, int64_t n, int64_t k, const uint8_t *A4,
                                   int64_t lda4, const uint8_t *Bt4, int64_t ldbt4, uint8_t *C, int64_t ldc,
                                   void *stream) {
    if (!plan || plan->path != QMM_PATH_FP4) return fail(QMM_EINVAL, "an FP4 plan is required");
    qmm_status st = qmm_validate_plan(plan, m, n, k);
    if (st != QMM_OK) return st;
    if (bad_matrix(m, n, C, ldc)) return fail(QMM_EINVAL, "C: bad pointer or ldc");
    if (bad_fp4_operand(m, k, A4, lda4) || bad_fp4_operand(n, k, Bt4, ldbt4))
        return fail(QMM_EINVAL, "A4, Bt4: need 16-byte aligned pointers and leading dimensions that are "
                                "multiples of 128, >= k/2");
    if (m == 0 || n == 0) return QMM_OK;
    if (k == 0) return launch_fill_u8(C, m, n, ldc, 0, stream);
    return launch_gemm_fp4(*plan, m, n, k, A4, lda4, Bt4, ldbt4, C, ldc, stream);
}

extern "C" qmm_status qmm_gemm_right_packed(const qmm_plan *plan, int64_t m, int64_t n, int64_t k, const uint8_t *A,
                                            int64_t lda, const void *CBr, int64_t ldcbr, uint8_t *C, int64_t ldc,
                                            void *stream) {
    if (!plan || !path_is_redq(plan->path)) return fail(QMM_EINVAL, "a REDQ plan is required");
    if (plan->p > 256) return fail(QMM_EINVAL, "byte results need p <= 256");
    qmm_status st = qmm_validate_plan(plan, m, n, k);
    if (st != QMM_OK) return st;
    if (bad_matrix(m, k, A, lda) || bad_matrix(k, words_for(n, plan->d), CBr, ldcbr) || bad_matrix(m, n, C, ldc))
        return fail(QMM_EINVAL, "bad pointer or leading dimension");
    if (m == 0 || n == 0) return QMM_OK;
    if (k == 0) return launch_fill_u8(C, m, n, ldc, 0, stream);
    return launch_gemm_redq(*plan, m, n, k, A, lda, CBr, ldcbr, C, ldc, stream);
}

extern "C" qmm_status qmm_gemm_packed_compress(const qmm_plan *plan, int64_t m, int64_t n, int64_t k, const void *CA,
                                               int64_t ldca, const void *CB, int64_t ldcb, void *CC, int64_t ldcc,
                                               void *stream) {
    if (!plan) return fail(QMM_EINVAL, "plan is NULL");
    if (!path_is_qadic(plan->path)) return fail(QMM_EINVAL, "qmm_gemm_packed_compress takes a QADIC plan");
    if (plan->p > 256) return fail(QMM_EINVAL, "residues of the output words need p <= 256");
    if (plan->d + 1 > 128) return fail(QMM_EUNSUPPORTED, "compressed output needs d + 1 <= 128");
    qmm_status st = qmm_validate_plan(plan, m, n, k);
    if (st != QMM_OK) return st;
    if ((st = check_plan_for_words(plan)) != QMM_OK) return st;
    const int64_t nw = words_for(k < 1 ? 1 : k, plan->d);
    if (bad_matrix(m, nw, CA, ldca) || bad_matrix(nw, n, CB, ldcb) || bad_matrix(m, words_for(n, plan->d), CC, ldcc))
        return fail(QMM_EINVAL, "bad pointer or leading dimension");
    if (m == 0 || n == 0) return QMM_OK;
    if (k == 0) return fail(QMM_EUNSUPPORTED, "compressed output of an empty product (k = 0) is not produced");
    return launch_gemm_qadic_compress(*plan, m, n, k, CA, ldca, CB, ldcb, CC, ldcc, stream);
}

extern "C" qmm_status qmm_pack_left(const qmm_plan *plan, int64_t m, int64_t k, const uint8_t *A, int64_t lda,
                                    void *CAl, int64_t ldcal, void *stream) {
    qmm_status st = check_plan_for_words(plan);
    if (st != QMM_OK) return st;
    if (!path_is_left(plan->path) && !path_is_full(plan->path))
        return fail(QMM_EINVAL, "qmm_pack_left takes a LEFT or FULL plan");
    if (bad_matrix(m, k, A, lda)) return fail(QMM_EINVAL, "A: bad size, pointer or lda");
    if (bad_matrix(words_for(m, plan->d), k, CAl, ldcal)) return fail(QMM_EINVAL, "CAl: bad pointer or ldcal");
    return launch_pack_cols_fwd(*plan, m, k, A, lda, CAl, ldcal, stream);
}

extern "C" qmm_status qmm_pack_full_right(const qmm_plan *plan, int64_t k, int64_t n, const uint8_t *B, int64_t ldb,
                                          void *CBt, int64_t ldcbt, void *stream) {
    if (!plan) return fail(QMM_EINVAL, "plan is NULL");
    if (!path_is_full(plan->path)) return fail(QMM_EINVAL, "qmm_pack_full_right takes a FULL plan");
    if ((uint64_t)plan->t * (plan->d + 1) > 63 || plan->d2 > 63) return fail(QMM_EINVAL, "Theta = Q^(d+1) out of range");
    const qmm_plan tp = theta_plan(*plan);
    qmm_status st = check_plan_for_words(&tp);
    if (st != QMM_OK) return st;
    if (bad_matrix(k, n, B, ldb)) return fail(QMM_EINVAL, "B: bad size, pointer or ldb");
    if (bad_matrix(k, words_for(n, plan->d2), CBt, ldcbt)) return fail(QMM_EINVAL, "CBt: bad pointer or ldcbt");
    return launch_pack_rows_fwd(tp, k, n, B, ldb, CBt, ldcbt, stream);
}

extern "C" qmm_status qmm_gemm_left_packed(const qmm_plan *plan, int64_t m, int64_t n, int64_t k, const void *CAl,
                                           int64_t ldcal, const uint8_t *B, int64_t ldb, uint8_t *C, int64_t ldc,
                                           void *stream) {
    if (!plan || !path_is_left(plan->path)) return fail(QMM_EINVAL, "a LEFT plan is required");
    if (plan->p > 256) return fail(QMM_EINVAL, "byte results need p <= 256");
    qmm_status st = qmm_validate_plan(plan, m, n, k);
    if (st != QMM_OK) return st;
    if (bad_matrix(words_for(m, plan->d), k, CAl, ldcal) || bad_matrix(k, n, B, ldb) || bad_matrix(m, n, C, ldc))
        return fail(QMM_EINVAL, "bad pointer or leading dimension");
    if (m == 0 || n == 0) return QMM_OK;
    if (k == 0) return launch_fill_u8(C, m, n, ldc, 0, stream);
    return launch_gemm_left(*plan, m, n, k, CAl, ldcal, B, ldb, C, ldc, stream);
}

extern "C" qmm_status qmm_gemm_full_packed(const qmm_plan *plan, int64_t m, int64_t n, int64_t k, const void *CAl,
                                           int64_t ldcal, const void *CBt, int64_t ldcbt, uint8_t *C, int64_t ldc,
                                           void *stream) {
    if (!plan || !path_is_full(plan->path)) return fail(QMM_EINVAL, "a FULL plan is required");
    if (plan->p > 256) return fail(QMM_EINVAL, "byte results need p <= 256");
    qmm_status st = qmm_validate_plan(plan, m, n, k);
    if (st != QMM_OK) return st;
    if (bad_matrix(words_for(m, plan->d), k, CAl, ldcal) || bad_matrix(k, words_for(n, plan->d2), CBt, ldcbt) ||
        bad_matrix(m, n, C, ldc))
        return fail(QMM_EINVAL, "bad pointer or leading dimension");
    if (m == 0 || n == 0) return QMM_OK;
    if (k == 0) return launch_fill_u8(C, m, n, ldc, 0, stream);
    return launch_gemm_full(*plan, m, n, k, CAl, ldcal, CBt, ldcbt, C, ldc, stream);
}
