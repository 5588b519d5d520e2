/*
 * qmm.h -- Q-adic compressed modular matrix multiplication on AMD MI355X (gfx950).
 *
 * Computes C = A x B mod p for residue matrices stored as bytes, following
 * Dumas, Fousse and Salvy, "Compressed Modular Matrix Multiplication" (2008):
 *   - section 2: d+1 residues packed in one floating-point word in base Q = 2^t
 *     (rows of A reversed, columns of B forward); the product of packed matrices
 *     holds every dot product as its degree-d coefficient (procedures (1), (2));
 *   - section 3: a packed word times a single residue, followed by the
 *     simultaneous reduction REDQ (procedure (5));
 *   - section 4: full compression, A packed along m in Q and B along n in
 *     Theta = Q^(d+1), every product word holding a block of C (eqs. (6), (7));
 *   - section 5, Table 2: left compression (A packed along m) and the choice of
 *     the compressed dimension from the shape;
 *   - procedure (1): the product of compressed matrices returned compressed
 *     (ReduceAndCompress), so products chain without unpacking;
 *   - sections 2.4, 2.5 and 5: the bounds tying p, k, Q, d and the mantissa.
 * Two further forms go beyond the paper: INT8 matrix cores on centred residues
 * with int32 accumulation, and batches of independent products in one launch.
 *
 * Conventions for every call below.
 *   Matrices are row-major with an explicit leading dimension (elements, >= the
 *   row length).  Residue matrices are uint8 in [0, p-1]; results are the
 *   canonical residue in [0, p-1].  Packed matrices hold "words": double when
 *   plan->beta == 53, float when plan->beta == 24.
 *   Device pointers are HIP device addresses owned by the caller; the library
 *   never frees them.  `stream` is a hipStream_t (NULL = the null stream); every
 *   device call only enqueues work on it and returns.
 *   Errors are return codes; nothing is thrown.  qmm_last_error() describes the
 *   last failure of the calling thread.  Sizes of 0 are valid and do nothing
 *   (a product with k == 0 writes zeros).
 */
#ifndef QMM_H
#define QMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    QMM_OK = 0,
    QMM_EINVAL = 1,       /* bad argument: null pointer, negative size, short leading dimension */
    QMM_EBOUND = 2,       /* no (Q, d, block) meets the bounds, or a given plan violates them */
    QMM_EVALUE = 3,       /* p out of range for the path (INT8 needs p <= 256), or input
                             entries that are not residues (validation) */
    QMM_ENOSPACE = 4,     /* workspace smaller than qmm_gemm_workspace_size() */
    QMM_EDEVICE = 5,      /* a HIP runtime call failed (message in qmm_last_error) */
    QMM_EUNSUPPORTED = 6  /* combination not implemented (named in qmm_last_error) */
} qmm_status;

typedef enum {
    QMM_PATH_AUTO = 0,        /* let qmm_choose_Qd pick */
    QMM_PATH_FP64_QADIC = 1,  /* k-compressed words, FP64 matrix cores (procedure (2)) */
    QMM_PATH_FP64_REDQ = 2,   /* n-compressed words times residues + REDQ (procedure (5)) */
    QMM_PATH_FP32_QADIC = 3,  /* as FP64_QADIC with a 24-bit mantissa */
    QMM_PATH_FP32_REDQ = 4,   /* as FP64_REDQ with a 24-bit mantissa */
    QMM_PATH_INT8 = 5,        /* centred residues, int8 matrix cores, int32 accumulation */
    QMM_PATH_FP4 = 6,         /* centred residues as FP4 (e2m1) codes, FP4 matrix cores with
                                 FP32 accumulation that stays exact (p <= 8) */
    QMM_PATH_FP64_LEFT = 7,   /* m-compressed words (d+1 rows of A) times residues + REDQ
                                 (left compression, Table 2) */
    QMM_PATH_FP32_LEFT = 8,   /* as FP64_LEFT with a 24-bit mantissa */
    QMM_PATH_FP64_FULL = 9,   /* A packed along m (degree d in Q) times B packed along n (degree
                                 d2 in Theta = Q^(d+1)), two-variable REDQ (section 4) */
    QMM_PATH_FP32_FULL = 10   /* as FP64_FULL with a 24-bit mantissa */
} qmm_path;

typedef enum {
    QMM_REGIME_EXACT = 0,   /* every partial sum is an integer below 2^beta: no rounding */
    QMM_REGIME_OFFSET = 1,  /* accumulator starts at 2^(beta-1) Q^d; each rounding floors */
    QMM_REGIME_PAPER = 2,   /* the paper's rule only (informational, never executed) */
    QMM_REGIME_INT = 3      /* integer accumulation (INT8 path) */
} qmm_regime;

/* Flags for qmm_choose_Qd. */
#define QMM_BOUND_PROVEN   0u  /* default: plans whose exactness is proven (EXACT/OFFSET) */
#define QMM_BOUND_PAPER    1u  /* the paper's rule: smallest t with k(p-1)^2 < 2^t (eq. (3)),
                                  d = min(floor(beta/t), k) - 1 (section 5); not executable */
#define QMM_PLAN_UNBLOCKED 2u  /* keep k in one block (the paper's unblocked product) */
#define QMM_BOUND_G4       4u  /* assume 4 products may be summed before one rounding */
#define QMM_BOUND_EQ4      8u  /* also impose eq. (4) as printed, Q^(d+1) < 2^beta, instead of
                                  only its sharper sum form (section 2.5) */
#define QMM_PLAN_ANY_COMPRESSION 16u
                               /* with an FP64 (FP32) path: choose among the four compressions of
                                  that mantissa -- k (procedure (2)), n (procedure (5)), m (left)
                                  and m and n (full, section 4) -- the one with the fewest
                                  multiply-adds of packed words for this shape (Table 2 with the
                                  classical product; the compressed dimension is the largest one
                                  up to the rounding of each count), ties to k */

/* A plan: everything the kernels need to know about the packing.  Plans are
 * plain values; qmm_choose_Qd fills one, and the product calls re-validate any
 * plan they are handed (a plan that violates the bounds is refused, never run). */
typedef struct {
    uint32_t p;        /* modulus, 2 <= p */
    uint32_t t;        /* Q = 2^t */
    uint32_t d;        /* polynomial degree: d+1 residues per word */
    uint32_t beta;     /* mantissa bits: 53 (FP64), 24 (FP32); 31 for INT8 (int32) */
    int64_t  k_block;  /* k is cut into blocks of k_block (a multiple of d+1); the
                          residue of every block is reduced, then the blocks summed */
    uint32_t path;     /* qmm_path; never QMM_PATH_AUTO in a returned plan */
    uint32_t regime;   /* qmm_regime */
    uint32_t g;        /* products per rounding assumed by the offset regime (1 or 4) */
    uint32_t tile;     /* kernel tile variant: 0 = chosen from the shape (1 below 192 tiles
                          of 256 x 256; above, 4 for INT8 and 3 for FP4);
                          INT8 and FP4: 1 = 128 x 128 output tiles (4 wavefronts),
                          2 = 256 x 256 (8 wavefronts of 128 x 64),
                          3 = 256 x 256 (16 wavefronts of 64 x 64);
                          INT8 only: 4 = 256 x 256, 8 wavefronts of 128 x 64 with both
                          operands loaded straight into on-chip memory, which reads A's
                          rows whole as int8 (residues of p <= 128 when k is a multiple
                          of 128 and the uncentred sums fit int32, else a centred copy
                          qmm_gemm_mod_p makes); where it cannot (qmm_gemm_centred on
                          rows not 16-byte aligned) tile 3 runs instead;
                          other values are EINVAL */
    uint32_t d2;       /* FULL paths: degree in Theta = Q^(d+1), d2+1 columns of B per word
                          (d+1 rows of A per word); 0 on every other path */
} qmm_plan;

/* Choose (Q = 2^t, d, k_block, path) for a product of shape m x k times k x n
 * modulo p (sections 1, 2.4, 2.5, 5: the field, the sizes and the mantissa are
 * given, and they constrain Q and d).  beta = 0 takes the path's own mantissa.
 * Host only, synchronous.  Returns QMM_EBOUND when no plan exists for the path. */
qmm_status qmm_choose_Qd(uint32_t p, int64_t m, int64_t n, int64_t k, uint32_t beta,
                         qmm_path path, uint32_t flags, qmm_plan *out);

/* Checks a plan against the bounds for a product with inner dimension k.
 * QMM_OK if it may run, QMM_EBOUND otherwise.  Host only. */
qmm_status qmm_validate_plan(const qmm_plan *plan, int64_t m, int64_t n, int64_t k);

/* CompressRows (procedure (2); section 2.1 reversed word, section 2.3 padding):
 * CA[i][l] = sum_{s=0..d} A[i][l(d+1)+s] * Q^(d-s), residues past k read as 0.
 * A: m x k bytes (lda >= k).  CA: m x ceil(k/(d+1)) words (ldca >= that). */
qmm_status qmm_pack_rows_rev(const qmm_plan *plan, int64_t m, int64_t k,
                             const uint8_t *A, int64_t lda, void *CA, int64_t ldca,
                             void *stream);

/* CompressColumns (procedure (2); section 2.1 forward word):
 * CB[l][j] = sum_{s=0..d} B[l(d+1)+s][j] * Q^s.
 * B: k x n bytes (ldb >= n).  CB: ceil(k/(d+1)) x n words (ldcb >= n). */
qmm_status qmm_pack_cols_fwd(const qmm_plan *plan, int64_t k, int64_t n,
                             const uint8_t *B, int64_t ldb, void *CB, int64_t ldcb,
                             void *stream);

/* Row compression of the right operand (section 3):
 * CBr[i][J] = sum_{j=0..d} B[i][J(d+1)+j] * Q^j, columns past n read as 0.
 * B: k x n bytes.  CBr: k x ceil(n/(d+1)) words (ldcbr >= that). */
qmm_status qmm_pack_rows_fwd(const qmm_plan *plan, int64_t k, int64_t n,
                             const uint8_t *B, int64_t ldb, void *CBr, int64_t ldcbr,
                             void *stream);

/* Uncompress (procedure (5)): the inverse of one of the three packings.
 * which: 0 = rows reversed (out is rows x cols = m x k), 1 = columns forward
 * (out is k x n), 2 = rows forward (out is k x n).  Each residue is digit
 * (position) of its word, i.e. floor(w / Q^j) mod Q, stored as a byte; words must
 * come from the matching pack call (digits below 256). */
qmm_status qmm_unpack(const qmm_plan *plan, int which, int64_t rows, int64_t cols,
                      const void *packed, int64_t ldp, uint8_t *out, int64_t ldo,
                      void *stream);

/* Input validation (the products take residues in [0, p) and leave any other
 * byte undefined).  Counts the entries x >= p of the rows x cols byte matrix X
 * (device, row-major, leading dimension ldx >= cols) into *count (device, 4-byte
 * aligned, caller-owned; the call sets it to zero first, with a kernel, then
 * adds).  Asynchronous on `stream`.  The Python binding's validate=True runs it on
 * A and B, synchronises and reports QMM_EVALUE when the count is not zero.
 * Errors: QMM_EINVAL for p outside [2, 256], a bad size, pointer or ldx. */
qmm_status qmm_count_nonresidues(uint32_t p, int64_t rows, int64_t cols, const uint8_t *X,
                                 int64_t ldx, uint32_t *count, void *stream);

/* REDC of Table 2 (the per-entry extraction of section 2.5): C[i][j] = digit d of
 * the accumulated word T[i][j], reduced mod p.  EXACT regime: T holds the exact
 * sum S and the digit is floor(S / Q^d) mod Q.  OFFSET regime: T holds
 * 2^(beta-1) Q^d + floor(S / Q^d) Q^d and the digit is read from the low t bits of
 * the mantissa.  T: m x n words of one k-block.  C: m x n bytes. */
qmm_status qmm_extract(const qmm_plan *plan, int64_t m, int64_t n, const void *T, int64_t ldt,
                       uint8_t *C, int64_t ldc, void *stream);

/* REDQ + EXTRACT (section 3, Table 2): every word r = sum_{j<=d} c_j Q^j of CC
 * (m x ceil(n/(d+1)), EXACT regime) yields its d+1 residues c_j mod p, written to
 * C[i][J(d+1)+j] for J(d+1)+j < n.  One division by p per word. */
qmm_status qmm_redq(const qmm_plan *plan, int64_t m, int64_t n, const void *CC, int64_t ldcc,
                    uint8_t *C, int64_t ldc, void *stream);

/* Device workspace that qmm_gemm_mod_p needs for this plan and shape (INT8:
 * centred B transposed, plus A centred into aligned rows when k is not a multiple
 * of 16, or when the product runs on tile 4 and A's residues cannot be read as
 * they are: p > 128, k not a multiple of 128, or uncentred sums past int32; INT8
 * and FP4: plus the partial outputs of the split-K edge strips when the grid of
 * 256 x 256 tiles is just past whole rounds over the device's compute units, so
 * the size can depend on the current device; edge strips of at most 16 rows or
 * columns with 16-byte aligned operand rows run as dot products and leave that
 * part unused). */
qmm_status qmm_gemm_workspace_size(const qmm_plan *plan, int64_t m, int64_t n, int64_t k,
                                   size_t *bytes);

/* C = A x B mod p from bytes to bytes (procedure (2) for the QADIC paths,
 * procedure (5) for the REDQ paths, left and full compression for the LEFT and
 * FULL paths, INT8 / FP4 matrix cores for the INT8 / FP4 paths).
 * plan == NULL: qmm_choose_Qd(p, m, n, k, 0, QMM_PATH_AUTO, 0) is used.
 * A: m x k, B: k x n, C: m x n bytes (C must not overlap A or B).
 * ws: device workspace of ws_bytes >= qmm_gemm_workspace_size, 256-byte aligned
 * (QMM_EINVAL otherwise; it may be NULL when that size is 0); it holds the packed
 * operands between the kernels.  The REDQ and
 * LEFT paths also hold their residue operand there as words (one residue each,
 * procedure (5)'s Uncompress) and multiply two word matrices; the stage calls
 * qmm_gemm_right_packed / qmm_gemm_left_packed instead convert that operand on
 * the fly, with no workspace.  Small products on an unblocked FP64 Q-adic plan
 * (m n k <= 2^22) run in one launch that packs the operands in on-chip memory and
 * need no workspace (qmm_gemm_workspace_size returns 0); so do unblocked INT8
 * products of m n k <= 2^32 with plan->tile == 0, which run in one launch that
 * centres both operands in on-chip memory. */
qmm_status qmm_gemm_mod_p(const qmm_plan *plan, int64_t m, int64_t n, int64_t k, uint32_t p,
                          const uint8_t *A, int64_t lda, const uint8_t *B, int64_t ldb,
                          uint8_t *C, int64_t ldc, void *ws, size_t ws_bytes, void *stream);

/* Largest workspace, in bytes, that qmm_gemm_mod_p_noalloc can hold (64 MiB). */
#define QMM_NOALLOC_SCRATCH_BYTES (64u << 20)

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * serving loops, harnesses that forbid hipMalloc): qmm_gemm_mod_p with the same
 * arguments, plan choice and kernels, but the workspace is a scratch array of
 * QMM_NOALLOC_SCRATCH_BYTES that the library keeps in every GPU it runs on until
 * the process ends.  The call allocates nothing: no hipMalloc, no hipFree.  The
 * caller still passes A, B and C.  The first call on a device looks up that
 * device's scratch address (with the device current); later calls reuse it.
 * Every call on one GPU shares that GPU's scratch, which keeps the last call's
 * contents (no kernel needs it cleared), so calls that overlap on one GPU --
 * concurrent streams, or threads without ordering -- race and must be
 * serialised by the caller.
 * Errors: those of qmm_gemm_mod_p; QMM_ENOSPACE when the product's workspace
 * (qmm_gemm_workspace_size) exceeds QMM_NOALLOC_SCRATCH_BYTES (nothing is
 * launched); QMM_EDEVICE if the scratch address cannot be looked up. */
qmm_status qmm_gemm_mod_p_noalloc(const qmm_plan *plan, int64_t m, int64_t n, int64_t k, uint32_t p,
                                  const uint8_t *A, int64_t lda, const uint8_t *B, int64_t ldb,
                                  uint8_t *C, int64_t ldc, void *stream);

/* Procedure (1) on already compressed operands: C = digit d of CA x CB, mod p.
 * CA: m x ceil(k/(d+1)) words from qmm_pack_rows_rev; CB: ceil(k/(d+1)) x n words
 * from qmm_pack_cols_fwd, both with this plan.  QADIC paths only; p <= 256. */
qmm_status qmm_gemm_packed(const qmm_plan *plan, int64_t m, int64_t n, int64_t k,
                           const void *CA, int64_t ldca, const void *CB, int64_t ldcb,
                           uint8_t *C, int64_t ldc, void *stream);

/* Procedure (1) with ReduceAndCompress: the product of compressed matrices handed
 * back compressed.  CC[i][L] = sum_{s=0..d} C[i][L(d+1)+s] * Q^(d-s) (the
 * CompressRows layout, columns past n read as 0) where C = digit d of CA x CB, mod p;
 * CC is m x ceil(n/(d+1)) words (ldcc >= that) and can be the CA of a next product
 * with the same plan and k = n (chained products, e.g. powers of a matrix).
 * CA, CB as for qmm_gemm_packed.  QADIC paths only; plans with d + 1 <= 128. */
qmm_status qmm_gemm_packed_compress(const qmm_plan *plan, int64_t m, int64_t n, int64_t k,
                                    const void *CA, int64_t ldca, const void *CB, int64_t ldcb,
                                    void *CC, int64_t ldcc, void *stream);

/* Left compression (Table 2; section 3's packing applied to the rows of A):
 * CAl[I][l] = sum_{i=0..d} A[I(d+1)+i][l] * Q^i, rows past m read as 0.
 * A: m x k bytes (lda >= k).  CAl: ceil(m/(d+1)) x k words (ldcal >= k).
 * LEFT and FULL plans (the left operand of both). */
qmm_status qmm_pack_left(const qmm_plan *plan, int64_t m, int64_t k, const uint8_t *A, int64_t lda,
                         void *CAl, int64_t ldcal, void *stream);

/* Full compression (section 4), right operand packed along n in Theta = Q^(d+1):
 * CBt[l][J] = sum_{j=0..d2} B[l][J(d2+1)+j] * Theta^j, columns past n read as 0.
 * B: k x n bytes.  CBt: k x ceil(n/(d2+1)) words (ldcbt >= that).  FULL plans. */
qmm_status qmm_pack_full_right(const qmm_plan *plan, int64_t k, int64_t n, const uint8_t *B, int64_t ldb,
                               void *CBt, int64_t ldcbt, void *stream);

/* Left compression, product step: CC = CAl x B over exact words (every coefficient
 * below Q by eq. (3), every word below Q^(d+1) < 2^beta by eq. (4)), then REDQ of
 * each word into its d+1 residues, written to C[I(d+1)+i][j] for rows < m.
 * CAl from qmm_pack_left with this plan; B: k x n residues.  LEFT plans. */
qmm_status qmm_gemm_left_packed(const qmm_plan *plan, int64_t m, int64_t n, int64_t k,
                                const void *CAl, int64_t ldcal, const uint8_t *B, int64_t ldb,
                                uint8_t *C, int64_t ldc, void *stream);

/* Full compression, product step: CC = CAl x CBt over exact words (eq. (3) for every
 * coefficient, eq. (7) Q^((d+1)(d2+1)) < 2^beta for the word), then one REDQ per
 * word: the coefficient of Q^i Theta^j goes, mod p, to C[I(d+1)+i][J(d2+1)+j].
 * CAl from qmm_pack_left, CBt from qmm_pack_full_right, both with this plan. */
qmm_status qmm_gemm_full_packed(const qmm_plan *plan, int64_t m, int64_t n, int64_t k,
                                const void *CAl, int64_t ldcal, const void *CBt, int64_t ldcbt,
                                uint8_t *C, int64_t ldc, void *stream);

/* Procedure (5) on an already row-compressed right operand: C = REDQ(A x CBr).
 * A: m x k residues (converted to words on the fly); CBr: k x ceil(n/(d+1)) words
 * from qmm_pack_rows_fwd with this plan.  REDQ paths only. */
qmm_status qmm_gemm_right_packed(const qmm_plan *plan, int64_t m, int64_t n, int64_t k,
                                 const uint8_t *A, int64_t lda, const void *CBr, int64_t ldcbr,
                                 uint8_t *C, int64_t ldc, void *stream);

/* Leading dimension (bytes) of the packed operands of the INT8 and FP4 paths for an
 * inner dimension k: for an INT8 plan the row stride of Bt that qmm_gemm_mod_p uses
 * (k rounded up to 128, plus one 128-byte line when that is a multiple of 2048, so
 * that rows do not crowd a few HBM channels); for an FP4 plan the row stride of A4
 * and Bt4 (ceil(k/2) rounded the same way).  Callers of the stage entry points
 * allocate with it; any multiple of 128 >= k (>= k/2) is accepted too.
 * QMM_EINVAL for other paths, a NULL argument or k < 0.  Host only. */
qmm_status qmm_operand_ld(const qmm_plan *plan, int64_t k, int64_t *ld);

/* INT8 path, conversion step: Bt[j][l] = centred(B[l][j]) as int8, where
 * centred(x) = x - p if x > (p-1)/2, else x; Bt is n x ldbt with ldbt a multiple
 * of 128 and >= k, columns l >= k are zero.  Bt must be 16-byte aligned.
 * (The int8 matrix cores take both operands contiguous along k.) */
qmm_status qmm_pack_centred_cols(const qmm_plan *plan, int64_t k, int64_t n, const uint8_t *B,
                                 int64_t ldb, int8_t *Bt, int64_t ldbt, void *stream);

/* FP4 path (p <= 8): the product C = A x B mod p of section 1's problem, on a
 * number format the paper's hardware did not have.  Every centred residue of such a p (|x| <= 4) is an exact
 * e2m1 value (0, +-1, +-2, +-3, +-4), so the FP4 matrix cores of gfx950 multiply
 * them exactly and the FP32 accumulator stays an exact integer while
 * k_block floor(p/2)^2 + p - 1 <= 2^24; longer k is cut into blocks reduced mod p.
 * Packed operand layout: row-major rows of e2m1 codes (sign bit 8, magnitude code
 * 0 = 0, 2 = 1, 4 = 2, 5 = 3, 6 = 4), two per byte, the even k in the low nibble;
 * row stride ld4 bytes, a multiple of 128 with 2 ld4 >= k; codes past k are zero.
 * Both packed operands must be 16-byte aligned.
 * Conversion steps: A4 (m x ld4) from A (m x k residues, row-major) and Bt4
 * (n x ld4) from B (k x n residues) transposed, so both are contiguous along k.
 * All buffers are the caller's; every call is asynchronous on `stream`.
 * Errors: QMM_EINVAL for a plan that is not an FP4 plan, p outside [2, 8], a bad
 * size, pointer, alignment or leading dimension; the product step also returns
 * what qmm_validate_plan returns for the plan (QMM_EBOUND for a k_block past the
 * exact FP32 range, QMM_EVALUE for p > 8). */
qmm_status qmm_pack_fp4_rows(const qmm_plan *plan, int64_t m, int64_t k, const uint8_t *A,
                             int64_t lda, uint8_t *A4, int64_t lda4, void *stream);
qmm_status qmm_pack_fp4_cols(const qmm_plan *plan, int64_t k, int64_t n, const uint8_t *B,
                             int64_t ldb, uint8_t *Bt4, int64_t ldbt4, void *stream);

/* Both FP4 conversions in one launch: A4 from A as qmm_pack_fp4_rows and Bt4 from
 * B as qmm_pack_fp4_cols (what qmm_gemm_mod_p runs on this path). */
qmm_status qmm_pack_fp4(const qmm_plan *plan, int64_t m, int64_t n, int64_t k, const uint8_t *A,
                        int64_t lda, const uint8_t *B, int64_t ldb, uint8_t *A4, int64_t lda4,
                        uint8_t *Bt4, int64_t ldbt4, void *stream);

/* FP4 path, product step: C = (A4 x Bt4^T) mod p (values decoded from the codes),
 * FP32 accumulation, k cut into plan->k_block blocks reduced mod p.  plan->tile
 * picks the kernel tile as for INT8. */
qmm_status qmm_gemm_fp4(const qmm_plan *plan, int64_t m, int64_t n, int64_t k,
                        const uint8_t *A4, int64_t lda4, const uint8_t *Bt4, int64_t ldbt4,
                        uint8_t *C, int64_t ldc, void *stream);

/* INT8 path, product step: C = (centred(A) x Bt^T) mod p with int32 accumulation,
 * k cut into plan->k_block blocks reduced mod p.  A: m x k bytes; Bt from
 * qmm_pack_centred_cols with the same plan. */
qmm_status qmm_gemm_centred(const qmm_plan *plan, int64_t m, int64_t n, int64_t k,
                            const uint8_t *A, int64_t lda, const int8_t *Bt, int64_t ldbt,
                            uint8_t *C, int64_t ldc, void *stream);

/* ---- batches of independent products --------------------------------------- */
typedef struct {
    int64_t m, n, k;
    uint32_t p;
    const uint8_t *A; int64_t lda;   /* device, m x k */
    const uint8_t *B; int64_t ldb;   /* device, k x n */
    uint8_t *C; int64_t ldc;         /* device, m x n */
} qmm_problem;

typedef struct qmm_batched qmm_batched;

/* Plans every product (path and tile per product), builds the device-side
 * descriptor table, tile list and operand-block list, and records the launches in
 * one HIP graph: for INT8 products a pack kernel that centres every A_i and
 * centres and transposes every B_i once into a workspace, then one persistent
 * product kernel per tile shape.  probs is a host array; the device buffers it
 * names must stay valid until qmm_batched_destroy.  No output C_i may share a byte
 * with any A_j, B_j or other C_j (inputs may share bytes with each other): the
 * products run concurrently, raw tiles read A_j and B_j while other tiles write,
 * and QMM_BATCH_MEASURE replays the batch several times on these buffers.  The
 * library does not check this (outputs that are disjoint views into one larger
 * matrix are allowed and common).  The batch owns the device
 * memory it allocates, including the workspace of sum_i (mp_i + np_i) kp_i bytes
 * (kp_i = k_i rounded up to 64, mp_i and np_i = m_i and n_i rounded up to the
 * product's tile).
 * INT8 products of p <= 8 whose k is one exact FP32 block (k floor(p/2)^2 + p - 1 <=
 * 2^24) use FP4 codes instead (plan path QMM_PATH_FP4): half the workspace bytes
 * and the FP4 form of the MFMA in the same tile kernels.
 * flags: QMM_BATCH_FORCE_FP64 puts every product on the FP64 Q-adic tile path (the
 * paper's method, unblocked plans); QMM_BATCH_SHAPE_* fixes the INT8 output tile
 * instead of letting the autotuner pick it per product.  Products whose k would
 * need blocked int32 accumulation are refused (QMM_EUNSUPPORTED). */
#define QMM_BATCH_FORCE_FP64   1u
#define QMM_BATCH_INT8_ONLY    2u  /* keep products of p <= 8 on INT8 instead of FP4 codes */
#define QMM_BATCH_SHAPE_64x64   0x100u
#define QMM_BATCH_SHAPE_32x128  0x200u
#define QMM_BATCH_SHAPE_128x32  0x300u
#define QMM_BATCH_SHAPE_128x128 0x400u
#define QMM_BATCH_SHAPE_MASK    0x700u  /* other values under the mask are EINVAL */
/* QMM_BATCH_MEASURE: the autotuner's second stage.  Builds the cost-model
 * assignment and one batch per uniform INT8 tile shape, with packed operands and
 * again with raw tiles (QMM_BATCH_RAW), times each (three graph
 * replays after a warm-up, on a private stream, synchronised) on the problems' own
 * buffers, and keeps the fastest.  Every candidate computes the same C_i, so the
 * outputs hold the products when the call returns.  Not combinable with
 * QMM_BATCH_FORCE_FP64 or QMM_BATCH_SHAPE_* (EINVAL). */
#define QMM_BATCH_MEASURE       0x1000u
/* QMM_BATCH_RAW: every product on INT8 tiles that read the products' own residue
 * matrices in place (residues of p <= 128 used as they are when k (p-1)^2 < 2^31,
 * centred otherwise; B's rows read from on-chip memory with the transpose load):
 * no pack kernel and no operand workspace, the graph is one kernel per tile shape.
 * Products of p <= 8 stay on INT8.  The tiles address A and B with 32-bit offsets:
 * a product whose A or B data ((rows - 1) * ld + cols bytes) exceeds 2^32 - 64 is
 * refused (QMM_EUNSUPPORTED).  Not combinable with QMM_BATCH_FORCE_FP64 or
 * QMM_BATCH_MEASURE (EINVAL); QMM_BATCH_MEASURE times the raw assignments next to
 * the packed ones and keeps the fastest (skipping them when a product is refused). */
#define QMM_BATCH_RAW           0x2000u
qmm_status qmm_batched_create(int64_t count, const qmm_problem *probs, uint32_t flags,
                              qmm_batched **out);

/* Replays the recorded launch on `stream`: every product of the batch. */
qmm_status qmm_gemm_mod_p_batched(qmm_batched *batch, void *stream);

/* Autotuner calibration (the measured half of the cost model of section 5,
 * Table 2 being the prior): times whole batches of each tile shape on synthetic
 * m x n products at prime p, with k = 128 and k = 1024 (synchronising `stream`),
 * and fits per-tile cost = fixed + per_stage * (k / 128).  costs (may be NULL)
 * receives 8 doubles: (fixed, per_stage) for 64x64, 32x128, 128x32 and 128x128,
 * in units of one 128-byte K stage of a 64x64 tile.  The calibration products
 * read and write the caller's workspace ws (device, ws_bytes >=
 * qmm_batched_tune_workspace_size(m, n); its contents are overwritten); the only
 * device memory allocated is that of the calibration batches, inside
 * qmm_batched_create, freed before the call returns.  The fit becomes the
 * default costs of this process and is stored in the tune cache under (this
 * GPU's architecture, the encoding of p -- FP4 codes for p <= 8, centred int8
 * otherwise --, the shape bucket of m x n); when the environment variable
 * QMM_TUNE_CACHE names a file, the cache is written there.
 * Errors: QMM_EINVAL for p outside [2, 256] or m, n outside [1, 4096],
 * QMM_ENOSPACE for a short workspace, QMM_EDEVICE for runtime failures. */
qmm_status qmm_batched_tune(uint32_t p, int64_t m, int64_t n, void *ws, size_t ws_bytes, void *stream,
                            double *costs);

/* Workspace bytes qmm_batched_tune(p, m, n, ...) needs. */
qmm_status qmm_batched_tune_workspace_size(int64_t m, int64_t n, size_t *bytes);

/* Installs default costs (8 doubles, as qmm_batched_tune returns), used for
 * products that the tune cache has no entry for. */
qmm_status qmm_batched_set_costs(const double *costs);

/* The tune cache (host only).  Entries map (arch -- the device's gcnArchName up
 * to the first ':', e.g. "gfx950" --, encoding of p, shape bucket of max(m, n):
 * up to 128, up to 512, above) to the 8 costs of qmm_batched_tune.
 * qmm_batched_create reads the file named by QMM_TUNE_CACHE (if set) the first
 * time it runs in a process, then gives each product the costs of the entry with
 * its device's architecture and its encoding whose bucket is nearest its own,
 * or the default costs when there is none.  The file is JSON:
 *   {"version": 1, "entries": [{"arch": "gfx950", "enc": "fp4" | "int8",
 *    "bucket": "le128" | "le512" | "gt512", "costs": [8 numbers]}, ...]}
 * put stores (replacing an entry of the same key); get returns the entry of the
 * same arch and encoding with the nearest bucket (QMM_EVALUE if there is none);
 * load merges a file into memory (QMM_EINVAL if it is missing or malformed);
 * save writes every entry (to path.tmp, then renamed); clear empties memory. */
qmm_status qmm_tune_cache_put(const char *arch, uint32_t p, int64_t m, int64_t n, const double *costs);
qmm_status qmm_tune_cache_get(const char *arch, uint32_t p, int64_t m, int64_t n, double *costs);
qmm_status qmm_tune_cache_load(const char *path);
qmm_status qmm_tune_cache_save(const char *path);
qmm_status qmm_tune_cache_clear(void);

/* Plan chosen for product i of the batch (host copy); plan->tile holds the INT8
 * tile shape (0 = 64x64, 1 = 32x128, 2 = 128x32, 3 = 128x128). */
qmm_status qmm_batched_plan(const qmm_batched *batch, int64_t i, qmm_plan *out);

/* Frees the batch's device memory and graph.  NULL is accepted. */
qmm_status qmm_batched_destroy(qmm_batched *batch);

/* Thread-local description of the last error of this thread ("" if none). */
const char *qmm_last_error(void);

/* Library version, "major.minor.patch". */
const char *qmm_version(void);

#ifdef __cplusplus
}
#endif
#endif /* QMM_H */
