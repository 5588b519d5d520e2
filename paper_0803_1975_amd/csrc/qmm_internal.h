// Internal declarations shared by the library's translation units.
#pragma once

#include <cstdint>
#include <string>

#include "qmm.h"

namespace qmm {

// K-tile of the Q-adic GEMM kernels, in packed words.  A k-block always spans a
// whole number of K-tiles of words, so block boundaries fall between tiles.
constexpr int kQadicKT = 16;
// Largest K stage of the INT8 kernels, in bytes.  Blocks of the INT8 path are
// multiples of it (and so whole stages of every INT8 kernel).
constexpr int kInt8KT = 128;
constexpr int kFp4KB = 256;  // FP4 k-block granularity: one 128-byte K stage of packed codes
// Cost of one block boundary (extraction + reduction of every output) in units of
// one packed word of MFMA work per output; used to rank blocked plans.
constexpr int kBlockCostWords = 8;

void set_error(const std::string &msg);
qmm_status fail(qmm_status st, const std::string &msg);

#if defined(__HIP__)
#define QMM_HD __host__ __device__
#else
#define QMM_HD
#endif

QMM_HD inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Packed words along one packed dimension of size len.
QMM_HD inline int64_t words_for(int64_t len, uint32_t d) { return ceil_div(len, (int64_t)d + 1); }

// Multiplier of mod_u32: floor((2^64 - 1) / p) + 1, which is floor(2^64 / p) + 1 when
// p is not a power of two and exactly 2^64 / p when it is; both keep the quotient exact.
inline uint64_t mod_magic(uint32_t p) { return ~0ull / p + 1; }

bool path_is_fp64(uint32_t path);
bool path_is_fp32(uint32_t path);
bool path_is_qadic(uint32_t path);
bool path_is_redq(uint32_t path);
bool path_is_left(uint32_t path);
bool path_is_full(uint32_t path);

// The plan of full compression's right operand: words in base Theta = Q^(d+1)
// holding d2+1 residues (what qmm_pack_full_right packs with).
qmm_plan theta_plan(const qmm_plan &pl);

// True when every packed word (p-1)(1 + Q + ... + Q^d) is an exact float of the
// plan's mantissa and fits the 64-bit integer the pack kernels build it in.
bool words_exact(const qmm_plan &pl);

// Word size in bytes for a plan (8 for beta 53, 4 for beta 24).
int word_bytes(const qmm_plan &pl);

// Launchers (qmm_kernels_*.hip).  All sizes already validated.
qmm_status launch_pack_rows_rev(const qmm_plan &pl, int64_t m, int64_t k, const uint8_t *A,
                                int64_t lda, void *CA, int64_t ldca, void *stream);
qmm_status launch_pack_cols_fwd(const qmm_plan &pl, int64_t k, int64_t n, const uint8_t *B,
                                int64_t ldb, void *CB, int64_t ldcb, void *stream);
qmm_status launch_pack_rows_fwd(const qmm_plan &pl, int64_t k, int64_t n, const uint8_t *B,
                                int64_t ldb, void *CBr, int64_t ldcbr, void *stream);
qmm_status launch_unpack(const qmm_plan &pl, int which, int64_t rows, int64_t cols,
                         const void *packed, int64_t ldp, uint8_t *out, int64_t ldo, void *stream);
qmm_status launch_extract(const qmm_plan &pl, int64_t m, int64_t n, const void *T, int64_t ldt,
                          uint8_t *C, int64_t ldc, void *stream);
qmm_status launch_redq(const qmm_plan &pl, int64_t m, int64_t n, const void *CC, int64_t ldcc,
                       uint8_t *C, int64_t ldc, void *stream);
qmm_status launch_fill_u8(uint8_t *C, int64_t m, int64_t n, int64_t ldc, uint8_t v, void *stream);
qmm_status launch_count_nonresidues(uint32_t p, int64_t rows, int64_t cols, const uint8_t *X, int64_t ldx,
                                    uint32_t *count, void *stream);

// Q-adic GEMM on packed words (procedure (1)): C = digit d of CA x CB mod p.
qmm_status launch_gemm_qadic(const qmm_plan &pl, int64_t m, int64_t n, int64_t k,
                             const void *CA, int64_t ldca, const void *CB, int64_t ldcb,
                             uint8_t *C, int64_t ldc, void *stream);
// Procedure (1) with ReduceAndCompress: CC = CompressRows(digit d of CA x CB mod p).
qmm_status launch_gemm_qadic_compress(const qmm_plan &pl, int64_t m, int64_t n, int64_t k, const void *CA,
                                      int64_t ldca, const void *CB, int64_t ldcb, void *CC, int64_t ldcc,
                                      void *stream);
// Left compression + REDQ: C = REDQ(CAl x B), blocks of d+1 rows.
qmm_status launch_gemm_left(const qmm_plan &pl, int64_t m, int64_t n, int64_t k, const void *CAl, int64_t ldcal,
                            const uint8_t *B, int64_t ldb, uint8_t *C, int64_t ldc, void *stream);
// Full compression + two-variable REDQ: C = REDQ(CAl x CBt), blocks of (d+1) x (d2+1).
qmm_status launch_gemm_full(const qmm_plan &pl, int64_t m, int64_t n, int64_t k, const void *CAl, int64_t ldcal,
                            const void *CBt, int64_t ldcbt, uint8_t *C, int64_t ldc, void *stream);
// Procedure (2) for a small product in one launch (FP64, unblocked plans): each
// tile packs its operands from the bytes into LDS.
qmm_status launch_gemm_qadic_fused(const qmm_plan &pl, int64_t m, int64_t n, int64_t k, const uint8_t *A,
                                   int64_t lda, const uint8_t *B, int64_t ldb, uint8_t *C, int64_t ldc,
                                   void *stream);
// Largest m n k that qmm_gemm_mod_p runs on the fused Q-adic kernel.
constexpr double kFusedQadicMaxMacs = 4194304.0;  // 2^22: the staged path wins from between 160^3 and 192^3 (measured)
// Right-compressed GEMM + REDQ (procedure (5)): C = REDQ(A x CBr).
qmm_status launch_gemm_redq(const qmm_plan &pl, int64_t m, int64_t n, int64_t k,
                            const uint8_t *A, int64_t lda, const void *CBr, int64_t ldcbr,
                            uint8_t *C, int64_t ldc, void *stream);
// INT8: B is first centred and transposed into Bt (n x k, int8, ldbt = k rounded up).
qmm_status launch_centre_transpose(const qmm_plan &pl, int64_t k, int64_t n, const uint8_t *B,
                                   int64_t ldb, int8_t *Bt, int64_t ldbt, void *stream);
// A small unblocked INT8 product in one launch (B centred and transposed in LDS).
qmm_status launch_gemm_int8_small(const qmm_plan &pl, int64_t m, int64_t n, int64_t k, const uint8_t *A,
                                  int64_t lda, const uint8_t *B, int64_t ldb, uint8_t *C, int64_t ldc,
                                  void *stream);
// Longest operand data (bytes from the first element to one past the last) that
// kernels address with 32-bit offsets, with room for their 20-byte load windows.
constexpr int64_t kRawSpan = (int64_t)UINT32_MAX - 63;

// Autotuner cost fits: (fixed, per_stage) for each of the four batched INT8 tile
// shapes, cached per (GPU architecture, encoding, shape bucket).
constexpr int kTuneCosts = 8;
uint32_t tune_enc(uint32_t p);                     // 1: FP4 codes (p <= 8), 0: centred int8
uint32_t tune_bucket(int64_t m, int64_t n);        // max(m, n) <= 128, <= 512, larger
void tune_cache_put(const std::string &arch, uint32_t enc, uint32_t bucket, const double *costs);
// The entry of this architecture and encoding with the nearest bucket, if any.
bool tune_cache_lookup(const std::string &arch, uint32_t enc, uint32_t bucket, double *costs);
qmm_status tune_cache_load_env_once();             // QMM_TUNE_CACHE, read once per process
qmm_status tune_cache_save_env();                  // QMM_TUNE_CACHE, if set
// Largest m n k that qmm_gemm_mod_p runs on the one-launch INT8 kernel.
constexpr double kSmallInt8MaxMacs = 4294967296.0;  // 2^32: one launch measured faster up to 1536^3
// tail_ws, tail_bytes: workspace for the split-K strip of a partial last round of
// 256 x 256 tiles (lowp_tail_bytes); without it (nullptr) the product runs whole.
qmm_status launch_gemm_int8(const qmm_plan &pl, int64_t m, int64_t n, int64_t k,
                            const uint8_t *A, int64_t lda, const int8_t *Bt, int64_t ldbt,
                            uint8_t *C, int64_t ldc, void *stream, uint8_t *tail_ws = nullptr,
                            size_t tail_bytes = 0);
// INT8 with k not a multiple of 16: A is first centred into Ac (m x ldac int8,
// ldac = int8_bt_ld(k), zero past k), so the product reads it with aligned 16-byte
// loads and centres nothing (launch_gemm_int8_centred_a).
qmm_status launch_centre_rows(const qmm_plan &pl, int64_t m, int64_t k, const uint8_t *A, int64_t lda, int8_t *Ac,
                              int64_t ldac, void *stream);
qmm_status launch_gemm_int8_centred_a(const qmm_plan &pl, int64_t m, int64_t n, int64_t k, const int8_t *Ac,
                                      int64_t ldac, const int8_t *Bt, int64_t ldbt, uint8_t *C, int64_t ldc,
                                      void *stream, uint8_t *tail_ws = nullptr, size_t tail_bytes = 0);
// Bytes of the partial outputs qmm_gemm_mod_p's INT8 or FP4 product uses for the
// rows of a partial last round of 256 x 256 tiles (0: no split).
size_t lowp_tail_bytes(const qmm_plan &pl, int64_t m, int64_t n, int64_t k);
int64_t int8_bt_ld(int64_t k);
int64_t fp4_ld(int64_t k);
void fp4_lut(uint32_t p, uint32_t &lo, uint32_t &hi);  // e2m1 codes of the residues 0..7, as bytes
qmm_status launch_pack_fp4_rows(const qmm_plan &pl, int64_t m, int64_t k, const uint8_t *A, int64_t lda,
                                uint8_t *A4, int64_t lda4, void *stream);
qmm_status launch_pack_fp4_cols(const qmm_plan &pl, int64_t k, int64_t n, const uint8_t *B, int64_t ldb,
                                uint8_t *Bt4, int64_t ldbt4, void *stream);
qmm_status launch_pack_fp4_both(const qmm_plan &pl, int64_t m, int64_t n, int64_t k, const uint8_t *A, int64_t lda,
                                const uint8_t *B, int64_t ldb, uint8_t *A4, int64_t lda4, uint8_t *Bt4, int64_t ldbt4,
                                void *stream);
qmm_status launch_gemm_fp4(const qmm_plan &pl, int64_t m, int64_t n, int64_t k, const uint8_t *A4, int64_t lda4,
                           const uint8_t *Bt4, int64_t ldbt4, uint8_t *C, int64_t ldc, void *stream,
                           uint8_t *tail_ws = nullptr, size_t tail_bytes = 0);
int int8_tile_for(int64_t m, int64_t n, bool fp4);
// Whether qmm_gemm_mod_p's INT8 product centres A into aligned rows first (k not a
// multiple of 16, or the direct-load tile 4, which reads both operands as rows).
bool int8_centres_a(const qmm_plan &pl, int64_t m, int64_t n, int64_t k);

}  // namespace qmm
