// Conversions between residues and packed words, and the standalone reductions.
//
//   pack_rows_rev   CompressRows  (section 2.1 reversed word, section 2.3 padding)
//   pack_cols_fwd   CompressColumns (section 2.1 forward word)
//   pack_rows_fwd   row compression of the right operand (section 3)
//   unpack          Uncompress (procedure (5))
//   extract         REDC of Table 2: digit d of an accumulated word, mod p (section 2.5)
//   redq            REDQ + EXTRACT of Table 2 (section 3)
//   count_nonresidues  input validation: entries x >= p of a byte matrix
//
// All are HBM-bound elementwise passes: one thread per output word (or residue),
// consecutive threads on consecutive outputs so both the byte reads and the word
// writes of a wavefront are contiguous.  Two-dimensional grid-stride loops: rows
// on the grid's y, positions in a row on x, so no thread divides a flat 64-bit
// index (rows longer than 2^31 entries are refused, and the in-row divisions of
// unpack are 32-bit).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "qmm_device.h"
#include "qmm_internal.h"

namespace qmm {
namespace {

constexpr int kThreads = 256;

// Grid for a rows x cols pass: enough x blocks to cover a row (at most 4096), and
// as many rows per launch as keep the grid near kPassBlocks workgroups; each
// workgroup then strides over rows.  Workgroups of one output row each (2^18 of
// them for the graph workload's operands) left these passes bound by launching
// workgroups rather than by HBM.
#ifndef QMM_PASS_BLOCKS
#define QMM_PASS_BLOCKS 4096
#endif
constexpr int64_t kPassBlocks = QMM_PASS_BLOCKS;
inline dim3 grid2(int64_t rows, int64_t cols) {
    const int64_t x = std::max<int64_t>(1, std::min<int64_t>(ceil_div(cols, kThreads), 4096));
    const int64_t y = std::max<int64_t>(1, std::min<int64_t>({rows, (int64_t)65535, std::max<int64_t>(1, kPassBlocks / x)}));
    return dim3((unsigned)x, (unsigned)y);
}

#define QMM_FOR_ROWS(r, rows) for (int64_t r = blockIdx.y; r < (rows); r += gridDim.y)
#define QMM_FOR_COLS(c, cols) \
    for (int64_t c = (int64_t)blockIdx.x * kThreads + threadIdx.x; c < (cols); c += (int64_t)gridDim.x * kThreads)

// CA[i][l] = sum_s A[i][l(d+1)+s] Q^(d-s): Horner from the first residue of the chunk,
// which ends with the top power (the paper's init3 order).
template <typename W>
__global__ __launch_bounds__(kThreads) void pack_rows_rev_kernel(int64_t m, int64_t k, int64_t nw,
                                                                  const uint8_t *__restrict__ A, int64_t lda,
                                                                  W *__restrict__ CA, int64_t ldca,
                                                                  uint32_t t, uint32_t d) {
    QMM_FOR_ROWS(i, m) {
        const uint8_t *a = A + i * lda;
        QMM_FOR_COLS(l, nw) {
            const int64_t base = (int64_t)l * (d + 1);
            uint64_t w = 0;
            for (uint32_t s = 0; s <= d; ++s) {
                const int64_t c = base + s;
                w = (w << t) | (c < k ? (uint64_t)a[c] : 0ull);
            }
            CA[i * ldca + l] = word_from_u64<W>(w);
        }
    }
}

// CB[l][j] = sum_s B[l(d+1)+s][j] Q^s.
template <typename W>
__global__ __launch_bounds__(kThreads) void pack_cols_fwd_kernel(int64_t k, int64_t n, int64_t nw,
                                                                  const uint8_t *__restrict__ B, int64_t ldb,
                                                                  W *__restrict__ CB, int64_t ldcb,
                                                                  uint32_t t, uint32_t d) {
    QMM_FOR_ROWS(l, nw) {
        const int64_t base = l * (d + 1);
        QMM_FOR_COLS(j, n) {
            uint64_t w = 0;
            for (int32_t s = (int32_t)d; s >= 0; --s) {
                const int64_t r = base + s;
                w = (w << t) | (r < k ? (uint64_t)B[r * ldb + j] : 0ull);
            }
            CB[l * ldcb + j] = word_from_u64<W>(w);
        }
    }
}

// The same, four words per thread when rows of A are 4-byte aligned and d+1 <= 8:
// the thread's 4 (d+1) residues are d+1 aligned dwords of the row (one load each,
// consecutive threads on consecutive dwords), and its four words go out as one run.
// Words whose residues run past k take the byte path.
template <typename W, int D1>
__global__ __launch_bounds__(kThreads) void pack_rows_rev4_kernel(int64_t m, int64_t k, int64_t nw,
                                                                   const uint8_t *__restrict__ A, int64_t lda,
                                                                   W *__restrict__ CA, int64_t ldca, uint32_t t) {
    const int64_t groups = ceil_div(nw, 4);
    QMM_FOR_ROWS(i, m) {
        const uint8_t *a = A + i * lda;
        W *ca = CA + i * ldca;
        QMM_FOR_COLS(gi, groups) {
            const int64_t l0 = 4 * gi, b0 = l0 * D1;
            if (b0 + 4 * D1 <= k) {
                uint32_t dw[D1];
#pragma unroll
                for (int q = 0; q < D1; ++q) dw[q] = *(const uint32_t *)(a + b0 + 4 * q);
#pragma unroll
                for (int w = 0; w < 4; ++w) {
                    uint64_t v = 0;
#pragma unroll
                    for (int s2 = 0; s2 < D1; ++s2) {
                        const int j = w * D1 + s2;
                        v = (v << t) | ((dw[j >> 2] >> (8 * (j & 3))) & 0xffu);
                    }
                    if (l0 + w < nw) ca[l0 + w] = word_from_u64<W>(v);
                }
            } else {
                for (int64_t l = l0; l < nw && l < l0 + 4; ++l) {
                    uint64_t v = 0;
                    for (int s2 = 0; s2 < D1; ++s2) {
                        const int64_t c = l * D1 + s2;
                        v = (v << t) | (c < k ? (uint64_t)a[c] : 0ull);
                    }
                    ca[l] = word_from_u64<W>(v);
                }
            }
        }
    }
}

// CompressColumns, four columns per thread when rows of B are 4-byte aligned: each
// of the d+1 residue rows of a word row is one dword load for the four columns;
// columns past n take byte loads.
template <typename W>
__global__ __launch_bounds__(kThreads) void pack_cols_fwd4_kernel(int64_t k, int64_t n, int64_t nw,
                                                                   const uint8_t *__restrict__ B, int64_t ldb,
                                                                   W *__restrict__ CB, int64_t ldcb,
                                                                   uint32_t t, uint32_t d) {
    const int64_t groups = ceil_div(n, 4);
    QMM_FOR_ROWS(l, nw) {
        const int64_t base = l * (d + 1);
        W *cb = CB + l * ldcb;
        QMM_FOR_COLS(gi, groups) {
            const int64_t j0 = 4 * gi;
            uint64_t v[4] = {0, 0, 0, 0};
            const bool whole = j0 + 4 <= n;
            for (int32_t s2 = (int32_t)d; s2 >= 0; --s2) {
                const int64_t r = base + s2;
                uint32_t x = 0;
                if (r < k) {
                    const uint8_t *row = B + r * ldb + j0;
                    if (whole) {
                        x = *(const uint32_t *)row;
                    } else {
                        for (int q = 0; j0 + q < n; ++q) x |= (uint32_t)row[q] << (8 * q);
                    }
                }
#pragma unroll
                for (int q = 0; q < 4; ++q) v[q] = (v[q] << t) | ((x >> (8 * q)) & 0xffu);
            }
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (j0 + q < n) cb[j0 + q] = word_from_u64<W>(v[q]);
        }
    }
}

// CBr[i][J] = sum_j B[i][J(d+1)+j] Q^j.
template <typename W>
__global__ __launch_bounds__(kThreads) void pack_rows_fwd_kernel(int64_t k, int64_t n, int64_t nw,
                                                                  const uint8_t *__restrict__ B, int64_t ldb,
                                                                  W *__restrict__ CBr, int64_t ldcbr,
                                                                  uint32_t t, uint32_t d) {
    QMM_FOR_ROWS(i, k) {
        const uint8_t *b = B + i * ldb;
        QMM_FOR_COLS(J, nw) {
            const int64_t base = (int64_t)J * (d + 1);
            uint64_t w = 0;
            for (int32_t j = (int32_t)d; j >= 0; --j) {
                const int64_t c = base + j;
                w = (w << t) | (c < n ? (uint64_t)b[c] : 0ull);
            }
            CBr[i * ldcbr + J] = word_from_u64<W>(w);
        }
    }
}

// One thread per residue: which = 0 rows reversed, 1 columns forward, 2 rows forward.
template <typename W>
__global__ __launch_bounds__(kThreads) void unpack_kernel(int which, int64_t rows, int64_t cols,
                                                           const W *__restrict__ P, int64_t ldp,
                                                           uint8_t *__restrict__ out, int64_t ldo,
                                                           uint32_t t, uint32_t d) {
    const uint64_t qmask = (t >= 64) ? ~0ull : ((1ull << t) - 1);
    const uint32_t e = d + 1;
    QMM_FOR_ROWS(r, rows) {
        QMM_FOR_COLS(c, cols) {
            uint64_t w;
            uint32_t pos;
            if (which == 0) {  // residue (r, c) is digit d - s of word (r, c / (d+1))
                w = u64_from_word(P[r * ldp + (uint32_t)c / e]);
                pos = d - (uint32_t)c % e;
            } else if (which == 1) {  // residue (r, c) is digit s of word (r / (d+1), c)
                w = u64_from_word(P[(r / e) * ldp + c]);
                pos = (uint32_t)(r % e);
            } else {  // residue (r, c) is digit j of word (r, c / (d+1))
                w = u64_from_word(P[r * ldp + (uint32_t)c / e]);
                pos = (uint32_t)c % e;
            }
            out[r * ldo + c] = (uint8_t)((w >> (t * pos)) & qmask);
        }
    }
}

template <typename W>
__global__ __launch_bounds__(kThreads) void extract_kernel(int64_t m, int64_t n, const W *__restrict__ T,
                                                            int64_t ldt, uint8_t *__restrict__ C, int64_t ldc,
                                                            uint32_t td, uint64_t qmask, bool offset, uint32_t p,
                                                            double invp) {
    QMM_FOR_ROWS(i, m) {
        QMM_FOR_COLS(j, n) {
            const uint32_t c = qadic_digit<W>(T[i * ldt + j], offset, td, qmask);
            C[i * ldc + j] = (uint8_t)mod_u64(c, p, invp);
        }
    }
}

// REDQ on r = sum_{j<=d} c_j Q^j: s = floor(r/p) once; mu_j = (r >> tj) - p (s >> tj)
// equals floor(r/Q^j) mod p (since floor(floor(r/p)/Q^j) = floor(floor(r/Q^j)/p));
// c_j = floor(r/Q^j) - Q floor(r/Q^(j+1)) gives c_j mod p = (mu_j - (Q mod p) mu_{j+1}) mod p.
template <typename W>
__global__ __launch_bounds__(kThreads) void redq_kernel(int64_t m, int64_t n, int64_t nw,
                                                         const W *__restrict__ CC, int64_t ldcc,
                                                         uint8_t *__restrict__ C, int64_t ldc,
                                                         uint32_t t, uint32_t d, uint32_t p, double invp,
                                                         uint32_t qmodp) {
    QMM_FOR_ROWS(i, m) QMM_FOR_COLS(J, nw) {
        const uint64_t r = u64_from_word(CC[i * ldcc + J]);
        const uint64_t s = div_u64(r, p, invp);  // floor(r / p), the one division
        uint32_t mu_next = 0;  // mu_{d+1} = 0
        // walk j downwards so mu_{j+1} is at hand
        for (int32_t j = (int32_t)d; j >= 0; --j) {
            const uint32_t sh = t * (uint32_t)j;
            const uint32_t mu = (uint32_t)((r >> sh) - (uint64_t)p * (s >> sh));
            const uint64_t v = (uint64_t)mu + (uint64_t)qmodp * p - (uint64_t)qmodp * mu_next;
            const int64_t col = (int64_t)J * (d + 1) + j;
            if (col < n) C[i * ldc + col] = (uint8_t)mod_u64(v, p, invp);
            mu_next = mu;
        }
    }
}

__global__ __launch_bounds__(kThreads) void fill_u8_kernel(uint8_t *C, int64_t m, int64_t n, int64_t ldc,
                                                            uint8_t v) {
    QMM_FOR_ROWS(i, m) QMM_FOR_COLS(j, n) C[i * ldc + j] = v;
}

qmm_status row_too_long(int64_t cols) {
    return cols > INT32_MAX ? fail(QMM_EUNSUPPORTED, "rows longer than 2^31 entries are not supported") : QMM_OK;
}

qmm_status check_launch(const char *what) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(QMM_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
    return QMM_OK;
}

}  // namespace

qmm_status launch_pack_rows_rev(const qmm_plan &pl, int64_t m, int64_t k, const uint8_t *A, int64_t lda,
                                void *CA, int64_t ldca, void *stream) {
    const int64_t nw = words_for(k, pl.d);
    if (m * nw == 0) return QMM_OK;
    if (row_too_long(nw) != QMM_OK) return QMM_EUNSUPPORTED;
    hipStream_t s = (hipStream_t)stream;
    const bool aligned = (uintptr_t)A % 4 == 0 && lda % 4 == 0;
    if (aligned && pl.d + 1 <= 8) {
        const dim3 grid = grid2(m, ceil_div(nw, 4));
        auto go = [&](auto d1) {
            constexpr int D1 = decltype(d1)::value;
            if (pl.beta == 24)
                pack_rows_rev4_kernel<float, D1><<<grid, kThreads, 0, s>>>(m, k, nw, A, lda, (float *)CA, ldca, pl.t);
            else
                pack_rows_rev4_kernel<double, D1><<<grid, kThreads, 0, s>>>(m, k, nw, A, lda, (double *)CA, ldca, pl.t);
        };
        switch (pl.d + 1) {
        case 1: go(std::integral_constant<int, 1>{}); break;
        case 2: go(std::integral_constant<int, 2>{}); break;
        case 3: go(std::integral_constant<int, 3>{}); break;
        case 4: go(std::integral_constant<int, 4>{}); break;
        case 5: go(std::integral_constant<int, 5>{}); break;
        case 6: go(std::integral_constant<int, 6>{}); break;
        case 7: go(std::integral_constant<int, 7>{}); break;
        default: go(std::integral_constant<int, 8>{}); break;
        }
        return check_launch("pack_rows_rev4");
    }
    if (pl.beta == 24)
        pack_rows_rev_kernel<float><<<grid2(m, nw), kThreads, 0, s>>>(m, k, nw, A, lda, (float *)CA, ldca, pl.t, pl.d);
    else
        pack_rows_rev_kernel<double><<<grid2(m, nw), kThreads, 0, s>>>(m, k, nw, A, lda, (double *)CA, ldca, pl.t, pl.d);
    return check_launch("pack_rows_rev");
}

qmm_status launch_pack_cols_fwd(const qmm_plan &pl, int64_t k, int64_t n, const uint8_t *B, int64_t ldb,
                                void *CB, int64_t ldcb, void *stream) {
    const int64_t nw = words_for(k, pl.d);
    if (nw * n == 0) return QMM_OK;
    if (row_too_long(n) != QMM_OK) return QMM_EUNSUPPORTED;
    hipStream_t s = (hipStream_t)stream;
    if ((uintptr_t)B % 4 == 0 && ldb % 4 == 0) {
        const dim3 grid = grid2(nw, ceil_div(n, 4));
        if (pl.beta == 24)
            pack_cols_fwd4_kernel<float><<<grid, kThreads, 0, s>>>(k, n, nw, B, ldb, (float *)CB, ldcb, pl.t, pl.d);
        else
            pack_cols_fwd4_kernel<double><<<grid, kThreads, 0, s>>>(k, n, nw, B, ldb, (double *)CB, ldcb, pl.t, pl.d);
        return check_launch("pack_cols_fwd4");
    }
    if (pl.beta == 24)
        pack_cols_fwd_kernel<float><<<grid2(nw, n), kThreads, 0, s>>>(k, n, nw, B, ldb, (float *)CB, ldcb, pl.t, pl.d);
    else
        pack_cols_fwd_kernel<double><<<grid2(nw, n), kThreads, 0, s>>>(k, n, nw, B, ldb, (double *)CB, ldcb, pl.t, pl.d);
    return check_launch("pack_cols_fwd");
}

qmm_status launch_pack_rows_fwd(const qmm_plan &pl, int64_t k, int64_t n, const uint8_t *B, int64_t ldb,
                                void *CBr, int64_t ldcbr, void *stream) {
    const int64_t nw = words_for(n, pl.d);
    if (k * nw == 0) return QMM_OK;
    if (row_too_long(nw) != QMM_OK) return QMM_EUNSUPPORTED;
    hipStream_t s = (hipStream_t)stream;
    if (pl.beta == 24)
        pack_rows_fwd_kernel<float><<<grid2(k, nw), kThreads, 0, s>>>(k, n, nw, B, ldb, (float *)CBr, ldcbr, pl.t, pl.d);
    else
        pack_rows_fwd_kernel<double><<<grid2(k, nw), kThreads, 0, s>>>(k, n, nw, B, ldb, (double *)CBr, ldcbr, pl.t, pl.d);
    return check_launch("pack_rows_fwd");
}

qmm_status launch_unpack(const qmm_plan &pl, int which, int64_t rows, int64_t cols, const void *packed,
                         int64_t ldp, uint8_t *out, int64_t ldo, void *stream) {
    if (rows * cols == 0) return QMM_OK;
    if (row_too_long(cols) != QMM_OK) return QMM_EUNSUPPORTED;
    hipStream_t s = (hipStream_t)stream;
    if (pl.beta == 24)
        unpack_kernel<float><<<grid2(rows, cols), kThreads, 0, s>>>(which, rows, cols, (const float *)packed, ldp, out, ldo, pl.t, pl.d);
    else
        unpack_kernel<double><<<grid2(rows, cols), kThreads, 0, s>>>(which, rows, cols, (const double *)packed, ldp, out, ldo, pl.t, pl.d);
    return check_launch("unpack");
}

qmm_status launch_extract(const qmm_plan &pl, int64_t m, int64_t n, const void *T, int64_t ldt, uint8_t *C,
                          int64_t ldc, void *stream) {
    if (m * n == 0) return QMM_OK;
    if (row_too_long(n) != QMM_OK) return QMM_EUNSUPPORTED;
    hipStream_t s = (hipStream_t)stream;
    const uint64_t qmask = (1ull << pl.t) - 1;
    const bool offset = pl.regime == QMM_REGIME_OFFSET;
    const double invp = 1.0 / (double)pl.p;
    if (pl.beta == 24)
        extract_kernel<float><<<grid2(m, n), kThreads, 0, s>>>(m, n, (const float *)T, ldt, C, ldc, pl.t * pl.d, qmask, offset, pl.p, invp);
    else
        extract_kernel<double><<<grid2(m, n), kThreads, 0, s>>>(m, n, (const double *)T, ldt, C, ldc, pl.t * pl.d, qmask, offset, pl.p, invp);
    return check_launch("extract");
}

qmm_status launch_redq(const qmm_plan &pl, int64_t m, int64_t n, const void *CC, int64_t ldcc, uint8_t *C,
                       int64_t ldc, void *stream) {
    const int64_t nw = words_for(n, pl.d);
    if (m * nw == 0) return QMM_OK;
    if (row_too_long(nw) != QMM_OK) return QMM_EUNSUPPORTED;
    hipStream_t s = (hipStream_t)stream;
    const double invp = 1.0 / (double)pl.p;
    const uint32_t qmodp = (uint32_t)((1ull << pl.t) % pl.p);
    if (pl.beta == 24)
        redq_kernel<float><<<grid2(m, nw), kThreads, 0, s>>>(m, n, nw, (const float *)CC, ldcc, C, ldc, pl.t, pl.d, pl.p, invp, qmodp);
    else
        redq_kernel<double><<<grid2(m, nw), kThreads, 0, s>>>(m, n, nw, (const double *)CC, ldcc, C, ldc, pl.t, pl.d, pl.p, invp, qmodp);
    return check_launch("redq");
}

// Entries x >= p of a byte matrix (input validation): a grid-stride loop over rows
// (y) and 16-byte column segments (x); a segment is one vector load when the row
// is 16-byte aligned and the segment lies inside it, else byte loads.  Each byte
// of the loaded words is compared with p; then a wavefront sum and one atomic add
// per wavefront.
__device__ __forceinline__ uint32_t count_ge(uint32_t w, uint32_t p) {
    uint32_t c = 0;
#pragma unroll
    for (int b = 0; b < 4; ++b) c += ((w >> (8 * b)) & 0xffu) >= p ? 1u : 0u;
    return c;
}

__global__ __launch_bounds__(kThreads) void count_nonresidues_kernel(uint32_t p, int64_t rows, int64_t cols,
                                                                     const uint8_t *__restrict__ X, int64_t ldx,
                                                                     uint32_t *count) {
    uint32_t bad = 0;
    const int64_t segs = ceil_div(cols, 16);
    for (int64_t r = blockIdx.y; r < rows; r += gridDim.y) {
        const uint8_t *row = X + r * ldx;
        const bool aligned = ((uintptr_t)row & 15) == 0;
        for (int64_t sg = (int64_t)blockIdx.x * kThreads + threadIdx.x; sg < segs; sg += (int64_t)gridDim.x * kThreads) {
            const int64_t c0 = 16 * sg;
            if (aligned && c0 + 16 <= cols) {
                const uint4 v = *(const uint4 *)(row + c0);
                bad += count_ge(v.x, p) + count_ge(v.y, p) + count_ge(v.z, p) + count_ge(v.w, p);
            } else {
                for (int64_t c = c0; c < cols && c < c0 + 16; ++c) bad += row[c] >= p ? 1u : 0u;
            }
        }
    }
    for (int off = 32; off > 0; off >>= 1) bad += __shfl_down(bad, off, 64);
    if ((threadIdx.x & 63) == 0 && bad != 0) atomicAdd(count, bad);
}

__global__ void zero_u32_kernel(uint32_t *x) { *x = 0; }

qmm_status launch_count_nonresidues(uint32_t p, int64_t rows, int64_t cols, const uint8_t *X, int64_t ldx,
                                    uint32_t *count, void *stream) {
    zero_u32_kernel<<<1, 1, 0, (hipStream_t)stream>>>(count);
    if (rows == 0 || cols == 0) return check_launch("zero");
    const dim3 grid((unsigned)std::min<int64_t>(ceil_div(ceil_div(cols, 16), kThreads), 64),
                    (unsigned)std::min<int64_t>(rows, 4096));
    count_nonresidues_kernel<<<grid, kThreads, 0, (hipStream_t)stream>>>(p, rows, cols, X, ldx, count);
    return check_launch("count_nonresidues");
}

qmm_status launch_fill_u8(uint8_t *C, int64_t m, int64_t n, int64_t ldc, uint8_t v, void *stream) {
    if (m * n == 0) return QMM_OK;
    if (row_too_long(n) != QMM_OK) return QMM_EUNSUPPORTED;
    fill_u8_kernel<<<grid2(m, n), kThreads, 0, (hipStream_t)stream>>>(C, m, n, ldc, v);
    return check_launch("fill");
}

}  // namespace qmm
