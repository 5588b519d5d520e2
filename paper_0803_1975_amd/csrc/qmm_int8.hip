// INT8 path: centred residues on the int8 matrix cores with int32 accumulation.
//
// A residue x in [0, p-1] is replaced by x - p when x > (p-1)/2, so |x| <= p/2
// fits a signed byte for p <= 256 and k products of two centred residues stay in
// int32 while k (p/2)^2 < 2^31 (longer k is cut into blocks reduced mod p).
//
//   centre_transpose  B (k x n bytes) -> Bt (n x ldbt int8, k contiguous, zero
//                     padded to a multiple of 128): the int8 MFMA wants both
//                     operands contiguous along k.  HBM-bound, 128 x 128 tiles
//                     through LDS so reads and writes are both row-contiguous.
//   gemm_int8         C = (A_centred x Bt^T) mod p.  A is centred in registers on
//                     its way into LDS, four residues per 32-bit word.  MFMA
//                     i32_32x32x32_i8 (on gfx950 it sustains about 1.6x the
//                     rate of i32_16x16x64_i8), workgroups of 2 x 2 or 2 x 4 wavefronts,
//                     double-buffered LDS stages.  Two tile shapes: 256 x 256 with
//                     512 threads (2 x 4 wavefronts of 128 x 64) and 128-byte K
//                     stages (one workgroup per CU, 144 KB of LDS; each row of a
//                     stage is one 128-byte line) for products that fill the chip;
//                     128 x 128 with 256 threads (2 x 2 wavefronts of 64 x 64) and
//                     64-byte stages below that.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <type_traits>

#include "qmm_device.h"
#include "qmm_internal.h"

namespace qmm {
namespace {

typedef int ix4 __attribute__((ext_vector_type(4)));
typedef int ix8 __attribute__((ext_vector_type(8)));
typedef int ix16 __attribute__((ext_vector_type(16)));
typedef float fx16 __attribute__((ext_vector_type(16)));
typedef unsigned int ux2 __attribute__((ext_vector_type(2)));
typedef unsigned int ux4 __attribute__((ext_vector_type(4)));

// Transposed operand rows are padded to a multiple of the largest K stage.
constexpr int kBtAlign = 128;
static_assert(kBtAlign % kInt8KT == 0, "blocks must be whole stages");

// Centre four packed residues: x -> x - p where x > h = (p-1)/2.  With x <= p-1
// every byte of w + (127-h) stays below 256, so its top bit is exactly [x > h];
// adding (256-p) to the flagged bytes is x - p mod 256 (the int8 encoding) and
// cannot carry since x + 256 - p <= 255.
__device__ __forceinline__ uint32_t centre4(uint32_t w, uint32_t add_h, uint32_t neg_p) {
    const uint32_t flag = ((w + add_h) >> 7) & 0x01010101u;
    return w + flag * neg_p;
}

// Bt[n0 + c][k0 + r] = centred(B[k0 + r][n0 + c]) for a 128 (k) x 128 (n) tile:
// each thread reads 16 consecutive bytes of four B rows (vector loads when the
// row segments are aligned and whole, all four in flight together) into an LDS
// tile of 32-bit words.  Then thread t reads the word of columns 4 cg .. 4 cg + 3
// (cg = t % 32) in 16 consecutive k rows (k group t / 32), transposes the 16 x 4
// bytes in registers (4 x 4 blocks by byte permutes) and writes four 16-byte
// k-runs, one per column, into Bt.
constexpr int CT = 128;

// The four 16-byte row segments a thread of a 128 x 128 transposing tile reads: B
// rows k0 + r0 + 32 i, columns nn .. nn + 15 (bytes past k or n read as zero).
// B_VEC (B and ldb 16-byte aligned): whole segments are one 16-byte load each,
// and a segment cut by n (only in the last column tile) is read byte by byte.
// Otherwise every segment is a dword-aligned window (raw_issue_ptr), all four
// issued before the first is aligned, where byte loads would each wait for the one
// before.
template <bool B_VEC>
__device__ __forceinline__ void load_tile_segments(const uint8_t *__restrict__ B, int64_t ldb, int64_t k, int64_t n,
                                                   int64_t k0, int r0, int64_t nn, uint4 (&v)[4]) {
    if constexpr (B_VEC) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t kk = k0 + r0 + 32 * i;
            v[i] = make_uint4(0, 0, 0, 0);
            if (kk < k) {
                const uint8_t *src = B + kk * ldb + nn;
                if (nn + 16 <= n) {
                    v[i] = *(const uint4 *)src;
                } else {
                    uint32_t w[4] = {0, 0, 0, 0};
                    for (int b = 0; b < 16; ++b)
                        if (nn + b < n) w[b >> 2] |= (uint32_t)src[b] << (8 * (b & 3));
                    v[i] = make_uint4(w[0], w[1], w[2], w[3]);
                }
            }
        }
        return;
    }
    const uint8_t *end = B + (k - 1) * ldb + n;  // one past B's data
    uint32_t w[4][5];
    int32_t meta[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int64_t kk = k0 + r0 + 32 * i;
        v[i] = make_uint4(0, 0, 0, 0);
        meta[i] = 0;
        if (kk < k && nn < n) {
            raw_issue_ptr(w[i], meta[i], B + kk * ldb + nn, n - nn, end);
        }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        if (meta[i] != 0) {
            uint32_t o[4];
            raw_finish(w[i], meta[i], o);
            v[i] = make_uint4(o[0], o[1], o[2], o[3]);
        }
    }
}

template <bool B_VEC>
__global__ __launch_bounds__(256) void centre_transpose_kernel(int64_t k, int64_t n, const uint8_t *__restrict__ B,
                                                                int64_t ldb, int8_t *__restrict__ Bt, int64_t ldbt,
                                                                uint32_t add_h, uint32_t neg_p) {
    __shared__ uint32_t tile[CT][CT / 4 + 1];  // k rows x 128 column bytes, padded by one word
    const int64_t k0 = (int64_t)blockIdx.y * CT, n0 = (int64_t)blockIdx.x * CT;
    const int t = threadIdx.x;
    {
        const int seg = t & 7, r0 = t >> 3;  // 16-byte segment of a 128-byte row; rows r0 + 32 i
        const int64_t nn = n0 + 16 * seg;
        uint4 v[4];
        load_tile_segments<B_VEC>(B, ldb, k, n, k0, r0, nn, v);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            uint32_t *dst = &tile[r0 + 32 * i][4 * seg];
            dst[0] = centre4(v[i].x, add_h, neg_p);
            dst[1] = centre4(v[i].y, add_h, neg_p);
            dst[2] = centre4(v[i].z, add_h, neg_p);
            dst[3] = centre4(v[i].w, add_h, neg_p);
        }
    }
    __syncthreads();
    const int cg = t & 31, kg = t >> 5;  // columns 4 cg .. 4 cg + 3; k rows 16 kg .. 16 kg + 15
    uint32_t out[4][4];                  // [column q][k word d]
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        const uint32_t r0 = tile[16 * kg + 4 * d + 0][cg], r1 = tile[16 * kg + 4 * d + 1][cg];
        const uint32_t r2 = tile[16 * kg + 4 * d + 2][cg], r3 = tile[16 * kg + 4 * d + 3][cg];
        const uint32_t lo01 = __builtin_amdgcn_perm(r1, r0, 0x05010400u);  // r0b0 r1b0 r0b1 r1b1
        const uint32_t lo23 = __builtin_amdgcn_perm(r3, r2, 0x05010400u);
        const uint32_t hi01 = __builtin_amdgcn_perm(r1, r0, 0x07030602u);  // r0b2 r1b2 r0b3 r1b3
        const uint32_t hi23 = __builtin_amdgcn_perm(r3, r2, 0x07030602u);
        out[0][d] = __builtin_amdgcn_perm(lo23, lo01, 0x05040100u);
        out[1][d] = __builtin_amdgcn_perm(lo23, lo01, 0x07060302u);
        out[2][d] = __builtin_amdgcn_perm(hi23, hi01, 0x05040100u);
        out[3][d] = __builtin_amdgcn_perm(hi23, hi01, 0x07060302u);
    }
    // rows past k were loaded as zero (and centre4(0) = 0), so Bt's padding is zero
    const int64_t kk = k0 + 16 * kg;
    if (kk >= ldbt) return;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int64_t nn = n0 + 4 * cg + q;
        if (nn < n) *(uint4 *)(Bt + nn * ldbt + kk) = make_uint4(out[q][0], out[q][1], out[q][2], out[q][3]);
    }
}

// FP4 conversion.  Residue x (0 <= x < p <= 8) -> e2m1 code of centred(x), four
// at a time: the codes of x = 0..7 sit in the bytes of (lut_hi:lut_lo) and one byte
// permute looks all four up (selector bytes 0..7 pick those bytes).  Two words of
// codes (each code < 16, one per byte) pack into one word of eight nibbles,
// the lower k in the lower nibble.
__device__ __forceinline__ uint32_t fp4_codes(uint32_t x4, uint32_t lut_lo, uint32_t lut_hi) {
    return __builtin_amdgcn_perm(lut_hi, lut_lo, x4);
}
__device__ __forceinline__ uint32_t fp4_pack(uint32_t c_lo, uint32_t c_hi) {
    const uint32_t a = c_lo | (c_lo >> 4), b = c_hi | (c_hi >> 4);  // bytes 0 and 2 hold nibble pairs
    return __builtin_amdgcn_perm(b, a, 0x06040200u);
}

// A4 rows: residues 32 sg .. 32 sg + 31 of row r (zero past k) become the 16 bytes of
// codes at byte 16 sg of the packed row.
__device__ __forceinline__ void fp4_row_segment(int64_t r, int64_t sg, int64_t k, const uint8_t *__restrict__ A,
                                                int64_t lda, uint8_t *__restrict__ A4, int64_t lda4, uint32_t lut_lo,
                                                uint32_t lut_hi, int a_vec, const uint8_t *a_end) {
    const uint8_t *row = A + r * lda;
    const int64_t k0 = 32 * sg;
    uint32_t w[8];
    if (a_vec && k0 + 32 <= k) {
        const uint4 v0 = *(const uint4 *)(row + k0), v1 = *(const uint4 *)(row + k0 + 16);
        w[0] = v0.x; w[1] = v0.y; w[2] = v0.z; w[3] = v0.w;
        w[4] = v1.x; w[5] = v1.y; w[6] = v1.z; w[7] = v1.w;
    } else {
        // two dword-aligned windows (a_end: one past A's data), both issued first
        uint32_t x0[5], x1[5], o0[4], o1[4];
        int32_t m0, m1;
        raw_issue_ptr(x0, m0, row + k0, k - k0, a_end);
        raw_issue_ptr(x1, m1, row + k0 + 16, k - k0 - 16, a_end);
        raw_finish(x0, m0, o0);
        raw_finish(x1, m1, o1);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            w[i] = o0[i];
            w[4 + i] = o1[i];
        }
    }
    uint32_t o[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) o[i] = fp4_pack(fp4_codes(w[2 * i], lut_lo, lut_hi), fp4_codes(w[2 * i + 1], lut_lo, lut_hi));
    *(ux4 *)(A4 + r * lda4 + 16 * sg) = ux4{o[0], o[1], o[2], o[3]};
}

__global__ __launch_bounds__(256) void pack_fp4_rows_kernel(int64_t m, int64_t k, const uint8_t *__restrict__ A,
                                                            int64_t lda, uint8_t *__restrict__ A4, int64_t lda4,
                                                            uint32_t lut_lo, uint32_t lut_hi, int a_vec) {
    const int64_t segs = lda4 / 16;
    for (int64_t r = blockIdx.y; r < m; r += gridDim.y)
        for (int64_t sg = (int64_t)blockIdx.x * 256 + threadIdx.x; sg < segs; sg += (int64_t)gridDim.x * 256)
            fp4_row_segment(r, sg, k, A, lda, A4, lda4, lut_lo, lut_hi, a_vec, A + (m - 1) * lda + k);
}

// Bt4[n0 + c][(k0 + r) / 2] = code(B[k0 + r][n0 + c]) for the 128 (k) x 128 (n) tile
// (tx, ty): the loads, LDS tile and register transposes of centre_transpose_kernel,
// with the codes looked up on the way into LDS and each column's 16 k packed into 8
// bytes.  Every thread of the workgroup calls it (it holds a barrier).
template <bool B_VEC>
__device__ __forceinline__ void fp4_cols_tile(int64_t tx, int64_t ty, int64_t k, int64_t n,
                                              const uint8_t *__restrict__ B, int64_t ldb, uint8_t *__restrict__ Bt4,
                                              int64_t ldbt4, uint32_t lut_lo, uint32_t lut_hi,
                                              uint32_t (*tile)[CT / 4 + 1]) {
    const int64_t k0 = ty * CT, n0 = tx * CT;
    const int t = threadIdx.x;
    {
        const int seg = t & 7, r0 = t >> 3;
        const int64_t nn = n0 + 16 * seg;
        uint4 v[4];
        load_tile_segments<B_VEC>(B, ldb, k, n, k0, r0, nn, v);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            uint32_t *dst = &tile[r0 + 32 * i][4 * seg];
            dst[0] = fp4_codes(v[i].x, lut_lo, lut_hi);
            dst[1] = fp4_codes(v[i].y, lut_lo, lut_hi);
            dst[2] = fp4_codes(v[i].z, lut_lo, lut_hi);
            dst[3] = fp4_codes(v[i].w, lut_lo, lut_hi);
        }
    }
    __syncthreads();
    const int cg = t & 31, kg = t >> 5;
    uint32_t out[4][4];
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        const uint32_t r0 = tile[16 * kg + 4 * d + 0][cg], r1 = tile[16 * kg + 4 * d + 1][cg];
        const uint32_t r2 = tile[16 * kg + 4 * d + 2][cg], r3 = tile[16 * kg + 4 * d + 3][cg];
        const uint32_t lo01 = __builtin_amdgcn_perm(r1, r0, 0x05010400u);
        const uint32_t lo23 = __builtin_amdgcn_perm(r3, r2, 0x05010400u);
        const uint32_t hi01 = __builtin_amdgcn_perm(r1, r0, 0x07030602u);
        const uint32_t hi23 = __builtin_amdgcn_perm(r3, r2, 0x07030602u);
        out[0][d] = __builtin_amdgcn_perm(lo23, lo01, 0x05040100u);
        out[1][d] = __builtin_amdgcn_perm(lo23, lo01, 0x07060302u);
        out[2][d] = __builtin_amdgcn_perm(hi23, hi01, 0x05040100u);
        out[3][d] = __builtin_amdgcn_perm(hi23, hi01, 0x07060302u);
    }
    // rows past k were loaded as zero, whose code is 0, so Bt4's padding is zero
    const int64_t kb = (k0 + 16 * kg) / 2;  // packed byte offset of this thread's 16 k
    if (kb >= ldbt4) return;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int64_t nn = n0 + 4 * cg + q;
        if (nn < n)
            *(ux2 *)(Bt4 + nn * ldbt4 + kb) = ux2{fp4_pack(out[q][0], out[q][1]), fp4_pack(out[q][2], out[q][3])};
    }
}

template <bool B_VEC>
__global__ __launch_bounds__(256) void pack_fp4_cols_kernel(int64_t k, int64_t n, const uint8_t *__restrict__ B,
                                                            int64_t ldb, uint8_t *__restrict__ Bt4, int64_t ldbt4,
                                                            uint32_t lut_lo, uint32_t lut_hi) {
    __shared__ uint32_t tile[CT][CT / 4 + 1];
    fp4_cols_tile<B_VEC>(blockIdx.x, blockIdx.y, k, n, B, ldb, Bt4, ldbt4, lut_lo, lut_hi, tile);
}

// Both conversions of an FP4 product in one launch (two kernels this size each
// spend a good part of their time filling and draining the GPU): workgroups
// 0 .. a_blocks-1 pack A, 256 row segments each; the rest transpose B tiles.
struct Fp4PackArgs {
    int64_t m, n, k;
    const uint8_t *A;
    int64_t lda;
    uint8_t *A4;
    int64_t lda4;
    const uint8_t *B;
    int64_t ldb;
    uint8_t *Bt4;
    int64_t ldbt4;
    uint32_t lut_lo, lut_hi;
    int a_vec;
    int64_t a_blocks, b_tiles_x;
};
template <bool B_VEC>
__global__ __launch_bounds__(256) void pack_fp4_both_kernel(Fp4PackArgs g) {
    __shared__ uint32_t tile[CT][CT / 4 + 1];
    const int64_t blk = blockIdx.x;
    if (blk < g.a_blocks) {
        const int64_t segs = g.lda4 / 16;
        const int64_t idx = blk * 256 + threadIdx.x;
        if (idx < g.m * segs) {
            const int64_t r = idx / segs;
            fp4_row_segment(r, idx - r * segs, g.k, g.A, g.lda, g.A4, g.lda4, g.lut_lo, g.lut_hi, g.a_vec,
                            g.A + (g.m - 1) * g.lda + g.k);
        }
        return;
    }
    const int64_t tb = blk - g.a_blocks;
    fp4_cols_tile<B_VEC>(tb % g.b_tiles_x, tb / g.b_tiles_x, g.k, g.n, g.B, g.ldb, g.Bt4, g.ldbt4, g.lut_lo,
                         g.lut_hi, tile);
}

template <int BM, int BN>
__device__ __forceinline__ void tile_coords(int64_t m, int64_t n, int &tm, int &tn) {
    const int tiles_m = (int)ceil_div(m, BM), tiles_n = (int)ceil_div(n, BN);
    const int nb = gridDim.x;
    int bid = blockIdx.x;
    if ((nb & 7) == 0) bid = (bid & 7) * (nb >> 3) + (bid >> 3);
    constexpr int GROUP = 8;
    const int per_group = GROUP * tiles_n;
    const int group = bid / per_group;
    const int first_m = group * GROUP;
    const int gsize = min(tiles_m - first_m, GROUP);
    const int local = bid - group * per_group;
    tm = first_m + local % gsize;
    tn = local / gsize;
}

struct Int8Args {
    int64_t m, n, k;
    const uint8_t *A;
    int64_t lda;
    const int8_t *Bt;
    int64_t ldbt;
    uint8_t *C;
    int64_t ldc;
    int32_t kb_tiles;  // K stages per block (0 = unblocked)
    uint32_t p, add_h, neg_p;
    uint64_t magic;    // floor(2^64 / p) + 1
    uint32_t off;      // p floor(2^31 / p)
    uint32_t magic32;  // floor(2^32 / p)
    bool a_vec;        // A rows 16-byte aligned: vector loads allowed
    bool c_vec;        // C and ldc 4-byte aligned: whole tiles are stored as dwords
    int64_t kc;           // split K (gridDim.y > 1): bytes of k per chunk
    int64_t part_stride;  // split K: bytes between the chunks' partial outputs
};

// BM x BN output tile, WGM x WGN wavefronts, K stage of KT bytes.  Each wavefront
// owns a (BM/WGM) x (BN/WGN) sub-tile of 32 x 32 MFMA blocks (i32_32x32x32_i8:
// lane l holds 16 k-bytes of row l % 32 for k-chunk l / 32, and outputs
// D[8 (r/4) + 4 (l/32) + r % 4][l % 32] in register r).  Rows of both LDS stages
// are padded by 16 bytes: the 8 lanes that one LDS cycle serves then read 8
// consecutive rows on distinct bank groups.
// AVEC: every row of A is 16-byte aligned and k is a multiple of 16, so each
// 16-byte segment below k is one vector load; segments past k or rows past m
// load from a clamped, valid address and are zeroed by a select (no branches in
// the loop).  Otherwise each segment is a dword-aligned window, all of a stage's
// issued before any is aligned (byte loads would each wait for the one before).
// FP4: both operands are packed e2m1 codes (two k per byte, A already converted,
// g.k counts packed bytes), and each 16-byte fragment feeds the FP4 form of the
// MFMA, v_mfma_scale_f32_32x32x64_f8f6f4 with unit scales: 64 k per instruction
// into FP32 accumulators (lane l holds 32 codes of row l % 32 for k-half l / 32,
// in the same order for both operands; outputs as for the int8 form).
template <int BM, int BN, int KT, int WGM, int WGN, bool BLOCKED, bool AVEC, bool FP4>
__global__ __launch_bounds__(64 * WGM * WGN, (BM * BN * 4 >= 256 * 256 * WGM * WGN) ? 1 : 2) void gemm_int8_kernel(Int8Args g) {
    using AccT = typename std::conditional<FP4, fx16, ix16>::type;
    constexpr int NT = 64 * WGM * WGN;
    constexpr int PITCH = KT + 16;
    constexpr int WTM = BM / WGM, WTN = BN / WGN;
    constexpr int FM = WTM / 32, FN = WTN / 32;
    constexpr int SEGS = KT / 16;
    constexpr int A_LOADS = BM * SEGS / NT, B_LOADS = BN * SEGS / NT;
    static_assert(BM * SEGS % NT == 0 && BN * SEGS % NT == 0, "staging must divide evenly");
    static_assert(KT % 32 == 0 && WTM % 32 == 0 && WTN % 32 == 0, "whole MFMA blocks");
    __shared__ __attribute__((aligned(16))) uint8_t sA[2][BM * PITCH];
    __shared__ __attribute__((aligned(16))) uint8_t sB[2][BN * PITCH];

    if (gridDim.y > 1) {
        // one K chunk of a split product: its slice of A's and Bt's rows, and its own
        // partial output (the residue of the chunk's sum), combined afterwards
        const int64_t k0 = (int64_t)blockIdx.y * g.kc;
        g.A += k0;
        g.Bt += k0;
        g.C += (int64_t)blockIdx.y * g.part_stride;
        g.k = min(g.kc, g.k - k0);
    }
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave / WGN, wn = wave % WGN;
    int tm, tn;
    tile_coords<BM, BN>(g.m, g.n, tm, tn);
    const int64_t row0 = (int64_t)tm * BM, col0 = (int64_t)tn * BN;

    AccT acc[FM][FN];
#pragma unroll
    for (int mi = 0; mi < FM; ++mi)
#pragma unroll
        for (int ni = 0; ni < FN; ++ni) acc[mi][ni] = AccT{};

    // Staging: segment c = tid + NT i covers row c / SEGS, bytes 16 (c % SEGS) .. +15.
    // Row pointers and validity are fixed for the whole k loop.
    uint4 ra[A_LOADS], rb[B_LOADS];
    const uint8_t *a_ptr[A_LOADS];
    const int8_t *b_ptr[B_LOADS];
    bool a_ok[A_LOADS], b_ok[B_LOADS];
#pragma unroll
    for (int i = 0; i < A_LOADS; ++i) {
        const int c = tid + NT * i;
        const int64_t arow = row0 + c / SEGS;
        a_ok[i] = arow < g.m;
        a_ptr[i] = g.A + (a_ok[i] ? arow : 0) * g.lda + (c % SEGS) * 16;
    }
#pragma unroll
    for (int i = 0; i < B_LOADS; ++i) {
        const int c = tid + NT * i;
        const int64_t brow = col0 + c / SEGS;
        b_ok[i] = brow < g.n;
        b_ptr[i] = g.Bt + (b_ok[i] ? brow : 0) * g.ldbt + (c % SEGS) * 16;
    }
    const uint8_t *a_end = g.A + (g.m - 1) * g.lda + g.k;  // one past A's data
    auto load_stage = [&](int kt) {
        const int64_t k0 = (int64_t)kt * KT;
        if constexpr (!AVEC && !FP4) {
            // unaligned A: every window of the stage issued, then all aligned
            uint32_t aw[A_LOADS][5];
            int32_t am[A_LOADS];
#pragma unroll
            for (int i = 0; i < A_LOADS; ++i) {
                const int64_t kk = k0 + ((tid + NT * i) % SEGS) * 16;
                raw_issue_ptr(aw[i], am[i], a_ptr[i] + k0, a_ok[i] ? g.k - kk : 0, a_end);
            }
#pragma unroll
            for (int i = 0; i < A_LOADS; ++i) {
                uint32_t o[4];
                raw_finish(aw[i], am[i], o);
                ra[i] = make_uint4(o[0], o[1], o[2], o[3]);
            }
        }
#pragma unroll
        for (int i = 0; i < A_LOADS; ++i) {
            const int64_t kk = k0 + ((tid + NT * i) % SEGS) * 16;
            if constexpr (FP4) {
                // packed rows are zero padded to whole stages; rows past m are clamped
                // to row 0 and only reach outputs that are not stored
                ra[i] = *(const uint4 *)(a_ptr[i] + k0);
            } else if constexpr (AVEC) {
                // a segment past k (or a row past m) reads A's first 16 bytes instead
                const bool ok = a_ok[i] && kk < g.k;
                const uint4 v = *(const uint4 *)(ok ? a_ptr[i] + k0 : g.A);
                ra[i] = ok ? v : make_uint4(0, 0, 0, 0);
            }
        }
#pragma unroll
        for (int i = 0; i < B_LOADS; ++i) {
            // Bt rows are zero-padded to ldbt (a multiple of the stage), so whole stages are in bounds.
            const uint4 v = *(const uint4 *)(b_ptr[i] + k0);
            if constexpr (FP4)
                rb[i] = v;  // rows past n (clamped to row 0) only reach outputs that are not stored
            else
                rb[i] = b_ok[i] ? v : make_uint4(0, 0, 0, 0);
        }
    };
    // The loads of a stage are only consumed here, after the MFMAs of the previous
    // stage, so their latency hides behind that work; A is centred on the way in.
    auto store_stage = [&](int buf) {
#pragma unroll
        for (int i = 0; i < A_LOADS; ++i) {
            const int c = tid + NT * i;
            uint4 v = ra[i];
            if constexpr (!FP4) {
                v.x = centre4(v.x, g.add_h, g.neg_p);
                v.y = centre4(v.y, g.add_h, g.neg_p);
                v.z = centre4(v.z, g.add_h, g.neg_p);
                v.w = centre4(v.w, g.add_h, g.neg_p);
            }
            *(uint4 *)&sA[buf][(c / SEGS) * PITCH + (c % SEGS) * 16] = v;
        }
#pragma unroll
        for (int i = 0; i < B_LOADS; ++i) {
            const int c = tid + NT * i;
            *(uint4 *)&sB[buf][(c / SEGS) * PITCH + (c % SEGS) * 16] = rb[i];
        }
    };

    const int ntiles = (int)ceil_div(g.k, KT);
    load_stage(0);
    store_stage(0);
    __syncthreads();
    for (int kt = 0; kt < ntiles; ++kt) {
        const int buf = kt & 1;
        if (kt + 1 < ntiles) load_stage(kt + 1);
        // Fragments of k-step ks+1 are read from LDS while the MFMAs of k-step ks run.
        ix4 af[2][FM], bf[2][FN];
        auto read_frags = [&](int ks, int slot) {
#pragma unroll
            for (int ni = 0; ni < FN; ++ni)
                bf[slot][ni] = *(const ix4 *)&sB[buf][(wn * WTN + ni * 32 + (lane & 31)) * PITCH + ks * 32 + 16 * (lane >> 5)];
#pragma unroll
            for (int mi = 0; mi < FM; ++mi)
                af[slot][mi] = *(const ix4 *)&sA[buf][(wm * WTM + mi * 32 + (lane & 31)) * PITCH + ks * 32 + 16 * (lane >> 5)];
        };
        read_frags(0, 0);
#pragma unroll
        for (int ks = 0; ks < KT / 32; ++ks) {
            const int cur = ks & 1;
            if (ks + 1 < KT / 32) read_frags(ks + 1, cur ^ 1);
#pragma unroll
            for (int mi = 0; mi < FM; ++mi)
#pragma unroll
                for (int ni = 0; ni < FN; ++ni)
                    if constexpr (FP4) {
                        const ix4 a = af[cur][mi], b = bf[cur][ni];
                        acc[mi][ni] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(
                            ix8{a.x, a.y, a.z, a.w, 0, 0, 0, 0}, ix8{b.x, b.y, b.z, b.w, 0, 0, 0, 0}, acc[mi][ni],
                            4, 4, 0, 127, 0, 127);  // e2m1 x e2m1, scales 2^(127-127) = 1
                    } else {
                        acc[mi][ni] = __builtin_amdgcn_mfma_i32_32x32x32_i8(af[cur][mi], bf[cur][ni], acc[mi][ni], 0, 0, 0);
                    }
            // Interleave: one MFMA, then one of the next k-step's LDS reads, so the
            // reads' latency hides behind the matrix core instead of stalling it.
            if (ks + 1 < KT / 32) {
#pragma unroll
                for (int x = 0; x < FM + FN; ++x) {
                    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
                    __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
                }
                if constexpr (FM * FN > FM + FN) __builtin_amdgcn_sched_group_barrier(0x008, FM * FN - (FM + FN), 0);
            }
        }
        if constexpr (BLOCKED) {
            if ((kt + 1) % g.kb_tiles == 0 && kt + 1 < ntiles) {
#pragma unroll
                for (int mi = 0; mi < FM; ++mi)
#pragma unroll
                    for (int ni = 0; ni < FN; ++ni)
#pragma unroll
                        for (int r = 0; r < 16; ++r) {
                            if constexpr (FP4)  // an exact integer below 2^24 in magnitude
                                acc[mi][ni][r] = (float)mod_u32_m32((uint32_t)(int32_t)acc[mi][ni][r] + g.off, g.p, g.magic32);
                            else
                                acc[mi][ni][r] = (int)mod_u32_m32((uint32_t)acc[mi][ni][r] + g.off, g.p, g.magic32);
                        }
            }
        }
        if (kt + 1 < ntiles) {
            store_stage(buf ^ 1);
            __syncthreads();
        }
    }

    if (g.c_vec && row0 + BM <= g.m && col0 + BN <= g.n) {
        // Whole tile: registers 4q .. 4q+3 of lane l are rows R .. R+3 of column l % 32
        // (R = 8q + 4 (l / 32)); packed into a dword and transposed across the lane's
        // quad, they become 4 consecutive bytes of row R + (l % 4), one dword store.
        const int j = lane & 3;
        uint8_t *cbase = g.C + (row0 + wm * WTM + 4 * (lane >> 5) + j) * g.ldc + col0 + wn * WTN + (lane & 31) - j;
#pragma unroll
        for (int mi = 0; mi < FM; ++mi)
#pragma unroll
            for (int ni = 0; ni < FN; ++ni)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    uint32_t w = 0;
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        w |= mod_u32_m32((uint32_t)(int32_t)acc[mi][ni][4 * q + i] + g.off, g.p, g.magic32) << (8 * i);
                    w = quad_transpose_bytes(w, j);
                    *(uint32_t *)(cbase + (int64_t)(mi * 32 + 8 * q) * g.ldc + ni * 32) = w;
                }
        return;
    }
#pragma unroll
    for (int mi = 0; mi < FM; ++mi)
#pragma unroll
        for (int ni = 0; ni < FN; ++ni)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int64_t row = row0 + wm * WTM + mi * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                const int64_t col = col0 + wn * WTN + ni * 32 + (lane & 31);
                if (row < g.m && col < g.n)
                    g.C[row * g.ldc + col] = (uint8_t)mod_i32_magic((int32_t)acc[mi][ni][r], g.p, g.magic, g.off);
            }
}

// Both operands as centred int8 rows (A as Ac from the centring pass, B as Bt), each
// row zero padded to its leading dimension (a multiple of 128 bytes, at least k), so
// every 128-byte K stage of a row is in bounds.  256 x 256 output tile, WGM x WGN
// wavefronts; the launch uses 2 x 4 wavefronts of 128 x 64 (4 x 2 blocks of
// i32_32x32x32_i8, two wavefronts per SIMD: six fragment reads per eight MFMAs,
// against four per four for 16 wavefronts of 64 x 64, which measured 4-6 % slower).
// The stages go from HBM straight into LDS (global_load_lds_dwordx4: no staging
// registers, no LDS store instructions, no VALU), two buffers of 64 KB.
// LDS layout of an operand's stage: 256 rows of 128 bytes, no padding; 16-byte chunk
// c of row r sits at position c ^ swz(r), swz(r) = (r % 8) ^ ((r / 8) % 2).  A
// fragment read (lane l: row base + l % 32, chunk 2 ks + l / 32) then touches 8
// distinct positions on any 8 consecutive rows and, on 16 consecutive rows, distinct
// positions among the rows of each parity, so it is free of bank conflicts whether
// the LDS serves 8 or 16 lanes of a 16-byte read per cycle.  A direct load writes
// 1 KB (8 rows) per instruction, lane j at bytes 16 j, so lane j reads chunk
// (j % 8) ^ swz(its row) of row j / 8 of the block.
// Schedule: stage kt computes from buffer kt % 2.  The fragments of k-step ks + 1
// are read during k-step ks's MFMAs; the last k-step reads the next stage's first
// fragments from the other buffer.  One barrier per stage, after the MFMAs of the
// second-to-last k-step, preceded by a wait for this wavefront's direct loads (the
// next stage's, issued a stage earlier) and its LDS reads: after it, the next stage
// is complete in LDS and every read of this stage's buffer is done, so the last
// k-step issues the loads of stage kt + 2 into this buffer.  The MFMAs after a
// barrier never wait on LDS: their fragments are already in registers.
template <bool BLOCKED, int WGM, int WGN>
__global__ __launch_bounds__(64 * WGM * WGN, 1) void gemm_int8_direct_kernel(Int8Args g) {
    constexpr int BM = 256, BN = 256, KT = 128, KS = KT / 32;
    constexpr int WAVES = WGM * WGN, WTM = BM / WGM, WTN = BN / WGN, FM = WTM / 32, FN = WTN / 32;
    constexpr int BLK = 32 / WAVES;  // 8-row blocks of each operand's stage per wavefront
    constexpr int STAGE = BM * KT;
    __shared__ __attribute__((aligned(1024))) uint8_t lds[2][2][STAGE];  // [buffer][A, B]

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave / WGN, wn = wave % WGN;
    int tm, tn;
    tile_coords<BM, BN>(g.m, g.n, tm, tn);
    const int64_t row0 = (int64_t)tm * BM, col0 = (int64_t)tn * BN;

    // Direct loads: wavefront w fills blocks q = BLK w + i (i < BLK, rows 8 q ..
    // 8 q + 7) of each operand's stage.  Rows past m (n) read row m - 1 (n - 1); they
    // only reach outputs that are not stored.
    const int8_t *a_src[BLK], *b_src[BLK];
#pragma unroll
    for (int i = 0; i < BLK; ++i) {
        const int q = BLK * wave + i, r = 8 * q + (lane >> 3);
        const int chunk = (lane & 7) ^ (r & 7) ^ ((r >> 3) & 1);
        const int64_t ar = min(row0 + r, g.m - 1), br = min(col0 + r, g.n - 1);
        a_src[i] = (const int8_t *)g.A + ar * g.lda + 16 * chunk;
        b_src[i] = g.Bt + br * g.ldbt + 16 * chunk;
    }
    auto issue = [&](int kt, int b) {
        const int64_t k0 = (int64_t)kt * KT;
#pragma unroll
        for (int i = 0; i < BLK; ++i) {
            __builtin_amdgcn_global_load_lds((const void *)(a_src[i] + k0),
                                             (__attribute__((address_space(3))) void *)&lds[b][0][(BLK * wave + i) * 1024],
                                             16, 0, 0);
            __builtin_amdgcn_global_load_lds((const void *)(b_src[i] + k0),
                                             (__attribute__((address_space(3))) void *)&lds[b][1][(BLK * wave + i) * 1024],
                                             16, 0, 0);
        }
    };

    ix16 acc[FM][FN];
#pragma unroll
    for (int mi = 0; mi < FM; ++mi)
#pragma unroll
        for (int ni = 0; ni < FN; ++ni) acc[mi][ni] = ix16{};

    // Fragment rows are 32 x + l % 32, so swz(row) = (l % 8) ^ ((l / 8) % 2), and the
    // chunk 2 ks + l / 32 sits at position (2 ks) ^ (l / 32) ^ swz.
    const int swz = (lane & 7) ^ ((lane >> 3) & 1) ^ (lane >> 5);
    const int a_row = (wm * WTM + (lane & 31)) * KT, b_row = (wn * WTN + (lane & 31)) * KT;
    ix4 af[2][FM], bf[2][FN];
    auto read_frags = [&](int b, int ks, int slot) {
        const int co = 16 * ((2 * ks) ^ swz);
#pragma unroll
        for (int ni = 0; ni < FN; ++ni) bf[slot][ni] = *(const ix4 *)&lds[b][1][b_row + ni * 32 * KT + co];
#pragma unroll
        for (int mi = 0; mi < FM; ++mi) af[slot][mi] = *(const ix4 *)&lds[b][0][a_row + mi * 32 * KT + co];
    };

    const int ntiles = (int)ceil_div(g.k, KT);
    issue(0, 0);
    if (ntiles > 1) issue(1, 1);
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    read_frags(0, 0, 0);
    for (int kt = 0; kt < ntiles; ++kt) {
        const int buf = kt & 1;
        const bool more = kt + 1 < ntiles;
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            const int cur = ks & 1;
            if (ks == KS - 1 && kt + 2 < ntiles) issue(kt + 2, buf);
            // on the last stage the other buffer's reads are not used
            read_frags(ks + 1 < KS ? buf : buf ^ 1, (ks + 1) % KS, cur ^ 1);
#pragma unroll
            for (int mi = 0; mi < FM; ++mi)
#pragma unroll
                for (int ni = 0; ni < FN; ++ni)
                    acc[mi][ni] = __builtin_amdgcn_mfma_i32_32x32x32_i8(af[cur][mi], bf[cur][ni], acc[mi][ni], 0, 0, 0);
#pragma unroll
            for (int x = 0; x < FM + FN; ++x) {
                __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
                __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
            }
            if constexpr (FM * FN > FM + FN) __builtin_amdgcn_sched_group_barrier(0x008, FM * FN - (FM + FN), 0);
            if (ks == KS - 2 && more) {
                asm volatile("s_waitcnt vmcnt(0) lgkmcnt(0)" ::: "memory");
                __syncthreads();
            }
        }
        if constexpr (BLOCKED) {
            if ((kt + 1) % g.kb_tiles == 0 && more) {
#pragma unroll
                for (int mi = 0; mi < FM; ++mi)
#pragma unroll
                    for (int ni = 0; ni < FN; ++ni)
#pragma unroll
                        for (int r = 0; r < 16; ++r)
                            acc[mi][ni][r] = (int)mod_u32_m32((uint32_t)acc[mi][ni][r] + g.off, g.p, g.magic32);
            }
        }
    }

    if (g.c_vec && row0 + BM <= g.m && col0 + BN <= g.n) {
        // Whole tile: registers 4q .. 4q+3 of lane l are rows R .. R+3 of column l % 32
        // (R = 8q + 4 (l / 32)); packed into a dword and transposed across the lane's
        // quad, they become 4 consecutive bytes of row R + (l % 4), one dword store.
        const int j = lane & 3;
        uint8_t *cbase = g.C + (row0 + wm * WTM + 4 * (lane >> 5) + j) * g.ldc + col0 + wn * WTN + (lane & 31) - j;
#pragma unroll
        for (int mi = 0; mi < FM; ++mi)
#pragma unroll
            for (int ni = 0; ni < FN; ++ni)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    uint32_t w = 0;
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        w |= mod_u32_m32((uint32_t)acc[mi][ni][4 * q + i] + g.off, g.p, g.magic32) << (8 * i);
                    w = quad_transpose_bytes(w, j);
                    *(uint32_t *)(cbase + (int64_t)(mi * 32 + 8 * q) * g.ldc + ni * 32) = w;
                }
        return;
    }
#pragma unroll
    for (int mi = 0; mi < FM; ++mi)
#pragma unroll
        for (int ni = 0; ni < FN; ++ni)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int64_t row = row0 + wm * WTM + mi * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                const int64_t col = col0 + wn * WTN + ni * 32 + (lane & 31);
                if (row < g.m && col < g.n)
                    g.C[row * g.ldc + col] = (uint8_t)mod_i32_magic((int32_t)acc[mi][ni][r], g.p, g.magic, g.off);
            }
}

qmm_status check_launch(const char *what) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(QMM_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
    return QMM_OK;
}

void centre_consts(uint32_t p, uint32_t &add_h, uint32_t &neg_p) {
    const uint32_t h = (p - 1) / 2;
    add_h = (127u - h) * 0x01010101u;
    neg_p = (256u - p) & 0xffu;
}

// A small INT8 product in one launch: one 256-thread workgroup per 64 x 64 tile of C
// (2 x 2 wavefronts, one i32_32x32x32_i8 block each), 64-byte K stages.  A's rows
// are centred on their way into LDS; B's rows are centred and stored as they are
// (k-major), and each wavefront reads its B fragments with the gfx950 LDS
// transpose load, so the product needs no conversion launch and no workspace.
// Unblocked plans only (k (p/2)^2 stays in int32).
//
// ds_read_b64_tr_b8 (measured with an in-bounds probe): within each group of 16
// lanes, lane i receives byte i of the 8 x 16 byte block whose row b is the 8 bytes
// at lane 2b's address followed by the 8 bytes at lane 2b+1's.  So if lane 2b + c of
// group g points at k-row k0 + b and columns n0 + 8c, lane i of the group gets the
// 8 bytes of column n0 + i from k-rows k0 .. k0 + 7: the MFMA B operand's order.
struct SmallInt8Args {
    int64_t m, n, k;
    const uint8_t *A;
    int64_t lda;
    const uint8_t *B;
    int64_t ldb;
    uint8_t *C;
    int64_t ldc;
    int32_t tiles_n;
    uint32_t p, add_h, neg_p, off, magic32;
};
constexpr int SM_T = 64, SM_KT = 64, SM_PITCH = SM_KT + 16, SM_BPITCH = SM_T + 16;
typedef int v2i __attribute__((ext_vector_type(2)));

// 16 bytes of row `row` of X from column c0 (zero past rows or cols), as four words:
// one 16-byte load when they are whole and aligned, byte loads otherwise.
__device__ __forceinline__ void load16(const uint8_t *__restrict__ X, int64_t ld, int64_t rows, int64_t cols,
                                       int64_t row, int64_t c0, uint32_t w[4]) {
    w[0] = w[1] = w[2] = w[3] = 0;
    if (row >= rows || c0 >= cols) return;
    const uint8_t *src = X + row * ld + c0;
    if (c0 + 16 <= cols && ((uintptr_t)src & 15) == 0) {
        const uint4 v = *(const uint4 *)src;
        w[0] = v.x;
        w[1] = v.y;
        w[2] = v.z;
        w[3] = v.w;
        return;
    }
    for (int b = 0; b < 16; ++b)
        if (c0 + b < cols) w[b >> 2] |= (uint32_t)src[b] << (8 * (b & 3));
}

// WINDOWED: for operands with rows that are not whole aligned 16-byte segments;
// both stage loads go out through raw_issue32 before either is waited for (the
// byte loads of load16 would each wait for the one before).
template <bool WINDOWED>
__global__ __launch_bounds__(256) void small_int8_kernel(SmallInt8Args g) {
    __shared__ __attribute__((aligned(16))) uint8_t sA[SM_T * SM_PITCH];
    __shared__ __attribute__((aligned(16))) uint8_t sB[SM_KT * SM_BPITCH];  // rows: k, as B is stored
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int64_t row0 = (int64_t)(blockIdx.x / (uint32_t)g.tiles_n) * SM_T;
    const int64_t col0 = (int64_t)(blockIdx.x % (uint32_t)g.tiles_n) * SM_T;
    const int r = tid >> 2, seg = tid & 3;  // staging: row r, bytes 16 seg .. 16 seg + 15
    const uint32_t a_size = (uint32_t)((g.m - 1) * g.lda + g.k), b_size = (uint32_t)((g.k - 1) * g.ldb + g.n);
    ix16 acc = ix16{};
    for (int64_t k0 = 0; k0 < g.k; k0 += SM_KT) {
        uint32_t wa[4], wb[4];
        if constexpr (WINDOWED) {
            uint32_t xa[5], xb[5];
            int32_t ma, mb;
            const int64_t ar = row0 + r, ac = k0 + 16 * seg, bk = k0 + r, bc = col0 + 16 * seg;
            raw_issue32(xa, ma, g.A, (uint32_t)(ar * g.lda + ac), ar < g.m ? (int32_t)min(g.k - ac, (int64_t)16) : 0,
                        a_size);
            raw_issue32(xb, mb, g.B, (uint32_t)(bk * g.ldb + bc), bk < g.k ? (int32_t)min(g.n - bc, (int64_t)16) : 0,
                        b_size);
            raw_finish(xa, ma, wa);
            raw_finish(xb, mb, wb);
        } else {
            load16(g.A, g.lda, g.m, g.k, row0 + r, k0 + 16 * seg, wa);       // A row, 16 k
            load16(g.B + col0, g.ldb, g.k, g.n - col0, k0 + r, 16 * seg, wb);  // B k-row, 16 n
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            wa[i] = centre4(wa[i], g.add_h, g.neg_p);
            wb[i] = centre4(wb[i], g.add_h, g.neg_p);
        }
        *(uint4 *)&sA[r * SM_PITCH + 16 * seg] = make_uint4(wa[0], wa[1], wa[2], wa[3]);
        *(uint4 *)&sB[r * SM_BPITCH + 16 * seg] = make_uint4(wb[0], wb[1], wb[2], wb[3]);
        __syncthreads();
        // B fragment of lane l: column wn 32 + l % 32, k-bytes 16 (l / 32) .. + 15 of the
        // k-step, as two transpose loads of 8 k each (group g = l / 16, lane 2b + c of it)
        const int g = lane >> 4, sl = lane & 15;
        const int b_off = (16 * (g >> 1) + (sl >> 1)) * SM_BPITCH + wn * 32 + 16 * (g & 1) + 8 * (sl & 1);
#pragma unroll
        for (int ks = 0; ks < SM_KT / 32; ++ks) {
            const ix4 a = *(const ix4 *)&sA[(wm * 32 + (lane & 31)) * SM_PITCH + ks * 32 + 16 * (lane >> 5)];
            const uint8_t *bp = &sB[b_off + ks * 32 * SM_BPITCH];
            const v2i b0 = __builtin_amdgcn_ds_read_tr8_b64_v2i32((__attribute__((address_space(3))) v2i *)bp);
            const v2i b1 = __builtin_amdgcn_ds_read_tr8_b64_v2i32(
                (__attribute__((address_space(3))) v2i *)(bp + 8 * SM_BPITCH));
            acc = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, ix4{b0.x, b0.y, b1.x, b1.y}, acc, 0, 0, 0);
        }
        __syncthreads();
    }
    // register q holds D[8 (q/4) + 4 (l/32) + q % 4][l % 32] of this wavefront's block
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int64_t row = row0 + wm * 32 + 8 * (q >> 2) + 4 * (lane >> 5) + (q & 3);
        const int64_t col = col0 + wn * 32 + (lane & 31);
        if (row < g.m && col < g.n)
            g.C[row * g.ldc + col] = (uint8_t)mod_u32_m32((uint32_t)acc[q] + g.off, g.p, g.magic32);
    }
}

}  // namespace

qmm_status launch_gemm_int8_small(const qmm_plan &pl, int64_t m, int64_t n, int64_t k, const uint8_t *A,
                                  int64_t lda, const uint8_t *B, int64_t ldb, uint8_t *C, int64_t ldc,
                                  void *stream) {
    if (m == 0 || n == 0) return QMM_OK;
    if (pl.path != QMM_PATH_INT8 || pl.k_block < k || pl.p > 256)
        return fail(QMM_EUNSUPPORTED, "the one-launch INT8 kernel takes unblocked INT8 plans");
    SmallInt8Args g{};
    g.m = m;
    g.n = n;
    g.k = k;
    g.A = A;
    g.lda = lda;
    g.B = B;
    g.ldb = ldb;
    g.C = C;
    g.ldc = ldc;
    g.p = pl.p;
    centre_consts(pl.p, g.add_h, g.neg_p);
    g.off = pl.p * ((1u << 31) / pl.p);
    g.magic32 = (uint32_t)((1ull << 32) / pl.p);
    const int64_t tiles_m = ceil_div(m, SM_T), tiles_n = ceil_div(n, SM_T);
    if (tiles_m * tiles_n > INT32_MAX) return fail(QMM_EUNSUPPORTED, "too many tiles for the one-launch INT8 kernel");
    g.tiles_n = (int32_t)tiles_n;
    // whole aligned 16-byte row segments everywhere: plain 16-byte loads; otherwise
    // the windowed loads, whose 32-bit offsets need data of at most kRawSpan bytes
    const bool aligned = lda % 16 == 0 && ldb % 16 == 0 && k % 16 == 0 && n % 16 == 0 &&
                         (uintptr_t)A % 16 == 0 && (uintptr_t)B % 16 == 0;
    const bool windowed = !aligned && (m - 1) * lda + k <= kRawSpan && (k - 1) * ldb + n <= kRawSpan;
    const dim3 grid((unsigned)(tiles_m * tiles_n));
    if (windowed)
        small_int8_kernel<true><<<grid, 256, 0, (hipStream_t)stream>>>(g);
    else
        small_int8_kernel<false><<<grid, 256, 0, (hipStream_t)stream>>>(g);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? QMM_OK : fail(QMM_EDEVICE, std::string("small_int8_kernel: ") + hipGetErrorString(e));
}

// Codes of the residues 0..7 (centred, then e2m1: magnitudes 0, 1, 2, 3, 4 are the
// codes 0, 2, 4, 5, 6, sign bit 8), bytes 0..3 in lo and 4..7 in hi; residues >= p
// (not valid input) get code 0.
void fp4_lut(uint32_t p, uint32_t &lo, uint32_t &hi) {
    static const uint32_t mag_code[5] = {0, 2, 4, 5, 6};
    uint64_t lut = 0;
    for (uint32_t x = 0; x < 8 && x < p; ++x) {
        const int32_t c = x > (p - 1) / 2 ? (int32_t)x - (int32_t)p : (int32_t)x;
        const uint32_t code = mag_code[c < 0 ? -c : c] | (c < 0 ? 8u : 0u);
        lut |= (uint64_t)code << (8 * x);
    }
    lo = (uint32_t)lut;
    hi = (uint32_t)(lut >> 32);
}

// k rounded up to the stage alignment; strides that are multiples of 2 KiB get one
// more 128-byte line (rows of Bt at such strides crowd fewer HBM channels: the
// conversion writes at n = k = 16384 run 1.2x faster with the extra line).
int64_t int8_bt_ld(int64_t k) {
    const int64_t r = ceil_div(k < 1 ? 1 : k, kBtAlign) * kBtAlign;
    return r % 2048 == 0 ? r + kBtAlign : r;
}

namespace {
// Ac[i][16 s .. 16 s + 15] = centred(A[i][16 s .. 16 s + 15]), zero past k: one
// thread per 16-byte segment of Ac, read as a dword-aligned window of A (rows of A
// may start anywhere) and stored as one 16-byte store.
__global__ __launch_bounds__(256) void centre_rows_kernel(int64_t m, int64_t k, const uint8_t *__restrict__ A,
                                                           int64_t lda, int8_t *__restrict__ Ac, int64_t ldac,
                                                           uint32_t add_h, uint32_t neg_p) {
    const int64_t segs = ldac / 16;
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= m * segs) return;
    const int64_t r = idx / segs, s = idx - r * segs;
    uint32_t w[5], o[4] = {0, 0, 0, 0};
    int32_t meta = 0;
    const int64_t c0 = 16 * s;
    if (c0 < k) raw_issue_ptr(w, meta, A + r * lda + c0, k - c0, A + (m - 1) * lda + k);
    if (meta != 0) raw_finish(w, meta, o);
    *(uint4 *)(Ac + r * ldac + c0) = make_uint4(centre4(o[0], add_h, neg_p), centre4(o[1], add_h, neg_p),
                                               centre4(o[2], add_h, neg_p), centre4(o[3], add_h, neg_p));
}
}  // namespace

qmm_status launch_centre_rows(const qmm_plan &pl, int64_t m, int64_t k, const uint8_t *A, int64_t lda, int8_t *Ac,
                              int64_t ldac, void *stream) {
    if (m == 0) return QMM_OK;
    uint32_t add_h, neg_p;
    centre_consts(pl.p, add_h, neg_p);
    const int64_t blocks = ceil_div(m * (ldac / 16), 256);
    if (blocks > INT32_MAX) return fail(QMM_EUNSUPPORTED, "centre_rows grid too large");
    centre_rows_kernel<<<(unsigned)blocks, 256, 0, (hipStream_t)stream>>>(m, k, A, lda, Ac, ldac, add_h, neg_p);
    return check_launch("centre_rows");
}

qmm_status launch_centre_transpose(const qmm_plan &pl, int64_t k, int64_t n, const uint8_t *B, int64_t ldb,
                                   int8_t *Bt, int64_t ldbt, void *stream) {
    if (n == 0) return QMM_OK;
    uint32_t add_h, neg_p;
    centre_consts(pl.p, add_h, neg_p);
    const dim3 grid((unsigned)ceil_div(n, CT), (unsigned)ceil_div(ldbt, CT));
    if (((uintptr_t)B % 16 == 0) && (ldb % 16 == 0))
        centre_transpose_kernel<true><<<grid, 256, 0, (hipStream_t)stream>>>(k, n, B, ldb, Bt, ldbt, add_h, neg_p);
    else
        centre_transpose_kernel<false><<<grid, 256, 0, (hipStream_t)stream>>>(k, n, B, ldb, Bt, ldbt, add_h, neg_p);
    return check_launch("centre_transpose");
}

namespace {
template <int BM, int BN, int KT, int WGM, int WGN>
qmm_status run_int8(const Int8Args &g, bool blocked, hipStream_t s, unsigned chunks = 1) {
    const dim3 grid((unsigned)(ceil_div(g.m, BM) * ceil_div(g.n, BN)), chunks);
    const bool avec = g.a_vec && g.k % 16 == 0;
    if (blocked && avec)
        gemm_int8_kernel<BM, BN, KT, WGM, WGN, true, true, false><<<grid, 64 * WGM * WGN, 0, s>>>(g);
    else if (blocked)
        gemm_int8_kernel<BM, BN, KT, WGM, WGN, true, false, false><<<grid, 64 * WGM * WGN, 0, s>>>(g);
    else if (avec)
        gemm_int8_kernel<BM, BN, KT, WGM, WGN, false, true, false><<<grid, 64 * WGM * WGN, 0, s>>>(g);
    else
        gemm_int8_kernel<BM, BN, KT, WGM, WGN, false, false, false><<<grid, 64 * WGM * WGN, 0, s>>>(g);
    return check_launch("gemm_int8");
}

// FP4: packed rows are 16-byte aligned with whole 16-byte segments (ld4 a multiple
// of 128, g.k rounded up to 16 packed bytes), so A always takes the vector loads.
// Only the blocked variant is built: an unblocked product runs it with one block
// longer than k (the per-stage block test is one scalar step; the variant without
// it is scheduled by the compiler into more registers than four wavefronts per
// SIMD allow, and spills).
template <int BM, int BN, int KT, int WGM, int WGN>
qmm_status run_fp4(const Int8Args &g, hipStream_t s, unsigned chunks = 1) {
    const dim3 grid((unsigned)(ceil_div(g.m, BM) * ceil_div(g.n, BN)), chunks);
    gemm_int8_kernel<BM, BN, KT, WGM, WGN, true, true, true><<<grid, 64 * WGM * WGN, 0, s>>>(g);
    return check_launch("gemm_fp4");
}
}  // namespace

// The direct-load tile reads A's rows as they are when every residue is already an
// int8 (p <= 128), the int32 sums stay in range with A in [0, p-1] instead of
// centred (a block of k_block terms of at most (p-1) floor(p/2) each, plus the
// residue carried from the block before), and whole 128-byte stages of every row
// lie inside the row (k a multiple of 128, rows 16-byte aligned).
bool int8_raw_a_ok(const qmm_plan &pl, int64_t k) {
    const int64_t kb = pl.k_block < k ? pl.k_block : k;
    return pl.p <= 128 && k % 128 == 0 &&
           (__int128)kb * (pl.p - 1) * (pl.p / 2) + (pl.p - 1) <= (((__int128)1 << 31) - 1);
}

bool int8_centres_a(const qmm_plan &pl, int64_t m, int64_t n, int64_t k) {
    const int tile = pl.tile ? (int)pl.tile : int8_tile_for(m, n, false);
    return k % 16 != 0 || (tile == 4 && !int8_raw_a_ok(pl, k));
}

int int8_tile_for(int64_t m, int64_t n, bool fp4) {
    // 256 x 256 tiles once they (nearly) fill the 256 CUs, 128 x 128 below that.
    // INT8: the direct-load tile (8 wavefronts of 128 x 64, both operands straight
    // from HBM into LDS, one barrier per K stage); the product kernels fall back to
    // tile 3 where A's rows cannot be read whole.  FP4: 16 wavefronts of 64 x 64
    // with register-staged loads (measured interleaved on one GPU against 8
    // wavefronts of 128 x 64: 2-6 % faster).
    if (ceil_div(m, 256) * ceil_div(n, 256) < 192) return 1;
    return fp4 ? 3 : 4;
}

// Packed FP4 rows: ceil(k/2) bytes rounded up to 128, plus one 128-byte line at
// multiples of 2 KiB (as for Bt).
int64_t fp4_ld(int64_t k) {
    const int64_t r = ceil_div(ceil_div(k < 1 ? 1 : k, 2), kBtAlign) * kBtAlign;
    return r % 2048 == 0 ? r + kBtAlign : r;
}

qmm_status launch_pack_fp4_rows(const qmm_plan &pl, int64_t m, int64_t k, const uint8_t *A, int64_t lda,
                                uint8_t *A4, int64_t lda4, void *stream) {
    if (m == 0) return QMM_OK;
    uint32_t lo, hi;
    fp4_lut(pl.p, lo, hi);
    const int64_t segs = lda4 / 16;
    const int64_t gx = std::max<int64_t>(1, std::min<int64_t>(ceil_div(segs, 256), 64));
    const int64_t gy = std::max<int64_t>(1, std::min<int64_t>(m, 65535));
    const int a_vec = ((uintptr_t)A % 16 == 0) && (lda % 16 == 0);
    pack_fp4_rows_kernel<<<dim3((unsigned)gx, (unsigned)gy), 256, 0, (hipStream_t)stream>>>(m, k, A, lda, A4, lda4, lo,
                                                                                             hi, a_vec);
    return check_launch("pack_fp4_rows");
}

qmm_status launch_pack_fp4_cols(const qmm_plan &pl, int64_t k, int64_t n, const uint8_t *B, int64_t ldb,
                                uint8_t *Bt4, int64_t ldbt4, void *stream) {
    if (n == 0) return QMM_OK;
    uint32_t lo, hi;
    fp4_lut(pl.p, lo, hi);
    const dim3 grid((unsigned)ceil_div(n, CT), (unsigned)ceil_div(2 * ldbt4, CT));
    if (((uintptr_t)B % 16 == 0) && (ldb % 16 == 0))
        pack_fp4_cols_kernel<true><<<grid, 256, 0, (hipStream_t)stream>>>(k, n, B, ldb, Bt4, ldbt4, lo, hi);
    else
        pack_fp4_cols_kernel<false><<<grid, 256, 0, (hipStream_t)stream>>>(k, n, B, ldb, Bt4, ldbt4, lo, hi);
    return check_launch("pack_fp4_cols");
}

qmm_status launch_pack_fp4_both(const qmm_plan &pl, int64_t m, int64_t n, int64_t k, const uint8_t *A, int64_t lda,
                                const uint8_t *B, int64_t ldb, uint8_t *A4, int64_t lda4, uint8_t *Bt4, int64_t ldbt4,
                                void *stream) {
    if (m == 0 && n == 0) return QMM_OK;
    Fp4PackArgs g{};
    g.m = m;
    g.n = n;
    g.k = k;
    g.A = A;
    g.lda = lda;
    g.A4 = A4;
    g.lda4 = lda4;
    g.B = B;
    g.ldb = ldb;
    g.Bt4 = Bt4;
    g.ldbt4 = ldbt4;
    fp4_lut(pl.p, g.lut_lo, g.lut_hi);
    g.a_vec = ((uintptr_t)A % 16 == 0) && (lda % 16 == 0);
    const bool b_vec = ((uintptr_t)B % 16 == 0) && (ldb % 16 == 0);
    g.a_blocks = ceil_div(m * (lda4 / 16), 256);
    g.b_tiles_x = ceil_div(n, CT);
    const int64_t blocks = g.a_blocks + (n > 0 ? g.b_tiles_x * ceil_div(2 * ldbt4, CT) : 0);
    if (blocks > INT32_MAX) return fail(QMM_EUNSUPPORTED, "FP4 conversion grid too large");
    if (b_vec)
        pack_fp4_both_kernel<true><<<(unsigned)blocks, 256, 0, (hipStream_t)stream>>>(g);
    else
        pack_fp4_both_kernel<false><<<(unsigned)blocks, 256, 0, (hipStream_t)stream>>>(g);
    return check_launch("pack_fp4_both");
}

namespace {
// Compute units of the current device, looked up once per device.
int device_cus() {
    static std::mutex mu;
    static int cache[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    std::lock_guard<std::mutex> lock(mu);
    if (cache[dev] == 0) {
        int c = 0;
        if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c <= 0) c = 256;
        cache[dev] = c;
    }
    return cache[dev];
}

// Tile quantisation: when m or n is a little past a multiple of 256 (4097^2: 17 x 17
// = 289 tiles of 256 x 256 on 256 CUs), the ragged last tile-row and tile-column make
// a second round of tiles that takes as long as the first.  Then the block
// [0, m0) x [0, n0) of whole 256 x 256 tiles runs on them in fewer rounds, and the two
// edge strips -- rows [m0, m) of all of C, and columns [n0, n) of rows [0, m0) --
// each run as a split-K product on 128 x 128 tiles: k cut into chunks of kc bytes
// (multiples of 128), chunks chosen so that tiles times chunks make about one round
// over the CUs (four chunk-tiles per CU measured no faster); each chunk's product
// mod p goes to a partial output in the workspace, and a small kernel sums the
// chunks mod p into C (a strip of one chunk is written to C directly).  kbytes:
// bytes of k per row (INT8: k; FP4: packed).
struct Strip {
    int64_t rows = 0, cols = 0;
    int64_t chunks = 1, kc = 0;
    size_t off = 0;  // partial outputs in the workspace (chunks > 1)
    size_t bytes() const { return chunks > 1 ? (size_t)chunks * (size_t)rows * (size_t)cols : 0; }
};
struct TailPlan {
    bool split = false;
    int64_t m0 = 0, n0 = 0;
    Strip bottom, right;
    size_t bytes = 0;
};

Strip strip_plan(int64_t rows, int64_t cols, int64_t kbytes, int64_t cus) {
    Strip st;
    st.rows = rows;
    st.cols = cols;
    if (rows == 0 || cols == 0) return st;
    const int64_t tiles = ceil_div(rows, 128) * ceil_div(cols, 128);
    const int64_t stages = ceil_div(kbytes, 128);
    const int64_t want = std::max<int64_t>(1, std::min<int64_t>(cus / tiles, stages));
    st.kc = ceil_div(stages, want) * 128;
    st.chunks = ceil_div(kbytes, st.kc);
    return st;
}

TailPlan tail_plan(int64_t m, int64_t n, int64_t kbytes, int64_t cus) {
    TailPlan t;
    const int64_t tiles = ceil_div(m, 256) * ceil_div(n, 256);
    const int64_t inner = (m / 256) * (n / 256);
    if (inner == 0 || ceil_div(inner, cus) >= ceil_div(tiles, cus)) return t;
    t.split = true;
    t.m0 = m / 256 * 256;
    t.n0 = n / 256 * 256;
    t.bottom = strip_plan(m - t.m0, n, kbytes, cus);
    t.right = strip_plan(t.m0, n - t.n0, kbytes, cus);
    t.bottom.off = 0;
    t.right.off = (t.bottom.bytes() + 255) / 256 * 256;
    t.bytes = t.right.off + t.right.bytes();
    return t;
}

// C = (sum of the chunks' partial residues) mod p, one output per thread.
__global__ __launch_bounds__(256) void tail_combine_kernel(const uint8_t *__restrict__ part, int64_t stride,
                                                           int32_t chunks, int64_t rows, int64_t n,
                                                           uint8_t *__restrict__ C, int64_t ldc, uint32_t p,
                                                           uint32_t magic32) {
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= rows * n) return;
    uint32_t sum = 0;
    for (int32_t c = 0; c < chunks; ++c) sum += part[c * stride + idx];
    const int64_t r = idx / n;
    C[r * ldc + (idx - r * n)] = (uint8_t)mod_u32_m32(sum, p, magic32);
}

// Four e2m1 codes (one per byte, as the FP4 rows hold them: magnitudes 0..4 as the
// codes 0, 2, 4, 5, 6, sign bit 8, never a negative zero) as four int8 values.
__device__ __forceinline__ uint32_t e2m1x4_to_int8x4(uint32_t codes) {
    const uint32_t mag = codes & 0x07070707u, sgn = (codes >> 3) & 0x01010101u;
    // byte c of the table (c = 0 .. 7) is the magnitude of code c: 0, 0.5, 1, 1.5, 2,
    // 3, 4, 6 (the halves never occur; they read 0)
    const uint32_t val = __builtin_amdgcn_perm(0x06040302u, 0x00010000u, mag);
    const uint32_t neg = sgn * 0xffu;  // 0xff in each negative byte
    return (val ^ neg) + sgn;          // two's complement of a non-zero byte: no carry
}

// A thin edge strip (at most 16 rows or columns): out[x][y] = (X[x] . Y[y]) mod p for
// x < nx, y < ny <= RMAX, X and Y rows 16-byte aligned, readable up to k16 bytes
// (zero past k): int8 values, or (FP4) e2m1 codes two per byte, the even k in the low
// nibble, decoded to int8 here.  Each dot product stays within int32 (INT8: the plan's
// bound; FP4: |x| <= 4, so 16 k per product at most).  out[x][y] goes to C[x sx + y sy].
// One wavefront per XR rows of X: each lane takes 16 bytes of k at a time (a
// wavefront reads 1 KB of a row per load), v_dot4 on four int8 pairs at a time; then
// the XR x RMAX sums are reduced across the wavefront by halving exchanges (each step
// keeps half the values and adds the partner's other half), which leaves lane l with
// the total of value (l >> (6 - log2 NV)).  Memory-bound on X, which the strip reads
// once (Y stays in the caches).
struct ThinStrip {
    const int8_t *X, *Y;
    int64_t ldx, ldy, nx;
    uint8_t *C;
    int64_t sx, sy;
    int32_t ny;
    uint32_t blocks;  // workgroups of this strip
};
struct ThinStrips {
    ThinStrip s[2];  // the bottom and the right strip of one product, one launch
    int64_t k16;
    uint32_t p, off;
    uint64_t magic;
};

template <int XR, int RMAX, bool FP4>
__global__ __launch_bounds__(256) void thin_strip_kernel(ThinStrips g) {
    constexpr int NV = XR * RMAX, LOGNV = NV == 32 ? 5 : NV == 16 ? 4 : NV == 8 ? 3 : NV == 4 ? 2 : NV == 2 ? 1 : 0;
    static_assert((1 << LOGNV) == NV && NV <= 32, "XR x RMAX is a power of two up to 32");
    constexpr int DW = FP4 ? 8 : 4;  // int8x4 words per 16 bytes of a row
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const bool second = blockIdx.x >= g.s[0].blocks;
    const ThinStrip &js = second ? g.s[1] : g.s[0];
    const int8_t *X = js.X, *Y = js.Y;
    const int64_t ldx = js.ldx, ldy = js.ldy, nx = js.nx, sx = js.sx, sy = js.sy, k16 = g.k16;
    const int32_t ny = js.ny;
    uint8_t *C = js.C;
    const int64_t x0 = ((int64_t)(blockIdx.x - (second ? g.s[0].blocks : 0u)) * 4 + wave) * XR;
    if (x0 >= nx) return;  // the whole wavefront
    const QMM_GLOBAL int8_t *xrow[XR];
#pragma unroll
    for (int i = 0; i < XR; ++i) xrow[i] = (const QMM_GLOBAL int8_t *)X + (x0 + i < nx ? x0 + i : nx - 1) * ldx;
    const QMM_GLOBAL int8_t *yb = (const QMM_GLOBAL int8_t *)Y;
    // 16 bytes of a row as DW int8x4 words (FP4: low nibbles then high nibbles of
    // each dword, the same k order for X and Y)
    auto words = [](const ix4 v, int32_t (&w)[DW]) {
        const int32_t in[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if constexpr (FP4) {
                w[2 * j] = (int32_t)e2m1x4_to_int8x4((uint32_t)in[j] & 0x0f0f0f0fu);
                w[2 * j + 1] = (int32_t)e2m1x4_to_int8x4(((uint32_t)in[j] >> 4) & 0x0f0f0f0fu);
            } else {
                w[j] = in[j];
            }
        }
    };
    int32_t v[NV];
#pragma unroll
    for (int j = 0; j < NV; ++j) v[j] = 0;
#pragma unroll 2
    for (int64_t c = 16 * lane; c < k16; c += 1024) {
        int32_t xw[XR][DW];
#pragma unroll
        for (int i = 0; i < XR; ++i) words(*(const QMM_GLOBAL ix4 *)(xrow[i] + c), xw[i]);
#pragma unroll
        for (int r = 0; r < RMAX; ++r) {
            if (r < ny) {
                int32_t yw[DW];
                words(*(const QMM_GLOBAL ix4 *)(yb + r * ldy + c), yw);
#pragma unroll
                for (int i = 0; i < XR; ++i) {
                    int32_t a = v[i * RMAX + r];
#pragma unroll
                    for (int j = 0; j < DW; ++j) a = __builtin_amdgcn_sdot4(xw[i][j], yw[j], a, false);
                    v[i * RMAX + r] = a;
                }
            }
        }
    }
#pragma unroll
    for (int s = 0; s < LOGNV; ++s) {
        const int o = 32 >> s, h = (NV >> s) / 2;
        const bool upper = (lane & o) != 0;
#pragma unroll
        for (int j = 0; j < h; ++j) {
            const int32_t keep = upper ? v[j + h] : v[j], send = upper ? v[j] : v[j + h];
            v[j] = keep + __shfl_xor(send, o);
        }
    }
#pragma unroll
    for (int o = 32 >> LOGNV; o >= 1; o >>= 1) v[0] += __shfl_xor(v[0], o);
    const int idx = (lane >> (6 - LOGNV)) & (NV - 1), i = idx / RMAX, r = idx % RMAX;
    if ((lane & ((64 >> LOGNV) - 1)) == 0 && x0 + i < nx && r < ny)
        C[(x0 + i) * sx + (int64_t)r * sy] = (uint8_t)mod_i32_magic(v[0], g.p, g.magic, g.off);
}

// Runs the thin strips of one product (each ny <= 16; an empty one has nx = 0) in one
// launch, with the smallest register block that holds the thicker.
template <bool FP4>
qmm_status run_thin_strips(ThinStrips t, const Int8Args &g, hipStream_t s) {
    constexpr int XR = 2;
    t.p = g.p;
    t.off = g.off;
    t.magic = g.magic;
    int32_t ny = 0;
    for (ThinStrip &j : t.s) {
        if (j.nx == 0 || j.ny == 0) j.nx = j.ny = 0;
        j.blocks = (uint32_t)ceil_div(j.nx, 4 * (int64_t)XR);
        ny = std::max(ny, j.ny);
    }
    const unsigned blocks = t.s[0].blocks + t.s[1].blocks;
    if (blocks == 0) return QMM_OK;
    if (ny <= 2) thin_strip_kernel<XR, 2, FP4><<<blocks, 256, 0, s>>>(t);
    else if (ny <= 4) thin_strip_kernel<XR, 4, FP4><<<blocks, 256, 0, s>>>(t);
    else if (ny <= 8) thin_strip_kernel<XR, 8, FP4><<<blocks, 256, 0, s>>>(t);
    else thin_strip_kernel<XR, 16, FP4><<<blocks, 256, 0, s>>>(t);
    return check_launch("thin_strip");
}
constexpr int64_t kThinStrip = 16;  // strips this thin or thinner take thin_strip_kernel

// One edge strip: args `a` already describe the strip's A rows, Bt rows and C; run
// it whole (one chunk) or as chunks into `part` and combine.
template <typename Run>
qmm_status run_strip(const Strip &st, Int8Args a, uint8_t *part, uint32_t p, hipStream_t s, Run run) {
    if (st.rows == 0 || st.cols == 0) return QMM_OK;
    a.m = st.rows;
    a.n = st.cols;
    if (st.chunks == 1) return run(a, 1u);
    uint8_t *C = a.C;
    const int64_t ldc = a.ldc;
    a.C = part;
    a.ldc = st.cols;
    a.c_vec = st.cols % 4 == 0 && (uintptr_t)part % 4 == 0;
    a.kc = st.kc;
    a.part_stride = st.rows * st.cols;
    qmm_status r = run(a, (unsigned)st.chunks);
    if (r != QMM_OK) return r;
    const int64_t blocks = ceil_div(st.rows * st.cols, 256);
    tail_combine_kernel<<<(unsigned)blocks, 256, 0, s>>>(part, st.rows * st.cols, (int32_t)st.chunks, st.rows, st.cols,
                                                         C, ldc, p, (uint32_t)((1ull << 32) / p));
    return check_launch("tail_combine");
}
}  // namespace

qmm_status launch_gemm_fp4(const qmm_plan &pl, int64_t m, int64_t n, int64_t k, const uint8_t *A4, int64_t lda4,
                           const uint8_t *Bt4, int64_t ldbt4, uint8_t *C, int64_t ldc, void *stream,
                           uint8_t *tail_ws, size_t tail_bytes) {
    if (m == 0 || n == 0) return QMM_OK;
    Int8Args g{};
    g.m = m;
    g.n = n;
    g.k = ceil_div(ceil_div(k, 2), 16) * 16;  // packed bytes, whole 16-byte segments (zero padded)
    g.A = A4;
    g.lda = lda4;
    g.Bt = (const int8_t *)Bt4;
    g.ldbt = ldbt4;
    g.C = C;
    g.ldc = ldc;
    const bool blocked = pl.k_block < k;
    g.p = pl.p;
    g.magic = mod_magic(pl.p);
    g.off = pl.p * ((1u << 31) / pl.p);
    g.magic32 = (uint32_t)((1ull << 32) / pl.p);
    g.c_vec = ((uintptr_t)C % 4 == 0) && (ldc % 4 == 0);
    g.a_vec = true;
    hipStream_t s = (hipStream_t)stream;
    const int tile = pl.tile ? (int)pl.tile : int8_tile_for(m, n, true);
    // one K stage of KT packed bytes holds 2 KT values of k
    const int32_t never = INT32_MAX;
    auto small_tiles = [&](Int8Args a) {
        a.kb_tiles = blocked ? (int32_t)(pl.k_block / 128) : never;
        return run_fp4<128, 128, 64, 2, 2>(a, s);
    };
    auto big_tiles = [&](Int8Args a) {
        a.kb_tiles = blocked ? (int32_t)(pl.k_block / 256) : never;
        return tile == 2 ? run_fp4<256, 256, 128, 2, 4>(a, s) : run_fp4<256, 256, 128, 4, 4>(a, s);
    };
    if (tile != 2 && tile != 3) return small_tiles(g);
    const TailPlan t = tail_plan(m, n, g.k, device_cus());
    if (!t.split || tail_ws == nullptr || tail_bytes < t.bytes) return big_tiles(g);
    // ragged edges past whole rounds of 256 x 256 tiles: split-K strips
    Int8Args head = g;
    head.m = t.m0;
    head.n = t.n0;
    qmm_status st = big_tiles(head);
    auto run = [&](Int8Args a, unsigned chunks) {
        a.kb_tiles = blocked ? (int32_t)(pl.k_block / 128) : never;
        return run_fp4<128, 128, 64, 2, 2>(a, s, chunks);
    };
    Int8Args bottom = g, right = g;
    bottom.A = A4 + t.m0 * lda4;
    bottom.C = C + t.m0 * ldc;
    right.Bt = (const int8_t *)(Bt4 + t.n0 * ldbt4);
    right.C = C + t.n0;
    // strips of at most kThinStrip rows (columns): dot products of decoded code rows
    const bool thin_ok = lda4 % 16 == 0 && ldbt4 % 16 == 0 && (uintptr_t)A4 % 16 == 0 && (uintptr_t)Bt4 % 16 == 0;
    const int8_t *a4 = (const int8_t *)A4, *b4 = (const int8_t *)Bt4;
    const bool tb = thin_ok && t.bottom.rows <= kThinStrip, tr = thin_ok && t.right.cols <= kThinStrip;
    ThinStrips ts{};
    ts.k16 = g.k;
    if (tb)  // C[m0 + y][x] = Bt4[x] . A4[m0 + y]
        ts.s[0] = ThinStrip{b4, a4 + t.m0 * lda4, ldbt4, lda4, n, bottom.C, 1, ldc, (int32_t)t.bottom.rows, 0};
    if (tr)  // C[x][n0 + y] = A4[x] . Bt4[n0 + y]
        ts.s[1] = ThinStrip{a4, right.Bt, lda4, ldbt4, t.m0, right.C, ldc, 1, (int32_t)t.right.cols, 0};
    if (st == QMM_OK && (tb || tr)) st = run_thin_strips<true>(ts, g, s);
    if (st == QMM_OK && !tb) st = run_strip(t.bottom, bottom, tail_ws + t.bottom.off, pl.p, s, run);
    if (st == QMM_OK && !tr) st = run_strip(t.right, right, tail_ws + t.right.off, pl.p, s, run);
    return st;
}

namespace {
qmm_status gemm_int8_impl(const qmm_plan &pl, int64_t m, int64_t n, int64_t k, const uint8_t *A, int64_t lda,
                          bool a_centred, const int8_t *Bt, int64_t ldbt, uint8_t *C, int64_t ldc, void *stream,
                          uint8_t *tail_ws, size_t tail_bytes);
}  // namespace

qmm_status launch_gemm_int8(const qmm_plan &pl, int64_t m, int64_t n, int64_t k, const uint8_t *A, int64_t lda,
                            const int8_t *Bt, int64_t ldbt, uint8_t *C, int64_t ldc, void *stream,
                            uint8_t *tail_ws, size_t tail_bytes) {
    return gemm_int8_impl(pl, m, n, k, A, lda, false, Bt, ldbt, C, ldc, stream, tail_ws, tail_bytes);
}

// Ac holds centred rows zero padded to ldac (a multiple of 128, at least k), so the
// product may run over k rounded up to 16: the padding adds zero terms.  With the
// centring constants zero, centre4 is the identity.
qmm_status launch_gemm_int8_centred_a(const qmm_plan &pl, int64_t m, int64_t n, int64_t k, const int8_t *Ac,
                                      int64_t ldac, const int8_t *Bt, int64_t ldbt, uint8_t *C, int64_t ldc,
                                      void *stream, uint8_t *tail_ws, size_t tail_bytes) {
    // an unblocked plan stays unblocked over the padded k (its zero terms keep every
    // sum within the plan's bound)
    const int64_t k16 = ceil_div(k, 16) * 16;
    qmm_plan p16 = pl;
    if (p16.k_block >= k) p16.k_block = k16;
    return gemm_int8_impl(p16, m, n, k16, (const uint8_t *)Ac, ldac, true, Bt, ldbt, C, ldc, stream, tail_ws,
                          tail_bytes);
}

size_t lowp_tail_bytes(const qmm_plan &pl, int64_t m, int64_t n, int64_t k) {
    if (m == 0 || n == 0 || k == 0) return 0;
    const bool fp4 = pl.path == QMM_PATH_FP4;
    const int tile = pl.tile ? (int)pl.tile : int8_tile_for(m, n, fp4);
    if (tile < 2 || tile > (fp4 ? 3 : 4)) return 0;
    // the product's k in bytes per row: INT8 rounds up to 16 when A is centred first
    const int64_t kbytes = fp4 ? ceil_div(ceil_div(k, 2), 16) * 16 : (k % 16 ? ceil_div(k, 16) * 16 : k);
    return tail_plan(m, n, kbytes, device_cus()).bytes;
}

namespace {
qmm_status gemm_int8_impl(const qmm_plan &pl, int64_t m, int64_t n, int64_t k, const uint8_t *A, int64_t lda,
                          bool a_centred, const int8_t *Bt, int64_t ldbt, uint8_t *C, int64_t ldc, void *stream,
                          uint8_t *tail_ws, size_t tail_bytes) {
    if (m == 0 || n == 0) return QMM_OK;
    Int8Args g{};
    g.m = m;
    g.n = n;
    g.k = k;
    g.A = A;
    g.lda = lda;
    g.Bt = Bt;
    g.ldbt = ldbt;
    g.C = C;
    g.ldc = ldc;
    const bool blocked = pl.k_block < k;
    g.p = pl.p;
    centre_consts(pl.p, g.add_h, g.neg_p);
    if (a_centred) g.add_h = g.neg_p = 0;  // centre4 is then the identity
    g.magic = mod_magic(pl.p);
    g.off = pl.p * ((1u << 31) / pl.p);
    g.magic32 = (uint32_t)((1ull << 32) / pl.p);
    g.c_vec = ((uintptr_t)C % 4 == 0) && (ldc % 4 == 0);
    g.a_vec = ((uintptr_t)A % 16 == 0) && (lda % 16 == 0);
    hipStream_t s = (hipStream_t)stream;
    // the direct-load tile reads A as int8 rows: centred (Ac, padded to whole
    // stages) or, where int8_raw_a_ok, the residues themselves; otherwise tile 3
    // runs instead
    const bool direct_a = a_centred ? lda % 128 == 0 : (int8_raw_a_ok(pl, k) && lda % 16 == 0);
    const bool direct = direct_a && ldbt % 128 == 0 && (uintptr_t)A % 16 == 0 && (uintptr_t)Bt % 16 == 0;
    int tile = pl.tile ? (int)pl.tile : int8_tile_for(m, n, false);
    if (tile == 4 && !direct) tile = 3;  // same 256 x 256 tile, register-staged loads
    auto small_tiles = [&](Int8Args a) {
        a.kb_tiles = blocked ? (int32_t)(pl.k_block / 64) : 0;
        return run_int8<128, 128, 64, 2, 2>(a, blocked, s);
    };
    auto big_tiles = [&](Int8Args a) {
        a.kb_tiles = blocked ? (int32_t)(pl.k_block / 128) : 0;
        if (tile == 2) return run_int8<256, 256, 128, 2, 4>(a, blocked, s);
        if (tile == 3) return run_int8<256, 256, 128, 4, 4>(a, blocked, s);
        const dim3 grid((unsigned)(ceil_div(a.m, 256) * ceil_div(a.n, 256)));
        if (blocked)
            gemm_int8_direct_kernel<true, 2, 4><<<grid, 512, 0, s>>>(a);
        else
            gemm_int8_direct_kernel<false, 2, 4><<<grid, 512, 0, s>>>(a);
        return check_launch("gemm_int8_direct");
    };
    if (tile < 2 || tile > 4) return small_tiles(g);
    const TailPlan t = tail_plan(m, n, k, device_cus());
    if (!t.split || tail_ws == nullptr || tail_bytes < t.bytes) return big_tiles(g);
    // ragged edges past whole rounds of 256 x 256 tiles: split-K strips
    Int8Args head = g;
    head.m = t.m0;
    head.n = t.n0;
    qmm_status st = big_tiles(head);
    auto run = [&](Int8Args a, unsigned chunks) {
        a.kb_tiles = blocked ? (int32_t)(pl.k_block / 64) : 0;
        return run_int8<128, 128, 64, 2, 2>(a, blocked, s, chunks);
    };
    Int8Args bottom = g, right = g;
    bottom.A = A + t.m0 * lda;
    bottom.C = C + t.m0 * ldc;
    right.Bt = Bt + t.n0 * ldbt;
    right.C = C + t.n0;
    // Strips of at most kThinStrip rows (columns) are dot products of int8 rows read
    // straight from A and Bt: A's rows must be int8 values already (centred, or
    // residues usable as they are) and both operands whole 16-byte segments.
    const bool thin_ok = !blocked && (a_centred || int8_raw_a_ok(pl, k)) && k % 16 == 0 && lda % 16 == 0 &&
                         ldbt % 16 == 0 && (uintptr_t)A % 16 == 0 && (uintptr_t)Bt % 16 == 0;
    const bool tb = thin_ok && t.bottom.rows <= kThinStrip, tr = thin_ok && t.right.cols <= kThinStrip;
    ThinStrips ts{};
    ts.k16 = k;
    if (tb)  // C[m0 + y][x] = Bt[x] . A[m0 + y]
        ts.s[0] = ThinStrip{Bt, (const int8_t *)bottom.A, ldbt, lda, n, bottom.C, 1, ldc, (int32_t)t.bottom.rows, 0};
    if (tr)  // C[x][n0 + y] = A[x] . Bt[n0 + y]
        ts.s[1] = ThinStrip{(const int8_t *)A, right.Bt, lda, ldbt, t.m0, right.C, ldc, 1, (int32_t)t.right.cols, 0};
    if (st == QMM_OK && (tb || tr)) st = run_thin_strips<false>(ts, g, s);
    if (st == QMM_OK && !tb) st = run_strip(t.bottom, bottom, tail_ws + t.bottom.off, pl.p, s, run);
    if (st == QMM_OK && !tr) st = run_strip(t.right, right, tail_ws + t.right.off, pl.p, s, run);
    return st;
}
}  // namespace

}  // namespace qmm
