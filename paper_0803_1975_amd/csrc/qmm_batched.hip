// Batches of independent products C_i = A_i x B_i mod p_i in one graph launch.
//
// Host side (qmm_batched_create):
//   - plans every product: INT8 on centred residues whenever p_i <= 256 (the fast
//     path on these matrix cores), or the FP64 Q-adic product when the batch is
//     forced onto it (QMM_BATCH_FORCE_FP64, the paper's method as a baseline);
//   - the autotuner picks the output tile shape per product (see tune_shape);
//   - one descriptor per product, one entry per output tile and one per operand
//     block to pack go to device memory once; tiles are sorted longest first and
//     dealt round-robin to the persistent workgroups (a static longest-processing-
//     time schedule: no atomics, no counters to reset between replays);
//   - the launches are recorded in a HIP graph; qmm_gemm_mod_p_batched replays it.
//
// Device side, INT8 (two stages in the graph):
//   pack    every operand byte is read once: A_i is centred (or FP4-coded) into a workspace copy
//           with rows of KP_i = k_i rounded up to 64 bytes, B_i is centred and
//           transposed (k contiguous) into another, both zero padded to whole
//           tiles and whole K stages, so the product needs no bounds checks and
//           only aligned 16-byte loads;
//   product one persistent kernel per tile class (tile shape x encoding), one after
//           another in the graph; each tile runs 128-byte K stages through LDS
//           into i32_32x32x32_i8 MFMAs (centred bytes) or the FP4 form of the
//           MFMA (e2m1 codes of p <= 8, 64 k per instruction), with the next
//           stage's loads in flight during the MFMAs, then reduces mod p and
//           stores its bytes.
// Device side, INT8 raw (QMM_BATCH_RAW: no pack stage, no workspace): one persistent
// kernel per tile shape reads A's rows and B's k-rows in place with unaligned 16-byte
// loads, from one self-contained record per tile, and pipelines K stages across
// its tiles (the next tile's first loads go out during the current tile's last
// stage).
// Device side, FP64 Q-adic: one persistent kernel whose tiles pack rows of A
// reversed and columns of B forward straight from the bytes on the way into LDS.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <type_traits>
#include <vector>

#include "qmm_device.h"
#include "qmm_internal.h"

namespace qmm {
namespace {

typedef int ix4 __attribute__((ext_vector_type(4)));
typedef int ix16 __attribute__((ext_vector_type(16)));
typedef int ix8 __attribute__((ext_vector_type(8)));
typedef float fx16 __attribute__((ext_vector_type(16)));
typedef unsigned int ux2 __attribute__((ext_vector_type(2)));
typedef double dx4 __attribute__((ext_vector_type(4)));
typedef unsigned int uint4v __attribute__((ext_vector_type(4)));
typedef int v2i __attribute__((ext_vector_type(2)));

// Global-address-space accesses: pointers read from a descriptor in memory are
// otherwise generic, and a generic (flat) access also counts against the LDS
// wait counter, so every LDS wait would wait for outstanding memory traffic too.

constexpr int NT = 256;
constexpr int KW = 16;          // FP64 K stage (packed words)

// Tile shapes of the batched kernel (rows x columns of C per tile).
enum Shape : uint32_t { SHAPE_64x64 = 0, SHAPE_32x128 = 1, SHAPE_128x32 = 2, SHAPE_128x128 = 3, SHAPE_COUNT = 4 };
constexpr int shape_bm(uint32_t s) { return s == SHAPE_32x128 ? 32 : (s == SHAPE_64x64 ? 64 : 128); }
constexpr int shape_bn(uint32_t s) { return s == SHAPE_128x32 ? 32 : (s == SHAPE_64x64 ? 64 : 128); }
// wavefront grid of a shape: 2 x 2 for the square tiles, 1 x 4 / 4 x 1 for the thin ones
constexpr int shape_wgm(uint32_t s) { return s == SHAPE_32x128 ? 1 : (s == SHAPE_128x32 ? 4 : 2); }

struct Desc {
    const uint8_t *A;
    const uint8_t *B;
    uint8_t *C;
    int64_t lda, ldb, ldc;
    int32_t m, n, k;
    uint32_t p;
    uint32_t path;    // QMM_PATH_INT8 or QMM_PATH_FP64_QADIC
    uint32_t shape;   // Shape (INT8); FP64 tiles are 64 x 64
    uint32_t add_h, neg_p, off;
    uint64_t magic;
    // FP64 Q-adic
    uint32_t t, d, offset_regime;
    double start, invp;
    // INT8 / FP4: centred, zero-padded workspace copies (rows of kpb bytes; mp and np
    // rows); kp = k rounded up to 64.  FP4 products hold e2m1 codes, two per byte
    // (kpb = kp / 2), INT8 products centred bytes (kpb = kp).
    int8_t *Ac;
    int8_t *Bt;
    int32_t kp, mp, np, kpb;
    uint32_t fp4, lut_lo, lut_hi;
    uint32_t magic32;  // floor(2^32 / p)
};

// One operand block for the pack kernel: kind 0 = rows r0 .. r0+63 of A at k bytes
// c0 .. c0+255; kind 1 = k rows r0 .. r0+255 of B at columns c0 .. c0+63
// (transposed into Bt); kind 2 = nothing (pads the list to a multiple of 8).
struct PackJob {
    int32_t desc;
    int32_t kind;
    int32_t r0, c0;
};

struct TileRef {
    int32_t desc;
    int32_t tm, tn;
    int32_t pad;
};

__device__ __forceinline__ uint32_t centre4(uint32_t w, uint32_t add_h, uint32_t neg_p) {
    const uint32_t flag = ((w + add_h) >> 7) & 0x01010101u;
    return w + flag * neg_p;
}


// 64 bytes of a byte matrix starting at src (any alignment), bytes at positions
// >= valid zero.  When the dword-aligned 68-byte window around them lies inside
// the matrix's data [lo, hi) (it may run into the next row: those bytes are masked)
// they come from four 16-byte and one 4-byte load and byte-aligning shifts;
// otherwise from single byte loads.
__device__ __forceinline__ void load64(const uint8_t *src, int valid, const uint8_t *lo, const uint8_t *hi,
                                       uint32_t out[16]) {
#pragma unroll
    for (int j = 0; j < 16; ++j) out[j] = 0;
    if (valid <= 0) return;
    const uintptr_t a = (uintptr_t)src;
    const uint8_t *base = (const uint8_t *)(a & ~(uintptr_t)3);
    if (base >= lo && base + 68 <= hi) {
        uint32_t w[17];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const u32x4a4 v = *(const QMM_GLOBAL u32x4a4 *)(base + 16 * q);
            w[4 * q] = v.x; w[4 * q + 1] = v.y; w[4 * q + 2] = v.z; w[4 * q + 3] = v.w;
        }
        w[16] = *(const QMM_GLOBAL uint32_t *)(base + 64);
        const uint32_t sh = (uint32_t)(a & 3);
#pragma unroll
        for (int j = 0; j < 16; ++j) out[j] = sh ? __builtin_amdgcn_alignbyte(w[j + 1], w[j], sh) : w[j];
        if (valid < 64) {
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                const int left = valid - 4 * j;  // valid bytes in this dword
                out[j] &= left >= 4 ? 0xffffffffu : (left <= 0 ? 0u : (1u << (8 * left)) - 1u);
            }
        }
    } else {
        const int nb = valid < 64 ? valid : 64;
        for (int b = 0; b < nb; ++b) out[b >> 2] |= (uint32_t)((const QMM_GLOBAL uint8_t *)src)[b] << (8 * (b & 3));
    }
}

// Pack one operand block (256 threads, one 64-byte run each, its loads in flight
// together).  A job: rows r0 .. r0+63 of A, k bytes c0 .. c0+255, encoded (centred
// bytes, or FP4 codes two per byte), zero past k (up to kp).  B job: k rows
// r0 .. r0+255, columns c0 .. c0+63 of B go through LDS encoded; thread t then reads
// 16 k rows of one 4-column word, transposes the 16 x 4 bytes in registers and
// writes the four k-runs into rows of Bt (zero past k, up to kp).  Rows of Ac past m and rows of Bt past n (the tile padding up
// to mp and np) are never written: they only reach outputs past m or n, which the
// product does not store, so any bytes there will do.
constexpr int PACK_K = 256;

// FP4 codes: residue x < p <= 8 -> e2m1 code of centred(x), four at a time by one
// byte permute over the codes of 0..7 held in (lut_hi:lut_lo); two words of codes
// (one code per byte) pack into one word of eight nibbles, the lower k low.
__device__ __forceinline__ uint32_t fp4_codes(uint32_t x4, uint32_t lut_lo, uint32_t lut_hi) {
    return __builtin_amdgcn_perm(lut_hi, lut_lo, x4);
}
__device__ __forceinline__ uint32_t fp4_pack(uint32_t c_lo, uint32_t c_hi) {
    const uint32_t a = c_lo | (c_lo >> 4), b = c_hi | (c_hi >> 4);
    return __builtin_amdgcn_perm(b, a, 0x06040200u);
}
__device__ __forceinline__ uint32_t encode4(const Desc &D, uint32_t w) {
    return D.fp4 ? fp4_codes(w, D.lut_lo, D.lut_hi) : centre4(w, D.add_h, D.neg_p);
}

__global__ __launch_bounds__(NT) void batched_pack_kernel(const Desc *__restrict__ descs,
                                                          const PackJob *__restrict__ jobs) {
    __shared__ uint32_t tile[PACK_K][17];  // k rows x 64 column bytes, padded by one word
    // Workgroups go to the 8 XCDs round-robin; the job list (padded to a multiple
    // of 8) is split into 8 contiguous ranges, one per XCD, so neighbouring jobs,
    // which share the cache lines at their edges, share one L2.
    const uint32_t nb = gridDim.x, b = blockIdx.x;
    const PackJob J = jobs[(b & 7) * (nb >> 3) + (b >> 3)];
    if (J.kind > 1) return;  // padding
    const Desc &D = descs[J.desc];
    const int t = threadIdx.x;
    if (J.kind == 0) {
        // thread t: row r0 + t / 4, k bytes c0 + 64 (t % 4) .. + 63
        const int32_t row = J.r0 + (t >> 2), kk = J.c0 + 64 * (t & 3);
        if (row >= D.m || kk >= D.kp) return;
        uint32_t w[16];
        load64(D.A + (int64_t)row * D.lda + kk, D.k - kk, D.A, D.A + (int64_t)(D.m - 1) * D.lda + D.k, w);
        if (D.fp4) {
            uint32_t o[8];
#pragma unroll
            for (int i = 0; i < 8; ++i)
                o[i] = fp4_pack(fp4_codes(w[2 * i], D.lut_lo, D.lut_hi), fp4_codes(w[2 * i + 1], D.lut_lo, D.lut_hi));
            QMM_GLOBAL uint4v *dst = (QMM_GLOBAL uint4v *)(D.Ac + (int64_t)row * D.kpb + kk / 2);
            dst[0] = uint4v{o[0], o[1], o[2], o[3]};
            dst[1] = uint4v{o[4], o[5], o[6], o[7]};
        } else {
            QMM_GLOBAL uint4v *dst = (QMM_GLOBAL uint4v *)(D.Ac + (int64_t)row * D.kpb + kk);
#pragma unroll
            for (int q = 0; q < 4; ++q)
                dst[q] = uint4v{centre4(w[4 * q], D.add_h, D.neg_p), centre4(w[4 * q + 1], D.add_h, D.neg_p),
                                centre4(w[4 * q + 2], D.add_h, D.neg_p), centre4(w[4 * q + 3], D.add_h, D.neg_p)};
        }
        return;
    }
    {
        // thread t: k row r0 + t, columns c0 .. c0 + 63, encoded into LDS row t
        const int32_t kk = J.r0 + t;
        uint32_t w[16];
        if (kk < D.k)
            load64(D.B + (int64_t)kk * D.ldb + J.c0, D.n - J.c0, D.B, D.B + (int64_t)(D.k - 1) * D.ldb + D.n, w);
        else
#pragma unroll
            for (int j = 0; j < 16; ++j) w[j] = 0;
#pragma unroll
        for (int j = 0; j < 16; ++j) tile[t][j] = encode4(D, w[j]);
    }
    __syncthreads();
    const int cg = t & 15, kg = t >> 4;  // columns 4 cg .. 4 cg + 3, k rows 16 kg .. 16 kg + 15
    uint32_t out[4][4];                  // [column q][k dword d]
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
    const int32_t kk = J.r0 + 16 * kg;
    if (kk >= D.kp) return;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int32_t orow = J.c0 + 4 * cg + q;
        if (orow >= D.n) continue;
        if (D.fp4)
            *(QMM_GLOBAL ux2 *)(D.Bt + (int64_t)orow * D.kpb + kk / 2) =
                ux2{fp4_pack(out[q][0], out[q][1]), fp4_pack(out[q][2], out[q][3])};
        else
            *(QMM_GLOBAL uint4v *)(D.Bt + (int64_t)orow * D.kpb + kk) = uint4v{out[q][0], out[q][1], out[q][2], out[q][3]};
    }
}

// One INT8 tile of BM x BN outputs from the packed operands: wavefronts laid out
// WGM x WGN, each owning (BM/WGM) x (BN/WGN) outputs in 32 x 32 MFMA blocks
// (i32_32x32x32_i8: lane l holds 16 k-bytes of row l % 32 for k-chunk l / 32 and
// outputs D[8 (r/4) + 4 (l/32) + r % 4][l % 32] in register r).  K goes in
// 128-byte stages through ONE LDS buffer per workgroup (so seven workgroups fit
// a CU): a stage is published from registers, and the loads of the next stage
// are issued before its MFMAs, so they are in flight during the MFMAs and the
// barrier.  Loads are aligned 16-byte loads inside the padded workspace; the
// segments of a last, 64-byte stage past kp are not loaded.
__device__ __forceinline__ ix4 gload16(const int8_t *p) { return *(const QMM_GLOBAL ix4 *)p; }

// An accumulator register as an integer: int32 for INT8 tiles, an FP32 exact
// integer (|x| <= 2^24) for FP4 tiles.
__device__ __forceinline__ int32_t acc_value(int32_t bits, bool fp4) {
    return fp4 ? (int32_t)__builtin_bit_cast(float, bits) : bits;
}

constexpr int KT = 128;            // K stage (bytes)
constexpr int PT = KT + 16;        // LDS row pitch: 8 lanes reading 8 rows hit distinct banks
constexpr int KP_ALIGN = 64;       // workspace rows: k rounded up to this
// LDS pitch of B's k-rows in raw tiles narrower than 128 bytes: 8 lanes reading 8
// consecutive rows at one column hit distinct banks for the widths used (32, 64).
constexpr int raw_bpitch(int bn) { return bn + 16; }
// LDS bytes of one packed tile: A rows, then B's n-rows of packed codes
constexpr int tile_lds_bytes(int bm, int bn) { return (bm + bn) * PT; }
template <int BM, int BN, int WGM, int WGN, bool FP4>
__device__ __forceinline__ void int8_tile(const Desc &D, int tm, int tn, uint8_t *lds) {
    constexpr int WTM = BM / WGM, WTN = BN / WGN, FM = WTM / 32, FN = WTN / 32;
    constexpr int SEGS = KT / 16;
    constexpr int A_SEGS = BM * SEGS, B_SEGS = BN * SEGS;
    constexpr int A_LOADS = (A_SEGS + NT - 1) / NT, B_LOADS = (B_SEGS + NT - 1) / NT;
    static_assert(WGM * WGN == NT / 64, "one wavefront per sub-tile");
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave / WGN, wn = wave % WGN;
    const int64_t row0 = (int64_t)tm * BM, col0 = (int64_t)tn * BN;
    const int kp = D.kpb;  // bytes per packed row (k values for INT8, half of them for FP4)
    constexpr bool fp4 = FP4;  // the tile list of an FP4 class holds only FP4 products
    const int stages = (kp + KT - 1) / KT;

    // Thread tid stages the 16-byte segment seg = tid % 8 of rows tid / 8 + 32 i: the
    // same k offset in every row, so one predicate per stage covers all its loads.
    static_assert(A_SEGS % NT == 0 && B_SEGS % NT == 0, "whole rows per load step");
    constexpr int RSTEP = NT / SEGS;
    const int seg = tid % SEGS, rfirst = tid / SEGS;
    const int8_t *a_base = D.Ac + (row0 + rfirst) * kp + 16 * seg;
    const int8_t *b_base = D.Bt + (col0 + rfirst) * kp + 16 * seg;
    const int slot = rfirst * PT + 16 * seg;
    const int64_t rstride = (int64_t)RSTEP * kp;
    ix4 ra[A_LOADS], rb[B_LOADS];
    auto fetch = [&](int st) __attribute__((always_inline)) {
        const int k0 = st * KT;
        const bool ok = k0 + 16 * seg < kp;
#pragma unroll
        for (int i = 0; i < A_LOADS; ++i) ra[i] = ok ? gload16(a_base + i * rstride + k0) : ix4{0, 0, 0, 0};
#pragma unroll
        for (int i = 0; i < B_LOADS; ++i) rb[i] = ok ? gload16(b_base + i * rstride + k0) : ix4{0, 0, 0, 0};
    };

    ix16 acc[FM][FN];
#pragma unroll
    for (int mi = 0; mi < FM; ++mi)
#pragma unroll
        for (int ni = 0; ni < FN; ++ni) acc[mi][ni] = ix16{};
    auto publish = [&]() __attribute__((always_inline)) {
#pragma unroll
        for (int i = 0; i < A_LOADS; ++i) *(ix4 *)&lds[slot + i * RSTEP * PT] = ra[i];
#pragma unroll
        for (int i = 0; i < B_LOADS; ++i) *(ix4 *)&lds[BM * PT + slot + i * RSTEP * PT] = rb[i];
        __syncthreads();
    };
    auto compute = [&](int st) __attribute__((always_inline)) {
        const uint8_t *sA = lds, *sB = lds + BM * PT;
        // 32 bytes of each row per MFMA step: 32 k of int8, or 64 k of e2m1 codes into
        // the FP4 form (FP32 accumulators in the same registers, bit-cast)
        const int ksteps = (min(KT, kp - st * KT) + 31) / 32;  // bytes past k are zero
        for (int ks = 0; ks < ksteps; ++ks) {
            ix4 bf[FN];
#pragma unroll
            for (int ni = 0; ni < FN; ++ni)
                bf[ni] = *(const ix4 *)&sB[(wn * WTN + ni * 32 + (lane & 31)) * PT + ks * 32 + 16 * (lane >> 5)];
#pragma unroll
            for (int mi = 0; mi < FM; ++mi) {
                const ix4 af = *(const ix4 *)&sA[(wm * WTM + mi * 32 + (lane & 31)) * PT + ks * 32 + 16 * (lane >> 5)];
#pragma unroll
                for (int ni = 0; ni < FN; ++ni) {
                    if constexpr (fp4) {
                        const ix4 b = bf[ni];
                        const fx16 f = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(
                            ix8{af.x, af.y, af.z, af.w, 0, 0, 0, 0}, ix8{b.x, b.y, b.z, b.w, 0, 0, 0, 0},
                            __builtin_bit_cast(fx16, acc[mi][ni]), 4, 4, 0, 127, 0, 127);
                        acc[mi][ni] = __builtin_bit_cast(ix16, f);
                    } else {
                        acc[mi][ni] = __builtin_amdgcn_mfma_i32_32x32x32_i8(af, bf[ni], acc[mi][ni], 0, 0, 0);
                    }
                }
            }
        }
        __syncthreads();  // the stage's LDS is read before the next one (or tile) overwrites it
    };
    // The last stage is peeled off: it loads nothing, so no load is in flight when
    // the epilogue's stores go out, and the next tile's first loads need not wait
    // for those stores (a load that might still be pending would make them wait).
    // A product with k = 0 (no stages) loads nothing at all.
    if (stages > 0) {
        fetch(0);
        for (int st = 0; st + 1 < stages; ++st) {
            publish();
            fetch(st + 1);
            compute(st);
        }
        publish();
        compute(stages - 1);
    }
    // Epilogue: every C offset of a product fits 32 bits (checked on the host), so a
    // store is a uniform base plus one 32-bit lane offset.  Register r of a block
    // holds row 8 (r/4) + 4 (l/32) + r % 4 of column l % 32.
    QMM_GLOBAL uint8_t *cbase = (QMM_GLOBAL uint8_t *)D.C;
    const uint32_t ldc = (uint32_t)D.ldc;
    const bool full = row0 + BM <= D.m && col0 + BN <= D.n;
    auto residue = [&](int32_t bits) __attribute__((always_inline)) {
        return mod_u32_m32((uint32_t)acc_value(bits, fp4) + D.off, D.p, D.magic32);
    };
    if (full) {
        // Interior tile: registers 4q .. 4q+3 (rows R .. R+3 of one column) packed
        // into a dword and transposed across the lane's quad become 4 consecutive
        // bytes of row R + l % 4: one dword store each, unaligned when ldc or C is
        // not a multiple of 4 (served like the unaligned loads of load16_any).
        const int j = lane & 3;
        const uint32_t b0 = (uint32_t)(row0 + wm * WTM + 4 * (lane >> 5) + j) * ldc +
                            (uint32_t)(col0 + wn * WTN + (lane & 31) - j);
#pragma unroll
        for (int mi = 0; mi < FM; ++mi)
#pragma unroll
            for (int ni = 0; ni < FN; ++ni)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    uint32_t w = 0;
#pragma unroll
                    for (int i = 0; i < 4; ++i) w |= residue(acc[mi][ni][4 * q + i]) << (8 * i);
                    w = quad_transpose_bytes(w, j);
                    *(QMM_GLOBAL u32a1 *)(cbase + b0 + (uint32_t)(mi * 32 + 8 * q) * ldc + ni * 32) = w;
                }
    } else {
#pragma unroll
        for (int mi = 0; mi < FM; ++mi)
#pragma unroll
            for (int ni = 0; ni < FN; ++ni) {
                const uint32_t rl = (uint32_t)(row0 + wm * WTM + mi * 32 + 4 * (lane >> 5));
                const uint32_t cl = (uint32_t)(col0 + wn * WTN + ni * 32 + (lane & 31));
                const uint32_t off0 = rl * ldc + cl;
                if (full) {
#pragma unroll
                    for (int r = 0; r < 16; ++r)
                        cbase[off0 + (uint32_t)(8 * (r >> 2) + (r & 3)) * ldc] = (uint8_t)residue(acc[mi][ni][r]);
                } else {
#pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        const uint32_t rr = (uint32_t)(8 * (r >> 2) + (r & 3));
                        if (rl + rr < (uint32_t)D.m && cl < (uint32_t)D.n) cbase[off0 + rr * ldc] = (uint8_t)residue(acc[mi][ni][r]);
                    }
                }
            }
    }
}

// One FP64 Q-adic tile of 64 x 64 outputs: rows of A packed reversed and columns
// of B packed forward straight from the bytes (Horner over the d+1 residues of a
// chunk), 16 words per stage, MFMA f64 16x16x4, digit d of every word mod p.
__device__ __forceinline__ void fp64_tile(const Desc &D, int tm, int tn, double *sA, double *sB) {
    // sA: 64 rows x (KW + 1) words; sB: KW rows x 64 words
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int64_t row0 = (int64_t)tm * 64, col0 = (int64_t)tn * 64;
    const uint32_t e = D.d + 1;
    const int nw = (int)((D.k + e - 1) / e);
    dx4 acc[2][2];
    const double start = D.start;
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int ni = 0; ni < 2; ++ni) acc[mi][ni] = dx4{start, start, start, start};
    const int nst = (nw + KW - 1) / KW;
    for (int st = 0; st < nst; ++st) {
        const int l0 = st * KW;
        // 64 x 16 A words and 16 x 64 B words: four of each per thread
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int c = tid + NT * i;
            {   // A word (row r, word l)
                const int r = c >> 4, l = l0 + (c & 15);
                const int64_t row = row0 + r;
                uint64_t w = 0;
                if (row < D.m && l < nw) {
                    const uint8_t *a = D.A + row * D.lda;
                    for (uint32_t s = 0; s < e; ++s) {
                        const int64_t kk = (int64_t)l * e + s;
                        w = (w << D.t) | (kk < D.k ? (uint64_t)a[kk] : 0ull);
                    }
                }
                sA[r * (KW + 1) + (c & 15)] = (double)w;
            }
            {   // B word (word l, column j)
                const int lr = c >> 6, j = c & 63;
                const int l = l0 + lr;
                const int64_t col = col0 + j;
                uint64_t w = 0;
                if (col < D.n && l < nw) {
                    for (int32_t s = (int32_t)e - 1; s >= 0; --s) {
                        const int64_t kk = (int64_t)l * e + s;
                        w = (w << D.t) | (kk < D.k ? (uint64_t)D.B[kk * D.ldb + col] : 0ull);
                    }
                }
                sB[lr * 64 + j] = (double)w;
            }
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < KW / 4; ++ks) {
            double af[2], bf[2];
#pragma unroll
            for (int mi = 0; mi < 2; ++mi) af[mi] = sA[(wm * 32 + mi * 16 + (lane & 15)) * (KW + 1) + ks * 4 + (lane >> 4)];
#pragma unroll
            for (int ni = 0; ni < 2; ++ni) bf[ni] = sB[(ks * 4 + (lane >> 4)) * 64 + wn * 32 + ni * 16 + (lane & 15)];
#pragma unroll
            for (int mi = 0; mi < 2; ++mi)
#pragma unroll
                for (int ni = 0; ni < 2; ++ni)
                    acc[mi][ni] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[mi], bf[ni], acc[mi][ni], 0, 0, 0);
        }
        __syncthreads();
    }
    const uint32_t td = D.t * D.d;
    const uint64_t qmask = (1ull << D.t) - 1;
    const bool offset = D.offset_regime != 0;
    // lane l, register r holds D[(l >> 4) + 4 r][l & 15]
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int ni = 0; ni < 2; ++ni)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t row = row0 + wm * 32 + mi * 16 + (lane >> 4) + 4 * r;
                const int64_t col = col0 + wn * 32 + ni * 16 + (lane & 15);
                if (row < D.m && col < D.n)
                    D.C[row * D.ldc + col] = (uint8_t)mod_u64(qadic_digit<double>(acc[mi][ni][r], offset, td, qmask), D.p, D.invp);
            }
}

// One persistent kernel per tile class (so each gets the registers and occupancy
// of its own shape).  Workgroup w takes tiles w, w + G, w + 2G, ... of its class's
// list, which is sorted longest first.
template <uint32_t SHAPE, bool FP4>
__global__ __launch_bounds__(NT, SHAPE == SHAPE_128x128 ? 3 : (SHAPE == SHAPE_64x64 && !FP4 ? 7 : 5))
void batched_int8_kernel(const Desc *__restrict__ descs, const TileRef *__restrict__ tiles, int32_t ntiles) {
    __shared__ __attribute__((aligned(16))) uint8_t lds[tile_lds_bytes(shape_bm(SHAPE), shape_bn(SHAPE))];
    for (int32_t i = blockIdx.x; i < ntiles; i += gridDim.x) {
        const TileRef tr = tiles[i];
        const Desc D = descs[tr.desc];
        int8_tile<shape_bm(SHAPE), shape_bn(SHAPE), shape_wgm(SHAPE), 4 / shape_wgm(SHAPE), FP4>(D, tr.tm, tr.tn, lds);
    }
}

// One tile of a raw batch: everything its workgroup needs in one record, the
// operand bases moved to the tile's origin (row0, col0), so a tile starts without
// a dependent descriptor lookup.  Sizes are bytes of data from the moved bases.
struct RawTile {
    const uint8_t *A;          // A + row0 lda
    const uint8_t *B;          // B + col0
    uint8_t *C;                // C + row0 ldc + col0
    uint32_t lda, ldb, ldc;
    int32_t rows, cols, k;     // m - row0, n - col0, k
    uint32_t a_size, b_size;   // (rows - 1) lda + k and (k - 1) ldb + cols (0 when k = 0)
    uint32_t p, off, magic32;  // modulus, epilogue offset (0 for uncentred sums), floor(2^32 / p)
    uint32_t add_h, neg_p;     // centring constants (0: residues used as they are)
    uint32_t pad[5];
};
static_assert(sizeof(RawTile) == 96, "RawTile is 24 dwords");
constexpr int kRawTileDwords = (int)(sizeof(RawTile) / 4);

// The record of the next tile, loaded by lanes 0 .. 23 as vector loads (so its
// wait is ordered with the operand loads', not with the LDS traffic), then read
// back into uniform registers lane by lane.
__device__ __forceinline__ uint32_t raw_record_issue(const RawTile *recs, int32_t i, int lane) {
    const QMM_GLOBAL uint32_t *w = (const QMM_GLOBAL uint32_t *)(recs + i);
    return w[lane < kRawTileDwords ? lane : 0];  // every lane loads: no branch around the load
}
__device__ __forceinline__ RawTile raw_record_read(uint32_t v) {
    uint32_t d[kRawTileDwords];
#pragma unroll
    for (int j = 0; j < kRawTileDwords; ++j) d[j] = __builtin_amdgcn_readlane(v, j);
    return __builtin_bit_cast(RawTile, d);
}

// Persistent raw tiles of one shape: A's rows and B's k-rows come straight from the
// products' residue matrices as unaligned 16-byte loads (A centred in registers when
// the product needs it; B's k-rows go to LDS as they are and the MFMA's B fragments
// are read from them with the LDS transpose load).  Workgroup w takes records w,
// w + G, ... and runs their K stages as one pipeline: while a stage computes, the
// next stage's loads are in flight, and the next tile's first stage and record are
// loaded during the current tile's last stage, so neither a tile's first loads nor
// its record wait in the open.  One LDS buffer (so several workgroups share a CU).
template <uint32_t SHAPE>
__global__ __launch_bounds__(NT, SHAPE == SHAPE_128x128 ? 3 : 5)
void batched_raw_kernel(const RawTile *__restrict__ recs, int32_t ntiles) {
    constexpr int BM = shape_bm(SHAPE), BN = shape_bn(SHAPE), WGM = shape_wgm(SHAPE), WGN = 4 / WGM;
    constexpr int WTM = BM / WGM, WTN = BN / WGN, FM = WTM / 32, FN = WTN / 32;
    constexpr int SEGS = KT / 16, CSEG = BN / 16, RSTEP = NT / SEGS;
    constexpr int A_LOADS = BM * SEGS / NT, B_LOADS = KT * CSEG / NT;
    // LDS: A's stage as BM rows of 128 bytes, B's as KT k-rows of BN bytes.  A (and B
    // when BN = 128) without padding, 16-byte chunk c of row r at position
    // c ^ swz(r), swz(r) = (r % 8) ^ ((r / 8) % 2): the register writes (8 lanes per
    // row, 16 lanes on two rows), the A fragment reads (16 lanes on 16 rows at one
    // chunk) and the B transpose reads (32 lanes on 8 rows, two chunks) each touch
    // every bank once.  Narrower B keeps rows of BN + 16 bytes.
    constexpr bool BSWZ = BN == 128;
    constexpr int BP = BSWZ ? BN : raw_bpitch(BN);
    constexpr int A_BYTES = BM * KT;
    static_assert(A_LOADS * NT == BM * SEGS && B_LOADS * NT == KT * CSEG, "whole load steps");
    __shared__ __attribute__((aligned(16))) uint8_t lds[A_BYTES + KT * BP];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave / WGN, wn = wave % WGN;
    // thread tid loads 16-byte segment seg of A rows rfirst + RSTEP i, and B segment
    // c = tid + NT i: k-row c / CSEG of the stage, columns 16 (c % CSEG) ..
    const int seg = tid % SEGS, rfirst = tid / SEGS;
    const uint32_t bcol = 16u * (uint32_t)(tid % CSEG);
    // swizzles: of this thread's A rows rfirst + RSTEP i (RSTEP = 32), of its B k-rows
    // (tid + NT i) / 8 when BN = 128, of the fragment rows 32 x + l % 32
    const int a_swz = (rfirst & 7) ^ ((rfirst >> 3) & 1);
    const int b_swz = ((tid >> 3) & 7) ^ ((tid >> 6) & 1);
    const int f_swz = (lane & 7) ^ ((lane >> 3) & 1);

    ix4 ra[A_LOADS], rb[B_LOADS];
    uint32_t sa[A_LOADS], sb[B_LOADS];
    auto as_ix4 = [](uint4v_t v) { return ix4{(int)v.x, (int)v.y, (int)v.z, (int)v.w}; };
    // Issue stage st of tile t.  A's bytes past k in a row are the next row's: they
    // meet B's k-rows past k, which are zero, so they add nothing.  B's columns past
    // the product's n reach only outputs that are not stored.
    auto fetch = [&](const RawTile &t, int st) __attribute__((always_inline)) {
        const int32_t kk = st * KT + 16 * seg;
        const bool bcol_ok = (int32_t)bcol < t.cols;
        if (t.a_size >= 16u && t.b_size >= 16u) {
#pragma unroll
            for (int i = 0; i < A_LOADS; ++i) {
                const int32_t r = rfirst + i * RSTEP;
                ra[i] = as_ix4(load16_clamped(t.A, (uint32_t)r * t.lda + (uint32_t)kk, r < t.rows && kk < t.k, t.a_size, sa[i]));
            }
#pragma unroll
            for (int i = 0; i < B_LOADS; ++i) {
                const int32_t kr = st * KT + (tid + NT * i) / CSEG;
                rb[i] = as_ix4(load16_clamped(t.B, (uint32_t)kr * t.ldb + bcol, kr < t.k && bcol_ok, t.b_size, sb[i]));
            }
        } else {  // an operand under 16 bytes from the tile's origin: byte loads
#pragma unroll
            for (int i = 0; i < A_LOADS; ++i) {
                const int32_t r = rfirst + i * RSTEP;
                ra[i] = as_ix4(load16_tiny(t.A, (uint32_t)r * t.lda + (uint32_t)kk, r < t.rows && kk < t.k, t.a_size));
                sa[i] = 0;
            }
#pragma unroll
            for (int i = 0; i < B_LOADS; ++i) {
                const int32_t kr = st * KT + (tid + NT * i) / CSEG;
                rb[i] = as_ix4(load16_tiny(t.B, (uint32_t)kr * t.ldb + bcol, kr < t.k && bcol_ok, t.b_size));
                sb[i] = 0;
            }
        }
    };
    auto publish = [&](const RawTile &t) __attribute__((always_inline)) {
        auto fix = [](ix4 v, uint32_t sh) {
            return sh ? __builtin_bit_cast(ix4, shift_down_bytes(__builtin_bit_cast(uint4v_t, v), sh)) : v;
        };
#pragma unroll
        for (int i = 0; i < A_LOADS; ++i) ra[i] = fix(ra[i], sa[i]);
#pragma unroll
        for (int i = 0; i < B_LOADS; ++i) rb[i] = fix(rb[i], sb[i]);
        if (t.neg_p != 0) {
            auto centre = [&](ix4 v) {
                return ix4{(int)centre4((uint32_t)v.x, t.add_h, t.neg_p), (int)centre4((uint32_t)v.y, t.add_h, t.neg_p),
                           (int)centre4((uint32_t)v.z, t.add_h, t.neg_p), (int)centre4((uint32_t)v.w, t.add_h, t.neg_p)};
            };
#pragma unroll
            for (int i = 0; i < A_LOADS; ++i) ra[i] = centre(ra[i]);
#pragma unroll
            for (int i = 0; i < B_LOADS; ++i) rb[i] = centre(rb[i]);
        }
#pragma unroll
        for (int i = 0; i < A_LOADS; ++i) *(ix4 *)&lds[(rfirst + i * RSTEP) * KT + 16 * (seg ^ a_swz)] = ra[i];
#pragma unroll
        for (int i = 0; i < B_LOADS; ++i) {
            const int c = tid + NT * i, kr = c / CSEG, cs = c % CSEG;
            *(ix4 *)&lds[A_BYTES + kr * BP + 16 * (BSWZ ? cs ^ b_swz : cs)] = rb[i];
        }
        __syncthreads();
    };
    ix16 acc[FM][FN];
    auto compute = [&](const RawTile &t, int st) __attribute__((always_inline)) {
        const uint8_t *sA = lds, *sB = lds + A_BYTES;
        const int ksteps = (min(KT, t.k - st * KT) + 31) / 32;
        const int g = lane >> 4, sl = lane & 15;
        for (int ks = 0; ks < ksteps; ++ks) {
            // lane l's B fragment: column l % 32 of the block, k-bytes 16 (l / 32) .. + 15
            // of the step, as two transpose loads of 8 k-rows: group g = l / 16 reads rows
            // 16 (g / 2) .., columns 16 (g % 2) .., lane 2b + c of the group giving bytes
            // 8c .. 8c + 7 of row b
            ix4 bf[FN];
#pragma unroll
            for (int ni = 0; ni < FN; ++ni) {
                // rows 16 (g / 2) + sl / 2 and 8 more: swz = sl / 2 and sl / 2 ^ 1
                const int row = ks * 32 + 16 * (g >> 1) + (sl >> 1), chunk = (wn * WTN + ni * 32) / 16 + (g & 1);
                const uint8_t *bp0, *bp1;
                if constexpr (BSWZ) {
                    bp0 = &sB[row * BP + 16 * (chunk ^ (sl >> 1)) + 8 * (sl & 1)];
                    bp1 = &sB[(row + 8) * BP + 16 * (chunk ^ (sl >> 1) ^ 1) + 8 * (sl & 1)];
                } else {
                    bp0 = &sB[row * BP + 16 * chunk + 8 * (sl & 1)];
                    bp1 = bp0 + 8 * BP;
                }
                const v2i b0 = __builtin_amdgcn_ds_read_tr8_b64_v2i32((__attribute__((address_space(3))) v2i *)bp0);
                const v2i b1 = __builtin_amdgcn_ds_read_tr8_b64_v2i32((__attribute__((address_space(3))) v2i *)bp1);
                bf[ni] = ix4{b0.x, b0.y, b1.x, b1.y};
            }
#pragma unroll
            for (int mi = 0; mi < FM; ++mi) {
                const ix4 af = *(const ix4 *)&sA[(wm * WTM + mi * 32 + (lane & 31)) * KT + 16 * ((2 * ks + (lane >> 5)) ^ f_swz)];
#pragma unroll
                for (int ni = 0; ni < FN; ++ni) acc[mi][ni] = __builtin_amdgcn_mfma_i32_32x32x32_i8(af, bf[ni], acc[mi][ni], 0, 0, 0);
            }
        }
        __syncthreads();  // the stage's LDS is read before the next stage overwrites it
    };
    // Epilogue: register r of a block holds row 8 (r/4) + 4 (l/32) + r % 4 of column
    // l % 32; every C offset of a product fits 32 bits (checked on the host).
    auto epilogue = [&](const RawTile &t) __attribute__((always_inline)) {
        QMM_GLOBAL uint8_t *cbase = (QMM_GLOBAL uint8_t *)t.C;
        auto residue = [&](int32_t v) { return mod_u32_m32((uint32_t)v + t.off, t.p, t.magic32); };
        // Registers 4q .. 4q+3 (rows R .. R+3 of one column) packed into a dword and
        // transposed across the lane's quad become 4 consecutive bytes of row R + l % 4,
        // columns c .. c+3 (c a multiple of 4): one dword store (unaligned when ldc or C
        // is not a multiple of 4); on a tile's edge, byte stores for a quad that the
        // product's last column cuts, nothing past its last row.
        const int j = lane & 3;
        const int32_t r0 = wm * WTM + 4 * (lane >> 5) + j, c0 = wn * WTN + (lane & 31) - j;
        const bool whole = t.rows >= BM && t.cols >= BN;
#pragma unroll
        for (int mi = 0; mi < FM; ++mi)
#pragma unroll
            for (int ni = 0; ni < FN; ++ni)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    uint32_t w = 0;
#pragma unroll
                    for (int i = 0; i < 4; ++i) w |= residue(acc[mi][ni][4 * q + i]) << (8 * i);
                    w = quad_transpose_bytes(w, j);
                    const int32_t r = r0 + mi * 32 + 8 * q, c = c0 + ni * 32;
                    QMM_GLOBAL uint8_t *dst = cbase + (uint32_t)r * t.ldc + (uint32_t)c;
                    if (whole || (r < t.rows && c + 4 <= t.cols)) {
                        *(QMM_GLOBAL u32a1 *)dst = w;
                    } else if (r < t.rows && c < t.cols) {
                        const int32_t nb = t.cols - c;  // 1 .. 3 bytes
                        dst[0] = (uint8_t)w;
                        if (nb > 1) dst[1] = (uint8_t)(w >> 8);
                        if (nb > 2) dst[2] = (uint8_t)(w >> 16);
                    }
                }
    };

    int32_t i = blockIdx.x;
    if (i >= ntiles) return;
    RawTile t = recs[i];
    fetch(t, 0);
    for (;;) {
        const int32_t inext = i + (int32_t)gridDim.x;
        const bool more = inext < ntiles;
        // the next record stays in one vector register (lane j: dword j) until used
        const uint32_t rv = raw_record_issue(recs, more ? inext : i, lane);
#pragma unroll
        for (int mi = 0; mi < FM; ++mi)
#pragma unroll
            for (int ni = 0; ni < FN; ++ni) acc[mi][ni] = ix16{};
        const int stages = (t.k + KT - 1) / KT;
        for (int st = 0; st < stages; ++st) {
            publish(t);
            if (st + 1 < stages)
                fetch(t, st + 1);
            else if (more)
                fetch(raw_record_read(rv), 0);
            compute(t, st);
        }
        if (more && stages == 0) fetch(raw_record_read(rv), 0);  // k = 0: nothing to wait for
        epilogue(t);
        if (!more) break;
        t = raw_record_read(rv);
        i = inext;
    }
}

__global__ __launch_bounds__(NT) void batched_fp64_kernel(const Desc *__restrict__ descs,
                                                          const TileRef *__restrict__ tiles, int32_t ntiles) {
    __shared__ __attribute__((aligned(16))) double lds[64 * (KW + 1) + KW * 64];
    for (int32_t i = blockIdx.x; i < ntiles; i += gridDim.x) {
        const TileRef tr = tiles[i];
        const Desc D = descs[tr.desc];
        fp64_tile(D, tr.tm, tr.tn, lds, lds + 64 * (KW + 1));
    }
}

// Autotuner cost model of one INT8 tile: a fixed part (tile set-up, epilogue) and a
// part per 128-byte K stage, in units of one K stage of the 64 x 64 shape.  Every
// shape does the same MFMA work per stage (four 32x32x32 blocks per wavefront);
// the defaults are the analytic prior and qmm_batched_tune replaces them with a
// fit to timed launches of each shape.
struct ShapeCost {
    double fixed, per_stage;
};
ShapeCost g_costs[SHAPE_COUNT] = {{2.0, 1.0}, {2.0, 1.1}, {2.0, 1.1}, {3.0, 3.0}};

double tile_cost(const ShapeCost *costs, uint32_t shape, int64_t m, int64_t n, int64_t k) {
    const int64_t tiles = ceil_div(m, shape_bm(shape)) * ceil_div(n, shape_bn(shape));
    return (double)tiles * (costs[shape].fixed + costs[shape].per_stage * (double)ceil_div(k, KT));
}

uint32_t tune_shape(const ShapeCost *costs, int64_t m, int64_t n, int64_t k) {
    uint32_t best = SHAPE_64x64;
    double bc = tile_cost(costs, SHAPE_64x64, m, n, k);
    for (uint32_t s = 1; s < SHAPE_COUNT; ++s) {
        const double c = tile_cost(costs, s, m, n, k);
        if (c < bc) {
            bc = c;
            best = s;
        }
    }
    return best;
}

qmm_status hip_fail(hipError_t e, const char *what) {
    return fail(QMM_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// Architecture name of the current device ("gfx950"), the key of the tune cache.
qmm_status device_arch(std::string &arch) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    hipDeviceProp_t prop;
    if ((e = hipGetDeviceProperties(&prop, dev)) != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
    arch = prop.gcnArchName;
    const size_t colon = arch.find(':');
    if (colon != std::string::npos) arch.resize(colon);
    return QMM_OK;
}

// A single small product on the FP64 Q-adic path in one launch: one workgroup per
// 64 x 64 tile packs its rows of A (reversed) and columns of B (forward) straight
// from the bytes into LDS, as the batched FP64 tiles do; no packed operands in HBM
// and no separate pack launches.
__global__ __launch_bounds__(NT) void fused_qadic_kernel(Desc D, int32_t tiles_n) {
    __shared__ __attribute__((aligned(16))) double lds[64 * (KW + 1) + KW * 64];
    const int tm = (int)(blockIdx.x / (uint32_t)tiles_n), tn = (int)(blockIdx.x % (uint32_t)tiles_n);
    fp64_tile(D, tm, tn, lds, lds + 64 * (KW + 1));
}

}  // namespace

qmm_status launch_gemm_qadic_fused(const qmm_plan &pl, int64_t m, int64_t n, int64_t k, const uint8_t *A,
                                   int64_t lda, const uint8_t *B, int64_t ldb, uint8_t *C, int64_t ldc,
                                   void *stream) {
    if (m == 0 || n == 0) return QMM_OK;
    if (pl.beta != 53 || !path_is_qadic(pl.path) || pl.k_block < k || pl.t > 63 ||
        (uint64_t)pl.t * (pl.d + 1) > 64 || m > INT32_MAX || n > INT32_MAX || k > INT32_MAX)
        return fail(QMM_EUNSUPPORTED, "the fused Q-adic kernel takes unblocked FP64 plans and 32-bit sizes");
    Desc D;
    std::memset(&D, 0, sizeof(D));
    D.A = A;
    D.B = B;
    D.C = C;
    D.lda = lda;
    D.ldb = ldb;
    D.ldc = ldc;
    D.m = (int32_t)m;
    D.n = (int32_t)n;
    D.k = (int32_t)k;
    D.p = pl.p;
    D.path = QMM_PATH_FP64_QADIC;
    D.invp = 1.0 / (double)pl.p;
    D.t = pl.t;
    D.d = pl.d;
    D.offset_regime = pl.regime == QMM_REGIME_OFFSET;
    D.start = D.offset_regime ? std::ldexp(1.0, 52 + (int)(pl.t * pl.d)) : 0.0;
    const int64_t tiles_m = ceil_div(m, 64), tiles_n = ceil_div(n, 64);
    if (tiles_m * tiles_n > INT32_MAX) return fail(QMM_EUNSUPPORTED, "too many tiles for the fused Q-adic kernel");
    fused_qadic_kernel<<<dim3((unsigned)(tiles_m * tiles_n)), NT, 0, (hipStream_t)stream>>>(D, (int32_t)tiles_n);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? QMM_OK : hip_fail(e, "fused_qadic_kernel");
}

}  // namespace qmm

using namespace qmm;

// Tile classes: the three INT8 shapes and the FP64 Q-adic tile.
// Tile classes: the four INT8 shapes, the same four for FP4 products, and the FP64
// Q-adic tile.
constexpr int kFp4Class = SHAPE_COUNT, kFp64Class = 2 * SHAPE_COUNT;
constexpr int kClasses = 2 * SHAPE_COUNT + 1;
constexpr int kXcds = 8;  // accelerator complex dies, one L2 each

struct qmm_batched {
    int64_t count = 0;
    std::vector<qmm_plan> plans;
    Desc *d_desc = nullptr;
    TileRef *d_tiles = nullptr;
    RawTile *d_raw = nullptr;  // raw batches: one record per INT8 tile, in d_tiles' order
    int32_t ntiles = 0;
    PackJob *d_jobs = nullptr;
    int32_t njobs = 0;
    int8_t *d_ws = nullptr;   // centred, padded INT8 operands
    size_t ws_bytes = 0;
    int32_t class_first[kClasses] = {}, class_count[kClasses] = {};
    bool raw = false;               // INT8 tiles read the residue matrices themselves (no pack kernel)
    hipStream_t capture = nullptr;  // the stream the graph was recorded on
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

void release(qmm_batched *b) {
    if (!b) return;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->capture) (void)hipStreamDestroy(b->capture);
    if (b->d_desc) (void)hipFree(b->d_desc);
    if (b->d_tiles) (void)hipFree(b->d_tiles);
    if (b->d_raw) (void)hipFree(b->d_raw);
    if (b->d_jobs) (void)hipFree(b->d_jobs);
    if (b->d_ws) (void)hipFree(b->d_ws);
    delete b;
}

qmm_status build_batch(int64_t count, const qmm_problem *probs, uint32_t flags, qmm_batched *b) {
    b->count = count;
    b->raw = (flags & QMM_BATCH_RAW) != 0;
    if (b->raw) flags |= QMM_BATCH_INT8_ONLY;  // raw tiles centre bytes; FP4 codes need the pack
    b->plans.resize((size_t)count);
    const qmm_status st0 = tune_cache_load_env_once();
    if (st0 != QMM_OK) return st0;
    std::string arch;        // the device's, looked up at the first tile-cost lookup
    bool arch_known = false;
    std::vector<Desc> descs((size_t)count);
    std::vector<std::pair<double, TileRef>> tiles[kClasses];
    std::vector<PackJob> jobs;
    std::vector<size_t> a_off((size_t)count, 0), b_off((size_t)count, 0);
    size_t ws = 0;
    for (int64_t i = 0; i < count; ++i) {
        const qmm_problem &P = probs[i];
        if (P.p < 2 || P.p > 256) return fail(QMM_EINVAL, "problem " + std::to_string(i) + ": byte residues need 2 <= p <= 256");
        if (P.m < 0 || P.n < 0 || P.k < 0 || P.m > INT32_MAX / 2 || P.n > INT32_MAX / 2 || P.k > INT32_MAX / 2)
            return fail(QMM_EINVAL, "problem " + std::to_string(i) + ": bad size");
        if ((P.m && P.k && (!P.A || P.lda < P.k)) || (P.k && P.n && (!P.B || P.ldb < P.n)) ||
            (P.m && P.n && (!P.C || P.ldc < P.n)))
            return fail(QMM_EINVAL, "problem " + std::to_string(i) + ": bad pointer or leading dimension");
        qmm_plan pl;
        qmm_status st;
        if (flags & QMM_BATCH_FORCE_FP64) {
            st = qmm_choose_Qd(P.p, P.m, P.n, P.k, 53, QMM_PATH_FP64_QADIC, QMM_PLAN_UNBLOCKED, &pl);
        } else {
            // FP4 codes when every centred residue is an e2m1 value (p <= 8) and the
            // whole k is one exact FP32 block; INT8 otherwise
            st = QMM_EINVAL;
            if (!(flags & QMM_BATCH_INT8_ONLY) && P.p <= 8) {
                st = qmm_choose_Qd(P.p, P.m, P.n, P.k, 0, QMM_PATH_FP4, 0, &pl);
                if (st == QMM_OK && pl.k_block < P.k) st = QMM_EBOUND;
            }
            if (st != QMM_OK) st = qmm_choose_Qd(P.p, P.m, P.n, P.k, 0, QMM_PATH_INT8, 0, &pl);
        }
        if (st != QMM_OK) return st;
        const bool lowp = pl.path == QMM_PATH_INT8 || pl.path == QMM_PATH_FP4;
        if (pl.path == QMM_PATH_INT8 && pl.k_block < P.k)
            return fail(QMM_EUNSUPPORTED, "problem " + std::to_string(i) + ": k needs blocked int32 accumulation, "
                                          "which the batched kernel does not do");
        if (lowp && b->raw && ((P.m > 0 && P.k > 0 && (P.m - 1) * P.lda + P.k > kRawSpan) ||
                               (P.k > 0 && P.n > 0 && (P.k - 1) * P.ldb + P.n > kRawSpan)))
            return fail(QMM_EUNSUPPORTED, "problem " + std::to_string(i) + ": A or B spans more than 2^32 - 64 bytes, "
                                          "past the raw tiles' 32-bit operand offsets");
        if (lowp && P.m > 0 && P.n > 0 && (P.m - 1) * P.ldc + P.n > (int64_t)UINT32_MAX)
            return fail(QMM_EUNSUPPORTED, "problem " + std::to_string(i) + ": C spans more than 2^32 bytes, "
                                          "past the batched kernel's 32-bit output offsets");
        Desc &D = descs[(size_t)i];
        std::memset(&D, 0, sizeof(D));
        D.A = P.A;
        D.B = P.B;
        D.C = P.C;
        D.lda = P.lda;
        D.ldb = P.ldb;
        D.ldc = P.ldc;
        D.m = (int32_t)P.m;
        D.n = (int32_t)P.n;
        D.k = (int32_t)P.k;
        D.p = P.p;
        D.path = pl.path;
        D.magic = mod_magic(P.p);
        D.off = P.p * ((1u << 31) / P.p);
        D.magic32 = (uint32_t)((1ull << 32) / P.p);
        D.invp = 1.0 / (double)P.p;
        int bm = 64, bn = 64;
        ShapeCost costs[SHAPE_COUNT];  // the product's tile costs (INT8 and FP4 tiles)
        if (lowp) {
            const uint32_t h = (P.p - 1) / 2;
            D.add_h = (127u - h) * 0x01010101u;
            D.neg_p = (256u - P.p) & 0xffu;
            D.fp4 = pl.path == QMM_PATH_FP4;
            if (D.fp4) fp4_lut(P.p, D.lut_lo, D.lut_hi);
            const uint32_t forced = (flags & QMM_BATCH_SHAPE_MASK) >> 8;  // 1 + shape, 0 = autotuned
            // costs tuned for this architecture, encoding and shape bucket when the
            // cache has them, else the current defaults
            double cached[kTuneCosts];
            if (!arch_known) {
                if (device_arch(arch) != QMM_OK) arch.clear();  // no device: no cached costs apply
                arch_known = true;
            }
            if (!arch.empty() && tune_cache_lookup(arch, D.fp4 ? 1u : 0u, tune_bucket(P.m, P.n), cached)) {
                for (uint32_t sh = 0; sh < SHAPE_COUNT; ++sh) costs[sh] = ShapeCost{cached[2 * sh], cached[2 * sh + 1]};
            } else {
                for (uint32_t sh = 0; sh < SHAPE_COUNT; ++sh) costs[sh] = g_costs[sh];
            }
            D.shape = forced ? forced - 1 : tune_shape(costs, P.m, P.n, P.k);
            pl.tile = D.shape;
            bm = shape_bm(D.shape);
            bn = shape_bn(D.shape);
        } else {
            D.t = pl.t;
            D.d = pl.d;
            D.offset_regime = pl.regime == QMM_REGIME_OFFSET;
            D.start = D.offset_regime ? std::ldexp(1.0, 52 + (int)(pl.t * pl.d)) : 0.0;
        }
        // Raw tiles read residues in place: below 128 they are already int8 values
        // (non-negative), and when k (p-1)^2 fits int32 the uncentred sum is exact, so
        // these products skip the centring and the epilogue's offset (neg_p = 0 says so).
        if (lowp && b->raw && P.p <= 128 && (uint64_t)P.k * (P.p - 1) * (P.p - 1) <= (uint64_t)INT32_MAX)
            D.add_h = D.neg_p = D.off = 0;
        b->plans[(size_t)i] = pl;
        if (P.m == 0 || P.n == 0) continue;
        if (lowp && b->raw) {
            D.kp = D.kpb = D.k;  // operands read in place
        } else if (lowp) {
            // workspace: Ac (mp x kpb) then Bt (np x kpb), each 256-byte aligned
            D.kp = (int32_t)(ceil_div(P.k, KP_ALIGN) * KP_ALIGN);
            D.kpb = D.fp4 ? D.kp / 2 : D.kp;
            D.mp = (int32_t)(ceil_div(P.m, bm) * bm);
            D.np = (int32_t)(ceil_div(P.n, bn) * bn);
            a_off[(size_t)i] = ws;
            ws += (size_t)ceil_div((int64_t)D.mp * D.kpb, 256) * 256;
            b_off[(size_t)i] = ws;
            ws += (size_t)ceil_div((int64_t)D.np * D.kpb, 256) * 256;
            for (int32_t r0 = 0; r0 < D.m; r0 += 64)
                for (int32_t c0 = 0; c0 < D.kp; c0 += PACK_K) jobs.push_back(PackJob{(int32_t)i, 0, r0, c0});
            for (int32_t r0 = 0; r0 < D.kp; r0 += PACK_K)
                for (int32_t c0 = 0; c0 < D.n; c0 += 64) jobs.push_back(PackJob{(int32_t)i, 1, r0, c0});
        }
        const int32_t tmax = (int32_t)ceil_div(P.m, bm), nmax = (int32_t)ceil_div(P.n, bn);
        // cost in K-stage units: an FP4 tile streams half the bytes of an INT8 one
        const double cost = lowp ? tile_cost(costs, D.shape, bm, bn, D.fp4 ? ceil_div(P.k, 2) : P.k)
                                 : (double)ceil_div(words_for(P.k < 1 ? 1 : P.k, pl.d), KW) * 4.0;
        const int cls = lowp ? (int)D.shape + (D.fp4 ? kFp4Class : 0) : kFp64Class;
        for (int32_t tm = 0; tm < tmax; ++tm)
            for (int32_t tn = 0; tn < nmax; ++tn) tiles[cls].push_back({cost, TileRef{(int32_t)i, tm, tn, 0}});
    }
    hipError_t e;
    int dev = 0, cus = 0;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return hip_fail(e, "hipGetDevice");
    if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return hip_fail(e, "attribute");
    // persistent grid of each class: as many workgroups as fit the CUs at once
    const void *kfun[kClasses] = {
        (const void *)batched_int8_kernel<SHAPE_64x64, false>,  (const void *)batched_int8_kernel<SHAPE_32x128, false>,
        (const void *)batched_int8_kernel<SHAPE_128x32, false>, (const void *)batched_int8_kernel<SHAPE_128x128, false>,
        (const void *)batched_int8_kernel<SHAPE_64x64, true>,   (const void *)batched_int8_kernel<SHAPE_32x128, true>,
        (const void *)batched_int8_kernel<SHAPE_128x32, true>,  (const void *)batched_int8_kernel<SHAPE_128x128, true>,
        (const void *)batched_fp64_kernel};
    const void *kraw[SHAPE_COUNT] = {
        (const void *)batched_raw_kernel<SHAPE_64x64>, (const void *)batched_raw_kernel<SHAPE_32x128>,
        (const void *)batched_raw_kernel<SHAPE_128x32>, (const void *)batched_raw_kernel<SHAPE_128x128>};
    int grid[kClasses];
    for (int c = 0; c < kClasses; ++c) {
        int per_cu = 1;
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (b->raw && c < SHAPE_COUNT) ? kraw[c] : kfun[c], NT, 0);
        grid[c] = (int)std::max<int64_t>(1, std::min<int64_t>((int64_t)tiles[c].size(), (int64_t)cus * std::max(1, per_cu)));
    }
    // Per class, longest first (stable, so the tiles of a product stay together).
    // Workgroup w takes list entries w, w + G, ...; the hardware hands workgroups
    // to the XCDs round-robin (w mod 8), and each XCD has its own L2.  Within every
    // full round of G entries the sorted tiles are placed XCD-major, so the tiles
    // of one product run at the same time on one XCD and share its L2 copy of the
    // product's operand panels.
    std::vector<TileRef> flat;
    for (int c = 0; c < kClasses; ++c) {
        std::stable_sort(tiles[c].begin(), tiles[c].end(), [](const auto &a, const auto &b) { return a.first > b.first; });
        const int64_t first = (int64_t)flat.size(), nt = (int64_t)tiles[c].size(), G = grid[c];
        b->class_first[c] = (int32_t)first;
        b->class_count[c] = (int32_t)nt;
        flat.resize((size_t)(first + nt));
        for (int64_t i = 0; i < nt; ++i) {
            const int64_t round = i / G, q = i % G;
            int64_t slot = q;
            if ((round + 1) * G <= nt && G % kXcds == 0) {
                const int64_t per = G / kXcds;
                slot = kXcds * (q % per) + q / per;
            }
            flat[(size_t)(first + round * G + slot)] = tiles[c][(size_t)i].second;
        }
    }
    b->ntiles = (int32_t)flat.size();

    if (jobs.size() > (size_t)INT32_MAX - kXcds) return fail(QMM_EUNSUPPORTED, "batch too large");
    while (jobs.size() % kXcds) jobs.push_back(PackJob{0, 2, 0, 0});  // padding jobs do nothing
    b->njobs = (int32_t)jobs.size();
    b->ws_bytes = ws;
    if (ws > 0) {
        if ((e = hipMalloc(&b->d_ws, ws)) != hipSuccess) return hip_fail(e, "hipMalloc (workspace)");
        for (int64_t i = 0; i < count; ++i) {
            Desc &D = descs[(size_t)i];
            if ((D.path != QMM_PATH_INT8 && D.path != QMM_PATH_FP4) || D.m == 0 || D.n == 0) continue;
            D.Ac = b->d_ws + a_off[(size_t)i];
            D.Bt = b->d_ws + b_off[(size_t)i];
        }
    }
    if (!jobs.empty()) {
        if ((e = hipMalloc(&b->d_jobs, sizeof(PackJob) * jobs.size())) != hipSuccess) return hip_fail(e, "hipMalloc");
        if ((e = hipMemcpy(b->d_jobs, jobs.data(), sizeof(PackJob) * jobs.size(), hipMemcpyHostToDevice)) != hipSuccess)
            return hip_fail(e, "hipMemcpy");
    }
    if ((e = hipMalloc(&b->d_desc, sizeof(Desc) * std::max<size_t>(1, descs.size()))) != hipSuccess) return hip_fail(e, "hipMalloc");
    if ((e = hipMalloc(&b->d_tiles, sizeof(TileRef) * std::max<size_t>(1, flat.size()))) != hipSuccess) return hip_fail(e, "hipMalloc");
    if (!descs.empty() && (e = hipMemcpy(b->d_desc, descs.data(), sizeof(Desc) * descs.size(), hipMemcpyHostToDevice)) != hipSuccess)
        return hip_fail(e, "hipMemcpy");
    if (!flat.empty() && (e = hipMemcpy(b->d_tiles, flat.data(), sizeof(TileRef) * flat.size(), hipMemcpyHostToDevice)) != hipSuccess)
        return hip_fail(e, "hipMemcpy");
    if (b->raw && !flat.empty()) {
        // raw tiles: one self-contained record per INT8 tile (FP64 entries stay empty)
        std::vector<RawTile> recs(flat.size());
        std::memset(recs.data(), 0, sizeof(RawTile) * recs.size());
        for (uint32_t c = 0; c < SHAPE_COUNT; ++c)
            for (int64_t j = b->class_first[c]; j < (int64_t)b->class_first[c] + b->class_count[c]; ++j) {
                const TileRef &tr = flat[(size_t)j];
                const Desc &D = descs[(size_t)tr.desc];
                const int64_t row0 = (int64_t)tr.tm * shape_bm(c), col0 = (int64_t)tr.tn * shape_bn(c);
                RawTile &r = recs[(size_t)j];
                r.A = D.A + row0 * D.lda;
                r.B = D.B + col0;
                r.C = D.C + row0 * D.ldc + col0;
                r.lda = (uint32_t)D.lda;
                r.ldb = (uint32_t)D.ldb;
                r.ldc = (uint32_t)D.ldc;
                r.rows = (int32_t)(D.m - row0);
                r.cols = (int32_t)(D.n - col0);
                r.k = D.k;
                r.a_size = D.k > 0 ? (uint32_t)((r.rows - 1) * D.lda + D.k) : 0u;
                r.b_size = D.k > 0 ? (uint32_t)((int64_t)(D.k - 1) * D.ldb + r.cols) : 0u;
                r.p = D.p;
                r.off = D.off;
                r.magic32 = D.magic32;
                r.add_h = D.add_h;
                r.neg_p = D.neg_p;
            }
        if ((e = hipMalloc(&b->d_raw, sizeof(RawTile) * recs.size())) != hipSuccess) return hip_fail(e, "hipMalloc");
        if ((e = hipMemcpy(b->d_raw, recs.data(), sizeof(RawTile) * recs.size(), hipMemcpyHostToDevice)) != hipSuccess)
            return hip_fail(e, "hipMemcpy");
    }

    // Record the launches in one graph: the pack kernel, then each class's persistent
    // kernel in turn, each with the whole GPU (measured marginally faster than the
    // classes as parallel branches, whose later kernels wait for the earlier ones'
    // persistent workgroups anyway).  The schedule is static, so the graph holds only
    // kernel nodes and nothing needs clearing between replays.
    if ((e = hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking)) != hipSuccess) return hip_fail(e, "stream");
    hipStream_t s0 = b->capture;
    if ((e = hipStreamBeginCapture(s0, hipStreamCaptureModeThreadLocal)) != hipSuccess) return hip_fail(e, "capture");
    hipError_t le = hipSuccess;
    if (b->njobs > 0) {
        batched_pack_kernel<<<b->njobs, NT, 0, s0>>>(b->d_desc, b->d_jobs);
        le = hipGetLastError();
    }
    for (int c = 0; c < kClasses; ++c) {
        if (b->class_count[c] == 0) continue;
        const Desc *dd = b->d_desc;
        const TileRef *tt = b->d_tiles + b->class_first[c];
        const int32_t nt = b->class_count[c];
        if (b->raw && c < SHAPE_COUNT) {
            const RawTile *rr = b->d_raw + b->class_first[c];
            switch (c) {
            case 0: batched_raw_kernel<SHAPE_64x64><<<grid[c], NT, 0, s0>>>(rr, nt); break;
            case 1: batched_raw_kernel<SHAPE_32x128><<<grid[c], NT, 0, s0>>>(rr, nt); break;
            case 2: batched_raw_kernel<SHAPE_128x32><<<grid[c], NT, 0, s0>>>(rr, nt); break;
            default: batched_raw_kernel<SHAPE_128x128><<<grid[c], NT, 0, s0>>>(rr, nt); break;
            }
            if (le == hipSuccess) le = hipGetLastError();
            continue;
        }
        switch (c) {
        case 0: batched_int8_kernel<SHAPE_64x64, false><<<grid[c], NT, 0, s0>>>(dd, tt, nt); break;
        case 1: batched_int8_kernel<SHAPE_32x128, false><<<grid[c], NT, 0, s0>>>(dd, tt, nt); break;
        case 2: batched_int8_kernel<SHAPE_128x32, false><<<grid[c], NT, 0, s0>>>(dd, tt, nt); break;
        case 3: batched_int8_kernel<SHAPE_128x128, false><<<grid[c], NT, 0, s0>>>(dd, tt, nt); break;
        case 4: batched_int8_kernel<SHAPE_64x64, true><<<grid[c], NT, 0, s0>>>(dd, tt, nt); break;
        case 5: batched_int8_kernel<SHAPE_32x128, true><<<grid[c], NT, 0, s0>>>(dd, tt, nt); break;
        case 6: batched_int8_kernel<SHAPE_128x32, true><<<grid[c], NT, 0, s0>>>(dd, tt, nt); break;
        case 7: batched_int8_kernel<SHAPE_128x128, true><<<grid[c], NT, 0, s0>>>(dd, tt, nt); break;
        default: batched_fp64_kernel<<<grid[c], NT, 0, s0>>>(dd, tt, nt); break;
        }
        if (le == hipSuccess) le = hipGetLastError();
    }
    if ((e = hipStreamEndCapture(s0, &b->graph)) != hipSuccess) return hip_fail(e, "end capture");
    if (le != hipSuccess) return hip_fail(le, "batched launch");
    if ((e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0)) != hipSuccess) return hip_fail(e, "instantiate");
    return QMM_OK;
}

}  // namespace

namespace {

// Mean time of `reps` replays of a batch's graph on `stream` (after one warm-up).
qmm_status time_batch(qmm_batched *b, hipStream_t stream, hipEvent_t e0, hipEvent_t e1, int reps, float *ms) {
    hipError_t e;
    if (b->ntiles == 0) {
        *ms = 0.f;
        return QMM_OK;
    }
    if ((e = hipGraphLaunch(b->exec, stream)) != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    if ((e = hipEventRecord(e0, stream)) != hipSuccess) return hip_fail(e, "hipEventRecord");
    for (int r = 0; r < reps; ++r)
        if ((e = hipGraphLaunch(b->exec, stream)) != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    if ((e = hipEventRecord(e1, stream)) != hipSuccess) return hip_fail(e, "hipEventRecord");
    if ((e = hipEventSynchronize(e1)) != hipSuccess) return hip_fail(e, "hipEventSynchronize");
    if ((e = hipEventElapsedTime(ms, e0, e1)) != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
    *ms /= (float)reps;
    return QMM_OK;
}

// QMM_BATCH_MEASURE: build the cost-model assignment and one batch per uniform
// tile shape, time each on the batch's own buffers (every candidate writes the
// same, correct C_i), keep the fastest.
qmm_status create_measured(int64_t count, const qmm_problem *probs, uint32_t flags, qmm_batched **out) {
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e;
    if ((e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking)) != hipSuccess) return hip_fail(e, "stream");
    qmm_status st = QMM_OK;
    if ((e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess) st = hip_fail(e, "event");
    qmm_batched *best = nullptr;
    float best_ms = 0.f;
    // candidates 0 .. SHAPE_COUNT: the packed operands (cost model, then each shape
    // everywhere); the same again with raw tiles (no pack kernel), skipped when some
    // product cannot take them
    for (uint32_t c = 0; c <= 2 * SHAPE_COUNT + 1 && st == QMM_OK; ++c) {
        const bool raw = c > SHAPE_COUNT;
        const uint32_t shape = raw ? c - SHAPE_COUNT - 1 : c;  // 0 = cost model, else 1 + shape
        qmm_batched *b = new qmm_batched();
        st = build_batch(count, probs, flags | (shape << 8) | (raw ? QMM_BATCH_RAW : 0u), b);
        if (raw && st == QMM_EUNSUPPORTED) {
            release(b);
            st = QMM_OK;
            continue;
        }
        float ms = 0.f;
        if (st == QMM_OK) st = time_batch(b, s, e0, e1, 3, &ms);
        if (st == QMM_OK && (!best || ms < best_ms)) {
            release(best);
            best = b;
            best_ms = ms;
        } else {
            release(b);
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipStreamDestroy(s);
    if (st != QMM_OK) {
        release(best);
        return st;
    }
    *out = best;
    return QMM_OK;
}

}  // namespace

extern "C" qmm_status qmm_batched_create(int64_t count, const qmm_problem *probs, uint32_t flags, qmm_batched **out) {
    if (!out) return fail(QMM_EINVAL, "out is NULL");
    *out = nullptr;
    if (count < 0 || (count > 0 && !probs)) return fail(QMM_EINVAL, "bad problem array");
    if (flags & ~(QMM_BATCH_FORCE_FP64 | QMM_BATCH_SHAPE_MASK | QMM_BATCH_MEASURE | QMM_BATCH_INT8_ONLY | QMM_BATCH_RAW))
        return fail(QMM_EINVAL, "unknown flags");
    if ((flags & QMM_BATCH_RAW) && (flags & (QMM_BATCH_FORCE_FP64 | QMM_BATCH_MEASURE)))
        return fail(QMM_EINVAL, "QMM_BATCH_RAW is an INT8 layout; QMM_BATCH_MEASURE tries it by itself");
    if (((flags & QMM_BATCH_SHAPE_MASK) >> 8) > SHAPE_COUNT) return fail(QMM_EINVAL, "unknown tile shape flag");
    if ((flags & QMM_BATCH_MEASURE) && (flags & (QMM_BATCH_FORCE_FP64 | QMM_BATCH_SHAPE_MASK)))
        return fail(QMM_EINVAL, "QMM_BATCH_MEASURE chooses the INT8 tile shapes itself");
    if (flags & QMM_BATCH_MEASURE) return create_measured(count, probs, flags & ~QMM_BATCH_MEASURE, out);
    qmm_batched *b = new qmm_batched();
    const qmm_status st = build_batch(count, probs, flags, b);
    if (st != QMM_OK) {
        release(b);
        return st;
    }
    *out = b;
    return QMM_OK;
}

extern "C" qmm_status qmm_gemm_mod_p_batched(qmm_batched *batch, void *stream) {
    if (!batch) return fail(QMM_EINVAL, "batch is NULL");
    if (batch->ntiles == 0) return QMM_OK;
    const hipError_t e = hipGraphLaunch(batch->exec, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    return QMM_OK;
}

namespace {
// Calibration batches of qmm_batched_tune: `count` products of m x n x k (k = 128
// and 1024), all reading one A (m x 1024) and one B (1024 x n) and writing their
// own C, enough tiles to fill the GPU.
int64_t tune_count(int64_t m, int64_t n) {
    const int64_t c = ((int64_t)1 << 24) / std::max<int64_t>(1, m * n);
    return std::min<int64_t>(1024, std::max<int64_t>(16, c));
}
constexpr int64_t kTuneKMax = 1024;
struct TuneLayout {
    size_t a = 0, b = 0, c = 0, bytes = 0;
};
TuneLayout tune_layout(int64_t m, int64_t n) {
    TuneLayout L;
    auto up = [](size_t x) { return (x + 255) / 256 * 256; };
    L.b = up((size_t)m * kTuneKMax);
    L.c = L.b + up((size_t)kTuneKMax * n);
    L.bytes = L.c + up((size_t)tune_count(m, n) * m * n);
    return L;
}
}  // namespace

extern "C" qmm_status qmm_batched_tune_workspace_size(int64_t m, int64_t n, size_t *bytes) {
    if (!bytes) return fail(QMM_EINVAL, "bytes is NULL");
    if (m < 1 || n < 1 || m > 4096 || n > 4096) return fail(QMM_EINVAL, "calibration products need 1 <= m, n <= 4096");
    *bytes = tune_layout(m, n).bytes;
    return QMM_OK;
}

extern "C" qmm_status qmm_batched_tune(uint32_t p, int64_t m, int64_t n, void *ws, size_t ws_bytes, void *stream,
                                       double *costs) {
    // Times whole batches (pack and product) of each tile shape on two synthetic
    // workloads of m x n products at prime p (a short and a long k) and fits
    // cost = fixed + per_stage * stages per tile, in units of one 128-byte stage of
    // the 64 x 64 shape.  The buffers are the caller's workspace.
    if (p < 2 || p > 256) return fail(QMM_EINVAL, "p must be in [2, 256]");
    if (m < 1 || n < 1 || m > 4096 || n > 4096) return fail(QMM_EINVAL, "calibration products need 1 <= m, n <= 4096");
    const TuneLayout L = tune_layout(m, n);
    if (!ws || ws_bytes < L.bytes)
        return fail(QMM_ENOSPACE, "calibration workspace needs " + std::to_string(L.bytes) + " bytes");
    const int64_t reps = 10, count = tune_count(m, n);
    const int64_t ks[2] = {128, kTuneKMax};
    uint8_t *buf = (uint8_t *)ws;
    qmm_status st = launch_fill_u8(buf, 1, (int64_t)L.c, (int64_t)L.c, 1, stream);  // A and B: residue 1
    if (st != QMM_OK) return st;
    std::string arch;
    if ((st = device_arch(arch)) != QMM_OK) return st;
    double ms[SHAPE_COUNT][2];
    hipEvent_t e0, e1;
    hipError_t e;
    if ((e = hipEventCreate(&e0)) != hipSuccess) return hip_fail(e, "hipEventCreate");
    if ((e = hipEventCreate(&e1)) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return hip_fail(e, "hipEventCreate");
    }
    for (uint32_t sh = 0; sh < SHAPE_COUNT && st == QMM_OK; ++sh) {
        for (int ki = 0; ki < 2 && st == QMM_OK; ++ki) {
            std::vector<qmm_problem> probs((size_t)count);
            for (int64_t i = 0; i < count; ++i)
                probs[(size_t)i] = qmm_problem{m, n, ks[ki], p, buf, kTuneKMax, buf + L.b, n,
                                               buf + L.c + (size_t)i * m * n, n};
            qmm_batched *b = nullptr;
            st = qmm_batched_create(count, probs.data(), (sh + 1) << 8, &b);
            if (st != QMM_OK) break;
            (void)qmm_gemm_mod_p_batched(b, stream);
            (void)hipEventRecord(e0, (hipStream_t)stream);
            for (int r = 0; r < reps; ++r) (void)qmm_gemm_mod_p_batched(b, stream);
            (void)hipEventRecord(e1, (hipStream_t)stream);
            if ((e = hipEventSynchronize(e1)) != hipSuccess) st = hip_fail(e, "hipEventSynchronize");
            float t = 0.f;
            (void)hipEventElapsedTime(&t, e0, e1);
            const double tiles = (double)(ceil_div(m, shape_bm(sh)) * ceil_div(n, shape_bn(sh)) * count);
            ms[sh][ki] = (double)t / reps / tiles;  // per tile
            qmm_batched_destroy(b);
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != QMM_OK) return st;
    // per-tile time = fixed + per_stage * stages; unit: one stage of the 64 x 64 shape
    const double s0 = (double)ceil_div(ks[0], KT), s1 = (double)ceil_div(ks[1], KT);
    const double unit = (ms[0][1] - ms[0][0]) / (s1 - s0);
    if (!(unit > 0)) return fail(QMM_EDEVICE, "tuning runs gave no usable timing");
    double fit[kTuneCosts];
    for (uint32_t sh = 0; sh < SHAPE_COUNT; ++sh) {
        const double per = (ms[sh][1] - ms[sh][0]) / (s1 - s0) / unit;
        const double fixed = ms[sh][0] / unit - per * s0;
        g_costs[sh].per_stage = per > 0.05 ? per : 0.05;
        g_costs[sh].fixed = fixed > 0 ? fixed : 0;
        fit[2 * sh] = g_costs[sh].fixed;
        fit[2 * sh + 1] = g_costs[sh].per_stage;
    }
    if (costs) std::memcpy(costs, fit, sizeof(fit));
    // the calibration batches ran FP4 codes for p <= 8 and centred bytes otherwise
    if ((st = tune_cache_load_env_once()) != QMM_OK) return st;
    tune_cache_put(arch, tune_enc(p), tune_bucket(m, n), fit);
    return tune_cache_save_env();
}

extern "C" qmm_status qmm_batched_set_costs(const double *costs) {
    if (!costs) return fail(QMM_EINVAL, "costs is NULL");
    for (uint32_t sh = 0; sh < SHAPE_COUNT; ++sh) {
        if (!(costs[2 * sh] >= 0) || !(costs[2 * sh + 1] > 0)) return fail(QMM_EINVAL, "costs must be positive");
    }
    for (uint32_t sh = 0; sh < SHAPE_COUNT; ++sh) g_costs[sh] = ShapeCost{costs[2 * sh], costs[2 * sh + 1]};
    return QMM_OK;
}

extern "C" qmm_status qmm_batched_plan(const qmm_batched *batch, int64_t i, qmm_plan *out) {
    if (!batch || !out) return fail(QMM_EINVAL, "NULL argument");
    if (i < 0 || i >= batch->count) return fail(QMM_EINVAL, "index out of range");
    *out = batch->plans[(size_t)i];
    return QMM_OK;
}

extern "C" qmm_status qmm_batched_destroy(qmm_batched *batch) {
    release(batch);
    return QMM_OK;
}
