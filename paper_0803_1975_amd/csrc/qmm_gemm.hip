// Compressed GEMMs on the FP64 / FP32 matrix cores of gfx950.
//
//   EPI_QADIC  procedure (1)/(2): T = start + CA x CB over packed words (CA rows
//              reversed, CB columns forward), then digit d of every word mod p.
//   EPI_REDQ   words that hold a (d_q+1) x (d_theta+1) block of C, split by
//              REDQ into all their coefficients mod p:
//              procedure (5) (A residues times the row-compressed CBr, d_q = 0),
//              left compression (Table 2: CAl packed along m times B residues,
//              d_theta = 0) and full compression (section 4: CAl times CBt packed
//              along n in Theta = Q^(d_q+1)).  Residue operands are converted to
//              words on the way into LDS.
//   EPI_PACK   procedure (1) with ReduceAndCompress: as EPI_QADIC, then the
//              reduced tile goes through LDS and leaves as CompressRows words
//              (reversed, d+1 columns per word), so products can be chained.
//              Tiles stay 128 columns wide when d+1 residues fit the bytes of a
//              word: a word cut by a tile edge gets its residues as bytes in its
//              own slot from both tiles, and a small pass packs those slots
//              afterwards (no tile count grows by rounding to whole words).
//
// Tiling: 128 x 128 output tile per 256-thread workgroup, 2 x 2 wavefronts of
// 64 x 64 each, i.e. 4 x 4 MFMA 16x16x4 tiles per wavefront.  K advances 16
// elements per LDS stage (four MFMA steps), double-buffered so that the global
// loads of stage s+1 are in flight while stage s is multiplied; one barrier per
// stage.  The A stage is stored row-major with one word of padding (the MFMA A
// fragment reads 16 rows at the same k: the padding spreads them over all banks);
// the B stage is stored row-major (the B fragment reads 16 consecutive columns).
//
// Exactness (see the planner): the MFMA on gfx950 adds each product to the
// accumulator with one fused, correctly rounded step, in k order.  In the EXACT
// regime nothing rounds; in the OFFSET regime the accumulator starts at
// M = 2^(beta-1) Q^d and each step floors onto a multiple of Q^d.  Blocked plans collect digit d of every finished block in integer registers:
// for t <= 15 as plain sums in 16-bit fields, two outputs to a register (four
// integer operations per pair of outputs and block), reduced mod p only every
// few blocks, before a field could overflow; for larger t each block's digit is
// reduced mod p into a byte field at once.  The accumulators then restart at M.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "qmm_device.h"
#include "qmm_internal.h"

namespace qmm {
namespace {

typedef double dx4 __attribute__((ext_vector_type(4)));
typedef float fx4 __attribute__((ext_vector_type(4)));

template <typename W> struct Mma;
template <> struct Mma<double> {
    using acc_t = dx4;
    __device__ __forceinline__ static acc_t mma(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    // lane l, register r holds D[(l >> 4) + 4 r][l & 15]
    __device__ __forceinline__ static int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};
template <> struct Mma<float> {
    using acc_t = fx4;
    __device__ __forceinline__ static acc_t mma(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    // lane l, register r holds D[4 (l >> 4) + r][l & 15]
    __device__ __forceinline__ static int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

constexpr int BM = 128, BN = 128, KT = kQadicKT, NT = 256, APAD = 1;
static_assert(KT == 16, "the staging maps below assume 16-element K stages");

enum { EPI_QADIC = 0, EPI_REDQ = 1, EPI_PACK = 2 };
// Blocked k (reading of section 2.4's bound per block): none, digits reduced mod p
// into byte fields at every block, or summed into 16-bit fields (t <= 15).
enum { BLK_NONE = 0, BLK_BYTE = 1, BLK_SUM16 = 2 };

struct GemmArgs {
    int64_t m, n, kdim;      // rows and columns of the product of (packed) operands, inner length
    const void *A;
    int64_t lda;             // words, or residues (bytes) for procedure (5)
    const void *B;
    int64_t ldb;             // words, or residues (bytes) for left compression
    uint8_t *C;
    int64_t ldc;
    int64_t m_out, n_out;    // rows and columns of C
    uint32_t dq, dth;        // EPI_REDQ: a word holds C's (dq+1) x (dth+1) block
    int32_t tiles_m, tiles_n;
    int32_t col_step;        // output columns per tile: BN, or whole words of BN (EPI_PACK)
    int32_t tile_words;      // EPI_PACK, whole-word tiles: words per tile row
    int32_t pack_slots;      // EPI_PACK: 128-column tiles, cut words left as bytes in their slots
    void *CW;                // EPI_PACK: compressed output, words
    int64_t ldcw, n_words;
    int32_t kb_tiles;        // K stages per block (blocked Q-adic plans)
    int32_t fold_blocks;     // BLK_SUM16: blocks summed into a 16-bit field between reductions
    uint32_t p, t, d, td;
    uint64_t qmask;
    double invp;
    double start;            // accumulator start value (M or 0)
    uint32_t m32;            // mod_u32_m32 multiplier for p, floor(2^32 / p)
    double inv_qd, inv_q, q; // 2^-td, 2^-t, 2^t (exact-regime digit)
    int32_t small_digit;     // t <= 31: digits fit 32 bits
    int32_t lds_epi;         // C and ldc 4-byte aligned and 4 x 512 E bytes fit the staging buffers
    int32_t c_vec;           // C and ldc 4-byte aligned
};

// Output tile of this workgroup.  Workgroups are dealt round-robin to the 8 XCDs;
// the first remap gives each XCD a contiguous range of tiles, the second walks
// them in groups of 8 tile-rows so neighbours share A row-panels and B panels in
// that XCD's L2.
__device__ __forceinline__ void tile_coords(int tiles_m, int tiles_n, int &tm, int &tn) {
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

template <typename W, typename AT, typename BT, int EPI, bool OFFSET, int BLK>
__global__ __launch_bounds__(NT, 2) void gemm_kernel(GemmArgs g) {
    constexpr bool BLOCKED = BLK != BLK_NONE;
    using MM = Mma<W>;
    using acc_t = typename MM::acc_t;
    __shared__ W sA[2][BM][KT + APAD];
    // FP32: B's k-rows padded by 64 bytes, so the four groups of 16 lanes of a
    // fragment read (four consecutive k-rows at the same columns) start 16 banks apart
    // (measured: square FP32 products 1.3 % faster; FP64 unchanged, so left unpadded)
    constexpr int BPAD = sizeof(W) == 4 ? 16 : 0;
    __shared__ W sB[2][KT][BN + BPAD];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    int tm, tn;
    tile_coords(g.tiles_m, g.tiles_n, tm, tn);
    const int64_t row0 = (int64_t)tm * BM, col0 = (int64_t)tn * g.col_step;

    const W start = (W)g.start;
    acc_t acc[4][4];
#pragma unroll
    for (int mi = 0; mi < 4; ++mi)
#pragma unroll
        for (int ni = 0; ni < 4; ++ni) acc[mi][ni] = acc_t{start, start, start, start};
    // Blocked plans: what the finished blocks left for each output.  BLK_BYTE: their
    // digits reduced mod p (< 256, since results are bytes), four to a register;
    // BLK_SUM16: the sum of their digits (a residue after each fold), two to a register.
    constexpr int RES_W = BLK == BLK_SUM16 ? 2 : 1;
    uint32_t res[4][4][RES_W];
    if constexpr (BLOCKED) {
#pragma unroll
        for (int mi = 0; mi < 4; ++mi)
#pragma unroll
            for (int ni = 0; ni < 4; ++ni)
#pragma unroll
                for (int h = 0; h < RES_W; ++h) res[mi][ni][h] = 0;
    }

    // Staging, in pairs of elements: the A stage (BM rows of KT words) and the B stage
    // (KT rows of BN words) are each cut into pairs p = tid + NT i (i < 4) in row-major
    // order, so the lanes of one load or store instruction cover consecutive pairs --
    // whole 128-byte rows of A (8 lanes a row) and 1 KB rows of B (64 lanes) -- for
    // coalesced loads and LDS stores on distinct banks (A rows are padded by one word).
    // A: rows ar0 + 32 i, elements ak, ak + 1; B: k-rows bk0 + 4 i, columns bc, bc + 1.
    static_assert(BM * KT == 8 * NT && KT * BN == 8 * NT, "four pairs of each operand per thread");
    const int ar0 = tid >> 3, ak = 2 * (tid & 7);
    const int bk0 = tid >> 6, bc = 2 * (tid & 63);
    const int64_t a_row = row0 + ar0;
    const AT *__restrict__ Ap = (const AT *)g.A + a_row * g.lda;  // row ar0 + 32 i at Ap + 32 i lda
    const BT *__restrict__ Bp = (const BT *)g.B;
    W ra[8], rb[8];

    auto load_stage = [&](int kt) {
        const int64_t k0 = (int64_t)kt * KT;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const bool row_ok = a_row + 32 * i < g.m;
            const AT *arow = Ap + (row_ok ? (int64_t)(32 * i) * g.lda : -a_row * g.lda);  // row 0 when past m
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                const int64_t kk = k0 + ak + e;
                ra[2 * i + e] = (row_ok && kk < g.kdim) ? (W)arow[kk] : (W)0;
            }
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t gk = k0 + bk0 + 4 * i;
            const bool krow_ok = gk < g.kdim;
            const BT *brow = Bp + (krow_ok ? gk : 0) * g.ldb;
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                const int64_t cc = col0 + bc + e;
                rb[2 * i + e] = (krow_ok && cc < g.n) ? (W)brow[cc] : (W)0;
            }
        }
    };
    auto store_stage = [&](int buf) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            sA[buf][ar0 + 32 * i][ak] = ra[2 * i];
            sA[buf][ar0 + 32 * i][ak + 1] = ra[2 * i + 1];
            sB[buf][bk0 + 4 * i][bc] = rb[2 * i];
            sB[buf][bk0 + 4 * i][bc + 1] = rb[2 * i + 1];
        }
    };
    // Digit d of one accumulated word (t <= 31 when blocked, so it fits 32 bits).
    auto digit32 = [&](W a) -> uint32_t {
        if constexpr (OFFSET) return low_mantissa_bits(a) & (uint32_t)g.qmask;
        else return exact_digit<W>(a, (W)g.inv_qd, (W)g.inv_q, (W)g.q);
    };
    // End of a block: its digits join the finished blocks'.
    auto reduce_block = [&]() {
#pragma unroll
        for (int mi = 0; mi < 4; ++mi)
#pragma unroll
            for (int ni = 0; ni < 4; ++ni) {
                if constexpr (BLK == BLK_SUM16) {
#pragma unroll
                    for (int h = 0; h < 2; ++h)
                        res[mi][ni][h] += digit32(acc[mi][ni][2 * h]) | digit32(acc[mi][ni][2 * h + 1]) << 16;
                } else {
                    uint32_t packed = 0;
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        packed |= mod_u32_m32(((res[mi][ni][0] >> (8 * r)) & 0xffu) + digit32(acc[mi][ni][r]), g.p,
                                              g.m32) << (8 * r);
                    res[mi][ni][0] = packed;
                }
            }
    };
    // BLK_SUM16: every field back to a residue, so fold_blocks more digits fit.
    auto fold = [&]() {
#pragma unroll
        for (int mi = 0; mi < 4; ++mi)
#pragma unroll
            for (int ni = 0; ni < 4; ++ni)
#pragma unroll
                for (int h = 0; h < RES_W; ++h) {
                    const uint32_t v = res[mi][ni][h];
                    res[mi][ni][h] = mod_u32_m32(v & 0xffffu, g.p, g.m32) | mod_u32_m32(v >> 16, g.p, g.m32) << 16;
                }
    };
    // Doubles take the schedule below; floats, whose MFMAs take half as long, keep
    // the plain double-buffered one (measured: the one-barrier schedule raises the
    // FP64 products 1.5-2 points of peak and costs the FP32 ones registers and a
    // wavefront per SIMD).
    if constexpr (sizeof(W) == 8) {
        // One barrier per K stage, and none between a barrier and the MFMAs after it:
        // stage kt computes from LDS buffer kt % 2; the registers loaded during stage
        // kt - 1 (stage kt + 1's words) are stored into the other buffer after the first
        // k-step, and stage kt + 2's loads are issued into the freed registers.  The
        // barrier follows the second-to-last k-step; the last k-step's MFMAs run while
        // the next stage's first fragments are read.  So every read of a buffer precedes
        // (in each wavefront) the barrier before its next overwrite, and every store
        // precedes the barrier before its first read.
        constexpr int KS = KT / 4;
        W af[2][4], bf[2][4];
        auto read_frags = [&](int b, int ks, int slot) {
    #pragma unroll
            for (int mi = 0; mi < 4; ++mi) af[slot][mi] = sA[b][wm * 64 + mi * 16 + (lane & 15)][ks * 4 + (lane >> 4)];
    #pragma unroll
            for (int ni = 0; ni < 4; ++ni) bf[slot][ni] = sB[b][ks * 4 + (lane >> 4)][wn * 64 + ni * 16 + (lane & 15)];
        };

        const int ntiles = (int)ceil_div(g.kdim, KT);
        load_stage(0);
        store_stage(0);
        if (ntiles > 1) load_stage(1);
        __syncthreads();
        read_frags(0, 0, 0);
        int blk_left = g.kb_tiles;      // stages left in the current block (blocked plans)
        int fold_left = g.fold_blocks;  // blocks before the next fold (BLK_SUM16)
        for (int kt = 0; kt < ntiles; ++kt) {
            const int buf = kt & 1;
            const bool more = kt + 1 < ntiles;
    #pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                const int cur = ks & 1;
                // the next k-step's fragments (on the last k-step: the next stage's first,
                // read unconditionally; on the last stage they are not used)
                read_frags(ks + 1 < KS ? buf : buf ^ 1, (ks + 1) % KS, cur ^ 1);
    #pragma unroll
                for (int mi = 0; mi < 4; ++mi)
    #pragma unroll
                    for (int ni = 0; ni < 4; ++ni) acc[mi][ni] = MM::mma(af[cur][mi], bf[cur][ni], acc[mi][ni]);
                if (ks == 0 && more) {
                    store_stage(buf ^ 1);
                    if (kt + 2 < ntiles) load_stage(kt + 2);
                }
                if (ks == KS - 2 && more) __syncthreads();
            }
            if constexpr (BLOCKED) {
                if (--blk_left == 0 && more) {
                    blk_left = g.kb_tiles;
                    reduce_block();
    #pragma unroll
                    for (int mi = 0; mi < 4; ++mi)
    #pragma unroll
                        for (int ni = 0; ni < 4; ++ni) acc[mi][ni] = acc_t{start, start, start, start};
                    if constexpr (BLK == BLK_SUM16) {
                        if (--fold_left == 0) {
                            fold_left = g.fold_blocks;
                            fold();
                        }
                    }
                }
            }
        }
    } else {
        // The four k-steps of one LDS stage.
        auto mma_stage = [&](int buf) {
    #pragma unroll
            for (int ks = 0; ks < KT / 4; ++ks) {
                W af[4], bf[4];
    #pragma unroll
                for (int mi = 0; mi < 4; ++mi) af[mi] = sA[buf][wm * 64 + mi * 16 + (lane & 15)][ks * 4 + (lane >> 4)];
    #pragma unroll
                for (int ni = 0; ni < 4; ++ni) bf[ni] = sB[buf][ks * 4 + (lane >> 4)][wn * 64 + ni * 16 + (lane & 15)];
    #pragma unroll
                for (int mi = 0; mi < 4; ++mi)
    #pragma unroll
                    for (int ni = 0; ni < 4; ++ni) {
                        acc[mi][ni] = MM::mma(af[mi], bf[ni], acc[mi][ni]);
                    }
            }
        };

        const int ntiles = (int)ceil_div(g.kdim, KT);
        load_stage(0);
        store_stage(0);
        __syncthreads();
        int blk_left = g.kb_tiles;      // stages left in the current block (blocked plans)
        int fold_left = g.fold_blocks;  // blocks before the next fold (BLK_SUM16)
        for (int kt = 0; kt < ntiles; ++kt) {
            const int buf = kt & 1;
            if (kt + 1 < ntiles) load_stage(kt + 1);
            mma_stage(buf);
            if constexpr (BLOCKED) {
                if (--blk_left == 0 && kt + 1 < ntiles) {
                    blk_left = g.kb_tiles;
                    reduce_block();
    #pragma unroll
                    for (int mi = 0; mi < 4; ++mi)
    #pragma unroll
                        for (int ni = 0; ni < 4; ++ni) acc[mi][ni] = acc_t{start, start, start, start};
                    if constexpr (BLK == BLK_SUM16) {
                        if (--fold_left == 0) {
                            fold_left = g.fold_blocks;
                            fold();
                        }
                    }
                }
            }
            if (kt + 1 < ntiles) {
                store_stage(buf ^ 1);
                __syncthreads();
            }
        }

    }
    __syncthreads();  // the epilogue may reuse the staging buffers

    // Epilogue.
    // Digit d of the accumulated word at (mi, ni, r), reduced mod p.
    auto qadic_value = [&](int mi, int ni, int r) -> uint32_t {
        if constexpr (BLK == BLK_SUM16)
            return mod_u32_m32(((res[mi][ni][r >> 1] >> (16 * (r & 1))) & 0xffffu) + digit32(acc[mi][ni][r]), g.p, g.m32);
        else if constexpr (BLOCKED)
            return mod_u32_m32(((res[mi][ni][0] >> (8 * r)) & 0xffu) + digit32(acc[mi][ni][r]), g.p, g.m32);
        else if (g.small_digit) return mod_u32_m32(digit32(acc[mi][ni][r]), g.p, g.m32);
        else return mod_u64(qadic_digit<W>(acc[mi][ni][r], OFFSET, g.td, g.qmask), g.p, g.invp);
    };
    if constexpr (EPI == EPI_PACK) {
        // ReduceAndCompress: the tile's residues go to LDS (the staging buffers are
        // free once every wavefront has read the last stage), then each thread packs
        // whole words of d+1 columns, first column in the top power (CompressRows).
        // Columns past n read as 0, the padding of a short last word.
        constexpr int LDS_C = BN + 4;
        static_assert(sizeof(sA) >= BM * LDS_C, "the reduced tile must fit the A staging buffers");
        uint8_t *sC = (uint8_t *)&sA[0][0][0];
        __syncthreads();
#pragma unroll
        for (int mi = 0; mi < 4; ++mi)
#pragma unroll
            for (int ni = 0; ni < 4; ++ni)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int rl = wm * 64 + mi * 16 + MM::row(lane, r);
                    const int cl = wn * 64 + ni * 16 + (lane & 15);
                    const bool in = row0 + rl < g.m && col0 + cl < g.n && cl < g.col_step;
                    sC[rl * LDS_C + cl] = in ? (uint8_t)qadic_value(mi, ni, r) : (uint8_t)0;
                }
        __syncthreads();
        // Words overlapping this tile's columns [col0, col0 + col_step).  A word inside
        // them is packed (Horner in the word's own type: every partial value is an
        // integer below the word bound, so exact) and stored; a word cut by an edge
        // (only with 128-column tiles) gets the residues of its columns below n as
        // bytes s of its slot, and the slot pass packs it.  Each thread walks the
        // flattened (row, word) list NT entries at a time without dividing.
        const int e = (int)g.d + 1;
        const int64_t cend = col0 + g.col_step;
        const int64_t L0 = col0 / e;
        const int64_t L1 = min((cend - 1) / e, g.n_words - 1);
        const int nwt = (int)(L1 - L0 + 1);
        const W q = (W)g.q;
        W *CW = (W *)g.CW;
        if (nwt > 0) {
            const int step_r = NT / nwt, step_l = NT - step_r * nwt;
            int rl = tid / nwt, li = tid - rl * nwt;
            for (; rl < BM; rl += step_r) {
                const int64_t row = row0 + rl;
                if (row < g.m) {
                    const int64_t L = L0 + li, w0 = L * e;
                    const uint8_t *srow = sC + rl * LDS_C;
                    if (w0 >= col0 && w0 + e <= cend) {
                        const int c0 = (int)(w0 - col0);
                        W w = (W)0;
                        for (int s = 0; s < e; ++s) w = w * q + (W)srow[c0 + s];
                        CW[row * g.ldcw + L] = w;
                    } else {
                        uint8_t *slot = (uint8_t *)(CW + row * g.ldcw + L);
                        for (int s = 0; s < e; ++s) {
                            const int64_t c = w0 + s;
                            if (c >= col0 && c < cend && c < g.n) slot[s] = srow[c - col0];
                        }
                    }
                }
                li += step_l;
                if (li >= nwt) {
                    li -= nwt;
                    ++rl;
                }
            }
        }
        return;
    }
    // Residue (i, j) of the word at (mi, ni, r): entry (i, j) of the word's
    // (dq+1) x (dth+1) block of C.  The exact word r = sum_q c_q Q^q holds every
    // coefficient c_q < Q (eq. (3)) as the bit field [tq, tq + t): REDQ's output,
    // c_q mod p, is that field reduced with a 32-bit multiply-high (t <= 32) or the
    // double reciprocal; coefficient q = i + j (dq+1).
    auto redq_value = [&](uint64_t w, int32_t i, int32_t j) -> uint32_t {
        const uint32_t sh = g.t * (uint32_t)(i + j * (int32_t)(g.dq + 1));
        if (g.small_digit) return mod_u32_m32(bit_field(w, sh, (uint32_t)g.qmask), g.p, g.m32);
        return mod_u64((w >> sh) & g.qmask, g.p, g.invp);
    };
    if constexpr (EPI == EPI_QADIC) {
        if (g.lds_epi && row0 + BM <= g.m && col0 + BN <= g.n) {
            // Whole tile, one residue per word: the four registers of a lane are four
            // rows of one column, and the four lanes of a quad hold four consecutive
            // columns of the same rows.  Packed into a dword and transposed across the
            // quad (two DPP exchanges), they become four consecutive bytes of one row
            // per lane: one dword store per lane and block instead of four byte stores.
            const int j = lane & 3;
#pragma unroll
            for (int mi = 0; mi < 4; ++mi)
#pragma unroll
                for (int ni = 0; ni < 4; ++ni) {
                    uint32_t w = 0;
#pragma unroll
                    for (int r = 0; r < 4; ++r) w |= qadic_value(mi, ni, r) << (8 * r);
                    w = quad_transpose_bytes(w, j);
                    const int64_t row = row0 + wm * 64 + mi * 16 + MM::row(lane, j);
                    const int64_t col = col0 + wn * 64 + ni * 16 + (lane & 15) - j;
                    *(uint32_t *)(g.C + row * g.ldc + col) = w;
                }
            return;
        }
    }
    if constexpr (EPI == EPI_REDQ) {
        const int dq1 = (int)g.dq + 1, dt1 = (int)g.dth + 1;
        const bool whole = (row0 + BM) * dq1 <= g.m_out && (col0 + BN) * dt1 <= g.n_out;
        if (g.c_vec && whole && g.dth == 0) {
            // Left compression, whole tile: output row R (dq+1) + i of word row R holds
            // residue i of each word, so for each i the four registers of a lane (four
            // word rows) and the four lanes of a quad (four columns) transpose into a
            // dword of one output row per lane, as for the Q-adic words.
            const int j = lane & 3;
#pragma unroll
            for (int mi = 0; mi < 4; ++mi)
#pragma unroll
                for (int ni = 0; ni < 4; ++ni) {
                    const int64_t wrow = row0 + wm * 64 + mi * 16 + MM::row(lane, j);
                    uint8_t *dst = g.C + wrow * dq1 * g.ldc + col0 + wn * 64 + ni * 16 + (lane & 15) - j;
                    for (int32_t i = 0; i < dq1; ++i) {
                        uint32_t v = 0;
#pragma unroll
                        for (int r = 0; r < 4; ++r) v |= redq_value(exact_word_bits(acc[mi][ni][r]), i, 0) << (8 * r);
                        *(uint32_t *)(dst + (int64_t)i * g.ldc) = quad_transpose_bytes(v, j);
                    }
                }
            return;
        }
        if (g.c_vec && whole && (dt1 == 2 || dt1 == 4)) {
            // Right or full compression with 2 or 4 residues per word along a row, whole
            // tile: residues (i, 0 .. dt1-1) of a word are consecutive bytes of output row
            // (dq+1) R + i, stored as one 2- or 4-byte store; the lanes of a row write
            // consecutive runs.
            auto store_words = [&](auto dt_c, auto one_row_c) __attribute__((always_inline)) {
                constexpr int DT = decltype(dt_c)::value;
                constexpr bool ONE_ROW = decltype(one_row_c)::value;  // right compression: dq = 0
                const uint32_t qm = (uint32_t)g.qmask;
                const int64_t rs = (int64_t)dq1 * g.ldc;
                uint8_t *base = g.C + (row0 + wm * 64 + MM::row(lane, 0)) * rs + (col0 + wn * 64 + (lane & 15)) * DT;
#pragma unroll
                for (int mi = 0; mi < 4; ++mi)
#pragma unroll
                    for (int ni = 0; ni < 4; ++ni)
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const uint64_t w = exact_word_bits(acc[mi][ni][r]);
                            uint8_t *dst = base + (int64_t)(mi * 16 + MM::row(lane, r) - MM::row(lane, 0)) * rs + ni * 16 * DT;
                            for (int32_t i = 0; i < (ONE_ROW ? 1 : dq1); ++i) {
                                uint32_t v = 0;
#pragma unroll
                                for (int jj = 0; jj < DT; ++jj)
                                    v |= mod_u32_m32(bit_field(w, g.t * (uint32_t)(i + jj * dq1), qm), g.p, g.m32) << (8 * jj);
                                if constexpr (DT == 2) *(uint16_t *)(dst + (int64_t)i * g.ldc) = (uint16_t)v;
                                else *(uint32_t *)(dst + (int64_t)i * g.ldc) = v;
                            }
                        }
            };
            // dt1 >= 2 residues of t bits share a word of at most 53 bits: t <= 26, the
            // digits fit 32 bits.
            if (dq1 == 1) {
                if (dt1 == 2) store_words(std::integral_constant<int, 2>{}, std::true_type{});
                else store_words(std::integral_constant<int, 4>{}, std::true_type{});
            } else {
                if (dt1 == 2) store_words(std::integral_constant<int, 2>{}, std::false_type{});
                else store_words(std::integral_constant<int, 4>{}, std::false_type{});
            }
            return;
        }
    }
    if (EPI != EPI_QADIC && g.lds_epi) {
        // Coalesced stores: one 16 x 16 MFMA block of words at a time, each wavefront
        // lays its words' residues out in LDS as the bytes of C they become (a block
        // of 16 (dq+1) rows by 16 (dth+1) bytes), then every lane reads back whole
        // dwords of those rows and stores them: E = (dq+1)(dth+1) dword stores per
        // lane and block instead of 4 E scattered byte stores.  The staging buffers
        // are free once every wavefront has read the last stage; each wavefront
        // alternates between two regions of 256 E bytes, so one barrier per block
        // orders the writes before the reads (and the reads of a region before its
        // next writes, two blocks later).
        const int dq1 = EPI == EPI_QADIC ? 1 : (int)g.dq + 1, dt1 = EPI == EPI_QADIC ? 1 : (int)g.dth + 1;
        const int E = dq1 * dt1, rowb = 16 * dt1, row_dw = 4 * dt1;
        uint8_t *region = (uint8_t *)&sA[0][0][0] + wave * 512 * E;
        // lane's first dword of a block: row lr0, dword ld0; then 64 dwords further on
        const int step_r = 64 / row_dw, step_d = 64 - step_r * row_dw;
        const int lr0 = lane / row_dw, ld0 = lane - lr0 * row_dw;
        __syncthreads();
#pragma unroll
        for (int mi = 0; mi < 4; ++mi)
#pragma unroll
            for (int ni = 0; ni < 4; ++ni) {
                uint8_t *blk = region + ((mi * 4 + ni) & 1) * 256 * E;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int wr = MM::row(lane, r), wc = lane & 15;
                    if constexpr (EPI == EPI_QADIC) {
                        blk[wr * 16 + wc] = (uint8_t)qadic_value(mi, ni, r);
                    } else {
                        const uint64_t w = exact_word_bits(acc[mi][ni][r]);
                        for (int32_t j = 0; j < dt1; ++j)
                            for (int32_t i = 0; i < dq1; ++i)
                                blk[(wr * dq1 + i) * rowb + wc * dt1 + j] = (uint8_t)redq_value(w, i, j);
                    }
                }
                __syncthreads();
                const int64_t orow = (row0 + wm * 64 + mi * 16) * dq1, ocol = (col0 + wn * 64 + ni * 16) * dt1;
                int lr = lr0, ld = ld0;
                for (int u = 0; u < E; ++u) {
                    const uint32_t v = *(const uint32_t *)(blk + lr * rowb + 4 * ld);
                    const int64_t ro = orow + lr, co = ocol + 4 * ld;
                    if (ro < g.m_out) {
                        uint8_t *dst = g.C + ro * g.ldc + co;
                        if (co + 4 <= g.n_out) {
                            *(uint32_t *)dst = v;
                        } else {
#pragma unroll
                            for (int b = 0; b < 4; ++b)
                                if (co + b < g.n_out) dst[b] = (uint8_t)(v >> (8 * b));
                        }
                    }
                    lr += step_r;
                    ld += step_d;
                    if (ld >= row_dw) {
                        ld -= row_dw;
                        ++lr;
                    }
                }
            }
        return;
    }
#pragma unroll
    for (int mi = 0; mi < 4; ++mi)
#pragma unroll
        for (int ni = 0; ni < 4; ++ni)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t row = row0 + wm * 64 + mi * 16 + MM::row(lane, r);
                const int64_t col = col0 + wn * 64 + ni * 16 + (lane & 15);
                if (row >= g.m || col >= g.n) continue;
                if constexpr (EPI == EPI_QADIC) {
                    g.C[row * g.ldc + col] = (uint8_t)qadic_value(mi, ni, r);
                } else {
                    const uint64_t w = exact_word_bits(acc[mi][ni][r]);
                    for (int32_t j = 0; j <= (int32_t)g.dth; ++j) {
                        const int64_t co = col * (g.dth + 1) + j;
                        if (co >= g.n_out) break;
                        for (int32_t i = 0; i <= (int32_t)g.dq; ++i) {
                            const int64_t ro = row * (g.dq + 1) + i;
                            if (ro >= g.m_out) break;
                            g.C[ro * g.ldc + co] = (uint8_t)redq_value(w, i, j);
                        }
                    }
                }
            }
}

// The words of a compressed output that a tile edge cuts (column c = 128 b, for
// b = 1 .. tiles_n, inside word L = (c - 1) / (d+1) when c is not a multiple of
// d+1): both tiles left the word's residues as bytes in its slot; pack them.
// Residues of columns at or past n are the zero padding, whatever the slot holds.
template <typename W>
__global__ __launch_bounds__(64) void pack_cut_words_kernel(int64_t m, int32_t tiles_n, int64_t n, int64_t n_words,
                                                              uint32_t e, uint32_t t, W *CW, int64_t ldcw) {
    const int32_t b = (int32_t)(blockIdx.x * 64 + threadIdx.x) + 1;
    if (b > tiles_n) return;
    const int64_t c = (int64_t)b * BN;
    if (c % e == 0) return;
    const int64_t L = (c - 1) / e;
    if (L >= n_words) return;
    for (int64_t row = blockIdx.y; row < m; row += gridDim.y) {
        W *slot = CW + row * ldcw + L;
        uint8_t bytes[sizeof(W)];
        __builtin_memcpy(bytes, slot, sizeof(W));
        uint64_t w = 0;
        for (uint32_t s = 0; s < e; ++s) w = (w << t) | (L * e + s < n ? (uint64_t)bytes[s] : 0ull);
        *slot = word_from_u64<W>(w);
    }
}

qmm_status check_launch(const char *what) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(QMM_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
    return QMM_OK;
}

// Fields every variant needs, from the plan.
void common_args(GemmArgs &g, const qmm_plan &pl) {
    g.p = pl.p;
    g.t = pl.t;
    g.d = pl.d;
    g.td = pl.t * pl.d;
    g.qmask = (1ull << pl.t) - 1;
    g.invp = 1.0 / (double)pl.p;
    g.m32 = (uint32_t)((1ull << 32) / pl.p);
    g.small_digit = pl.t <= 31;
    g.col_step = BN;
}

// The coalesced epilogue stores C as dwords (C and ldc 4-byte aligned) and stages
// each wavefront's block of E residues per word twice over in the A staging buffers.
template <typename W>
void set_lds_epi(GemmArgs &g, int64_t E) {
    const size_t staging = sizeof(W) * 2 * BM * (KT + APAD);
    g.c_vec = ((uintptr_t)g.C % 4 == 0) && (g.ldc % 4 == 0);
    g.lds_epi = g.c_vec && (size_t)(4 * 512 * E) <= staging;
}

dim3 grid_for(GemmArgs &g) {
    g.tiles_m = (int32_t)ceil_div(g.m, BM);
    g.tiles_n = (int32_t)ceil_div(g.n, g.col_step);
    return dim3((unsigned)((int64_t)g.tiles_m * g.tiles_n));
}

// Procedure (1)/(2), bytes out (EPI_QADIC) or compressed out (EPI_PACK: CW is
// m x ceil(n/(d+1)) words, leading dimension ldcw).
template <typename W, int EPI>
qmm_status launch_qadic_w(const qmm_plan &pl, int64_t m, int64_t n, int64_t k, const void *CA, int64_t ldca,
                          const void *CB, int64_t ldcb, uint8_t *C, int64_t ldc, void *CW, int64_t ldcw,
                          hipStream_t s) {
    GemmArgs g{};
    common_args(g, pl);
    g.m = g.m_out = m;
    g.n = g.n_out = n;
    g.kdim = words_for(k, pl.d);
    g.A = CA;
    g.lda = ldca;
    g.B = CB;
    g.ldb = ldcb;
    g.C = C;
    g.ldc = ldc;
    const bool blocked = pl.k_block < k;
    g.kb_tiles = blocked ? (int32_t)((pl.k_block / (pl.d + 1)) / KT) : 0;
    // A 16-bit field holds a residue (< p) plus fold_blocks digits (each < Q).
    const int64_t fold_blocks = pl.t <= 15 ? (int64_t)(0xffff - (pl.p - 1)) / (int64_t)((1u << pl.t) - 1) : 0;
    const bool sum16 = blocked && fold_blocks >= 1;
    g.fold_blocks = sum16 ? (int32_t)std::min<int64_t>(fold_blocks, 1 << 30) : 0;
    const bool offset = pl.regime == QMM_REGIME_OFFSET;
    g.start = offset ? ldexp(1.0, WordTraits<W>::beta - 1 + (int)(pl.t * pl.d)) : 0.0;
    g.inv_qd = ldexp(1.0, -(int)(pl.t * pl.d));
    g.inv_q = ldexp(1.0, -(int)pl.t);
    g.q = ldexp(1.0, (int)pl.t);
    g.small_digit = pl.t <= 31;
    if (blocked && pl.t > 31) return fail(QMM_EUNSUPPORTED, "blocked plans need t <= 31");
    if (EPI == EPI_PACK) {
        g.CW = CW;
        g.ldcw = ldcw;
        g.n_words = words_for(n, pl.d);
        // Residues fit a word's bytes: 128-column tiles and the slot pass for cut
        // words.  Otherwise a tile covers whole words, the largest multiple of d+1
        // columns in BN.
        g.pack_slots = pl.d + 1 <= sizeof(W);
        g.tile_words = BN / (int32_t)(pl.d + 1);
        if (g.tile_words < 1) return fail(QMM_EUNSUPPORTED, "compressed output needs d + 1 <= 128");
        if (!g.pack_slots) g.col_step = g.tile_words * (int32_t)(pl.d + 1);
    }
    set_lds_epi<W>(g, 1);
    const dim3 grid = grid_for(g);
    if (offset && sum16)
        gemm_kernel<W, W, W, EPI, true, BLK_SUM16><<<grid, NT, 0, s>>>(g);
    else if (offset && blocked)
        gemm_kernel<W, W, W, EPI, true, BLK_BYTE><<<grid, NT, 0, s>>>(g);
    else if (offset)
        gemm_kernel<W, W, W, EPI, true, BLK_NONE><<<grid, NT, 0, s>>>(g);
    else if (sum16)
        gemm_kernel<W, W, W, EPI, false, BLK_SUM16><<<grid, NT, 0, s>>>(g);
    else if (blocked)
        gemm_kernel<W, W, W, EPI, false, BLK_BYTE><<<grid, NT, 0, s>>>(g);
    else
        gemm_kernel<W, W, W, EPI, false, BLK_NONE><<<grid, NT, 0, s>>>(g);
    if (EPI == EPI_PACK && g.pack_slots && BN % (pl.d + 1) != 0) {
        const qmm_status st = check_launch("gemm_qadic_compress");
        if (st != QMM_OK) return st;
        const dim3 sgrid((unsigned)ceil_div(g.tiles_n, 64), (unsigned)std::min<int64_t>(m, 4096));
        pack_cut_words_kernel<W><<<sgrid, 64, 0, s>>>(m, g.tiles_n, n, g.n_words, pl.d + 1, pl.t, (W *)CW, ldcw);
        return check_launch("pack_cut_words");
    }
    return check_launch(EPI == EPI_PACK ? "gemm_qadic_compress" : "gemm_qadic");
}

// The REDQ family: the product of (packed) operands is rows x cols words, each
// holding a (dq+1) x (dth+1) block of the m x n result.
template <typename W, typename AT, typename BT>
qmm_status launch_redq_w(const qmm_plan &pl, uint32_t dq, uint32_t dth, int64_t m, int64_t n, int64_t k,
                         const void *A, int64_t lda, const void *B, int64_t ldb, uint8_t *C, int64_t ldc,
                         hipStream_t s, const char *what) {
    GemmArgs g{};
    common_args(g, pl);
    g.m = words_for(m, dq);
    g.n = words_for(n, dth);
    g.m_out = m;
    g.n_out = n;
    g.dq = dq;
    g.dth = dth;
    g.kdim = k;
    g.A = A;
    g.lda = lda;
    g.B = B;
    g.ldb = ldb;
    g.C = C;
    g.ldc = ldc;
    g.start = 0.0;
    set_lds_epi<W>(g, (int64_t)(dq + 1) * (dth + 1));
    const dim3 grid = grid_for(g);
    gemm_kernel<W, AT, BT, EPI_REDQ, false, BLK_NONE><<<grid, NT, 0, s>>>(g);
    return check_launch(what);
}

}  // namespace

qmm_status launch_gemm_qadic(const qmm_plan &pl, int64_t m, int64_t n, int64_t k, const void *CA, int64_t ldca,
                             const void *CB, int64_t ldcb, uint8_t *C, int64_t ldc, void *stream) {
    if (m == 0 || n == 0) return QMM_OK;
    const hipStream_t s = (hipStream_t)stream;
    if (pl.beta == 24) return launch_qadic_w<float, EPI_QADIC>(pl, m, n, k, CA, ldca, CB, ldcb, C, ldc, nullptr, 0, s);
    return launch_qadic_w<double, EPI_QADIC>(pl, m, n, k, CA, ldca, CB, ldcb, C, ldc, nullptr, 0, s);
}

qmm_status launch_gemm_qadic_compress(const qmm_plan &pl, int64_t m, int64_t n, int64_t k, const void *CA,
                                      int64_t ldca, const void *CB, int64_t ldcb, void *CC, int64_t ldcc,
                                      void *stream) {
    if (m == 0 || n == 0) return QMM_OK;
    const hipStream_t s = (hipStream_t)stream;
    if (pl.beta == 24) return launch_qadic_w<float, EPI_PACK>(pl, m, n, k, CA, ldca, CB, ldcb, nullptr, 0, CC, ldcc, s);
    return launch_qadic_w<double, EPI_PACK>(pl, m, n, k, CA, ldca, CB, ldcb, nullptr, 0, CC, ldcc, s);
}

qmm_status launch_gemm_redq(const qmm_plan &pl, int64_t m, int64_t n, int64_t k, const uint8_t *A, int64_t lda,
                            const void *CBr, int64_t ldcbr, uint8_t *C, int64_t ldc, void *stream) {
    if (m == 0 || n == 0) return QMM_OK;
    const hipStream_t s = (hipStream_t)stream;
    if (pl.beta == 24)
        return launch_redq_w<float, uint8_t, float>(pl, 0, pl.d, m, n, k, A, lda, CBr, ldcbr, C, ldc, s, "gemm_redq");
    return launch_redq_w<double, uint8_t, double>(pl, 0, pl.d, m, n, k, A, lda, CBr, ldcbr, C, ldc, s, "gemm_redq");
}

qmm_status launch_gemm_left(const qmm_plan &pl, int64_t m, int64_t n, int64_t k, const void *CAl, int64_t ldcal,
                            const uint8_t *B, int64_t ldb, uint8_t *C, int64_t ldc, void *stream) {
    if (m == 0 || n == 0) return QMM_OK;
    const hipStream_t s = (hipStream_t)stream;
    if (pl.beta == 24)
        return launch_redq_w<float, float, uint8_t>(pl, pl.d, 0, m, n, k, CAl, ldcal, B, ldb, C, ldc, s, "gemm_left");
    return launch_redq_w<double, double, uint8_t>(pl, pl.d, 0, m, n, k, CAl, ldcal, B, ldb, C, ldc, s, "gemm_left");
}

qmm_status launch_gemm_full(const qmm_plan &pl, int64_t m, int64_t n, int64_t k, const void *CAl, int64_t ldcal,
                            const void *CBt, int64_t ldcbt, uint8_t *C, int64_t ldc, void *stream) {
    if (m == 0 || n == 0) return QMM_OK;
    const hipStream_t s = (hipStream_t)stream;
    if (pl.beta == 24)
        return launch_redq_w<float, float, float>(pl, pl.d, pl.d2, m, n, k, CAl, ldcal, CBt, ldcbt, C, ldc, s, "gemm_full");
    return launch_redq_w<double, double, double>(pl, pl.d, pl.d2, m, n, k, CAl, ldcal, CBt, ldcbt, C, ldc, s, "gemm_full");
}

}  // namespace qmm
