// Compressed GEMMs on the FP64 / FP32 matrix cores of gfx950.
//
//   EPI_QADIC  procedure (1)/(2): T = start + CA x CB over packed words (CA rows
//              reversed, CB columns forward), then digit d of every word mod p.
//   EPI_REDQ   procedure (5): CC = A x CBr with A residues (converted to words on
//              the way into LDS) and CBr the row-compressed right operand; every
//              word is then split by REDQ into d+1 residues of consecutive columns.
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
// M = 2^(beta-1) Q^d and each step floors onto a multiple of Q^d.  Blocked plans
// reduce digit d of every block mod p into integer registers at block boundaries
// and restart the accumulator at M.
#include <hip/hip_runtime.h>

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

enum { EPI_QADIC = 0, EPI_REDQ = 1 };

struct GemmArgs {
    int64_t m, n, kdim;      // output rows, output word-columns, inner length of the K loop
    const void *A;
    int64_t lda;             // Q-adic: CA words; REDQ: residues (bytes)
    const void *B;
    int64_t ldb;             // words
    uint8_t *C;
    int64_t ldc;
    int64_t n_out;           // columns of C (REDQ: n; Q-adic: n)
    int32_t kb_tiles;        // K stages per block (blocked Q-adic plans)
    uint32_t p, t, d, td;
    uint64_t qmask;
    double invp;
    double start;            // accumulator start value (M or 0)
    uint32_t qmodp;          // Q mod p (REDQ)
    uint64_t magic;          // mod_u32 multiplier for p
    double inv_qd, inv_q, q; // 2^-td, 2^-t, 2^t (exact-regime digit)
    int32_t small_digit;     // t <= 31: digits fit 32 bits
};

// Output tile of this workgroup.  Workgroups are dealt round-robin to the 8 XCDs;
// the first remap gives each XCD a contiguous range of tiles, the second walks
// them in groups of 8 tile-rows so neighbours share A row-panels and B panels in
// that XCD's L2.
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

template <typename W, typename AT, int EPI, bool OFFSET, bool BLOCKED>
__global__ __launch_bounds__(NT, 2) void gemm_kernel(GemmArgs g) {
    using MM = Mma<W>;
    using acc_t = typename MM::acc_t;
    __shared__ W sA[2][BM][KT + APAD];
    __shared__ W sB[2][KT][BN];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    int tm, tn;
    tile_coords(g.m, g.n, tm, tn);
    const int64_t row0 = (int64_t)tm * BM, col0 = (int64_t)tn * BN;

    const W start = (W)g.start;
    acc_t acc[4][4];
#pragma unroll
    for (int mi = 0; mi < 4; ++mi)
#pragma unroll
        for (int ni = 0; ni < 4; ++ni) acc[mi][ni] = acc_t{start, start, start, start};
    // Blocked plans: the residues of the finished blocks, reduced mod p (< 256, since
    // results are bytes), four to a register.
    uint32_t res[4][4];
    if constexpr (BLOCKED) {
#pragma unroll
        for (int mi = 0; mi < 4; ++mi)
#pragma unroll
            for (int ni = 0; ni < 4; ++ni) res[mi][ni] = 0;
    }

    // Staging: A row ra_r, elements ra_k..ra_k+7; B row rb_k, columns rb_c..rb_c+7.
    const int ra_r = tid >> 1, ra_k = (tid & 1) * 8;
    const int rb_k = tid >> 4, rb_c = (tid & 15) * 8;
    const int64_t a_row = row0 + ra_r;
    const bool a_row_ok = a_row < g.m;
    const AT *__restrict__ Ap = (const AT *)g.A + (a_row_ok ? a_row : 0) * g.lda;
    const W *__restrict__ Bp = (const W *)g.B;
    W ra[8], rb[8];

    auto load_stage = [&](int kt) {
        const int64_t k0 = (int64_t)kt * KT;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int64_t kk = k0 + ra_k + e;
            ra[e] = (a_row_ok && kk < g.kdim) ? (W)Ap[kk] : (W)0;
        }
        const int64_t gk = k0 + rb_k;
        const bool krow_ok = gk < g.kdim;
        const W *brow = Bp + (krow_ok ? gk : 0) * g.ldb;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int64_t cc = col0 + rb_c + e;
            rb[e] = (krow_ok && cc < g.n) ? brow[cc] : (W)0;
        }
    };
    auto store_stage = [&](int buf) {
#pragma unroll
        for (int e = 0; e < 8; ++e) sA[buf][ra_r][ra_k + e] = ra[e];
#pragma unroll
        for (int e = 0; e < 8; ++e) sB[buf][rb_k][rb_c + e] = rb[e];
    };
    // Digit d of one accumulated word (t <= 31 when blocked, so it fits 32 bits).
    auto digit32 = [&](W a) -> uint32_t {
        if constexpr (OFFSET) return low_mantissa_bits(a) & (uint32_t)g.qmask;
        else return exact_digit<W>(a, (W)g.inv_qd, (W)g.inv_q, (W)g.q);
    };
    auto reduce_block = [&]() {
#pragma unroll
        for (int mi = 0; mi < 4; ++mi)
#pragma unroll
            for (int ni = 0; ni < 4; ++ni) {
                uint32_t packed = 0;
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    packed |= mod_u32(((res[mi][ni] >> (8 * r)) & 0xffu) + digit32(acc[mi][ni][r]), g.p, g.magic) << (8 * r);
                res[mi][ni] = packed;
                acc[mi][ni] = acc_t{start, start, start, start};
            }
    };

    const int ntiles = (int)ceil_div(g.kdim, KT);
    load_stage(0);
    store_stage(0);
    __syncthreads();
    for (int kt = 0; kt < ntiles; ++kt) {
        const int buf = kt & 1;
        if (kt + 1 < ntiles) load_stage(kt + 1);
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
                for (int ni = 0; ni < 4; ++ni) acc[mi][ni] = MM::mma(af[mi], bf[ni], acc[mi][ni]);
        }
        if constexpr (BLOCKED) {
            if ((kt + 1) % g.kb_tiles == 0 && kt + 1 < ntiles) reduce_block();
        }
        if (kt + 1 < ntiles) {
            store_stage(buf ^ 1);
            __syncthreads();
        }
    }

    // Epilogue.
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
                    uint32_t v;
                    if constexpr (BLOCKED)
                        v = mod_u32(((res[mi][ni] >> (8 * r)) & 0xffu) + digit32(acc[mi][ni][r]), g.p, g.magic);
                    else if (g.small_digit) v = mod_u32(digit32(acc[mi][ni][r]), g.p, g.magic);
                    else v = mod_u64(qadic_digit<W>(acc[mi][ni][r], OFFSET, g.td, g.qmask), g.p, g.invp);
                    g.C[row * g.ldc + col] = (uint8_t)v;
                } else {
                    // REDQ of the exact word, then its d+1 residues to consecutive columns.
                    const uint64_t w = u64_from_word(acc[mi][ni][r]);
                    const uint64_t s = div_u64(w, g.p, g.invp);
                    uint8_t *crow = g.C + row * g.ldc;
                    uint32_t mu_next = 0;
                    for (int32_t j = (int32_t)g.d; j >= 0; --j) {
                        const uint32_t sh = g.t * (uint32_t)j;
                        const uint32_t mu = (uint32_t)((w >> sh) - (uint64_t)g.p * (s >> sh));
                        const uint64_t v = (uint64_t)mu + (uint64_t)g.qmodp * g.p - (uint64_t)g.qmodp * mu_next;
                        const int64_t c = col * (g.d + 1) + j;
                        if (c < g.n_out) crow[c] = (uint8_t)mod_u64(v, g.p, g.invp);
                        mu_next = mu;
                    }
                }
            }
}

qmm_status check_launch(const char *what) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(QMM_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
    return QMM_OK;
}

template <typename W>
qmm_status launch_qadic_w(const qmm_plan &pl, int64_t m, int64_t n, int64_t k, const void *CA, int64_t ldca,
                          const void *CB, int64_t ldcb, uint8_t *C, int64_t ldc, hipStream_t s) {
    GemmArgs g{};
    g.m = m;
    g.n = n;
    g.kdim = words_for(k, pl.d);
    g.A = CA;
    g.lda = ldca;
    g.B = CB;
    g.ldb = ldcb;
    g.C = C;
    g.ldc = ldc;
    g.n_out = n;
    const bool blocked = pl.k_block < k;
    g.kb_tiles = blocked ? (int32_t)((pl.k_block / (pl.d + 1)) / KT) : 0;
    g.p = pl.p;
    g.t = pl.t;
    g.d = pl.d;
    g.td = pl.t * pl.d;
    g.qmask = (1ull << pl.t) - 1;
    g.invp = 1.0 / (double)pl.p;
    const bool offset = pl.regime == QMM_REGIME_OFFSET;
    g.start = offset ? ldexp(1.0, WordTraits<W>::beta - 1 + (int)(pl.t * pl.d)) : 0.0;
    g.magic = mod_magic(pl.p);
    g.inv_qd = ldexp(1.0, -(int)(pl.t * pl.d));
    g.inv_q = ldexp(1.0, -(int)pl.t);
    g.q = ldexp(1.0, (int)pl.t);
    g.small_digit = pl.t <= 31;
    if (blocked && pl.t > 31) return fail(QMM_EUNSUPPORTED, "blocked plans need t <= 31");
    const dim3 grid((unsigned)(ceil_div(m, BM) * ceil_div(n, BN)));
    if (offset && blocked)
        gemm_kernel<W, W, EPI_QADIC, true, true><<<grid, NT, 0, s>>>(g);
    else if (offset)
        gemm_kernel<W, W, EPI_QADIC, true, false><<<grid, NT, 0, s>>>(g);
    else if (blocked)
        gemm_kernel<W, W, EPI_QADIC, false, true><<<grid, NT, 0, s>>>(g);
    else
        gemm_kernel<W, W, EPI_QADIC, false, false><<<grid, NT, 0, s>>>(g);
    return check_launch("gemm_qadic");
}

template <typename W>
qmm_status launch_redq_w(const qmm_plan &pl, int64_t m, int64_t n, int64_t k, const uint8_t *A, int64_t lda,
                         const void *CBr, int64_t ldcbr, uint8_t *C, int64_t ldc, hipStream_t s) {
    GemmArgs g{};
    g.m = m;
    g.n = words_for(n, pl.d);
    g.kdim = k;
    g.A = A;
    g.lda = lda;
    g.B = CBr;
    g.ldb = ldcbr;
    g.C = C;
    g.ldc = ldc;
    g.n_out = n;
    g.kb_tiles = 0;
    g.p = pl.p;
    g.t = pl.t;
    g.d = pl.d;
    g.td = pl.t * pl.d;
    g.qmask = (1ull << pl.t) - 1;
    g.invp = 1.0 / (double)pl.p;
    g.start = 0.0;
    g.qmodp = (uint32_t)((1ull << pl.t) % pl.p);
    const dim3 grid((unsigned)(ceil_div(m, BM) * ceil_div(g.n, BN)));
    gemm_kernel<W, uint8_t, EPI_REDQ, false, false><<<grid, NT, 0, s>>>(g);
    return check_launch("gemm_redq");
}

}  // namespace

qmm_status launch_gemm_qadic(const qmm_plan &pl, int64_t m, int64_t n, int64_t k, const void *CA, int64_t ldca,
                             const void *CB, int64_t ldcb, uint8_t *C, int64_t ldc, void *stream) {
    if (m == 0 || n == 0) return QMM_OK;
    if (pl.beta == 24) return launch_qadic_w<float>(pl, m, n, k, CA, ldca, CB, ldcb, C, ldc, (hipStream_t)stream);
    return launch_qadic_w<double>(pl, m, n, k, CA, ldca, CB, ldcb, C, ldc, (hipStream_t)stream);
}

qmm_status launch_gemm_redq(const qmm_plan &pl, int64_t m, int64_t n, int64_t k, const uint8_t *A, int64_t lda,
                            const void *CBr, int64_t ldcbr, uint8_t *C, int64_t ldc, void *stream) {
    if (m == 0 || n == 0) return QMM_OK;
    if (pl.beta == 24) return launch_redq_w<float>(pl, m, n, k, A, lda, CBr, ldcbr, C, ldc, (hipStream_t)stream);
    return launch_redq_w<double>(pl, m, n, k, A, lda, CBr, ldcbr, C, ldc, (hipStream_t)stream);
}

}  // namespace qmm
