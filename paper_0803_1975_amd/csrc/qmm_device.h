// Device-side helpers shared by the kernels: reductions mod p and word access.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace qmm {

// x mod p for 0 <= x < 2^53, with invp = RN(1/p).  The float quotient is within
// one of floor(x/p) (relative error of x * invp below 2^-51 and x/p < 2^52), so a
// single correction in each direction gives the exact remainder.
__device__ __forceinline__ uint32_t mod_u64(uint64_t x, uint32_t p, double invp) {
    const uint64_t q = (uint64_t)((double)x * invp);
    int64_t r = (int64_t)x - (int64_t)(q * (uint64_t)p);
    if (r < 0) r += p;
    if (r >= (int64_t)p) r -= p;
    return (uint32_t)r;
}

// floor(x / p) for 0 <= x < 2^53 (same error argument as mod_u64).
__device__ __forceinline__ uint64_t div_u64(uint64_t x, uint32_t p, double invp) {
    uint64_t q = (uint64_t)((double)x * invp);
    const int64_t r = (int64_t)x - (int64_t)(q * (uint64_t)p);
    if (r < 0) q -= 1;
    else if (r >= (int64_t)p) q += 1;
    return q;
}

// u mod p for any 32-bit u and 2 <= p < 2^32, with magic = 2^64/p + e, 0 <= e <= 1
// (mod_magic).  Then u/p <= u * magic / 2^64 < u/p + 2^-32, which never reaches the
// next integer since the fractional part of u/p is at most 1 - 1/p: the high word
// is floor(u/p) exactly.
__device__ __forceinline__ uint32_t mod_u32(uint32_t u, uint32_t p, uint64_t magic) {
    const uint64_t lo = (uint64_t)u * (uint32_t)magic;
    const uint64_t hi = (uint64_t)u * (uint32_t)(magic >> 32);
    const uint32_t q = (uint32_t)((hi + (lo >> 32)) >> 32);
    return u - q * p;
}

// u mod p for any 32-bit u and 2 <= p < 2^31, with m32 = floor(2^32 / p): then
// u/p - 1 < u m32 / 2^32 <= u/p, so the high word q is floor(u/p) or one less, the
// remainder u - q p lies in [0, 2p), and min(r, r - p) (unsigned, r - p wraps when
// r < p) is the residue.  Five 32-bit operations in place of mod_u32's 64-bit ones.
__device__ __forceinline__ uint32_t mod_u32_m32(uint32_t u, uint32_t p, uint32_t m32) {
    const uint32_t r = u - __umulhi(u, m32) * p;
    return min(r, r - p);
}

// 4 x 4 byte transpose across the 4 lanes of a quad: lane j holds bytes
// M[j][0..3] (byte i in bits 8i..8i+7) and gets M[0..3][j].  Two DPP exchanges:
// 16-bit halves with lane j ^ 2, then bytes with lane j ^ 1.
__device__ __forceinline__ uint32_t quad_transpose_bytes(uint32_t w, int j) {
    // quad_perm [2,3,0,1]: lane j reads lane j ^ 2
    const uint32_t o = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)w, 0x4E, 0xF, 0xF, false);
    // j < 2 keeps [w0 w1 o0 o1], j >= 2 keeps [o2 o3 w2 w3]
    const uint32_t t = __builtin_amdgcn_perm(o, w, (j & 2) ? 0x03020706u : 0x05040100u);
    // quad_perm [1,0,3,2]: lane j reads lane j ^ 1
    const uint32_t u = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)t, 0xB1, 0xF, 0xF, false);
    // even j: [t0 u0 t2 u2], odd j: [u1 t1 u3 t3]
    return __builtin_amdgcn_perm(u, t, (j & 1) ? 0x03070105u : 0x06020400u);
}

// x mod p for a signed 32-bit x with |x| <= 2^31 - p: off = p floor(2^31 / p) is a
// multiple of p that makes x + off land in [1, 2^32).
__device__ __forceinline__ uint32_t mod_i32_magic(int32_t x, uint32_t p, uint64_t magic, uint32_t off) {
    return mod_u32((uint32_t)x + off, p, magic);
}

// x mod p in [0, p) for a signed 32-bit x.
__device__ __forceinline__ uint32_t mod_i32(int32_t x, uint32_t p, double invp) {
    const double q = floor((double)x * invp);
    int64_t r = (int64_t)x - (int64_t)q * (int64_t)p;
    if (r < 0) r += p;
    if (r >= (int64_t)p) r -= p;
    return (uint32_t)r;
}

// Word <-> integer conversions.  Packed words are non-negative integers that the
// plan's bounds keep exactly representable.
template <typename W> __device__ __forceinline__ W word_from_u64(uint64_t v);
template <> __device__ __forceinline__ double word_from_u64<double>(uint64_t v) { return (double)v; }
template <> __device__ __forceinline__ float word_from_u64<float>(uint64_t v) { return (float)v; }

__device__ __forceinline__ uint64_t u64_from_word(double w) { return (uint64_t)w; }
__device__ __forceinline__ uint64_t u64_from_word(float w) { return (uint64_t)w; }

// The bits of an exact word 0 <= w < 2^(beta-1) (a product word of the exact
// regime: every coefficient below Q and t (d+1) <= beta - 1) with one addition:
// w + 2^(beta-1) lies in [2^(beta-1), 2^beta), where the ulp is 1, so the sum is
// exact and its low beta-1 mantissa bits are w.  (A conversion to a 64-bit integer
// takes a sequence of instructions.)
__device__ __forceinline__ uint64_t exact_word_bits(double w) {
    return (uint64_t)__double_as_longlong(w + 4503599627370496.0) & ((1ull << 52) - 1);
}
__device__ __forceinline__ uint64_t exact_word_bits(float w) {
    return (uint64_t)(__float_as_uint(w + 8388608.0f) & ((1u << 23) - 1));
}

// Bit field [sh, sh + t) of a 64-bit value with t <= 32, from its 32-bit halves
// (alignbit shifts the pair hi:lo right by sh < 32).
__device__ __forceinline__ uint32_t bit_field(uint64_t x, uint32_t sh, uint32_t mask) {
    const uint32_t lo = (uint32_t)x, hi = (uint32_t)(x >> 32);
    const uint32_t v = sh < 32 ? __builtin_amdgcn_alignbit(hi, lo, sh) : hi >> (sh - 32);
    return v & mask;
}

// Low 32 bits of the encoding: in the OFFSET regime they are the low bits of
// floor(S / Q^d), i.e. digit d in the low t bits.
__device__ __forceinline__ uint32_t low_mantissa_bits(double w) {
    return (uint32_t)__double_as_longlong(w);
}
__device__ __forceinline__ uint32_t low_mantissa_bits(float w) { return __float_as_uint(w); }

// Digit d of an accumulated word with only exact floating-point steps, as the
// paper's init routine does: scale by Q^-d (a power of two), floor, and keep the
// low t bits as x - Q floor(x / Q).  Exact regime only (the word is S < 2^beta).
template <typename W>
__device__ __forceinline__ uint32_t exact_digit(W acc, W inv_qd, W inv_q, W q) {
    const W x = floor(acc * inv_qd);
    return (uint32_t)(x - q * floor(x * inv_q));
}

// Digit d of an accumulated word, for either regime.
template <typename W>
__device__ __forceinline__ uint32_t qadic_digit(W acc, bool offset, uint32_t td, uint64_t qmask) {
    if (offset) return low_mantissa_bits(acc) & (uint32_t)qmask;
    return (uint32_t)((u64_from_word(acc) >> td) & qmask);
}

// The accumulator start value of the OFFSET regime: 2^(beta-1) Q^d.
template <typename W> struct WordTraits;
template <> struct WordTraits<double> {
    static constexpr int beta = 53;
};
template <> struct WordTraits<float> {
    static constexpr int beta = 24;
};

// Global-address-space pointers: loads through them use the vector memory path
// only (a generic pointer would also hold the LDS wait counter).
#define QMM_GLOBAL __attribute__((address_space(1)))
typedef unsigned int u32x4a4 __attribute__((ext_vector_type(4), aligned(4)));  // 16 bytes, 4-byte aligned

// 16 bytes of a residue matrix from p (any alignment), bytes at positions >= valid
// zero, in two halves so that all of a stage's loads are in flight before any of
// them is waited for.  raw_issue32 starts the loads into w: one 16-byte
// and one 4-byte load of the dword-aligned 20-byte window when it lies inside the
// matrix's data, else the window's dwords that do and the last bytes of the data;
// it records the byte shift and the valid count in meta.  raw_finish, called once the data is needed, aligns the
// bytes and zeroes those past valid.
__device__ __forceinline__ void raw_finish(const uint32_t (&w)[5], int32_t meta, uint32_t (&o)[4]) {
    const uint32_t sh = (uint32_t)(meta >> 8) & 3u;
    const int32_t v = meta & 0xff;
#pragma unroll
    for (int j = 0; j < 4; ++j) o[j] = __builtin_amdgcn_alignbyte(w[j + 1], w[j], sh);
    if (v < 16) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int32_t left = v - 4 * j;
            o[j] &= left >= 4 ? 0xffffffffu : (left <= 0 ? 0u : (1u << (8 * left)) - 1u);
        }
    }
}

// The issue half, the matrix given as a uniform base X and a 32-bit byte offset
// (the caller has checked that the data is at most kRawSpan bytes long):
// the address is the scalar base plus one vector register, with no 64-bit
// arithmetic per load.  size is the length of the matrix's data from X.
__device__ __forceinline__ void raw_issue32(uint32_t (&w)[5], int32_t &meta, const uint8_t *X, uint32_t off,
                                            int32_t valid, uint32_t size) {
#pragma unroll
    for (int j = 0; j < 5; ++j) w[j] = 0;
    meta = 0;
    if (valid > 0) {
        const int32_t v = valid < 16 ? valid : 16;
        const uint32_t o4 = off & ~3u;
        if (o4 + 20u <= size) {
            const u32x4a4 x = *(const QMM_GLOBAL u32x4a4 *)(X + o4);
            w[0] = x.x;
            w[1] = x.y;
            w[2] = x.z;
            w[3] = x.w;
            w[4] = *(const QMM_GLOBAL uint32_t *)(X + o4 + 16u);
            meta = v | (int32_t)(off & 3u) << 8;
        } else {
            // the window runs past the data: the dwords wholly inside it, then the
            // bytes of the one the data ends in (none past it is read)
            const uint32_t whole = (size - o4) >> 2;  // dwords of the window inside the data
#pragma unroll
            for (int j = 0; j < 5; ++j)
                if ((uint32_t)j < whole) w[j] = *(const QMM_GLOBAL uint32_t *)(X + o4 + 4u * (uint32_t)j);
            if (whole < 5u) {
                const uint32_t last = o4 + 4u * whole;
                uint32_t x = 0;
#pragma unroll
                for (uint32_t b = 0; b < 3; ++b)
                    if (last + b < size) x |= (uint32_t)((const QMM_GLOBAL uint8_t *)X)[last + b] << (8 * b);
#pragma unroll
                for (int j = 0; j < 5; ++j)
                    if ((uint32_t)j == whole) w[j] = x;
            }
            meta = v | (int32_t)(off & 3u) << 8;
        }
    }
}

// Unaligned 16-byte access: the memory system serves vector loads and stores at
// any byte address (compute queues run with unaligned access enabled; the compiler
// emits one dwordx4 load for a 1-byte aligned 16-byte vector on this target).
typedef unsigned int u32x4a1 __attribute__((ext_vector_type(4), aligned(1)));
typedef unsigned int u32a1 __attribute__((aligned(1)));
typedef unsigned int uint4v_t __attribute__((ext_vector_type(4)));

// Issue half of a 16-byte load at X + off of a byte matrix whose data is size >= 16
// bytes from X: the load starts at min(off, size - 16), so it never leaves the
// data, and shift (0 for every load that fits) says how many bytes to move down
// when it is finished (shift_down_bytes).  Zero, with no load, when !ok.  Bytes past
// a row's end are NOT cleared: they are the next row's, and the caller must make
// them harmless.
__device__ __forceinline__ uint4v_t load16_clamped(const uint8_t *X, uint32_t off, bool ok, uint32_t size,
                                                  uint32_t &shift) {
    const uint32_t oc = off + 16u <= size ? off : size - 16u;
    uint4v_t v = {0u, 0u, 0u, 0u};
    shift = 0;
    if (ok) {
        const u32x4a1 x = *(const QMM_GLOBAL u32x4a1 *)(X + oc);
        v = uint4v_t{x.x, x.y, x.z, x.w};
        shift = off - oc;
    }
    return v;
}

// v moved down by s bytes (0 <= s < 16), zeros shifted in at the top.
__device__ __forceinline__ uint4v_t shift_down_bytes(uint4v_t v, uint32_t s) {
    const uint32_t q = s >> 2, r = s & 3u;
    auto dw = [&](uint32_t i) { return i == 0 ? v.x : i == 1 ? v.y : i == 2 ? v.z : i == 3 ? v.w : 0u; };
    uint32_t o[4];
#pragma unroll
    for (uint32_t j = 0; j < 4; ++j) o[j] = __builtin_amdgcn_alignbyte(dw(j + q + 1), dw(j + q), r);
    return uint4v_t{o[0], o[1], o[2], o[3]};
}

// 16 bytes at X + off of a byte matrix whose data is shorter than 16 bytes: byte
// loads of what lies inside it, zeros elsewhere (and none when !ok).
__device__ __forceinline__ uint4v_t load16_tiny(const uint8_t *X, uint32_t off, bool ok, uint32_t size) {
    uint64_t lo = 0, hi = 0;
    if (ok) {
        // one byte at a time (a rare path: kept rolled, so it holds few registers)
#pragma nounroll
        for (uint32_t b = 0; b < 16u; ++b) {
            const uint64_t x = off + b < size ? (uint64_t)((const QMM_GLOBAL uint8_t *)X)[off + b] << (8 * (b & 7)) : 0;
            if (b < 8) lo |= x; else hi |= x;
        }
    }
    return uint4v_t{(uint32_t)lo, (uint32_t)(lo >> 32), (uint32_t)hi, (uint32_t)(hi >> 32)};
}

// The issue half with a plain pointer p into data that ends at end (any length:
// the window is checked against end in 64 bits).
__device__ __forceinline__ void raw_issue_ptr(uint32_t (&w)[5], int32_t &meta, const uint8_t *p, int64_t valid,
                                              const uint8_t *end) {
#pragma unroll
    for (int j = 0; j < 5; ++j) w[j] = 0;
    meta = 0;
    if (valid > 0) {
        const int32_t v = valid < 16 ? (int32_t)valid : 16;
        const uint32_t sh = (uint32_t)((uintptr_t)p & 3);
        const uint8_t *W = p - sh;
        const int64_t avail = end - W;
        if (avail >= 20) {
            const u32x4a4 x = *(const QMM_GLOBAL u32x4a4 *)W;
            w[0] = x.x;
            w[1] = x.y;
            w[2] = x.z;
            w[3] = x.w;
            w[4] = *(const QMM_GLOBAL uint32_t *)(W + 16);
        } else {
            const uint32_t whole = (uint32_t)avail >> 2;
#pragma unroll
            for (int j = 0; j < 5; ++j)
                if ((uint32_t)j < whole) w[j] = *(const QMM_GLOBAL uint32_t *)(W + 4 * j);
            if (whole < 5u) {
                uint32_t x = 0;
#pragma unroll
                for (uint32_t b = 0; b < 3; ++b)
                    if (4u * whole + b < (uint32_t)avail)
                        x |= (uint32_t)((const QMM_GLOBAL uint8_t *)W)[4u * whole + b] << (8 * b);
#pragma unroll
                for (int j = 0; j < 5; ++j)
                    if ((uint32_t)j == whole) w[j] = x;
            }
        }
        meta = v | (int32_t)sh << 8;
    }
}

}  // namespace qmm
