// fp.hpp -- arithmetic in the P-256 prime field on gfx950.
//
// The field is F_p with p = 2^256 - 2^224 + 2^192 + 2^96 - 1 (the curve of the
// paper's implementation, Sec. 4.1).  An element lives in eight 32-bit VGPR
// limbs (little-endian) in Montgomery form x R mod p with R = 2^256, always
// fully reduced into [0, p), so equality and zero tests are limb compares.
//
// Montgomery multiplication is word-serial (one 32-bit digit of b per round).
// Because p = -1 (mod 2^32), the per-round quotient digit is the low word
// itself, and adding that digit times p is a handful of shifted additions:
//   t + m p = t - m + m 2^96 + m 2^192 - m 2^224 + m 2^256,
// so after the exact division by 2^32 the round adds m at word 2 and word 5
// and m (2^32 - 1) at words 6..7 -- no multiplications.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pcmm {

struct fe {
    uint32_t v[8];
};

// ---------------------------------------------------------------------------
// Compile-time constants (computed from p alone, no external tables).
// ---------------------------------------------------------------------------
struct fe_const {
    uint32_t v[8];
};

constexpr fe_const P_WORDS = {{0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0u, 0u, 0u, 1u, 0xFFFFFFFFu}};

constexpr bool c_geq(const fe_const &a, const fe_const &b) {
    for (int i = 7; i >= 0; --i) {
        if (a.v[i] != b.v[i]) return a.v[i] > b.v[i];
    }
    return true;
}

constexpr fe_const c_sub(const fe_const &a, const fe_const &b) {
    fe_const r{};
    uint64_t borrow = 0;
    for (int i = 0; i < 8; ++i) {
        uint64_t d = (uint64_t)a.v[i] - b.v[i] - borrow;
        r.v[i] = (uint32_t)d;
        borrow = (d >> 63) & 1;
    }
    return r;
}

// 2x mod p for x in [0, p)
constexpr fe_const c_dbl(const fe_const &a) {
    fe_const r{};
    uint32_t carry = 0;
    for (int i = 0; i < 8; ++i) {
        uint64_t s = (uint64_t)a.v[i] * 2 + carry;
        r.v[i] = (uint32_t)s;
        carry = (uint32_t)(s >> 32);
    }
    if (carry || c_geq(r, P_WORDS)) r = c_sub(r, P_WORDS);
    return r;
}

// x 2^k mod p by k doublings
constexpr fe_const c_shift(fe_const a, int k) {
    for (int i = 0; i < k; ++i) a = c_dbl(a);
    return a;
}

constexpr fe_const c_from_hex(const char *h) {
    fe_const r{};
    for (int i = 0; i < 64; ++i) {
        char ch = h[i];
        uint32_t d = (ch >= '0' && ch <= '9') ? (uint32_t)(ch - '0')
                   : (ch >= 'a' && ch <= 'f') ? (uint32_t)(ch - 'a' + 10)
                                              : (uint32_t)(ch - 'A' + 10);
        int bit = (63 - i) * 4;
        r.v[bit / 32] |= d << (bit % 32);
    }
    return r;
}

constexpr fe_const ONE_PLAIN = {{1, 0, 0, 0, 0, 0, 0, 0}};
constexpr fe_const R_MOD_P = c_shift(ONE_PLAIN, 256);   // Montgomery form of 1
constexpr fe_const R2_MOD_P = c_shift(R_MOD_P, 256);    // R^2 mod p

// ---------------------------------------------------------------------------
// Basic limb helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ fe fe_from(const fe_const &c) {
    fe r;
#pragma unroll
    for (int i = 0; i < 8; ++i) r.v[i] = c.v[i];
    return r;
}

__device__ __forceinline__ fe fe_zero() {
    fe r;
#pragma unroll
    for (int i = 0; i < 8; ++i) r.v[i] = 0;
    return r;
}

__device__ __forceinline__ fe fe_one_mont() { return fe_from(R_MOD_P); }

__device__ __forceinline__ bool fe_is_zero(const fe &a) {
    uint32_t x = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) x |= a.v[i];
    return x == 0;
}

__device__ __forceinline__ bool fe_eq(const fe &a, const fe &b) {
    uint32_t x = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) x |= a.v[i] ^ b.v[i];
    return x == 0;
}

// r = c ? b : a, limb-wise (no branch)
__device__ __forceinline__ fe fe_select(bool c, const fe &a, const fe &b) {
    fe r;
#pragma unroll
    for (int i = 0; i < 8; ++i) r.v[i] = c ? b.v[i] : a.v[i];
    return r;
}

// ---------------------------------------------------------------------------
// Addition and subtraction mod p (inputs and outputs in [0, p))
// ---------------------------------------------------------------------------
// Carries are propagated through 64-bit sums (s = a + b + c, digit = low
// word, carry = high word) rather than through the compiler's add-with-carry
// intrinsics.
__device__ __forceinline__ fe fe_add(const fe &a, const fe &b) {
    fe s, t;
    uint64_t c = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        c += (uint64_t)a.v[i] + b.v[i];
        s.v[i] = (uint32_t)c;
        c >>= 32;
    }
    // t = s - p; keep t when the sum overflowed 2^256 or s >= p
    uint64_t bw = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        uint64_t d = (uint64_t)s.v[i] - P_WORDS.v[i] - bw;
        t.v[i] = (uint32_t)d;
        bw = d >> 63;
    }
    bool use_t = (c != 0) || (bw == 0);
    return fe_select(use_t, s, t);
}

__device__ __forceinline__ fe fe_sub(const fe &a, const fe &b) {
    fe d, t;
    uint64_t bw = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        uint64_t x = (uint64_t)a.v[i] - b.v[i] - bw;
        d.v[i] = (uint32_t)x;
        bw = x >> 63;
    }
    uint64_t c = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        c += (uint64_t)d.v[i] + P_WORDS.v[i];
        t.v[i] = (uint32_t)c;
        c >>= 32;
    }
    return fe_select(bw != 0, d, t);
}

__device__ __forceinline__ fe fe_neg(const fe &a) { return fe_sub(fe_zero(), a); }

__device__ __forceinline__ fe fe_dbl(const fe &a) { return fe_add(a, a); }

// ---------------------------------------------------------------------------
// Montgomery multiplication: a b R^-1 mod p
// ---------------------------------------------------------------------------
__device__ __forceinline__ fe fe_mul(const fe &a, const fe &b) {
    // t holds a 9-word running value (t[8] is at most 1 between rounds)
    uint32_t t[9];
#pragma unroll
    for (int j = 0; j < 9; ++j) t[j] = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        // t += a * b_i
        uint32_t carry = 0;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            uint64_t s = (uint64_t)a.v[j] * b.v[i] + t[j] + carry;
            t[j] = (uint32_t)s;
            carry = (uint32_t)(s >> 32);
        }
        uint64_t s8 = (uint64_t)t[8] + carry;
        t[8] = (uint32_t)s8;
        const uint32_t c9 = (uint32_t)(s8 >> 32);
        // reduction by m = t[0]: u = t / 2^32 + m 2^64 + m 2^160 + m (2^32 - 1) 2^192
        const uint32_t m = t[0];
        const uint64_t mm = ((uint64_t)m << 32) - m;     // m (2^32 - 1)
        const uint32_t add[8] = {0u, 0u, m, 0u, 0u, m, (uint32_t)mm, (uint32_t)(mm >> 32)};
        uint64_t c = 0;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            c += (uint64_t)t[k + 1] + add[k];
            t[k] = (uint32_t)c;
            c >>= 32;
        }
        t[8] = c9 + (uint32_t)c;
    }
    // t < 2p: subtract p once if needed
    fe r, sb;
#pragma unroll
    for (int i = 0; i < 8; ++i) r.v[i] = t[i];
    uint64_t bw = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        uint64_t d = (uint64_t)r.v[i] - P_WORDS.v[i] - bw;
        sb.v[i] = (uint32_t)d;
        bw = d >> 63;
    }
    bool use_s = (t[8] != 0) || (bw == 0);
    return fe_select(use_s, r, sb);
}

__device__ __forceinline__ fe fe_sqr(const fe &a) { return fe_mul(a, a); }

__device__ __forceinline__ fe fe_sqr_n(fe a, int n) {
    for (int i = 0; i < n; ++i) a = fe_sqr(a);
    return a;
}

__device__ __forceinline__ fe fe_to_mont(const fe &a) { return fe_mul(a, fe_from(R2_MOD_P)); }

__device__ __forceinline__ fe fe_from_mont(const fe &a) { return fe_mul(a, fe_from(ONE_PLAIN)); }

// a^(p-2) = a^-1 for a != 0 (0 maps to 0).  p - 2 in 32-bit words from the
// top: ffffffff 00000001 00000000 00000000 00000000 ffffffff ffffffff fffffffd.
// x_k below is a^(2^k - 1); the chain uses 255 squarings and 12 products.
__device__ __noinline__ fe fe_inv(const fe &a) {
    fe x1 = a;
    fe x2 = fe_mul(fe_sqr(x1), x1);
    fe x3 = fe_mul(fe_sqr(x2), x1);
    fe x6 = fe_mul(fe_sqr_n(x3, 3), x3);
    fe x12 = fe_mul(fe_sqr_n(x6, 6), x6);
    fe x15 = fe_mul(fe_sqr_n(x12, 3), x3);
    fe x30 = fe_mul(fe_sqr_n(x15, 15), x15);
    fe x32 = fe_mul(fe_sqr_n(x30, 2), x2);
    fe r = x32;                               // word 7: 32 ones
    r = fe_mul(fe_sqr_n(r, 32), x1);          // word 6: 0x00000001
    r = fe_mul(fe_sqr_n(r, 128), x32);        // words 5..3 zero, word 2: 32 ones
    r = fe_mul(fe_sqr_n(r, 32), x32);         // word 1: 32 ones
    r = fe_mul(fe_sqr_n(r, 30), x30);         // word 0: 30 ones,
    r = fe_mul(fe_sqr_n(r, 2), x1);           //         then bits 0 1
    return r;
}

}  // namespace pcmm
