// fp.hpp -- arithmetic in the P-256 prime field on gfx950.
//
// The field is F_p with p = 2^256 - 2^224 + 2^192 + 2^96 - 1 (the curve of the
// paper's implementation, Sec. 4.1).
//
// Representation: nine 29-bit limbs in 32-bit VGPRs ("unsaturated"),
// value = sum_i v[i] 2^(29 i), in Montgomery form x R mod p with R = 2^261.
// Every fe produced by the functions below is in normal form:
//   limbs 0..7 < 2^29, limb 8 < 2^25, value < 2p (not necessarily < p).
// Why 29 bits: gfx950 issues the 32 x 32 -> 64-bit multiply-add at full rate,
// and with 29-bit limbs a whole column of a product (at most 9 partial
// products plus 4 reduction terms, < 2^62) fits one 64-bit accumulator, so
// every partial product is exactly one multiply-add into the accumulator and
// no carry is propagated inside the multiplication.
// Montgomery reduction: p = -1 (mod 2^29), so the per-column quotient digit m
// is simply the low 29 bits of the column.  In signed radix-2^29 digits
//   p = -1 + 2^9 B^3 + 2^18 B^6 - 2^21 B^7 + 2^24 B^8      (B = 2^29),
// so adding m p clears the low 29 bits of the column (the -1 digit: the
// carry out is just the column shifted right) and adds four multiples of m
// to later columns: four multiply-adds per quotient digit.  The column
// accumulators are therefore signed 64-bit.
// Carries between limbs are handled with plain 32/64-bit integer shifts and
// masks (no add-with-carry intrinsics).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pcmm {

constexpr int NL = 9;                       // limbs
constexpr int LB = 29;                      // bits per limb
constexpr uint32_t LMASK = (1u << LB) - 1;

struct fe {
    uint32_t v[NL];
};

// ---------------------------------------------------------------------------
// Compile-time constants, computed from p alone.
// fe_const: canonical value as eight 32-bit words (little-endian);
// fe29: the same value as nine 29-bit limbs.
// ---------------------------------------------------------------------------
struct fe_const {
    uint32_t v[8];
};

struct fe29 {
    uint32_t v[NL];
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

// bits [29 i, 29 i + 29) of a 256-bit value
constexpr fe29 c_to29(const fe_const &a) {
    fe29 r{};
    for (int i = 0; i < NL; ++i) {
        int bit = LB * i;
        uint64_t lo = a.v[bit / 32];
        uint64_t hi = (bit / 32 + 1 < 8) ? a.v[bit / 32 + 1] : 0;
        r.v[i] = (uint32_t)(((lo | (hi << 32)) >> (bit % 32)) & LMASK);
    }
    return r;
}

constexpr fe_const ONE_PLAIN = {{1, 0, 0, 0, 0, 0, 0, 0}};
constexpr fe_const R_MOD_P = c_shift(ONE_PLAIN, 261);    // Montgomery form of 1
constexpr fe_const R2_MOD_P = c_shift(R_MOD_P, 261);     // R^2 mod p
constexpr fe29 P29 = c_to29(P_WORDS);
constexpr fe29 TWO_P29 = {{0x1ffffffeu, 0x1fffffffu, 0x1fffffffu, 0x3ffu, 0u, 0u, 0x80000u, 0x1fc00000u, 0x1ffffffu}};
constexpr fe29 ONE29 = c_to29(ONE_PLAIN);
constexpr fe29 R29 = c_to29(R_MOD_P);
constexpr fe29 R2_29 = c_to29(R2_MOD_P);
constexpr fe_const R3_MOD_P = c_shift(R2_MOD_P, 261);    // R^3 mod p
constexpr fe29 R3_29 = c_to29(R3_MOD_P);

// 2p as limbs must be the radix-2^29 digits of 2p (checked at compile time)
constexpr bool c_check_2p() {
    fe_const two_p{};
    uint32_t carry = 0;
    for (int i = 0; i < 8; ++i) {
        uint64_t s = (uint64_t)P_WORDS.v[i] * 2 + carry;
        two_p.v[i] = (uint32_t)s;
        carry = (uint32_t)(s >> 32);
    }
    fe29 d = c_to29(two_p);
    d.v[8] |= carry << (256 - LB * 8);  // bit 256 of 2p lives in limb 8
    for (int i = 0; i < NL; ++i)
        if (d.v[i] != TWO_P29.v[i]) return false;
    return true;
}
static_assert(c_check_2p(), "2p limbs");

// K p as radix-2^29 digits: limbs 0..7 < 2^29, limb 8 the rest (exact)
struct fe29w {
    int64_t v[NL];
};

constexpr fe29w c_kp(int K) {
    fe29w r{};
    int64_t carry = 0;
    for (int i = 0; i < NL; ++i) {
        int64_t t = (int64_t)K * P29.v[i] + carry;
        if (i < NL - 1) {
            r.v[i] = t & LMASK;
            carry = t >> LB;
        } else {
            r.v[i] = t;
        }
    }
    return r;
}

constexpr fe29w KP4 = c_kp(4), KP6 = c_kp(6);

// K p as digits with limbs 0..7 in (-2^29, 0] (each positive digit lends
// 2^29 to the next limb) and limb 8 the rest
constexpr fe29w c_kp_nonpos(int K) {
    fe29w r = c_kp(K);
    for (int i = 0; i < NL - 1; ++i)
        if (r.v[i] > 0) {
            r.v[i] -= (int64_t)1 << LB;
            r.v[i + 1] += 1;
        }
    return r;
}

constexpr fe29w KN6 = c_kp_nonpos(6);

constexpr bool c_check_kn6() {
    int64_t carry = 0;
    for (int i = 0; i < NL; ++i) {
        if (i < NL - 1 && (KN6.v[i] > 0 || KN6.v[i] <= -((int64_t)1 << LB))) return false;
        const int64_t t = KN6.v[i] + carry;
        if (i == NL - 1) return t == KP6.v[i];
        const int64_t d = t & LMASK;  // the same value in radix-2^29 digits
        carry = (t - d) >> LB;
        if (d != KP6.v[i]) return false;
    }
    return false;
}
static_assert(c_check_kn6(), "6p with non-positive limbs");

// ---------------------------------------------------------------------------
// Limb helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ fe fe_from29(const fe29 &c) {
    fe r;
#pragma unroll
    for (int i = 0; i < NL; ++i) r.v[i] = c.v[i];
    return r;
}

__device__ __forceinline__ fe fe_zero() {
    fe r;
#pragma unroll
    for (int i = 0; i < NL; ++i) r.v[i] = 0;
    return r;
}

__device__ __forceinline__ fe fe_one_mont() { return fe_from29(R29); }

// r = c ? b : a, limb-wise (no branch)
__device__ __forceinline__ fe fe_select(bool c, const fe &a, const fe &b) {
    fe r;
#pragma unroll
    for (int i = 0; i < NL; ++i) r.v[i] = c ? b.v[i] : a.v[i];
    return r;
}

// value = 0 (mod p) for a normal-form value (which is then 0 or p)
__device__ __forceinline__ bool fe_is_zero(const fe &a) {
    uint32_t z = 0, q = 0;
#pragma unroll
    for (int i = 0; i < NL; ++i) {
        z |= a.v[i];
        q |= a.v[i] ^ P29.v[i];
    }
    return z == 0 || q == 0;
}

// raw limbs all zero (used only for the affine encoding of infinity)
__device__ __forceinline__ bool fe_is_raw_zero(const fe &a) {
    uint32_t z = 0;
#pragma unroll
    for (int i = 0; i < NL; ++i) z |= a.v[i];
    return z == 0;
}

// signed carry propagation over limbs 0..7 into limb 8 (limbs as int32)
__device__ __forceinline__ void fe_carry(fe &x) {
#pragma unroll
    for (int i = 0; i < NL - 1; ++i) {
        int32_t c = (int32_t)x.v[i] >> LB;
        x.v[i] &= LMASK;
        x.v[i + 1] += (uint32_t)c;
    }
}

// Normal form of a value 0 <= V < 2^260 held in signed limbs (|limb| < 2^31):
// propagate carries, fold the bits at and above 2^256 with
// 2^256 = 2^224 - 2^192 - 2^96 + 1 (mod p), i.e. V - h p with h = V >> 256,
// which lands in [0, 2p), and propagate again.
__device__ __forceinline__ fe fe_norm(fe x) {
    fe_carry(x);
    const uint32_t h = x.v[8] >> 24;         // 2^256 is bit 24 of limb 8
    x.v[8] &= (1u << 24) - 1;
    x.v[0] += h;                             // + h
    x.v[3] -= h << 9;                        // - h 2^96  (96 = 3 * 29 + 9)
    x.v[6] -= h << 18;                       // - h 2^192 (192 = 6 * 29 + 18)
    x.v[7] += h << 21;                       // + h 2^224 (224 = 7 * 29 + 21)
    fe_carry(x);
    return x;
}

// ---------------------------------------------------------------------------
// Addition and subtraction (normal form in, normal form out)
// ---------------------------------------------------------------------------
__device__ __forceinline__ fe fe_add(const fe &a, const fe &b) {
    fe x;
#pragma unroll
    for (int i = 0; i < NL; ++i) x.v[i] = a.v[i] + b.v[i];
    return fe_norm(x);
}

// a - b + 2p, in (0, 4p)
__device__ __forceinline__ fe fe_sub(const fe &a, const fe &b) {
    fe x;
#pragma unroll
    for (int i = 0; i < NL; ++i) x.v[i] = a.v[i] - b.v[i] + TWO_P29.v[i];
    return fe_norm(x);
}

// 2 (a - b), in (0, 8p)
__device__ __forceinline__ fe fe_sub2(const fe &a, const fe &b) {
    fe x;
#pragma unroll
    for (int i = 0; i < NL; ++i) x.v[i] = (a.v[i] - b.v[i] + TWO_P29.v[i]) << 1;
    return fe_norm(x);
}

__device__ __forceinline__ fe fe_neg(const fe &a) { return fe_sub(fe_zero(), a); }

__device__ __forceinline__ fe fe_dbl(const fe &a) {
    fe x;
#pragma unroll
    for (int i = 0; i < NL; ++i) x.v[i] = a.v[i] << 1;
    return fe_norm(x);
}

// 3a and 4a (value < 8p before normalisation)
__device__ __forceinline__ fe fe_mul3(const fe &a) {
    fe x;
#pragma unroll
    for (int i = 0; i < NL; ++i) x.v[i] = a.v[i] * 3u;
    return fe_norm(x);
}

__device__ __forceinline__ fe fe_mul4(const fe &a) {
    fe x;
#pragma unroll
    for (int i = 0; i < NL; ++i) x.v[i] = a.v[i] << 2;
    return fe_norm(x);
}

__device__ __forceinline__ bool fe_eq(const fe &a, const fe &b) { return fe_is_zero(fe_sub(a, b)); }

// ---------------------------------------------------------------------------
// Lazy forms.  A carry-only ("weak") result has limbs 0..7 in [0, 2^29) and
// the rest of the value in limb 8, without the fold below 2p.  fe_mul and
// fe_sqr accept such operands as long as the product of the operands' bounds
// is at most 32 p^2 (then a b < p 2^261 and the Montgomery result is again
// below 2p, in normal form), with limb 8 below 2^27 (column sums stay below
// 2^63).
// ---------------------------------------------------------------------------
// 2a with its limbs doubled and no carries (limbs 0..7 < 2^30, limb 8 <
// 2^27 for a weak or normal a, value < 8p).  Only as ONE operand of a
// product whose other operand has limbs 0..7 < 2^29: a column then holds
// at most 8 products below 2^59, the carry and 4 reduction terms below 2^55,
// so it stays below 2^63; the value bound a b <= 32 p^2 still applies.
__device__ __forceinline__ fe fe_x2(const fe &a) {
    fe x;
#pragma unroll
    for (int i = 0; i < NL; ++i) x.v[i] = a.v[i] << 1;
    return x;
}

// a - b + 2p in (0, 4p) for a, b normal; weak
__device__ __forceinline__ fe fe_sub_w(const fe &a, const fe &b) {
    fe x;
#pragma unroll
    for (int i = 0; i < NL; ++i) x.v[i] = a.v[i] - b.v[i] + TWO_P29.v[i];
    fe_carry(x);
    return x;
}

// a + b in [0, 4p) for a, b normal; weak
__device__ __forceinline__ fe fe_add_w(const fe &a, const fe &b) {
    fe x;
#pragma unroll
    for (int i = 0; i < NL; ++i) x.v[i] = a.v[i] + b.v[i];
    fe_carry(x);
    return x;
}

// 4a in [0, 8p) for a normal; weak
__device__ __forceinline__ fe fe_mul4_w(const fe &a) {
    fe x;
#pragma unroll
    for (int i = 0; i < NL; ++i) x.v[i] = a.v[i] << 2;
    fe_carry(x);
    return x;
}

// a - b - 2c (mod p) for a, b, c normal: one limb pass adding the digits of
// 6p (signed limb sums in (-3 2^29, 2^30), value in (0, 8p)), then
// normalised
__device__ __forceinline__ fe fe_sub_sub2(const fe &a, const fe &b, const fe &c) {
    fe x;
#pragma unroll
    for (int i = 0; i < NL; ++i) x.v[i] = a.v[i] - b.v[i] - (c.v[i] << 1) + (uint32_t)KP6.v[i];
    return fe_norm(x);
}

// 4a - b - 2c (mod p) for a, b, c normal: one limb pass adding the digits of
// 6p with limbs 0..7 in (-2^29, 0] (signed limb sums in (-2^31, 2^31), value
// in (0, 14p)), then normalised
__device__ __forceinline__ fe fe_4sub_sub2(const fe &a, const fe &b, const fe &c) {
    fe x;
#pragma unroll
    for (int i = 0; i < NL; ++i) x.v[i] = (a.v[i] << 2) - b.v[i] - (c.v[i] << 1) + (uint32_t)KN6.v[i];
    return fe_norm(x);
}

// a - 2b (mod p) for a, b normal: adds the digits of 4p, value in (0, 6p)
__device__ __forceinline__ fe fe_sub2x(const fe &a, const fe &b) {
    fe x;
#pragma unroll
    for (int i = 0; i < NL; ++i) x.v[i] = a.v[i] - (b.v[i] << 1) + (uint32_t)KP4.v[i];
    return fe_norm(x);
}

// ---------------------------------------------------------------------------
// Montgomery multiplication a b 2^-261 mod p (product scanning, the
// reduction interleaved column by column)
// ---------------------------------------------------------------------------
// red_terms adds to column c the contributions m_i p_j (i + j = c) of the
// earlier quotient digits m_i, for the nonzero signed digits p_3, p_6, p_7,
// p_8 of p (see the header).  The multipliers are kept opaque to the compiler
// so that each term stays one 32 x 32 -> 64-bit multiply-add instead of
// becoming a 64-bit shift plus an add.
struct red_consts {
    uint32_t k9, k18, k24;
    int32_t kn21;
};

__device__ __forceinline__ red_consts red_consts_make() {
    red_consts k{1u << 9, 1u << 18, 1u << 24, -(1 << 21)};
    asm("" : "+s"(k.k9), "+s"(k.k18), "+s"(k.k24), "+s"(k.kn21));
    return k;
}

// CHAIN = true sums each column as one chain of 32 x 32 + 64-bit
// multiply-adds: the accumulator passes through an empty register constraint
// after every term, which stops the compiler from splitting the column into
// parallel partial sums that cost one extra 64-bit add each (15 per product).
// That suits the point formulas, whose independent products give the
// scheduler parallelism enough; a lone serial chain of products (the
// inversion, prefix products) is latency-bound and keeps the split form.
template <bool CHAIN>
__device__ __forceinline__ void chain(int64_t &acc) {
    if constexpr (CHAIN) asm("" : "+v"(acc));
}

template <bool CHAIN>
__device__ __forceinline__ void red_terms(int64_t &acc, const uint32_t *m, int c, const red_consts &k) {
#pragma unroll
    for (int i = 0; i < NL; ++i) {
        const int j = c - i;
        if (i >= c) continue;
        if (j == 3) { acc += (int64_t)((uint64_t)m[i] * k.k9); chain<CHAIN>(acc); }
        if (j == 6) { acc += (int64_t)((uint64_t)m[i] * k.k18); chain<CHAIN>(acc); }
        if (j == 7) { acc += (int64_t)(int32_t)m[i] * (int64_t)k.kn21; chain<CHAIN>(acc); }
        if (j == 8) { acc += (int64_t)((uint64_t)m[i] * k.k24); chain<CHAIN>(acc); }
    }
}

// Loose quotient digits (LQ).  A quotient digit only has to agree with its
// column modulo 2^29: digits 0..7 take the column's whole low 32 bits (no
// mask), and the column then drops those 32 bits, its carry being the
// (signed) high half times 8 (one multiply-add instead of a mask and a
// shift).  With p's digits taken non-negative,
//   p = -1 + 2^9 B^3 + 2^18 B^6 + (2^29 - 2^21) B^7 + (2^24 - 1) B^8,
// every reduction term is an unsigned multiply-add below 2^61, so a column
// (at most 9 products below 2^59, 4 terms, a carry below 2^35) stays below
// 2^62.7.  Digit 8 keeps its mask, so M = sum m_i 2^(29 i) < R (1 + 2^-26)
// and the result (a b + M p) / R < a b / R + p (1 + 2^-26): normal form
// (< 2p) when a b / R < p (1 - 2^-26), i.e. for operand bounds multiplying
// to at most 31.99 p^2 (exact digits allow 32 p^2).
struct red_consts_lq {
    uint32_t k9, k18, k7, k8, eight;
};

__device__ __forceinline__ red_consts_lq red_consts_lq_make() {
    red_consts_lq k{1u << 9, 1u << 18, (1u << 29) - (1u << 21), (1u << 24) - 1u, 8u};
    asm("" : "+s"(k.k9), "+s"(k.k18), "+s"(k.k7), "+s"(k.k8), "+s"(k.eight));
    return k;
}

template <bool CHAIN>
__device__ __forceinline__ void red_terms_lq(int64_t &acc, const uint32_t *m, int c, const red_consts_lq &k) {
#pragma unroll
    for (int i = 0; i < NL; ++i) {
        const int j = c - i;
        if (i >= c) continue;
        if (j == 3) { acc += (int64_t)((uint64_t)m[i] * k.k9); chain<CHAIN>(acc); }
        if (j == 6) { acc += (int64_t)((uint64_t)m[i] * k.k18); chain<CHAIN>(acc); }
        if (j == 7) { acc += (int64_t)((uint64_t)m[i] * k.k7); chain<CHAIN>(acc); }
        if (j == 8) { acc += (int64_t)((uint64_t)m[i] * k.k8); chain<CHAIN>(acc); }
    }
}

// The column step after column c's terms: quotient digit (c < NL) or result
// limb (c >= NL), then the carry into column c + 1.
template <bool LQ>
__device__ __forceinline__ void column_out(int64_t &acc, int c, uint32_t *m, fe &r, uint32_t eight) {
    if (LQ && c < NL - 1) {
        m[c] = (uint32_t)acc;
        acc = (int64_t)(int32_t)(acc >> 32) * (int64_t)(int32_t)eight;  // |column| < 2^63
        return;
    }
    if (c < NL)
        m[c] = (uint32_t)acc & LMASK;
    else
        r.v[c - NL] = (uint32_t)acc & LMASK;
    acc >>= LB;  // exact after m p clears the low bits; arithmetic shift
}

template <bool CHAIN, bool LQ = false>
__device__ __forceinline__ fe fe_mul_t(const fe &a, const fe &b) {
    const red_consts k = red_consts_make();
    const red_consts_lq kl = red_consts_lq_make();
    int64_t acc = 0;
    uint32_t m[NL];
    fe r;
#pragma unroll
    for (int c = 0; c < 2 * NL - 1; ++c) {
#pragma unroll
        for (int i = 0; i < NL; ++i) {
            const int j = c - i;
            if (j >= 0 && j < NL) { acc += (int64_t)((uint64_t)a.v[i] * b.v[j]); chain<CHAIN>(acc); }
        }
        if constexpr (LQ) red_terms_lq<CHAIN>(acc, m, c, kl);
        else red_terms<CHAIN>(acc, m, c, k);
        column_out<LQ>(acc, c, m, r, kl.eight);
    }
    r.v[NL - 1] = (uint32_t)acc;
    return r;
}

template <bool CHAIN, bool LQ = false>
__device__ __forceinline__ fe fe_sqr_t(const fe &a) {
    const red_consts k = red_consts_make();
    const red_consts_lq kl = red_consts_lq_make();
    uint32_t d[NL];
#pragma unroll
    for (int i = 0; i < NL; ++i) d[i] = a.v[i] << 1;
    int64_t acc = 0;
    uint32_t m[NL];
    fe r;
#pragma unroll
    for (int c = 0; c < 2 * NL - 1; ++c) {
#pragma unroll
        for (int i = 0; i < NL; ++i) {
            const int j = c - i;
            if (i < j && j < NL) { acc += (int64_t)((uint64_t)d[i] * a.v[j]); chain<CHAIN>(acc); }
        }
        if ((c & 1) == 0 && c / 2 < NL) { acc += (int64_t)((uint64_t)a.v[c / 2] * a.v[c / 2]); chain<CHAIN>(acc); }
        if constexpr (LQ) red_terms_lq<CHAIN>(acc, m, c, kl);
        else red_terms<CHAIN>(acc, m, c, k);
        column_out<LQ>(acc, c, m, r, kl.eight);
    }
    r.v[NL - 1] = (uint32_t)acc;
    return r;
}

// one-chain forms for the point formulas, split forms for serial chains
// ---------------------------------------------------------------------------
// Products that absorb an addition.  Above column 8 the column sums are the
// result's limbs (the division by R = 2^261 keeps them), so a value e added
// there appears in the output unreduced: the column algorithm returns the
// exact integer (a b + M p) / R + e.  Outputs are carry-only (limbs 0..7 in
// [0, 2^29), limb 8 the rest); each caller bounds the value.
// ---------------------------------------------------------------------------

// 2p - x as signed limbs (each in (-2^29, 2^30)), value in (0, 2p], for x normal
__device__ __forceinline__ fe fe_2p_minus(const fe &x) {
    fe e;
#pragma unroll
    for (int i = 0; i < NL; ++i) e.v[i] = TWO_P29.v[i] - x.v[i];
    return e;
}

// REDC(a b) + e for e as signed limbs (|e_i| < 2^31): with a b < 4 p^2 and
// e = 2p - x, the result is a b / R - x (mod p), carry-only, in (0, 4p)
template <bool CHAIN, bool LQ = false>
__device__ __forceinline__ fe fe_mul_plus_t(const fe &a, const fe &b, const fe &e) {
    const red_consts k = red_consts_make();
    const red_consts_lq kl = red_consts_lq_make();
    int64_t acc = 0;
    uint32_t m[NL];
    fe r;
#pragma unroll
    for (int c = 0; c < 2 * NL - 1; ++c) {
#pragma unroll
        for (int i = 0; i < NL; ++i) {
            const int j = c - i;
            if (j >= 0 && j < NL) { acc += (int64_t)((uint64_t)a.v[i] * b.v[j]); chain<CHAIN>(acc); }
        }
        if constexpr (LQ) red_terms_lq<CHAIN>(acc, m, c, kl);
        else red_terms<CHAIN>(acc, m, c, k);
        if (c >= NL) acc += (int64_t)(int32_t)e.v[c - NL];
        column_out<LQ>(acc, c, m, r, kl.eight);
    }
    r.v[NL - 1] = (uint32_t)acc + e.v[NL - 1];
    return r;
}

// fe_norm without its first carry pass, for a carry-only value below 2^260
__device__ __forceinline__ fe fe_fold(fe x) {
    const uint32_t h = x.v[8] >> 24;
    x.v[8] &= (1u << 24) - 1;
    x.v[0] += h;
    x.v[3] -= h << 9;
    x.v[6] -= h << 18;
    x.v[7] += h << 21;
    fe_carry(x);
    return x;
}

// (a b - 2^SH c d) / R (mod p) in normal form, with one reduction: the
// column sums take a_i b_j and (-c_i)(2^SH d_j) (signed multiply-adds), p R
// is added above column 8, and the result is folded into [0, 2p).  For SH =
// 1 with a's limbs < 2^30 (fe_x2 of a carry-only value), or SH = 0 with a
// carry-only, b carry-only, c and d normal: each part of a column is below
// 9 2^59 in magnitude, so partial sums stay within 2^62.2 (2^62.7 with loose
// quotient digits); a b < 32 p^2 and 2^SH c d < 8 p^2 give a b - 2^SH c d +
// p R > 0 and a reduced value in (0, 3p) before the fold (below 3p (1 +
// 2^-26) with loose digits: still carry-only below 2^260).
template <bool CHAIN, bool LQ = false, int SH = 1>
__device__ __forceinline__ fe fe_mul_sub2_t(const fe &a, const fe &b, const fe &c, const fe &d) {
    const red_consts k = red_consts_make();
    const red_consts_lq kl = red_consts_lq_make();
    int32_t nc[NL];
    int32_t d2[NL];
#pragma unroll
    for (int i = 0; i < NL; ++i) {
        nc[i] = -(int32_t)c.v[i];
        d2[i] = (int32_t)(d.v[i] << SH);
    }
    int64_t acc = 0;
    uint32_t m[NL];
    fe r;
#pragma unroll
    for (int col = 0; col < 2 * NL - 1; ++col) {
#pragma unroll
        for (int i = 0; i < NL; ++i) {
            const int j = col - i;
            if (j >= 0 && j < NL) {
                acc += (int64_t)((uint64_t)a.v[i] * b.v[j]);
                chain<CHAIN>(acc);
                acc += (int64_t)nc[i] * (int64_t)d2[j];
                chain<CHAIN>(acc);
            }
        }
        if constexpr (LQ) red_terms_lq<CHAIN>(acc, m, col, kl);
        else red_terms<CHAIN>(acc, m, col, k);
        if (col >= NL) acc += (int64_t)P29.v[col - NL];
        column_out<LQ>(acc, col, m, r, kl.eight);
    }
    r.v[NL - 1] = (uint32_t)acc + P29.v[NL - 1];
    return fe_fold(r);
}

// (a b - c d) / R (mod p): fe_mul_sub2_t without the factor 2
template <bool CHAIN, bool LQ = false>
__device__ __forceinline__ fe fe_mul_sub_t(const fe &a, const fe &b, const fe &c, const fe &d) {
    return fe_mul_sub2_t<CHAIN, LQ, 0>(a, b, c, d);
}

__device__ __forceinline__ fe fe_mul(const fe &a, const fe &b) { return fe_mul_t<true>(a, b); }
__device__ __forceinline__ fe fe_sqr(const fe &a) { return fe_sqr_t<true>(a); }
__device__ __forceinline__ fe fe_mul_ilp(const fe &a, const fe &b) { return fe_mul_t<false>(a, b); }
__device__ __forceinline__ fe fe_sqr_ilp(const fe &a) { return fe_sqr_t<false>(a); }

// n squarings with loose quotient digits (a normal: every operand pair is
// below 4 p^2)
__device__ __forceinline__ fe fe_sqr_n(fe a, int n) {
    for (int i = 0; i < n; ++i) a = fe_sqr_t<false, true>(a);
    return a;
}

// ---------------------------------------------------------------------------
// Conversions between canonical 8 x 32-bit words and Montgomery limbs
// ---------------------------------------------------------------------------
// canonical words (any value < 2^256) -> limbs of the same integer
__device__ __forceinline__ fe fe_from_words(const uint32_t w[8]) {
    fe r;
#pragma unroll
    for (int i = 0; i < NL; ++i) {
        const int bit = LB * i;
        const int k = bit / 32, s = bit % 32;
        uint64_t x = w[k];
        if (k + 1 < 8) x |= (uint64_t)w[k + 1] << 32;
        r.v[i] = (uint32_t)(x >> s) & LMASK;
    }
    return r;
}

// fully reduced value (< p) of a normal-form element, as limbs
__device__ __forceinline__ fe fe_canon(const fe &a) {
    fe t;
#pragma unroll
    for (int i = 0; i < NL; ++i) t.v[i] = a.v[i] - P29.v[i];
    fe_carry(t);
    const bool neg = (int32_t)t.v[NL - 1] < 0;  // a < p: keep a
    return fe_select(neg, t, a);
}

// limbs of a value < 2^256 -> eight 32-bit words
__device__ __forceinline__ void fe_to_words(const fe &a, uint32_t w[8]) {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const int bit = 32 * k;
        const int i = bit / LB, s = bit % LB;
        uint64_t x = (uint64_t)a.v[i] >> s;
        if (i + 1 < NL) x |= (uint64_t)a.v[i + 1] << (LB - s);
        if (i + 2 < NL && 2 * LB - s < 32) x |= (uint64_t)a.v[i + 2] << (2 * LB - s);
        w[k] = (uint32_t)x;
    }
}

__device__ __forceinline__ fe fe_to_mont(const fe &a) { return fe_mul_ilp(a, fe_from29(R2_29)); }

// Montgomery limbs -> canonical integer limbs in [0, p)
__device__ __forceinline__ fe fe_from_mont(const fe &a) { return fe_canon(fe_mul_ilp(a, fe_from29(ONE29))); }

// a^(p-2) = a^-1 for a != 0 (0 maps to 0), by Fermat's little theorem.
// p - 2 in 32-bit words from the top: ffffffff 00000001 00000000 00000000
// 00000000 ffffffff ffffffff fffffffd.  x_k below is a^(2^k - 1); the chain
// uses 255 squarings and 12 products, all with loose quotient digits (for a
// below 4p every operand pair is below 16 p^2).  Kept as the cross-check of
// fe_inv.
__device__ __noinline__ fe fe_inv_fermat(const fe &a) {
    fe x1 = a;
    fe x2 = fe_mul_t<false, true>(fe_sqr_t<false, true>(x1), x1);
    fe x3 = fe_mul_t<false, true>(fe_sqr_t<false, true>(x2), x1);
    fe x6 = fe_mul_t<false, true>(fe_sqr_n(x3, 3), x3);
    fe x12 = fe_mul_t<false, true>(fe_sqr_n(x6, 6), x6);
    fe x15 = fe_mul_t<false, true>(fe_sqr_n(x12, 3), x3);
    fe x30 = fe_mul_t<false, true>(fe_sqr_n(x15, 15), x15);
    fe x32 = fe_mul_t<false, true>(fe_sqr_n(x30, 2), x2);
    fe r = x32;                               // word 7: 32 ones
    r = fe_mul_t<false, true>(fe_sqr_n(r, 32), x1);          // word 6: 0x00000001
    r = fe_mul_t<false, true>(fe_sqr_n(r, 128), x32);        // words 5..3 zero, word 2: 32 ones
    r = fe_mul_t<false, true>(fe_sqr_n(r, 32), x32);         // word 1: 32 ones
    r = fe_mul_t<false, true>(fe_sqr_n(r, 30), x30);         // word 0: 30 ones,
    r = fe_mul_t<false, true>(fe_sqr_n(r, 2), x1);           //         then bits 0 1
    return r;
}

// ---------------------------------------------------------------------------
// Inversion by divsteps (Bernstein and Yang, "Fast constant-time gcd
// computation and modular inversion", 2019).  A divstep maps (delta, f, g),
// f odd, to (1 - delta, g, (g - f) / 2) if delta > 0 and g is odd, to
// (1 + delta, f, (g + f) / 2) if g is odd otherwise, and to (1 + delta, f,
// g / 2) if g is even.  From (1, p, x) with 0 <= x < p < 2^256, g reaches 0
// (and f = +-1 when x != 0) within 742 divsteps (their bound
// floor((49 d + 80) / 17) for d = 256 bits); this runs 25 batches of 30 =
// 750.  The decisions of 30 divsteps depend only on the low 30 bits of f and
// g, so a batch runs on the low 32 bits and records its effect as an integer
// matrix (u v; q r): 2^30 (f', g') = (u f + v g, q f + r g), with |u| + |v|
// and |q| + |r| at most 2^30; the matrix is then applied to the full f, g
// and to d, e, which keep d x = f and e x = g (mod p): d' = (u d + v e) /
// 2^30 (mod p), exact after adding the multiple md p (md < 2^30) that
// clears the low 30 bits.  At the end d x = +-1, so x^-1 = +-d.
// State: signed radix-2^30 values, limbs 0..7 in [0, 2^30), limb 8 signed.
// |d|, |e| <= p throughout: |u d + v e| / 2^30 <= max(|d|, |e|) and md p /
// 2^30 < p, and a step of p toward zero after each batch keeps the bound.
// About 24 K VALU instructions per inversion against about 32 K for the
// Fermat chain, with a shorter critical path (no 64-bit multiply-add
// chains in the divsteps).
// ---------------------------------------------------------------------------
struct s30 {
    int32_t v[NL];
};
constexpr int32_t M30 = (1 << 30) - 1;

// 30 divsteps on the low 32 bits of f and g; d2 = 2 delta.
__device__ __forceinline__ void divsteps30(int32_t &d2, uint32_t f, uint32_t g, int32_t &u, int32_t &v, int32_t &q,
                                           int32_t &r) {
    u = 1;
    v = 0;
    q = 0;
    r = 1;
#pragma unroll
    for (int i = 0; i < 30; ++i) {
        const bool odd = (g & 1u) != 0;
        const bool swap = odd && d2 > 0;
        // swap: (f, g, u, v, q, r, delta) <- (g, -f, q, r, -u, -v, -delta),
        // after which every odd g is handled as g + f
        const uint32_t f1 = swap ? g : f, g1 = swap ? 0u - f : g;
        const int32_t u1 = swap ? q : u, v1 = swap ? r : v, q1 = swap ? -u : q, r1 = swap ? -v : r;
        d2 = (swap ? -d2 : d2) + 2;
        f = f1;
        g = (g1 + (odd ? f1 : 0u)) >> 1;
        q = q1 + (odd ? u1 : 0);
        r = r1 + (odd ? v1 : 0);
        u = (int32_t)((uint32_t)u1 << 1);
        v = (int32_t)((uint32_t)v1 << 1);
    }
}

// acc + x y for 32-bit signed x, y: one signed multiply-add.  The empty
// register constraints hide what the compiler knows of y (a masked limb is
// non-negative, which would turn the signed product into a widened one)
// and keep the sum one chain.
__device__ __forceinline__ int64_t smad(int64_t acc, int32_t x, int32_t y) {
    asm("" : "+v"(y));
    acc += (int64_t)x * (int64_t)y;
    asm("" : "+v"(acc));
    return acc;
}

// (u a + v b) / 2^30, exact (the caller's matrix makes the low 30 bits zero)
__device__ __forceinline__ s30 s30_row(int32_t u, int32_t v, const s30 &a, const s30 &b) {
    int64_t acc = smad(smad(0, u, a.v[0]), v, b.v[0]);
    acc >>= 30;
    s30 o;
#pragma unroll
    for (int i = 1; i < NL; ++i) {
        acc = smad(smad(acc, u, a.v[i]), v, b.v[i]);
        o.v[i - 1] = (int32_t)(acc & M30);
        acc >>= 30;
    }
    o.v[NL - 1] = (int32_t)acc;
    return o;
}

// limbs 0..7 back into [0, 2^30)
__device__ __forceinline__ void s30_carry(s30 &x) {
#pragma unroll
    for (int i = 0; i < NL - 1; ++i) {
        const int32_t c = x.v[i] >> 30;
        x.v[i] &= M30;
        x.v[i + 1] += c;
    }
}

// (u d + v e) / 2^30 (mod p), then a step of p toward zero.  p in signed
// radix-2^30 digits: -1 + 2^6 B^3 + 2^12 B^6 - 2^14 B^7 + 2^16 B^8 (B = 2^30),
// so p = -1 (mod 2^30) and md = (u d + v e) mod 2^30 clears the low bits.
__device__ __forceinline__ s30 s30_row_mod(int32_t u, int32_t v, const s30 &d, const s30 &e) {
    int64_t acc = smad(smad(0, u, d.v[0]), v, e.v[0]);
    const int64_t md = acc & M30;
    acc = (acc - md) >> 30;
    s30 o;
#pragma unroll
    for (int i = 1; i < NL; ++i) {
        acc = smad(smad(acc, u, d.v[i]), v, e.v[i]);
        if (i == 3) acc += md << 6;
        if (i == 6) acc += md << 12;
        if (i == 7) acc -= md << 14;
        if (i == 8) acc += md << 16;
        o.v[i - 1] = (int32_t)(acc & M30);
        acc >>= 30;
    }
    o.v[NL - 1] = (int32_t)acc;
    const int32_t sg = o.v[NL - 1] < 0 ? 1 : -1;  // + p below zero, - p from zero up
    o.v[0] -= sg;
    o.v[3] += sg * (1 << 6);
    o.v[6] += sg * (1 << 12);
    o.v[7] -= sg * (1 << 14);
    o.v[8] += sg * (1 << 16);
    s30_carry(o);
    return o;
}

// limbs of a value in [0, 2^256) -> radix 2^30
__device__ __forceinline__ s30 s30_from_fe(const fe &a) {
    s30 o;
#pragma unroll
    for (int j = 0; j < NL; ++j) {
        const int bit = 30 * j, i = bit / LB, sh = bit % LB;
        uint64_t x = (uint64_t)a.v[i] >> sh;
        if (i + 1 < NL) x |= (uint64_t)a.v[i + 1] << (LB - sh);
        if (i + 2 < NL) x |= (uint64_t)a.v[i + 2] << (2 * LB - sh);
        o.v[j] = (int32_t)(x & M30);
    }
    return o;
}

// a value in [0, 2^261) in radix 2^30 (limbs 0..7 in [0, 2^30)) -> 29-bit limbs
__device__ __forceinline__ fe fe_from_s30(const s30 &a) {
    fe o;
#pragma unroll
    for (int i = 0; i < NL; ++i) {
        const int bit = LB * i, j = bit / 30, sh = bit % 30;
        uint64_t x = (uint64_t)(uint32_t)a.v[j] >> sh;
        if (j + 1 < NL) x |= (uint64_t)(uint32_t)a.v[j + 1] << (30 - sh);
        o.v[i] = (uint32_t)(x & LMASK);
    }
    return o;
}

// x^-1 in Montgomery form for a = x R below 4p (0 maps to 0): the divsteps
// invert the integer a, and one product with R^3 turns a^-1 = x^-1 R^-1 into
// x^-1 R.
__device__ __noinline__ fe fe_inv(const fe &a) {
    s30 f = {{-1, 0, 0, 1 << 6, 0, 0, 1 << 12, -(1 << 14), 1 << 16}};
    s30_carry(f);
    s30 g = s30_from_fe(fe_canon(fe_norm(a)));
    s30 d = {{0, 0, 0, 0, 0, 0, 0, 0, 0}}, e = {{1, 0, 0, 0, 0, 0, 0, 0, 0}};
    int32_t d2 = 2;
#pragma unroll 1
    for (int b = 0; b < 25; ++b) {
        int32_t u, v, q, r;
        divsteps30(d2, (uint32_t)f.v[0] | ((uint32_t)f.v[1] << 30), (uint32_t)g.v[0] | ((uint32_t)g.v[1] << 30), u,
                   v, q, r);
        const s30 f1 = s30_row(u, v, f, g), g1 = s30_row(q, r, f, g);
        const s30 d1 = s30_row_mod(u, v, d, e), e1 = s30_row_mod(q, r, d, e);
        f = f1;
        g = g1;
        d = d1;
        e = e1;
    }
    // f = +-1 (f = p, d = 0 for a = 0): x^-1 = sign(f) d, brought into [0, p]
    const bool fneg = f.v[NL - 1] < 0;
#pragma unroll
    for (int i = 0; i < NL; ++i) d.v[i] = fneg ? -d.v[i] : d.v[i];
    s30_carry(d);
    const bool dneg = d.v[NL - 1] < 0;
    d.v[0] -= dneg ? 1 : 0;
    d.v[3] += dneg ? 1 << 6 : 0;
    d.v[6] += dneg ? 1 << 12 : 0;
    d.v[7] -= dneg ? 1 << 14 : 0;
    d.v[8] += dneg ? 1 << 16 : 0;
    s30_carry(d);
    return fe_mul_t<false, true>(fe_from_s30(d), fe_from29(R3_29));
}

}  // namespace pcmm
