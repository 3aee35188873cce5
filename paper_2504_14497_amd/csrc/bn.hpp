// bn.hpp -- arithmetic mod n^2 for Paillier ciphertexts, one residue per
// wavefront (device side, internal).
//
// The Paillier extension (Sec. "Extension to Paillier Encryption") replaces
// point addition by multiplication mod n^2 and scalar multiplication by
// exponentiation (Alg. 4).  For a 3072-bit n, a residue mod n^2 has 6144
// bits: far too many for one lane, so a wavefront of 64 lanes holds one
// residue, lane L owning limbs 4L .. 4L + 3 of 29 bits each (256 limbs,
// 7424 bits; 212 of them carry a residue below 2^6148).  All 64 lanes of a wavefront call these functions together
// with the same modulus; values and exponents are uniform per wavefront.
//
// Montgomery multiplication (operand scanning, the reduction interleaved):
// for i = 0 .. K-1, T <- (T + a_i b + q N) / 2^29 with q = -T N^-1 mod 2^29,
// R = 2^(29 K), K = 212.  Every limb position of T is a 64-bit accumulator
// that gains two products (each below 2^58 + 2^31 for operand limbs
// <= 2^29 + 1) per iteration.  The division by 2^29 moves every position
// down by one: within a lane that is a renaming of the 4 registers over 4
// unrolled iterations; across lanes only the low 29 bits of each lane's
// lowest position move (one 32-bit DPP move), its high part joining the
// lane's next position.  So every register is split once per 4 iterations
// and never holds more than about 8 products (below 2^62).  Three carry
// rounds then leave limbs <= 2^29 + 1.
// Since R >= 4 N, inputs below 2N give an output below 2N ("lazy" form, no
// final subtraction between products); only the conversion out of
// Montgomery form reduces fully, with carries and the borrow of the final
// subtraction resolved across lanes by wavefront ballots.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pcmm {

constexpr int BN_LB = 29;
constexpr uint32_t BN_MASK = (1u << BN_LB) - 1;
constexpr int BN_W = 4;           // limbs per lane
constexpr int BN_LIMBS = 256;     // limbs per residue (64 lanes)
constexpr int BN_K = 212;         // Montgomery iterations: R = 2^(29 * 212) = 2^6148
constexpr int BN_WORDS = 192;     // 32-bit words of a residue mod n^2
constexpr int BN_NWORDS = 96;     // 32-bit words of n

// this lane's four limbs of a residue
struct bn {
    uint32_t v[BN_W];
};

__device__ __forceinline__ int bn_lane() { return (int)(threadIdx.x & 63); }

// One-lane moves across the whole wavefront as DPP moves: wave_shl1 (lane L
// reads lane L + 1) and wave_shr1 (lane L reads lane L - 1); with bound_ctrl
// the lane without a source (63, resp. 0) reads zero.
constexpr int DPP_WAVE_SHL1 = 0x130;
constexpr int DPP_WAVE_SHR1 = 0x138;

__device__ __forceinline__ uint32_t lane_from_above(uint32_t x) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, DPP_WAVE_SHL1, 0xF, 0xF, true);
}

__device__ __forceinline__ uint64_t lane_from_below(uint64_t x) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)x, DPP_WAVE_SHR1, 0xF, 0xF, true);
    const uint32_t hi =
        (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(x >> 32), DPP_WAVE_SHR1, 0xF, 0xF, true);
    return (uint64_t)hi << 32 | lo;
}

__device__ __forceinline__ bn bn_load(const uint32_t *__restrict__ p) {
    const uint4 x = ((const uint4 *)p)[bn_lane()];
    return bn{{x.x, x.y, x.z, x.w}};
}

__device__ __forceinline__ void bn_store(uint32_t *__restrict__ p, const bn &a) {
    ((uint4 *)p)[bn_lane()] = make_uint4(a.v[0], a.v[1], a.v[2], a.v[3]);
}

__device__ __forceinline__ bn bn_select(bool c, const bn &a, const bn &b) {
    bn r;
#pragma unroll
    for (int t = 0; t < BN_W; ++t) r.v[t] = c ? b.v[t] : a.v[t];
    return r;
}

// Montgomery product a b R^-1 (mod N) for a, b < 2N with limbs <= 2^29 + 1;
// the result is below 2N with limbs <= 2^29 + 1.  n0 = -N^-1 mod 2^32.
__device__ __forceinline__ bn bn_mont(const bn &a, const bn &b, const bn &N, uint32_t n0) {
    uint64_t acc[BN_W] = {0, 0, 0, 0};
    for (int s = 0; s < BN_K / BN_W; ++s) {
#pragma unroll
        for (int w = 0; w < BN_W; ++w) {
            // limb 4s + w of a; position t of T is register (t + w) mod 4
            const uint32_t x = (uint32_t)__builtin_amdgcn_readlane((int)a.v[w], s);
#pragma unroll
            for (int t = 0; t < BN_W; ++t) acc[(t + w) & 3] += (uint64_t)x * b.v[t];
            const uint32_t t0 = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)acc[w], 0);
            const uint32_t q = (t0 * n0) & BN_MASK;
#pragma unroll
            for (int t = 0; t < BN_W; ++t) acc[(t + w) & 3] += (uint64_t)q * N.v[t];
            // position 0 (lane 0) is now divisible by 2^29.  Every lane
            // splits its lowest register: the part above 2^29 joins the
            // lane's next position, the low 29 bits move one lane down (as
            // the lane below's top position after the division by 2^29);
            // lane 0's low part is zero and drops out.
            acc[(w + 1) & 3] += acc[w] >> BN_LB;
            acc[w] = lane_from_above((uint32_t)acc[w] & BN_MASK);
        }
    }
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        uint64_t c[BN_W];
#pragma unroll
        for (int t = 0; t < BN_W; ++t) {
            c[t] = acc[t] >> BN_LB;
            acc[t] &= BN_MASK;
        }
        acc[0] += lane_from_below(c[BN_W - 1]);
#pragma unroll
        for (int t = 1; t < BN_W; ++t) acc[t] += c[t - 1];
    }
    bn out;
#pragma unroll
    for (int t = 0; t < BN_W; ++t) out.v[t] = (uint32_t)acc[t];
    return out;
}

// Carry-in of every lane from per-lane generate / propagate flags: bit L of
// ((G | P) + G) ^ (G | P) ^ G; *out receives the carry out of lane 63.
__device__ __forceinline__ bool bn_lookahead(bool gen, bool prop, bool *out) {
    const uint64_t G = __ballot(gen);
    const uint64_t X = G | __ballot(prop && !gen);
    const uint64_t S = X + G;
    *out = S < X;
    return ((S ^ X ^ G) >> bn_lane()) & 1;
}

// exact limbs (< 2^29) of a value with limbs <= 2^29 + 1 (below 2^7424)
__device__ __forceinline__ bn bn_carry_exact(const bn &x) {
    bn s0, s1;
    uint32_t c0 = 0, c1 = 1;
#pragma unroll
    for (int t = 0; t < BN_W; ++t) {
        const uint32_t v0 = x.v[t] + c0, v1 = x.v[t] + c1;
        s0.v[t] = v0 & BN_MASK;
        s1.v[t] = v1 & BN_MASK;
        c0 = v0 >> BN_LB;
        c1 = v1 >> BN_LB;
    }
    bool top;
    const bool cin = bn_lookahead(c0 != 0, c1 != 0, &top);
    return bn_select(cin, s0, s1);
}

// x - N when x >= N, else x, for exact limbs; *ge reports x >= N (uniform)
__device__ __forceinline__ bn bn_sub_if_ge(const bn &x, const bn &N, bool *ge) {
    bn d0, d1;
    uint32_t b0 = 0, b1 = 1;
#pragma unroll
    for (int t = 0; t < BN_W; ++t) {
        const uint32_t v0 = x.v[t] - N.v[t] - b0, v1 = x.v[t] - N.v[t] - b1;
        d0.v[t] = v0 & BN_MASK;
        d1.v[t] = v1 & BN_MASK;
        b0 = v0 >> 31;  // limbs < 2^29: a negative difference has its top bit set
        b1 = v1 >> 31;
    }
    bool borrow_out;
    const bool bin = bn_lookahead(b0 != 0, b1 != 0, &borrow_out);
    *ge = !borrow_out;
    return borrow_out ? x : bn_select(bin, d0, d1);
}

// canonical residue (< N, exact limbs) of a value below 2N with limbs <= 2^29 + 1
__device__ __forceinline__ bn bn_canon(const bn &x, const bn &N) {
    bool ge;
    return bn_sub_if_ge(bn_carry_exact(x), N, &ge);
}

__device__ __forceinline__ bool bn_is_zero(const bn &x) {
    return __ballot((x.v[0] | x.v[1] | x.v[2] | x.v[3]) != 0) == 0;
}

// 32-bit words (little-endian, `nwords` of them, the rest zero) -> limbs.
// lds: 256 words of this wavefront's LDS.
__device__ __forceinline__ bn bn_from_words(const uint32_t *__restrict__ words, int nwords, uint32_t *lds) {
    const int lane = bn_lane();
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int i = lane + 64 * k;
        lds[i] = i < nwords ? words[i] : 0u;
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    bn r;
#pragma unroll
    for (int t = 0; t < BN_W; ++t) {
        const int bit = BN_LB * (BN_W * lane + t);
        const int k = bit >> 5, o = bit & 31;
        const uint64_t x = (uint64_t)(k < 256 ? lds[k] : 0u) | ((uint64_t)(k + 1 < 256 ? lds[k + 1] : 0u) << 32);
        r.v[t] = (uint32_t)(x >> o) & BN_MASK;
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    return r;
}

// exact limbs -> the low `nwords` 32-bit words
__device__ __forceinline__ void bn_to_words(const bn &a, uint32_t *__restrict__ words, int nwords, uint32_t *lds) {
    const int lane = bn_lane();
#pragma unroll
    for (int t = 0; t < BN_W; ++t) lds[BN_W * lane + t] = a.v[t];
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int wi = lane + 64 * k;
        if (wi < nwords) {
            const int bit = 32 * wi;
            const int i = bit / BN_LB, o = bit % BN_LB;
            uint64_t x = (uint64_t)lds[i];
            if (i + 1 < BN_LIMBS) x |= (uint64_t)lds[i + 1] << BN_LB;
            if (i + 2 < BN_LIMBS) x |= (uint64_t)lds[i + 2] << (2 * BN_LB);
            words[wi] = (uint32_t)(x >> o);
        }
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
}

// Alg. 4: g^k for the low t bits of a uniform exponent k (Montgomery form in
// and out; one = R mod N): r0 = 1, r1 = g; per bit b, most significant first:
// r_{1-b} = r0 r1, r_b = r_b^2.
__device__ __forceinline__ bn bn_pow_small(const bn &g, uint32_t k, int t, const bn &one, const bn &N, uint32_t n0) {
    bn r0 = one, r1 = g;
    for (int i = t - 1; i >= 0; --i) {
        if ((k >> i) & 1u) {
            r0 = bn_mont(r0, r1, N, n0);
            r1 = bn_mont(r1, r1, N, n0);
        } else {
            r1 = bn_mont(r0, r1, N, n0);
            r0 = bn_mont(r0, r0, N, n0);
        }
    }
    return r0;
}

// the same over a long exponent given as 32-bit words in memory (uniform)
__device__ __forceinline__ bn bn_pow_words(const bn &g, const uint32_t *__restrict__ kw, int nbits, const bn &one,
                                           const bn &N, uint32_t n0) {
    bn r0 = one, r1 = g;
    for (int i = nbits - 1; i >= 0; --i) {
        const uint32_t bit = (kw[i >> 5] >> (i & 31)) & 1u;
        if (bit) {
            r0 = bn_mont(r0, r1, N, n0);
            r1 = bn_mont(r1, r1, N, n0);
        } else {
            r1 = bn_mont(r0, r1, N, n0);
            r0 = bn_mont(r0, r0, N, n0);
        }
    }
    return r0;
}

}  // namespace pcmm
