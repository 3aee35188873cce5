// common.hpp -- shared host/device helpers of libpcmm (internal).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <cmath>

#include "../../include/pcmm.h"
#include "ec.hpp"

namespace pcmm {

// ---------------------------------------------------------------------------
// Structure-of-arrays point matrices at the library boundary: limb w (32-bit
// word, canonical integer) of coordinate c of point pt of element e lives at
// d[((pt * form + c) * 8 + w) * ld + e].
// Internal workspaces keep Montgomery values in the same layout but with NL
// (= 9) 29-bit limbs per coordinate: d[((pt * form + c) * NL + w) * ld + e].
// ---------------------------------------------------------------------------
__device__ __forceinline__ fe fe_from_const(const fe_const &c) { return fe_from29(c_to29(c)); }

__device__ __forceinline__ bool fe_raw_eq(const fe &a, const fe &b) {
    uint32_t x = 0;
#pragma unroll
    for (int i = 0; i < NL; ++i) x |= a.v[i] ^ b.v[i];
    return x == 0;
}

// canonical words -> Montgomery limbs; values >= p are reduced
__device__ __forceinline__ fe soa_load_mont(const uint32_t *__restrict__ d, int64_t ld, int plane,
                                            int64_t e) {
    uint32_t w[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) w[k] = d[(int64_t)(plane * 8 + k) * ld + e];
    return fe_to_mont(fe_from_words(w));
}

// Montgomery limbs -> canonical words
__device__ __forceinline__ void soa_store_canon(uint32_t *__restrict__ d, int64_t ld, int plane,
                                                int64_t e, const fe &x) {
    uint32_t w[8];
    fe_to_words(fe_from_mont(x), w);
#pragma unroll
    for (int k = 0; k < 8; ++k) d[(int64_t)(plane * 8 + k) * ld + e] = w[k];
}

// internal Montgomery limbs
__device__ __forceinline__ fe soa_load_m(const uint32_t *__restrict__ d, int64_t ld, int plane, int64_t e) {
    fe r;
#pragma unroll
    for (int w = 0; w < NL; ++w) r.v[w] = d[(int64_t)(plane * NL + w) * ld + e];
    return r;
}

__device__ __forceinline__ void soa_store_m(uint32_t *__restrict__ d, int64_t ld, int plane, int64_t e,
                                            const fe &x) {
#pragma unroll
    for (int w = 0; w < NL; ++w) d[(int64_t)(plane * NL + w) * ld + e] = x.v[w];
}

// affine point `pt` of element e (form must be 2), canonical boundary layout
__device__ __forceinline__ apt load_affine(const uint32_t *__restrict__ d, int64_t ld, int pt,
                                           int64_t e) {
    apt a;
    a.x = soa_load_mont(d, ld, pt * 2 + 0, e);
    a.y = soa_load_mont(d, ld, pt * 2 + 1, e);
    return a;
}

__device__ __forceinline__ void store_affine(uint32_t *__restrict__ d, int64_t ld, int pt,
                                             int64_t e, const apt &a) {
    soa_store_canon(d, ld, pt * 2 + 0, e, a.x);
    soa_store_canon(d, ld, pt * 2 + 1, e, a.y);
}

__device__ __forceinline__ jpt load_jac(const uint32_t *__restrict__ d, int64_t ld, int pt,
                                        int64_t e) {
    jpt j;
    j.X = soa_load_mont(d, ld, pt * 3 + 0, e);
    j.Y = soa_load_mont(d, ld, pt * 3 + 1, e);
    j.Z = soa_load_mont(d, ld, pt * 3 + 2, e);
    return j;
}

__device__ __forceinline__ void store_jac(uint32_t *__restrict__ d, int64_t ld, int pt, int64_t e,
                                          const jpt &j) {
    soa_store_canon(d, ld, pt * 3 + 0, e, j.X);
    soa_store_canon(d, ld, pt * 3 + 1, e, j.Y);
    soa_store_canon(d, ld, pt * 3 + 2, e, j.Z);
}

// internal Montgomery Jacobian / affine points
__device__ __forceinline__ jpt load_jac_m(const uint32_t *__restrict__ d, int64_t ld, int pt,
                                          int64_t e) {
    jpt j;
    j.X = soa_load_m(d, ld, pt * 3 + 0, e);
    j.Y = soa_load_m(d, ld, pt * 3 + 1, e);
    j.Z = soa_load_m(d, ld, pt * 3 + 2, e);
    return j;
}

__device__ __forceinline__ void store_jac_m(uint32_t *__restrict__ d, int64_t ld, int pt, int64_t e,
                                            const jpt &j) {
    soa_store_m(d, ld, pt * 3 + 0, e, j.X);
    soa_store_m(d, ld, pt * 3 + 1, e, j.Y);
    soa_store_m(d, ld, pt * 3 + 2, e, j.Z);
}

__device__ __forceinline__ apt load_aff_m(const uint32_t *__restrict__ d, int64_t ld, int pt, int64_t e) {
    apt a;
    a.x = soa_load_m(d, ld, pt * 2 + 0, e);
    a.y = soa_load_m(d, ld, pt * 2 + 1, e);
    return a;
}

__device__ __forceinline__ void store_aff_m(uint32_t *__restrict__ d, int64_t ld, int pt, int64_t e,
                                            const apt &a) {
    soa_store_m(d, ld, pt * 2 + 0, e, a.x);
    soa_store_m(d, ld, pt * 2 + 1, e, a.y);
}

// words per internal (Montgomery) Jacobian matrix of two points per element
constexpr int JAC2_PLANES = 2 * 3 * NL;

// Alg. 1 (Montgomery ladder) over the low t bits of k, most significant
// first: R0 <- inf, R1 <- P; per bit b: R_{1-b} <- R0 + R1, R_b <- 2 R_b.
// Branch-free per lane (lanes may hold different k; t is uniform).
template <bool CHAIN = true>
__device__ __forceinline__ jpt ladder_small(uint32_t k, int t, const apt &P) {
    jpt R0 = jpt_infinity();
    jpt R1 = jpt_from_affine(P);
    for (int i = t - 1; i >= 0; --i) {
        bool b = (k >> i) & 1u;
        jpt S = jpt_add<CHAIN>(R1, R0);
        jpt D = jpt_dbl<CHAIN>(jpt_select(b, R0, R1));
        R0 = jpt_select(b, D, S);
        R1 = jpt_select(b, S, D);
    }
    return R0;
}

}  // namespace pcmm

#define PCMM_HIP_TRY(expr)                                   \
    do {                                                      \
        hipError_t _e = (expr);                               \
        if (_e != hipSuccess) return PCMM_EDEVICE;            \
    } while (0)

#define PCMM_LAUNCH_CHECK()                                   \
    do {                                                      \
        hipError_t _e = hipGetLastError();                    \
        if (_e != hipSuccess) return PCMM_EDEVICE;            \
    } while (0)
