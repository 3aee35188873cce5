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
// Structure-of-arrays point matrices: limb w of coordinate c of point pt of
// element e lives at d[((pt * form + c) * 8 + w) * ld + e].
// ---------------------------------------------------------------------------
struct soa {
    uint32_t *d;
    int64_t ld;
    int32_t form;  // coordinates per point (2 affine, 3 Jacobian)
};

__device__ __forceinline__ fe soa_load_raw(const uint32_t *__restrict__ d, int64_t ld, int plane,
                                           int64_t e) {
    fe r;
#pragma unroll
    for (int w = 0; w < 8; ++w) r.v[w] = d[(int64_t)(plane * 8 + w) * ld + e];
    return r;
}

__device__ __forceinline__ void soa_store_raw(uint32_t *__restrict__ d, int64_t ld, int plane,
                                              int64_t e, const fe &x) {
#pragma unroll
    for (int w = 0; w < 8; ++w) d[(int64_t)(plane * 8 + w) * ld + e] = x.v[w];
}

// canonical limbs -> Montgomery; values >= p are reduced by the multiplication
__device__ __forceinline__ fe soa_load_mont(const uint32_t *__restrict__ d, int64_t ld, int plane,
                                            int64_t e) {
    return fe_to_mont(soa_load_raw(d, ld, plane, e));
}

__device__ __forceinline__ void soa_store_canon(uint32_t *__restrict__ d, int64_t ld, int plane,
                                                int64_t e, const fe &x) {
    soa_store_raw(d, ld, plane, e, fe_from_mont(x));
}

// affine point `pt` of element e (form must be 2)
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

// Montgomery-form Jacobian planes (internal workspaces keep Montgomery form
// to skip conversions between kernels)
__device__ __forceinline__ jpt load_jac_m(const uint32_t *__restrict__ d, int64_t ld, int pt,
                                          int64_t e) {
    jpt j;
    j.X = soa_load_raw(d, ld, pt * 3 + 0, e);
    j.Y = soa_load_raw(d, ld, pt * 3 + 1, e);
    j.Z = soa_load_raw(d, ld, pt * 3 + 2, e);
    return j;
}

__device__ __forceinline__ void store_jac_m(uint32_t *__restrict__ d, int64_t ld, int pt, int64_t e,
                                            const jpt &j) {
    soa_store_raw(d, ld, pt * 3 + 0, e, j.X);
    soa_store_raw(d, ld, pt * 3 + 1, e, j.Y);
    soa_store_raw(d, ld, pt * 3 + 2, e, j.Z);
}

// Alg. 1 (Montgomery ladder) over the low t bits of k, most significant
// first: R0 <- inf, R1 <- P; per bit b: R_{1-b} <- R0 + R1, R_b <- 2 R_b.
// Branch-free per lane (lanes may hold different k; t is uniform).
__device__ __forceinline__ jpt ladder_small(uint32_t k, int t, const apt &P) {
    jpt R0 = jpt_infinity();
    jpt R1 = jpt_from_affine(P);
    for (int i = t - 1; i >= 0; --i) {
        bool b = (k >> i) & 1u;
        jpt S = jpt_add(R1, R0);
        jpt D = jpt_dbl(jpt_select(b, R0, R1));
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
