// normalize_dev.hpp -- device side of the batched Jacobian -> affine conversion.
//
// Montgomery's simultaneous-inversion trick: one thread walks its batch of
// points forward keeping the running product of the nonzero Z values (and
// storing each prefix), inverts the total once (fe_inv, by divsteps), then
// walks backward: Z_j^-1 = inv * prefix_{j-1}, inv <- inv * Z_j.  Per point
// that is 3 multiplications plus the affine conversion (x = X Z^-2,
// y = Y Z^-3), with one inversion per batch.  Z = 0 (the identity) maps to
// (0, 0) and is skipped in the product.
#pragma once
#include "common.hpp"

namespace pcmm {

// Thread t of T handles elements e = t + j * T (j < per_thread); both points
// of an element are handled by the same thread, and an element is written
// only after all of its inputs were read, so `out` may alias `in`.  Prefix
// slot s of thread t lives at column t + s * T of `prefix` (NL words).
template <bool IN_MONT, bool OUT_MONT>
__device__ __forceinline__ void normalize_points(const uint32_t *in, int64_t ld_in, uint32_t *out, int64_t ld_out,
                                                 int64_t n_elem, int npts, uint32_t *__restrict__ prefix,
                                                 int64_t ld_pre, int per_thread, int64_t t, int64_t T) {
    fe acc = fe_one_mont();
    int slot = 0;
    for (int j = 0; j < per_thread; ++j) {
        int64_t e = t + (int64_t)j * T;
        if (e >= n_elem) break;
        for (int pt = 0; pt < npts; ++pt, ++slot) {
            fe z = IN_MONT ? soa_load_m(in, ld_in, pt * 3 + 2, e) : soa_load_mont(in, ld_in, pt * 3 + 2, e);
            soa_store_m(prefix, ld_pre, 0, t + (int64_t)slot * T, acc);
            if (!fe_is_zero(z)) acc = fe_mul_ilp(acc, z);
        }
    }
    if (slot == 0) return;
    fe inv = fe_inv(acc);
    for (int j = per_thread - 1; j >= 0; --j) {
        int64_t e = t + (int64_t)j * T;
        if (e >= n_elem) continue;
        // npts is 1 or 2; the fixed-size loops keep P and A in registers
        jpt P[2];
        apt A[2];
#pragma unroll
        for (int pt = 0; pt < 2; ++pt) {
            if (pt < npts) P[pt] = IN_MONT ? load_jac_m(in, ld_in, pt, e) : load_jac(in, ld_in, pt, e);
        }
#pragma unroll
        for (int pt = 1; pt >= 0; --pt) {
            if (pt >= npts) continue;
            --slot;
            bool inf = fe_is_zero(P[pt].Z);
            fe pre = soa_load_m(prefix, ld_pre, 0, t + (int64_t)slot * T);
            fe zinv = fe_mul_ilp(inv, pre);
            if (!inf) inv = fe_mul_ilp(inv, P[pt].Z);
            A[pt] = jpt_to_affine_with(P[pt], zinv);
            if (inf) {
                A[pt].x = fe_zero();
                A[pt].y = fe_zero();
            }
        }
#pragma unroll
        for (int pt = 0; pt < 2; ++pt) {
            if (pt >= npts) continue;
            if (OUT_MONT) {
                store_aff_m(out, ld_out, pt, e, A[pt]);
            } else {
                store_affine(out, ld_out, pt, e, A[pt]);
            }
        }
    }
}

}  // namespace pcmm
