// Host build of the library's device field and point arithmetic (fp.hpp,
// ec.hpp, common.hpp), one lane per call, through the stand-in
// <hip/hip_runtime.h> of this folder.  The tests load it with ctypes and
// compare it with Python integers and with the oracle's affine group law, on
// the CPU, with the undefined-behaviour sanitizer watching the 64-bit column
// sums.  Test infrastructure only.
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <cmath>

#include "hip/hip_runtime.h"
#include "../../paper_2504_14497_amd/csrc/common.hpp"

using namespace pcmm;

namespace {

// canonical 8-word little-endian value -> Montgomery limbs (values >= p reduced)
fe mont_of(const uint32_t *w) {
    uint32_t c[8];
    memcpy(c, w, sizeof c);
    return fe_to_mont(fe_from_words(c));
}

void canon_out(const fe &x, uint32_t *w) { fe_to_words(fe_from_mont(x), w); }

fe raw_of(const uint32_t *v) {
    fe r;
    for (int i = 0; i < NL; ++i) r.v[i] = v[i];
    return r;
}

// affine canonical (x 8 words, y 8 words; all zero = identity) -> Montgomery
apt aff_of(const uint32_t *p) {
    apt a;
    a.x = mont_of(p);
    a.y = mont_of(p + 8);
    return a;
}

// Jacobian with a chosen Z: (x z^2, y z^3, z); z = 0 gives the identity
jpt jac_of(const uint32_t *p, const uint32_t *z) {
    const apt a = aff_of(p);
    jpt j = jpt_from_affine(a);
    if (jpt_is_inf(j) || !z) return j;
    const fe zz = mont_of(z);
    if (fe_is_zero(zz)) return jpt_infinity();
    const fe z2 = fe_sqr(zz);
    j.X = fe_mul(a.x, z2);
    j.Y = fe_mul(a.y, fe_mul(z2, zz));
    j.Z = zz;
    return j;
}

// XYZZ with a chosen Z: (x z^2, y z^3, z^2, z^3); z = 0 or the affine
// identity give the identity (flag set)
xpt xyzz_of(const uint32_t *p, const uint32_t *z, bool &inf) {
    const apt a = aff_of(p);
    xpt r = xpt_infinity();
    inf = apt_is_inf(a);
    if (inf) return r;
    fe zz = fe_one_mont();
    if (z) {
        zz = mont_of(z);
        if (fe_is_zero(zz)) {
            inf = true;
            return r;
        }
    }
    r.ZZ = fe_sqr(zz);
    r.ZZZ = fe_mul(r.ZZ, zz);
    r.X = fe_mul(a.x, r.ZZ);
    r.Y = fe_mul(a.y, r.ZZZ);
    return r;
}

// canonical affine of a Jacobian point (identity -> zeros)
void aff_out(const jpt &P, uint32_t *out) {
    if (jpt_is_inf(P)) {
        memset(out, 0, 64);
        return;
    }
    const apt a = jpt_to_affine_with(P, fe_inv(P.Z));
    canon_out(a.x, out);
    canon_out(a.y, out + 8);
}

}  // namespace

extern "C" {

// Element-wise field operation on raw limbs (9 words in, 9 words out), the
// same numbering as the library's raw-limb diagnostic kernel.
int hs_field_raw(int op, const uint32_t *a, const uint32_t *b, uint32_t *out) {
    const fe x = raw_of(a), y = raw_of(b);
    fe r = fe_zero();
    switch (op) {
        case 0: r = fe_add(x, y); break;
        case 1: r = fe_sub(x, y); break;
        case 2: r = fe_mul(x, y); break;
        case 3: r = fe_sqr(x); break;
        case 4: r = fe_sub2(x, y); break;
        case 5: r = fe_mul3(x); break;
        case 6: r = fe_mul4(x); break;
        case 7: r = fe_neg(x); break;
        case 8: r = fe_canon(x); break;
        case 9: r = fe_dbl(x); break;
        case 10: r = fe_norm(x); break;
        case 11: r.v[0] = fe_eq(x, y) ? 1u : 0u; break;
        case 12: r.v[0] = fe_is_zero(x) ? 1u : 0u; break;
        case 13: r = fe_sub_w(x, y); break;
        case 14: r = fe_mul4_w(x); break;
        case 15: r = fe_sub_sub2(x, y, y); break;
        case 16: r = fe_sub2x(x, y); break;
        case 17: r = fe_mul(fe_sub_w(x, y), fe_mul4_w(y)); break;
        case 18: r = fe_mul_plus_t<true>(x, y, fe_2p_minus(y)); break;
        case 19: r = fe_4sub_sub2(x, y, y); break;
        case 20: r = fe_mul_sub2_t<true>(fe_x2(x), y, fe_norm(y), fe_norm(y)); break;
        case 21: r = fe_mul_ilp(x, y); break;
        case 22: r = fe_sqr_ilp(x); break;
        case 23: r = fe_inv(x); break;
        case 24: r = fe_mul_t<true, true>(x, y); break;
        case 25: r = fe_sqr_t<true, true>(x); break;
        case 26: r = fe_mul_plus_t<true, true>(x, y, fe_2p_minus(y)); break;
        case 27: r = fe_mul_t<true, true>(x, fe_x2(y)); break;
        case 28: r = fe_mul_sub2_t<true, true>(fe_x2(x), y, fe_norm(y), fe_norm(y)); break;
        case 29: r = fe_mul_sub_t<true, true>(x, y, fe_norm(y), fe_norm(y)); break;
        case 30: r = fe_inv_fermat(x); break;
        default: return -1;
    }
    for (int i = 0; i < NL; ++i) out[i] = r.v[i];
    return 0;
}

// hs_field_raw over n elements (row-major n x 9 arrays)
int hs_field_raw_n(int op, const uint32_t *a, const uint32_t *b, uint32_t *out, int64_t n) {
    for (int64_t e = 0; e < n; ++e)
        if (hs_field_raw(op, a + e * NL, b + e * NL, out + e * NL)) return -1;
    return 0;
}

// Point operation on canonical affine inputs (16 words each; P given the
// Jacobian coordinate z_p, Q the coordinate z_q where the operation takes a
// Jacobian Q; a null z means Z = 1), result as canonical affine (16 words):
//   0 P + Q, Q affine (complete mixed addition)
//   1 P + Q, Q affine, the accumulation's form (identity flags carried)
//   2 P + Q, both Jacobian
//   3 2P
//   4 k P by the ladder over the low t bits of k (P affine)
//   5 -P
//   6 P + Q, Q affine, the accumulation's XYZZ form (identity flags
//     carried; P given in XYZZ coordinates at z_p)
int hs_point(int op, const uint32_t *P, const uint32_t *zp, const uint32_t *Q, const uint32_t *zq, uint32_t k,
             int t, uint32_t *out) {
    jpt r;
    switch (op) {
        case 0: r = jpt_add_affine(jac_of(P, zp), aff_of(Q)); break;
        case 1: {
            const jpt jp = jac_of(P, zp);
            const apt q = aff_of(Q);
            bool r_inf = false;
            r = jpt_add_affine_known(jp, jpt_is_inf(jp), q, apt_is_inf(q), r_inf);
            // the carried flag must agree with the result
            if (r_inf != jpt_is_inf(r)) return 1;
            break;
        }
        case 2: r = jpt_add(jac_of(P, zp), jac_of(Q, zq)); break;
        case 3: r = jpt_dbl(jac_of(P, zp)); break;
        case 4: r = ladder_small(k, t, aff_of(P)); break;
        case 5: r = jpt_neg(jac_of(P, zp)); break;
        case 6: {
            bool p_inf = false, r_inf = false;
            const xpt xp = xyzz_of(P, zp, p_inf);
            const apt q = aff_of(Q);
            const xpt s = xpt_add_affine_known(xp, p_inf, q, apt_is_inf(q), r_inf);
            // the carried flag must agree with the result's ZZ, ZZZ
            if (r_inf != (fe_is_zero(s.ZZ) || fe_is_zero(s.ZZZ))) return 1;
            r = xpt_to_jpt(s, r_inf);
            break;
        }
        default: return -1;
    }
    aff_out(r, out);
    return 0;
}

// The accumulation's loop on the host: the identity plus n affine points
// (16 canonical words each; neg[i] != 0 adds -P_i), in the XYZZ form with
// the identity flag carried, so that every addition after the first takes
// the previous one's loose outputs.  Result as canonical affine.
int hs_accumulate(const uint32_t *pts, const uint8_t *neg, int n, uint32_t *out) {
    xpt acc = xpt_infinity();
    bool inf = true;
    for (int i = 0; i < n; ++i) {
        apt q = aff_of(pts + 16 * i);
        const bool q_inf = apt_is_inf(q);
        if (neg[i]) q.y = fe_neg(q.y);
        acc = xpt_add_affine_known(acc, inf, q, q_inf, inf);
    }
    aff_out(xpt_to_jpt(acc, inf), out);
    return 0;
}

}  // extern "C"
