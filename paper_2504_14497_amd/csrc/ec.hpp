// ec.hpp -- P-256 point arithmetic on gfx950 (device side).
//
// Curve (Sec. 4.1): y^2 = x^3 - 3x + b over F_p, prime order q, cofactor 1.
// Points are held in VGPRs in Montgomery form:
//   jpt  Jacobian (X, Y, Z), x = X/Z^2, y = Y/Z^3; the identity has Z = 0;
//   apt  affine (x, y); the identity is (0, 0) (not on the curve since b != 0);
//   xpt  extended Jacobian (X, Y, ZZ, ZZZ), x = X/ZZ, y = Y/ZZZ, for the
//        accumulator (mixed addition 8M + 2S).
// Formulas are the standard Jacobian ones for a = -3 (doubling 3M + 5S,
// mixed addition 7M + 4S, general addition 11M + 5S).  Every exceptional
// case of the group law (Sec. 2.3) is handled:
//   identity operands         -> select the other operand;
//   P = -Q                    -> H = 0, r != 0: the formulas already give Z = 0;
//   P = Q                     -> H = 0, r = 0: the formulas break down, so the
//                                lanes that hit it take the doubling instead.
#pragma once
#include "fp.hpp"

namespace pcmm {

struct jpt {
    fe X, Y, Z;
};

struct apt {
    fe x, y;
};

// standard P-256 domain parameters (b, generator) in canonical hex
constexpr fe_const CURVE_B_PLAIN =
    c_from_hex("5ac635d8aa3a93e7b3ebbd55769886bc651d06b0cc53b0f63bce3c3e27d2604b");
constexpr fe_const GX_PLAIN =
    c_from_hex("6b17d1f2e12c4247f8bce6e563a440f277037d812deb33a0f4a13945d898c296");
constexpr fe_const GY_PLAIN =
    c_from_hex("4fe342e2fe1a7f9b8ee7eb4a7c0f9e162bce33576b315ececbb6406837bf51f5");
// group order q, for scalar handling
constexpr fe_const ORDER_Q =
    c_from_hex("ffffffff00000000ffffffffffffffffbce6faada7179e84f3b9cac2fc632551");

__device__ __forceinline__ jpt jpt_infinity() {
    jpt r;
    r.X = fe_one_mont();
    r.Y = fe_one_mont();
    r.Z = fe_zero();
    return r;
}

__device__ __forceinline__ bool jpt_is_inf(const jpt &P) { return fe_is_zero(P.Z); }

// Affine infinity is encoded as x = 0, y = 0 (not a curve point, since b != 0).
// x is compared by its raw limbs and y by value: negation maps y = 0 to the
// non-canonical limbs of p, and a curve point with x = 0 has y != 0.
__device__ __forceinline__ bool apt_is_inf(const apt &P) {
    return fe_is_raw_zero(P.x) && fe_is_zero(P.y);
}

__device__ __forceinline__ jpt jpt_from_affine(const apt &P) {
    jpt r;
    r.X = P.x;
    r.Y = P.y;
    r.Z = apt_is_inf(P) ? fe_zero() : fe_one_mont();
    return r;
}

__device__ __forceinline__ jpt jpt_select(bool c, const jpt &a, const jpt &b) {
    jpt r;
    r.X = fe_select(c, a.X, b.X);
    r.Y = fe_select(c, a.Y, b.Y);
    r.Z = fe_select(c, a.Z, b.Z);
    return r;
}

__device__ __forceinline__ apt apt_neg(const apt &P) {
    apt r;
    r.x = P.x;
    r.y = fe_neg(P.y);  // -infinity = (0, p), still recognised by apt_is_inf
    return r;
}

__device__ __forceinline__ jpt jpt_neg(const jpt &P) {
    jpt r = P;
    r.Y = fe_neg(P.Y);
    return r;
}

// The template parameter CHAIN of the point operations selects the product
// form of fp.hpp: one multiply-add chain per column (the default, for the
// accumulation, whose independent products hide the chains' latency) or the
// split form (for latency-bound callers such as the table build).

// 2P, a = -3 (dbl-2001-b).  Z = 0 stays Z = 0.  Lazy reduction as in
// jpt_add_affine: X1 -+ delta stay carry-only (their product is below
// 16 p^2), X3 = alpha^2 - 8 beta and Y3 = alpha (4 beta - X3) - 8 gamma^2 are
// one limb pass plus one normalisation each, and Z3 = (Y1 + Z1)^2 - gamma -
// delta is computed as the equal 2 Y1 Z1.
template <bool CHAIN = true>
__device__ __forceinline__ jpt jpt_dbl(const jpt &P) {
    fe delta = fe_sqr_t<CHAIN>(P.Z);
    fe gamma = fe_sqr_t<CHAIN>(P.Y);
    fe beta = fe_mul_t<CHAIN>(P.X, gamma);
    fe alpha = fe_mul3(fe_mul_t<CHAIN>(fe_sub_w(P.X, delta), fe_add_w(P.X, delta)));  // 3 (X - delta)(X + delta)
    jpt R;
    fe beta4 = fe_mul4(beta);
    R.X = fe_sub2x(fe_sqr_t<CHAIN>(alpha), beta4);
    R.Z = fe_dbl(fe_mul_t<CHAIN>(P.Y, P.Z));
    R.Y = fe_sub2x(fe_mul_t<CHAIN>(alpha, fe_sub_w(beta4, R.X)), fe_mul4(fe_sqr_t<CHAIN>(gamma)));
    return R;
}

// R <- 2P on the lanes where `same` holds.  The doubling runs only when some
// lane of the wavefront needs it, and then on the whole wavefront (a uniform
// branch) followed by a per-lane select.
template <bool CHAIN = true>
__device__ __forceinline__ jpt fix_equal_operands(bool same, const jpt &R, const jpt &P) {
    if (__ballot(same)) {
        jpt D = jpt_dbl<CHAIN>(P);
        return jpt_select(same, R, D);
    }
    return R;
}

// The formulas of madd-2007-bl (7M + 4S) for P + Q with Q affine, without
// the exceptional cases; hh = H^2 and r (r / 2 with LEAN) are returned for
// their tests.  Lazy reduction: H (< 4p) and I = 4 H^2 (< 8p) stay
// carry-only (their products are below 32 p^2), X3 = r^2 - J - 2V and
// Y3 = r (V - X3) - 2 Y1 J are each one limb pass plus one normalisation,
// and Z3 = (Z1 + H)^2 - Z1Z1 - HH is computed as the equal 2 Z1 H.
// LEAN (the table builds' form) folds additions into the products and
// doubles in an operand's limbs (fe_x2: below 2^30, valid for one operand of
// a product): H = U2 - X1 and r' = S2 - Y1 (= r / 2) come out of the products
// U2 and S2 with 2p - X1, 2p - Y1 added above R (carry-only, < 4p); r^2 =
// 4 r'^2 enters the X3 limb pass; Y3 = (2 r') (V - X3) - 2 Y1 J is one
// reduction of both products (fe_mul_sub2); Z3 = Z1 (2H) (below 16 p^2).
// Otherwise H and r are formed by limb passes, r is normalised and Z3 is the
// normalised doubling of Z1 H, which keeps fewer registers live in the
// latency-bound callers.
template <bool CHAIN, bool LEAN>
__device__ __forceinline__ jpt madd_formulas(const jpt &P, const apt &Q, fe &hh, fe &r) {
    jpt R;
    if constexpr (LEAN) {
        // Every product takes loose quotient digits (fp.hpp): a loose
        // product of a b is below a b / R + p (1 + 2^-26), which gives the
        // bounds in the comments (P's coordinates and Q normal, < 2p), and
        // the largest operand-bound product, 24.3 p^2 for Y3, is below the
        // 31.99 p^2 that keeps a loose result in normal form.
        constexpr bool LQ = true;
        fe z1z1 = fe_sqr_t<CHAIN, LQ>(P.Z);                                                      // < 1.13p
        fe h = fe_mul_plus_t<CHAIN, LQ>(Q.x, z1z1, fe_2p_minus(P.X));                            // (0, 3.08p)
        r = fe_mul_plus_t<CHAIN, LQ>(fe_mul_t<CHAIN, LQ>(Q.y, P.Z), z1z1, fe_2p_minus(P.Y));  // r / 2, (0, 3.05p)
        hh = fe_sqr_t<CHAIN, LQ>(h);        // 9.5 p^2 -> < 1.3p
        fe i4 = fe_mul4_w(hh);              // [0, 5.2p)
        fe j = fe_mul_t<CHAIN, LQ>(h, i4);  // 16 p^2 -> < 1.5p
        fe v = fe_mul_t<CHAIN, LQ>(P.X, i4);  // 10.4 p^2
        R.X = fe_4sub_sub2(fe_sqr_t<CHAIN, LQ>(r), j, v);
        R.Y = fe_mul_sub2_t<CHAIN, LQ>(fe_x2(r), fe_sub_w(v, R.X), P.Y, j);  // 6.1p x 4p, folded
        R.Z = fe_mul_t<CHAIN, LQ>(P.Z, fe_x2(h));  // 2p x 6.2p
    } else {
        fe z1z1 = fe_sqr_t<CHAIN>(P.Z);
        fe u2 = fe_mul_t<CHAIN>(Q.x, z1z1);
        fe s2 = fe_mul_t<CHAIN>(fe_mul_t<CHAIN>(Q.y, P.Z), z1z1);
        fe h = fe_sub_w(u2, P.X);           // (0, 4p)
        hh = fe_sqr_t<CHAIN>(h);
        fe i4 = fe_mul4_w(hh);              // [0, 8p)
        fe j = fe_mul_t<CHAIN>(h, i4);
        r = fe_sub2(s2, P.Y);
        fe v = fe_mul_t<CHAIN>(P.X, i4);
        R.X = fe_sub_sub2(fe_sqr_t<CHAIN>(r), j, v);
        R.Y = fe_sub2x(fe_mul_t<CHAIN>(r, fe_sub_w(v, R.X)), fe_mul_t<CHAIN>(P.Y, j));
        R.Z = fe_dbl(fe_mul_t<CHAIN>(P.Z, h));
    }
    return R;
}

// P + Q with Q affine, complete.
template <bool CHAIN = true>
__device__ __forceinline__ jpt jpt_add_affine(const jpt &P, const apt &Q) {
    fe hh, r;
    jpt R = madd_formulas<CHAIN, false>(P, Q, hh, r);
    bool p_inf = jpt_is_inf(P);
    bool q_inf = apt_is_inf(Q);
    bool same = fe_is_zero(hh) && fe_is_zero(r) && !p_inf && !q_inf;
    R = fix_equal_operands<CHAIN>(same, R, P);
    // infinity operands are rare: the selects run only when some lane of the
    // wavefront has one (uniform branches, then per-lane selects)
    if (__ballot(p_inf)) R = jpt_select(p_inf, R, jpt_from_affine(Q));
    if (__ballot(q_inf)) R = jpt_select(q_inf, R, P);
    return R;
}

// P + Q with Q affine, complete, for a caller that knows which operands
// are the identity: p_inf (Z1 = 0) and q_inf (Q is the affine
// identity) are given, and r_inf receives whether the result is the
// identity (its Z is then 0), so the caller carries the flag instead of
// testing Z1's limbs at every addition.  Exceptional cases: with neither
// operand the identity, H = 0 means P = +-Q; P = Q (r = 0) needs the
// doubling, P = -Q gives Z3 = 0, the identity.  The test of r runs only
// when some lane of the wavefront has H = 0.  A P-256 point is never of
// order 2, so 2P is not the identity.
template <bool CHAIN = true>
__device__ __forceinline__ jpt jpt_add_affine_known(const jpt &P, bool p_inf, const apt &Q, bool q_inf,
                                                    bool &r_inf) {
    fe hh, r;
    jpt R = madd_formulas<CHAIN, true>(P, Q, hh, r);
    const bool h_zero = fe_is_zero(hh) && !p_inf && !q_inf;
    bool inf = p_inf && q_inf;
    if (__ballot(h_zero)) {
        const bool r_zero = fe_is_zero(fe_norm(r));  // r / 2 is carry-only
        R = fix_equal_operands<CHAIN>(h_zero && r_zero, R, P);
        inf = inf || (h_zero && !r_zero);
    }
    if (__ballot(p_inf || q_inf)) {
        jpt Qj;
        Qj.X = Q.x;
        Qj.Y = Q.y;
        Qj.Z = q_inf ? fe_zero() : fe_one_mont();
        R = jpt_select(p_inf, R, Qj);
        R = jpt_select(q_inf, R, P);
    }
    r_inf = inf;
    return R;
}

// P + Q with Q affine, complete, in the lean form (the flags computed here):
// for dependent chains, whose latency tracks the products' instruction count.
template <bool CHAIN = true>
__device__ __forceinline__ jpt jpt_add_affine_lean(const jpt &P, const apt &Q) {
    bool r_inf;
    return jpt_add_affine_known<CHAIN>(P, jpt_is_inf(P), Q, apt_is_inf(Q), r_inf);
}

// Extended Jacobian ("XYZZ") coordinates for the accumulator: (X, Y, ZZ,
// ZZZ) stands for the affine (X / ZZ, Y / ZZZ), with ZZ^3 = ZZZ^2 (ZZ = Z^2
// and ZZZ = Z^3 for some Z); ZZ = ZZZ = 0 is the identity.  A mixed addition
// costs 8M + 2S here against 8M + 3S for the Jacobian form above (no Z1^2),
// and no doubled operands or 4 H^2 pass.
struct xpt {
    fe X, Y, ZZ, ZZZ;
};

__device__ __forceinline__ xpt xpt_infinity() {
    xpt r;
    r.X = fe_one_mont();
    r.Y = fe_one_mont();
    r.ZZ = fe_zero();
    r.ZZZ = fe_zero();
    return r;
}

__device__ __forceinline__ xpt xpt_select(bool c, const xpt &a, const xpt &b) {
    xpt r;
    r.X = fe_select(c, a.X, b.X);
    r.Y = fe_select(c, a.Y, b.Y);
    r.ZZ = fe_select(c, a.ZZ, b.ZZ);
    r.ZZZ = fe_select(c, a.ZZZ, b.ZZZ);
    return r;
}

// 2Q for a finite affine Q (the XYZZ doubling with ZZ1 = ZZZ1 = 1, a = -3):
// U = 2y, V = U^2, W = U V, S = x V, M = 3 (x - 1)(x + 1), X3 = M^2 - 2S,
// Y3 = M (S - X3) - W y, ZZ3 = V, ZZZ3 = W.  Normal operands throughout.
template <bool CHAIN = true>
__device__ __forceinline__ xpt xpt_dbl_affine(const apt &Q) {
    const fe one = fe_one_mont();
    const fe u = fe_dbl(Q.y);
    const fe v = fe_sqr_t<CHAIN>(u);
    const fe w = fe_mul_t<CHAIN>(u, v);
    const fe s = fe_mul_t<CHAIN>(Q.x, v);
    const fe m = fe_mul3(fe_mul_t<CHAIN>(fe_sub_w(Q.x, one), fe_add_w(Q.x, one)));
    xpt R;
    R.X = fe_sub2x(fe_sqr_t<CHAIN>(m), s);
    R.Y = fe_sub(fe_mul_t<CHAIN>(m, fe_sub_w(s, R.X)), fe_mul_t<CHAIN>(w, Q.y));
    R.ZZ = v;
    R.ZZZ = w;
    return R;
}

// P + Q with Q affine (the XYZZ mixed addition, madd-2008-s), complete, for
// the accumulation: identity flags carried as in jpt_add_affine_known (p_inf
// and q_inf given, r_inf returned).  With P's coordinates and Q normal (< 2p)
// and loose quotient digits in every product (a product of operands below
// a p and b p is below (a b / 32 + 1) p):
//   P  = X2 ZZ1 - X1          in (0, 3.13p), carry-only (2p - X1 absorbed)
//   R  = Y2 ZZZ1 - Y1         in (0, 3.13p), likewise
//   PP = P^2 < 1.31p, PPP = P PP < 1.13p, Q' = X1 PP < 1.09p
//   X3 = R^2 - PPP - 2 Q'     one limb pass, normalised
//   Y3 = R (Q' - X3) - Y1 PPP one reduction of both products (12.5 p^2 and
//                             2.3 p^2), folded into [0, 2p)
//   ZZ3 = ZZ1 PP, ZZZ3 = ZZZ1 PPP.
// Exceptional cases (neither operand the identity): P = 0 means P = +-Q; R =
// 0 then means P = Q, whose sum is the doubling of the affine Q, and
// otherwise P = -Q, for which PP = PPP = 0 already give ZZ3 = ZZZ3 = 0.
template <bool CHAIN = true>
__device__ __forceinline__ xpt xpt_add_affine_known(const xpt &P, bool p_inf, const apt &Q, bool q_inf,
                                                    bool &r_inf) {
    constexpr bool LQ = true;
    const fe h = fe_mul_plus_t<CHAIN, LQ>(Q.x, P.ZZ, fe_2p_minus(P.X));
    const fe r = fe_mul_plus_t<CHAIN, LQ>(Q.y, P.ZZZ, fe_2p_minus(P.Y));
    const fe pp = fe_sqr_t<CHAIN, LQ>(h);
    const fe ppp = fe_mul_t<CHAIN, LQ>(h, pp);
    const fe q = fe_mul_t<CHAIN, LQ>(P.X, pp);
    xpt R;
    R.X = fe_sub_sub2(fe_sqr_t<CHAIN, LQ>(r), ppp, q);
    R.Y = fe_mul_sub_t<CHAIN, LQ>(r, fe_sub_w(q, R.X), P.Y, ppp);
    R.ZZ = fe_mul_t<CHAIN, LQ>(P.ZZ, pp);
    R.ZZZ = fe_mul_t<CHAIN, LQ>(P.ZZZ, ppp);
    const bool h_zero = fe_is_zero(pp) && !p_inf && !q_inf;
    bool inf = p_inf && q_inf;
    if (__ballot(h_zero)) {
        const bool same = h_zero && fe_is_zero(fe_norm(r));  // r is carry-only
        if (__ballot(same)) R = xpt_select(same, R, xpt_dbl_affine<CHAIN>(Q));
        inf = inf || (h_zero && !same);
    }
    if (__ballot(p_inf || q_inf)) {
        xpt Qx;
        Qx.X = Q.x;
        Qx.Y = Q.y;
        Qx.ZZ = q_inf ? fe_zero() : fe_one_mont();
        Qx.ZZZ = Qx.ZZ;
        R = xpt_select(p_inf, R, Qx);
        R = xpt_select(q_inf, R, P);
    }
    r_inf = inf;
    return R;
}

// Jacobian form of an XYZZ point: (X ZZ^2, Y ZZZ^2, ZZZ), which with ZZ =
// Z^2, ZZZ = Z^3 is (X Z^4, Y Z^6, Z^3), the same affine point; Z = 0 for
// the identity (inf).
template <bool CHAIN = true>
__device__ __forceinline__ jpt xpt_to_jpt(const xpt &P, bool inf) {
    jpt R;
    R.X = fe_mul_t<CHAIN>(P.X, fe_sqr_t<CHAIN>(P.ZZ));
    R.Y = fe_mul_t<CHAIN>(P.Y, fe_sqr_t<CHAIN>(P.ZZZ));
    R.Z = inf ? fe_zero() : P.ZZZ;
    return R;
}

// P + Q, both Jacobian (add-2007-bl), complete.  Lazy reduction as in
// jpt_add_affine; I = (2H)^2 is computed as 4 H^2 and Z3 =
// ((Z1 + Z2)^2 - Z1Z1 - Z2Z2) H as the equal 2 Z1 Z2 H.
template <bool CHAIN = true>
__device__ __forceinline__ jpt jpt_add(const jpt &P, const jpt &Q) {
    fe z1z1 = fe_sqr_t<CHAIN>(P.Z);
    fe z2z2 = fe_sqr_t<CHAIN>(Q.Z);
    fe u1 = fe_mul_t<CHAIN>(P.X, z2z2);
    fe u2 = fe_mul_t<CHAIN>(Q.X, z1z1);
    fe s1 = fe_mul_t<CHAIN>(fe_mul_t<CHAIN>(P.Y, Q.Z), z2z2);
    fe s2 = fe_mul_t<CHAIN>(fe_mul_t<CHAIN>(Q.Y, P.Z), z1z1);
    fe h = fe_sub_w(u2, u1);           // (0, 4p)
    fe hh = fe_sqr_t<CHAIN>(h);
    fe i = fe_mul4_w(hh);              // [0, 8p)
    fe j = fe_mul_t<CHAIN>(h, i);
    fe r = fe_sub2(s2, s1);
    fe v = fe_mul_t<CHAIN>(u1, i);
    jpt R;
    R.X = fe_sub_sub2(fe_sqr_t<CHAIN>(r), j, v);
    R.Y = fe_sub2x(fe_mul_t<CHAIN>(r, fe_sub_w(v, R.X)), fe_mul_t<CHAIN>(s1, j));
    R.Z = fe_dbl(fe_mul_t<CHAIN>(fe_mul_t<CHAIN>(P.Z, Q.Z), h));
    bool p_inf = jpt_is_inf(P);
    bool q_inf = jpt_is_inf(Q);
    bool same = fe_is_zero(hh) && fe_is_zero(r) && !p_inf && !q_inf;
    R = fix_equal_operands<CHAIN>(same, R, P);
    if (__ballot(p_inf)) R = jpt_select(p_inf, R, Q);
    if (__ballot(q_inf)) R = jpt_select(q_inf, R, P);
    return R;
}

// affine (x, y) of a Jacobian point given zinv = Z^-1 (Z != 0)
// (a short dependent chain of products: the split forms have lower latency)
// (loose quotient digits: P's coordinates and zinv normal, every operand
// pair below 4 p^2)
__device__ __forceinline__ apt jpt_to_affine_with(const jpt &P, const fe &zinv) {
    fe z2 = fe_sqr_t<false, true>(zinv);
    apt r;
    r.x = fe_mul_t<false, true>(P.X, z2);
    r.y = fe_mul_t<false, true>(P.Y, fe_mul_t<false, true>(z2, zinv));
    return r;
}

}  // namespace pcmm
