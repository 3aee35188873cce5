"""The library's device field and point arithmetic (fp.hpp, ec.hpp,
common.hpp) compiled for the host with g++ and the undefined-behaviour
sanitizer (tests/hostshim), checked on the CPU: field operations against
exact integer arithmetic (the cases of the GPU raw-limb test), point
operations against the oracle's affine group law (Sec. 2.3), including every
exceptional case, and the ladder of Alg. 1 against the oracle's.

A mistake in a point formula or in the exceptional-case logic shows up here
without a GPU; a 64-bit column sum that overflows aborts the sanitized build.
"""
import random

import pytest

import field_cases as FC
import hostbuild


@pytest.fixture(scope="module")
def host():
    try:
        hostbuild.lib()
    except (RuntimeError, OSError) as e:  # no g++ or no sanitizer runtime
        pytest.skip(f"host build unavailable: {e}")
    return hostbuild


def test_host_raw_field_ops_vs_integers(host):
    FC.check_raw_field_ops(host.field_raw)


def test_host_raw_products_of_extreme_carry_only_operands(host):
    FC.check_extreme_carry_only_products(host.field_raw)


def test_host_loose_quotient_products(host):
    FC.check_loose_quotient_products(host.field_raw)


def test_host_raw_normalisation_of_signed_limbs(host):
    FC.check_signed_limb_normalisation(host.field_raw)


def test_host_split_form_products_and_inverse(host):
    """The split (ILP) product forms and the Fermat inverse of the
    latency-bound callers equal the plain definitions."""
    import numpy as np
    a, b = FC._operands(400, 3)
    A = np.array([FC.limbs(v) for v in a], dtype=np.int64)
    B = np.array([FC.limbs(v) for v in b], dtype=np.int64)
    P, RINV, R = FC.P, FC.RINV, FC.R
    out = host.field_raw(21, A, B)
    FC._check_normal(out)
    assert all(FC.value(out[i]) % P == (a[i] * b[i] * RINV) % P for i in range(len(a)))
    out = host.field_raw(22, A, B)
    FC._check_normal(out)
    assert all(FC.value(out[i]) % P == (a[i] * a[i] * RINV) % P for i in range(len(a)))
    out = host.field_raw(23, A, B)
    FC._check_normal(out)
    for i in range(len(a)):
        x = a[i] % P
        # Montgomery form: x R^-1 is the value, its inverse is x^-1 R^2 in limbs
        want = 0 if x == 0 else (pow(x, -1, P) * R * R) % P
        assert FC.value(out[i]) % P == want, i


def test_host_inversion_by_divsteps(host):
    """fe_inv (divsteps) equals the modular inverse and the Fermat chain on
    edge values, carry-only extremes and 20,000 random operands below 4p."""
    FC.check_inversion(host.field_raw)


def _random_point(orc, rnd):
    p_, b_, gx, gy, q = orc.curve_params()
    return orc.ladder_big(rnd.randrange(1, q), orc.generator())


def _cases(orc, count, seed):
    """(P, Q) pairs: random, P = Q, P = -Q, identities on either side, both."""
    rnd = random.Random(seed)
    out = []
    for k in range(count):
        P = _random_point(orc, rnd)
        Q = _random_point(orc, rnd)
        kind = k % 7
        if kind == 1:
            Q = P
        elif kind == 2:
            Q = orc.pt_neg(P)
        elif kind == 3:
            P = orc.INF
        elif kind == 4:
            Q = orc.INF
        elif kind == 5:
            P = Q = orc.INF
        out.append((P, Q))
    return out


def test_host_point_additions_vs_oracle(host, orc):
    """Mixed addition (both forms), general addition and doubling, with the
    Jacobian operands at random Z, equal the oracle on every case of the group
    law; the accumulation's form also carries the right identity flag."""
    p_ = orc.curve_params()[0]
    rnd = random.Random(77)
    for P, Q in _cases(orc, 210, 5):
        zp, zq = rnd.randrange(1, p_), rnd.randrange(1, p_)
        want = orc.pt_add(P, Q)
        for op in (0, 1, 6):
            assert host.point(op, P, Q, zp=zp) == want, (op, P.hex()[:16], Q.hex()[:16])
            assert host.point(op, P, Q) == want, (op, "Z = 1")
        assert host.point(2, P, Q, zp=zp, zq=zq) == want
        assert host.point(3, P, zp=zp) == orc.pt_dbl(P)
        assert host.point(5, P, zp=zp) == orc.pt_neg(P)


def test_host_xyzz_accumulation_chains_vs_oracle(host, orc):
    """The accumulation's XYZZ loop over chains of table-like entries equals
    the oracle's sum: every addition after the first takes loose outputs of
    the previous one, and the chains pass through every exceptional case
    (a repeated entry while the sum equals it, its negation, identities in
    the middle, a sum that returns to the identity and continues)."""
    rnd = random.Random(31)
    pts = [_random_point(orc, rnd) for _ in range(6)]
    for c in range(40):
        chain, negs = [], []
        for _ in range(rnd.randrange(1, 24)):
            kind = rnd.randrange(10)
            if kind == 0:
                chain.append(orc.INF)
            else:
                chain.append(pts[rnd.randrange(len(pts))])
            negs.append(rnd.random() < 0.4)
        if c % 4 == 1:  # P + P from the identity: the doubling case
            chain, negs = [pts[0], pts[0], pts[1]], [False, False, True]
        elif c % 4 == 2:  # P - P, then more: identity in the middle
            chain, negs = [pts[2], pts[2], pts[3], pts[3]], [False, True, True, True]
        elif c % 4 == 3:  # the sum (Z != 1) meets itself, then its negation
            S = orc.pt_add(pts[c % 6], pts[(c + 1) % 6])
            chain = [pts[c % 6], pts[(c + 1) % 6], S, S, S, S]
            negs = [False, False, False, False, True, True] if c % 8 == 3 else [False, False, True, False, False, False]
        want = orc.INF
        for P, ng in zip(chain, negs):
            want = orc.pt_add(want, orc.pt_neg(P) if ng else P)
        assert host.accumulate(chain, negs) == want, c


def test_host_ladder_vs_oracle(host, orc):
    """Alg. 1 over t bits equals the oracle's ladder, including k = 0, k with
    its top bit clear and k at 2^t - 1."""
    rnd = random.Random(9)
    for t in (1, 2, 4, 8, 12, 17):
        P = _random_point(orc, rnd)
        for k in {0, 1, 2, (1 << t) - 1, (1 << (t - 1)), rnd.randrange(1 << t), rnd.randrange(1 << t)}:
            assert host.point(4, P, k=k, t=t) == orc.ladder_small(k, t, P), (t, k)
