"""Pins of the CPU oracle's field and curve arithmetic.

Field and scalar arithmetic are checked against Python's big integers (an
independent implementation of the plain definitions: (a op b) mod M,
pow(a, -1, M)).  Curve constants and scalar multiples k*G are checked against
OpenSSL's prime256v1 (an independent library), and the group law against its
defining invariants (Sec. 2.3): identity, inverses, associativity, order q.
"""
import random

import pytest

from helpers import have_openssl, openssl_params, openssl_pubkey

P = 2**256 - 2**224 + 2**192 + 2**96 - 1  # Sec. 4.1


def _edge_values(M):
    return [0, 1, 2, 3, M - 1, M - 2, (M - 1) // 2, (M + 1) // 2, 2**255, 2**256 - 1 - M,
            2**224, 2**192, 2**128 - 1, 2**64, 2**32 - 1, (1 << 256) % M]


def test_prime_matches_paper(orc):
    p, b, gx, gy, q = orc.curve_params()
    assert p == P


@pytest.mark.parametrize("mod", [0, 1])
def test_mod_ops_vs_python_ints(orc, mod):
    p, _, _, _, q = orc.curve_params()
    M = p if mod == 0 else q
    rnd = random.Random(1234 + mod)
    vals = _edge_values(M) + [rnd.randrange(M) for _ in range(300)]
    for a in vals:
        b = rnd.choice(vals)
        a %= M
        b %= M
        assert orc.mod_op(mod, orc.OP_ADD, a, b) == (a + b) % M
        assert orc.mod_op(mod, orc.OP_SUB, a, b) == (a - b) % M
        assert orc.mod_op(mod, orc.OP_MUL, a, b) == (a * b) % M
        assert orc.mod_op(mod, orc.OP_NEG, a) == (-a) % M
        if a:
            assert orc.mod_op(mod, orc.OP_INV, a) == pow(a, -1, M)


def test_mod_reduces_unreduced_inputs(orc):
    # inputs >= p are reduced before use
    for a in [P, P + 1, 2**256 - 1]:
        assert orc.mod_op(0, orc.OP_MUL, a, 1) == a % P


@pytest.mark.skipif(not have_openssl(), reason="openssl CLI not available")
def test_constants_match_openssl(orc):
    p, a, b, gx, gy, q, h = openssl_params()
    assert (p, b, gx, gy, q) == orc.curve_params()
    assert a == p - 3  # y^2 = x^3 - 3x + b  (Sec. 4.1)
    assert h == 1


def test_generator_on_curve_and_order(orc):
    p, b, gx, gy, q = orc.curve_params()
    assert (gy * gy - (gx**3 - 3 * gx + b)) % p == 0
    G = orc.generator()
    assert orc.on_curve(G)
    assert orc.ladder_big(q, G) == orc.INF          # qG = infinity
    assert orc.ladder_big(q - 1, G) == orc.pt_neg(G)  # (q-1)G = -G
    assert orc.ladder_big(q + 1, G) == G


@pytest.mark.skipif(not have_openssl(), reason="openssl CLI not available")
def test_scalar_mult_known_answers_from_openssl(orc):
    rnd = random.Random(99)
    p, b, gx, gy, q = orc.curve_params()
    ks = [1, 2, 3, 7, 255, 2**32 + 1, q - 1, q - 2] + [rnd.randrange(1, q) for _ in range(6)]
    G = orc.generator()
    for k in ks:
        x, y = openssl_pubkey(k)
        assert orc.coords(orc.ladder_big(k, G)) == (x, y), hex(k)


def _rand_point(orc, rnd):
    p, b, gx, gy, q = orc.curve_params()
    return orc.ladder_big(rnd.randrange(1, q), orc.generator())


def test_group_law_invariants(orc):
    rnd = random.Random(5)
    G = orc.generator()
    for _ in range(20):
        Pp, Q, R = (_rand_point(orc, rnd) for _ in range(3))
        for X in (Pp, Q, R):
            assert orc.on_curve(X)
        assert orc.pt_add(Pp, orc.INF) == Pp
        assert orc.pt_add(orc.INF, Pp) == Pp
        assert orc.pt_add(Pp, orc.pt_neg(Pp)) == orc.INF
        assert orc.pt_add(Pp, Pp) == orc.pt_dbl(Pp)
        assert orc.pt_add(Pp, Q) == orc.pt_add(Q, Pp)
        lhs = orc.pt_add(orc.pt_add(Pp, Q), R)
        rhs = orc.pt_add(Pp, orc.pt_add(Q, R))
        assert lhs == rhs and orc.on_curve(lhs)
    assert orc.pt_dbl(orc.INF) == orc.INF
    assert orc.pt_neg(orc.INF) == orc.INF
    assert orc.on_curve(orc.INF)
    assert not orc.on_curve(orc.point(1, 1))
    assert orc.pt_add(G, orc.pt_neg(G)) == orc.INF


def test_scalar_mult_linearity(orc):
    rnd = random.Random(8)
    p, b, gx, gy, q = orc.curve_params()
    G = orc.generator()
    for _ in range(4):
        a, c = rnd.randrange(q), rnd.randrange(q)
        lhs = orc.ladder_big((a + c) % q, G)
        rhs = orc.pt_add(orc.ladder_big(a, G), orc.ladder_big(c, G))
        assert lhs == rhs
        assert orc.ladder_big(a * c % q, G) == orc.ladder_big(a, orc.ladder_big(c, G))


def test_ladder_small_vs_repeated_addition(orc):
    # Alg. 1 against the textbook definition kP = P + ... + P (Sec. 2.3)
    rnd = random.Random(3)
    P_ = _rand_point(orc, rnd)
    for k in range(0, 301):
        want = orc.repeated_add(k, P_)
        t = max(k.bit_length(), 1)
        assert orc.ladder_small(k, t, P_) == want, k
        assert orc.ladder_small(k, 9, P_) == want, k  # leading zero bits change nothing
    assert orc.ladder_small(5, 3, orc.INF) == orc.INF


def test_scalar_from_seed_range_and_spread(orc):
    p, b, gx, gy, q = orc.curve_params()
    seen = set()
    top = 0
    for idx in range(400):
        s = orc.scalar_from_seed(77, 1, idx)
        assert 1 <= s <= q - 1
        seen.add(s)
        top += s >> 255
    assert len(seen) == 400
    assert 150 < top < 250  # the top bit is roughly balanced
    assert orc.scalar_from_seed(77, 0, 0) != orc.scalar_from_seed(77, 1, 0)
    assert orc.scalar_from_seed(77, 1, 0) != orc.scalar_from_seed(78, 1, 0)
