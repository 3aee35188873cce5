"""GPU parity of the field arithmetic, the point formulas and the ladder.

Field operations are compared with Python's big integers (the plain
definitions) on random and edge operands; point operations with the CPU
oracle's affine group law, bit-exact after converting the GPU's Jacobian
result to affine.
"""
import random

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

P = 2**256 - 2**224 + 2**192 + 2**96 - 1


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_14497_amd import pcmm
    pcmm.lib()
    return pcmm


def _operands(n, seed):
    rnd = random.Random(seed)
    edge = [0, 1, 2, 3, P - 1, P - 2, P - 3, (P - 1) // 2, (P + 1) // 2, 2**255, 2**256 - P,
            2**224, 2**192, 2**96, 2**32 - 1, 2**64 - 1, (2**256) % P, (2**512) % P, P - 2**32]
    a = edge + [rnd.randrange(P) for _ in range(n - len(edge))]
    b = [rnd.choice(edge) if rnd.random() < 0.2 else rnd.randrange(P) for _ in range(n)]
    return a, b


def test_field_ops_vs_python(dev):
    a, b = _operands(20000, 1)
    assert dev.diag_field(0, a, b) == [(x + y) % P for x, y in zip(a, b)]
    assert dev.diag_field(1, a, b) == [(x - y) % P for x, y in zip(a, b)]
    assert dev.diag_field(2, a, b) == [(x * y) % P for x, y in zip(a, b)]
    assert dev.diag_field(3, a) == [(x * x) % P for x in a]
    assert dev.diag_field(5, a) == [(-x) % P for x in a]
    assert dev.diag_field(6, a) == a
    small = a[:3000]
    assert dev.diag_field(4, small) == [pow(x, -1, P) if x else 0 for x in small]


def test_field_ragged_sizes(dev):
    for n in (1, 63, 64, 65, 255, 257):
        a, b = _operands(max(n, 20), n)
        a, b = a[:n], b[:n]
        assert dev.diag_field(2, a, b) == [(x * y) % P for x, y in zip(a, b)]


def _affine(jac):
    X, Y, Z = jac
    if Z % P == 0:
        return bytes(64)
    zi = pow(Z, -1, P)
    x = X * zi * zi % P
    y = Y * zi * zi * zi % P
    return x.to_bytes(32, "big") + y.to_bytes(32, "big")


def _points(orc, n, seed):
    rnd = random.Random(seed)
    p_, b_, gx, gy, q = orc.curve_params()
    G = orc.generator()
    base = [orc.ladder_big(rnd.randrange(1, q), G) for _ in range(8)]
    pts = list(base)
    while len(pts) < n:
        pts.append(orc.pt_add(pts[-1], base[len(pts) % 8]))
    return pts[:n]


def _arr(pts):
    return np.frombuffer(b"".join(pts), dtype=np.uint8).reshape(len(pts), 64)


def test_point_ops_vs_oracle(dev, orc):
    Ps = _points(orc, 96, 3)
    Qs = _points(orc, 96, 4)
    # exceptional pairs: P = Q, P = -Q, identities
    Qs[0] = Ps[0]
    Qs[1] = orc.pt_neg(Ps[1])
    Ps[2] = orc.INF
    Qs[3] = orc.INF
    Ps[4] = orc.INF
    Qs[4] = orc.INF
    Qs[5] = Ps[5]
    # b is a square mod p, so (0, +-sqrt(b)) are curve points: an affine x of
    # zero that is not the identity, as an operand and in P = Q and P = -Q
    p_, b_ = orc.curve_params()[:2]
    y0 = pow(b_, (p_ + 1) // 4, p_)
    assert y0 * y0 % p_ == b_
    X0 = bytes(32) + y0.to_bytes(32, "big")
    X0n = bytes(32) + (p_ - y0).to_bytes(32, "big")
    Ps[6] = X0
    Qs[7] = X0
    Ps[8], Qs[8] = X0, X0
    Ps[9], Qs[9] = X0, X0n
    Ps[10], Qs[10] = X0n, orc.INF
    PA, QA = _arr(Ps), _arr(Qs)
    for op in (0, 1):
        got = [_affine(j) for j in dev.diag_point(op, PA, QA)]
        want = [orc.pt_add(p_, q_) for p_, q_ in zip(Ps, Qs)]
        assert got == want, op
    got = [_affine(j) for j in dev.diag_point(2, PA)]
    assert got == [orc.pt_dbl(p_) for p_ in Ps]
    got = [_affine(j) for j in dev.diag_point(4, PA)]
    assert got == [orc.pt_neg(p_) for p_ in Ps]


def test_ladder_vs_oracle(dev, orc):
    Ps = _points(orc, 64, 5)
    Ps[7] = orc.INF
    rnd = random.Random(6)
    for t in (1, 2, 4, 8):
        ks = [rnd.randrange(1 << t) for _ in Ps]
        ks[0] = 0
        ks[1] = (1 << t) - 1
        got = [_affine(j) for j in dev.diag_point(3, _arr(Ps), k=ks, t=t)]
        want = [orc.ladder_small(k, t, p_) for k, p_ in zip(ks, Ps)]
        assert got == want, t
