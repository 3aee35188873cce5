"""Cases for the field arithmetic on its internal representation (nine
29-bit limbs, Montgomery R = 2^261), checked against exact integer arithmetic;
shared by the GPU tests (the library's raw-limb diagnostic kernel) and the
CPU tests (the same headers compiled for the host).

Operands are arbitrary normal-form values -- every value in [0, 2p), including
the non-canonical [p, 2p) range that intermediate results can take -- plus
adversarial limb patterns.  Each result must equal the plain definition modulo
p and must itself be in normal form (limbs 0..7 < 2^29, limb 8 < 2^25,
value < 2p).  `raw(op, A, B)` applies field operation `op` (the diagnostic
numbering) to (count, 9) limb arrays.
"""
import random

import numpy as np

P = 2**256 - 2**224 + 2**192 + 2**96 - 1
R = 2**261
RINV = pow(R, -1, P)
LB, NL = 29, 9
MASK = (1 << LB) - 1


def limbs(v):
    return [(v >> (LB * i)) & MASK for i in range(NL)]


def value(row):
    return sum(int(x) << (LB * i) for i, x in enumerate(row))


def _operands(n, seed):
    rnd = random.Random(seed)
    edge = [0, 1, 2, P - 1, P, P + 1, 2 * P - 1, 2 * P - 2, 2**256 - 1, 2**256, 2**256 + 1,
            2**255, 2**224, 2**192, 2**96, P - 2**96, P + 2**96, (2**256) % P, 2**232 - 1,
            sum(MASK << (LB * i) for i in range(8)), R % P, (R * R) % P]
    edge = [v for v in edge if v < 2 * P]
    vals = edge + [rnd.randrange(2 * P) for _ in range(n)]
    a = list(vals)
    b = [rnd.choice(vals) for _ in vals]
    rnd.shuffle(b)
    # every pair of edge values
    for x in edge:
        for y in edge:
            a.append(x)
            b.append(y)
    return a, b


def _check_normal(out, bound=2 * P, top_bits=25):
    assert (out[:, :8] < (1 << LB)).all()
    assert (out[:, 8] < (1 << top_bits)).all()
    for row in out:
        assert value(row) < bound


def check_raw_field_ops(raw):
    a, b = _operands(6000, 11)
    A = np.array([limbs(v) for v in a], dtype=np.int64)
    B = np.array([limbs(v) for v in b], dtype=np.int64)
    cases = {
        0: lambda x, y: (x + y) % P,
        1: lambda x, y: (x - y) % P,
        2: lambda x, y: (x * y * RINV) % P,
        3: lambda x, y: (x * x * RINV) % P,
        4: lambda x, y: (2 * (x - y)) % P,
        5: lambda x, y: (3 * x) % P,
        6: lambda x, y: (4 * x) % P,
        7: lambda x, y: (-x) % P,
        9: lambda x, y: (2 * x) % P,
    }
    for op, f in cases.items():
        out = raw(op, A, B)
        _check_normal(out)
        bad = [i for i in range(len(a)) if value(out[i]) % P != f(a[i], b[i])]
        assert not bad, (op, bad[:5], [(hex(a[i]), hex(b[i])) for i in bad[:3]])
    # lazy (carry-only) forms and the operations that consume them
    lazy = {
        13: (lambda x, y: (x - y) % P, 4 * P, 26),
        14: (lambda x, y: (4 * x) % P, 8 * P, 27),
        15: (lambda x, y: (x - 3 * y) % P, 2 * P, 25),
        16: (lambda x, y: (x - 2 * y) % P, 2 * P, 25),
        17: (lambda x, y: ((x - y) * 4 * y * RINV) % P, 2 * P, 25),
        18: (lambda x, y: (x * y * RINV - y) % P, 4 * P, 26),
        19: (lambda x, y: (4 * x - 3 * y) % P, 2 * P, 25),
        20: (lambda x, y: (2 * (x - y) * y * RINV) % P, 2 * P, 25),
    }
    for op, (f, bound, top) in lazy.items():
        out = raw(op, A, B)
        _check_normal(out, bound, top)
        bad = [i for i in range(len(a)) if value(out[i]) % P != f(a[i], b[i])]
        assert not bad, (op, bad[:5], [(hex(a[i]), hex(b[i])) for i in bad[:3]])
    out = raw(8, A, B)  # full reduction
    assert all(value(out[i]) == a[i] % P for i in range(len(a)))
    eq = raw(11, A, B)[:, 0]
    assert all(bool(eq[i]) == ((a[i] - b[i]) % P == 0) for i in range(len(a)))
    z = raw(12, A, B)[:, 0]
    assert all(bool(z[i]) == (a[i] % P == 0) for i in range(len(a)))


def check_extreme_carry_only_products(raw):
    """The products that take a doubled operand (limbs < 2^30) and a
    subtracted product: operands carry-only below 4p with limbs 0..7 at or
    near 2^29 - 1, the largest column sums their bounds allow."""
    rnd = random.Random(8)
    rows, vals = [], []
    top = (4 * P - 1) >> (LB * 8)
    while len(rows) < 3000:
        mode = len(rows) % 3
        low = [MASK if mode == 0 else MASK - rnd.randrange(1 << (8 * mode)) for _ in range(8)]
        if mode == 2 and rnd.random() < 0.5:
            low = [rnd.randrange(1 << LB) for _ in range(8)]
        row = low + [rnd.randrange(top + 1)]
        v = value(row)
        if v < 4 * P:
            rows.append(row)
            vals.append(v)
    A = np.array(rows, dtype=np.int64)
    B = A[::-1].copy()
    vb = vals[::-1]
    out = raw(20, A, B)
    _check_normal(out)
    bad = [i for i in range(len(vals)) if value(out[i]) % P != (2 * (vals[i] - vb[i]) * vb[i] * RINV) % P]
    assert not bad, bad[:5]
    # the addend form with normal operands at their largest limbs
    nrows = [r for r, v in zip(rows, vals) if v < 2 * P and r[8] < (1 << 25)][:1000]
    N = np.array(nrows, dtype=np.int64)
    M = N[::-1].copy()
    out = raw(18, N, M)
    _check_normal(out, 4 * P, 26)
    for i in range(len(nrows)):
        x, y = value(nrows[i]), value(nrows[-1 - i])
        assert value(out[i]) % P == (x * y * RINV - y) % P


def _extreme_rows(bound, n, seed):
    """Carry-only values below `bound` with limbs 0..7 at or near 2^29 - 1
    (or random), the largest column sums such operands allow."""
    rnd = random.Random(seed)
    rows, vals = [], []
    top = (bound - 1) >> (LB * 8)
    while len(rows) < n:
        mode = len(rows) % 3
        low = [MASK if mode == 0 else MASK - rnd.randrange(1 << (8 * mode)) for _ in range(8)]
        if mode == 2 and rnd.random() < 0.5:
            low = [rnd.randrange(1 << LB) for _ in range(8)]
        row = low + [rnd.randrange(top + 1)]
        v = value(row)
        if v < bound:
            rows.append(row)
            vals.append(v)
    return np.array(rows, dtype=np.int64), vals


def check_loose_quotient_products(raw):
    """Products with loose quotient digits (ops 24-29; the mixed addition of
    the accumulation takes all its products in this form): random normal
    operands and carry-only operands at the largest limbs their bounds
    allow, up to 16 p^2 and 32 p^2 for the folded op 28 (16 p^2 for op 29).  Each result must
    equal the product times R^-1 modulo p and be in normal form (op 26:
    carry-only in (0, 4p))."""
    a, b = _operands(3000, 12)
    A = np.array([limbs(v) for v in a], dtype=np.int64)
    B = np.array([limbs(v) for v in b], dtype=np.int64)
    for op, f in {24: lambda x, y: (x * y * RINV) % P, 25: lambda x, y: (x * x * RINV) % P}.items():
        out = raw(op, A, B)
        _check_normal(out)
        bad = [i for i in range(len(a)) if value(out[i]) % P != f(a[i], b[i])]
        assert not bad, (op, bad[:5])
    out = raw(26, A, B)
    _check_normal(out, 4 * P, 26)
    bad = [i for i in range(len(a)) if value(out[i]) % P != (a[i] * b[i] * RINV - b[i]) % P]
    assert not bad, bad[:5]
    # carry-only operands: (< 4p) x (< 4p), (< 4p)^2, (< 8p) x (< 2p), and
    # (< 2p) x 2 (< 4p) with the doubled operand's limbs below 2^30
    R4, v4 = _extreme_rows(4 * P, 2000, 21)
    R8, v8 = _extreme_rows(8 * P, 2000, 22)
    R2, v2 = _extreme_rows(2 * P, 2000, 23)
    keep = [i for i in range(len(v2)) if R2[i, 8] < (1 << 25)]
    R2, v2 = R2[keep], [v2[i] for i in keep]
    cases = [
        (24, R4, R4[::-1].copy(), v4, v4[::-1], lambda x, y: x * y),
        (25, R4, R4, v4, v4, lambda x, y: x * x),
        (24, R8[:len(v2)], R2, v8[:len(v2)], v2, lambda x, y: x * y),
        (27, R2, R4[:len(v2)], v2, v4[:len(v2)], lambda x, y: 2 * x * y),
    ]
    for op, X, Y, vx, vy, f in cases:
        out = raw(op, X, Y)
        _check_normal(out)
        bad = [i for i in range(len(vx)) if value(out[i]) % P != (f(vx[i], vy[i]) * RINV) % P]
        assert not bad, (op, bad[:5])
    # (2a) b - 2 b' b' with one reduction and a fold, a and b below 4p
    Yr = R4[::-1].copy()
    out = raw(28, R4, Yr)
    _check_normal(out)
    vb = v4[::-1]
    bad = [i for i in range(len(v4)) if value(out[i]) % P != (2 * (v4[i] - vb[i]) * vb[i] * RINV) % P]
    assert not bad, bad[:5]
    # a b - b' b' with one reduction and a fold, a and b below 4p
    out = raw(29, R4, Yr)
    _check_normal(out)
    bad = [i for i in range(len(v4)) if value(out[i]) % P != ((v4[i] - vb[i]) * vb[i] * RINV) % P]
    assert not bad, bad[:5]


def check_inversion(raw, n=20000):
    """fe_inv (op 23, divsteps) on carry-only operands below 4p (its input
    range): edge values (0, 1, p - 1, p, 2p - 1, 2^256 - 1, ...), carry-only
    values at the largest limbs and random ones.  The result is x^-1 R for a
    = x R (a^-1 R^2 mod p), 0 for a = 0 (mod p), in normal form, and equal
    modulo p to the Fermat chain's (op 30) on every operand."""
    rnd = random.Random(29)
    edge, _ = _operands(0, 1)
    vals = sorted(set(edge)) + [3 * P, 4 * P - 1, 3 * P + 1, 2**257, 2**257 + 2**256 - 1]
    vals += [rnd.randrange(4 * P) for _ in range(n)]
    vals += [rnd.randrange(2**k) for k in (1, 2, 3, 8, 31, 32, 33, 64, 128, 200, 255) for _ in range(20)]
    rows = [limbs(v) for v in vals if v < 4 * P]
    R4, v4 = _extreme_rows(4 * P, 2000, 30)
    A = np.concatenate([np.array(rows, dtype=np.int64), R4])
    vals = [v for v in vals if v < 4 * P] + list(v4)
    out = raw(23, A, A)
    _check_normal(out)
    bad = [i for i, v in enumerate(vals)
           if value(out[i]) % P != (0 if v % P == 0 else pow(v, -1, P) * R * R % P)]
    assert not bad, [hex(vals[i]) for i in bad[:5]]
    ref = raw(30, A, A)
    _check_normal(ref)
    bad = [i for i in range(len(vals)) if value(out[i]) % P != value(ref[i]) % P]
    assert not bad, [hex(vals[i]) for i in bad[:5]]


def check_signed_limb_normalisation(raw):
    rnd = random.Random(5)
    rows, vals = [], []
    while len(rows) < 4000:
        row = [rnd.randrange(-(1 << 30) + 1, 1 << 30) for _ in range(NL)]
        v = sum(x << (LB * i) for i, x in enumerate(row))
        if 0 <= v < 2**259:
            rows.append(row)
            vals.append(v)
    A = np.array(rows, dtype=np.int64)
    out = raw(10, A, A)
    _check_normal(out)
    assert all(value(out[i]) % P == vals[i] % P for i in range(len(vals)))
