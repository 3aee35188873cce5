"""Pins of the oracle's EC-ElGamal and PC-MM (Sec. 2.4, Sec. 3.1, Alg. 3).

Every correct method yields the same group elements (the group is abelian and
the arithmetic exact), so schoolbook, Cussen and the closed form of
Eq. (ahe_5_elgamal) must agree byte for byte; brute force (repeated addition)
decides on tiny inputs; decryption must return (A.B) G with A.B computed in
exact integers.
"""
import itertools
import random

import numpy as np
import pytest

from paper_2504_14497_amd import workloads as W


def _random_cts(orc, rows, cols, rnd):
    p, b, gx, gy, q = orc.curve_params()
    G = orc.generator()
    ct = np.zeros((rows, cols, 128), dtype=np.uint8)
    for r in range(rows):
        for c in range(cols):
            for h in range(2):
                ct[r, c, 64 * h:64 * h + 64] = np.frombuffer(
                    orc.ladder_big(rnd.randrange(1, q), G), dtype=np.uint8)
    return ct


def _pt(arr):
    return bytes(np.asarray(arr, dtype=np.uint8))


def _brute(orc, A, B):
    """C_ij = sum_k a_ik B_kj by repeated addition (signed: add the negation)."""
    m, n = A.shape
    l = B.shape[1]
    C = np.zeros((m, l, 128), dtype=np.uint8)
    for i in range(m):
        for j in range(l):
            for h in range(2):
                acc = orc.INF
                for k in range(n):
                    a = int(A[i, k])
                    P_ = _pt(B[k, j, 64 * h:64 * h + 64])
                    if a < 0:
                        P_ = orc.pt_neg(P_)
                    for _ in range(abs(a)):
                        acc = orc.pt_add(acc, P_)
                C[i, j, 64 * h:64 * h + 64] = np.frombuffer(acc, dtype=np.uint8)
    return C


def test_every_2x2_matrix_in_0_3(orc):
    rnd = random.Random(21)
    B = _random_cts(orc, 2, 2, rnd)
    for vals in itertools.product(range(4), repeat=4):
        A = np.array(vals, dtype=np.uint8).reshape(2, 2)
        want = _brute(orc, A, B)
        assert (orc.pcmm_schoolbook(A, B, nthreads=1) == want).all(), vals
        assert (orc.pcmm_cussen(A, B, nthreads=1) == want).all(), vals


@pytest.mark.parametrize("shape", [(1, 1, 1), (3, 3, 3), (2, 5, 3), (5, 2, 1)])
def test_small_shapes_brute_force(orc, shape):
    m, n, l = shape
    rnd = random.Random(sum(shape))
    rng = np.random.default_rng(sum(shape))
    B = _random_cts(orc, n, l, rnd)
    for A in (rng.integers(0, 16, size=(m, n)).astype(np.uint8),
              rng.integers(-8, 8, size=(m, n)).astype(np.int8)):
        want = _brute(orc, A, B)
        assert (orc.pcmm_schoolbook(A, B) == want).all()
        for N in (1, 2, 4):
            assert (orc.pcmm_cussen(A, B, N=N) == want).all()


def test_special_matrices(orc):
    rnd = random.Random(4)
    n = 4
    B = _random_cts(orc, n, 3, rnd)
    I = np.eye(n, dtype=np.int8)
    for method in (orc.pcmm_schoolbook, orc.pcmm_cussen):
        assert (method(I.astype(np.uint8), B) == B).all()                    # A = I
        assert (method(np.zeros((2, n), np.uint8), B) == 0).all()            # A = 0 -> infinity
        C2 = method((2 * I).astype(np.uint8), B)                             # A = 2I -> 2B
        Cm = method(-I, B)                                                   # A = -I -> -B
        for k in range(n):
            for j in range(3):
                for h in range(2):
                    P_ = _pt(B[k, j, 64 * h:64 * h + 64])
                    assert _pt(C2[k, j, 64 * h:64 * h + 64]) == orc.pt_dbl(P_)
                    assert _pt(Cm[k, j, 64 * h:64 * h + 64]) == orc.pt_neg(P_)
        E = np.zeros((3, n), np.uint8)
        E[1, 2] = 1                                                          # A = e_1 e_2^T
        C = method(E, B)
        assert (C[1] == B[2]).all() and (C[0] == 0).all() and (C[2] == 0).all()


def test_forced_exceptional_cases(orc):
    # equal ciphertexts down a column: the accumulator meets P = Q; opposite
    # ciphertexts: it meets P = -Q.
    rnd = random.Random(9)
    B = _random_cts(orc, 4, 2, rnd)
    B[1] = B[0]
    for j in range(2):
        for h in range(2):
            B[2, j, 64 * h:64 * h + 64] = np.frombuffer(
                orc.pt_neg(_pt(B[0, j, 64 * h:64 * h + 64])), dtype=np.uint8)
    A = np.array([[1, 1, 0, 0], [1, 0, 1, 0], [3, 3, 6, 1], [2, 0, 2, 5]], dtype=np.int8)
    want = _brute(orc, A, B)
    assert (orc.pcmm_schoolbook(A, B) == want).all()
    assert (orc.pcmm_cussen(A, B) == want).all()
    assert (want[1] == 0).all()      # B0 + (-B0) = infinity
    for j in range(2):
        for h in range(2):
            assert _pt(want[0, j, 64 * h:64 * h + 64]) == orc.pt_dbl(_pt(B[0, j, 64 * h:64 * h + 64]))


def test_encrypt_decrypt_roundtrip(orc):
    sk, pk = orc.keygen(123)
    G = orc.generator()
    assert orc.ladder_big(sk, G) == pk
    msg = np.array([[0, 1, 2], [15, 255, 7]], dtype=np.int32)
    ct = orc.encrypt(pk, msg, seed=123)
    assert ct.shape == (2, 3, 128)
    pts = orc.decrypt_to_points(sk, ct)
    for (r, c), m in np.ndenumerate(msg):
        assert _pt(pts[r, c]) == orc.repeated_add(int(m), G)
        # C1 = rG with r from the nonce derivation
        rr = orc.scalar_from_seed(123, 1, r * 3 + c)
        assert _pt(ct[r, c, :64]) == orc.ladder_big(rr, G)
    neg = orc.encrypt(pk, np.array([-5], dtype=np.int32), seed=1)
    assert _pt(orc.decrypt_to_points(sk, neg)[0]) == orc.pt_neg(orc.repeated_add(5, G))


@pytest.mark.parametrize("signed", [False, True])
def test_closed_form_and_decryption(orc, signed):
    shape = W.PCMMShape(5, 6, 4, 8 if signed else 4, signed, 8, seed=17 if signed else 18)
    A, msg = W.make_inputs(shape)
    sk, pk = orc.keygen(shape.seed)
    B = orc.encrypt(pk, msg, shape.seed)
    C_s = orc.pcmm_schoolbook(A, B)
    C_c = orc.pcmm_cussen(A, B)
    assert (C_s == C_c).all()
    ii, jj = np.meshgrid(np.arange(shape.m), np.arange(shape.l), indexing="ij")
    C_f = orc.pcmm_closed_form(A, shape.l, sk, msg, shape.seed, ii.ravel(), jj.ravel())
    assert (C_f.reshape(C_c.shape) == C_c).all()
    # homomorphic check: Dec(C) = (A.B) G with A.B exact in int64
    AB = A.astype(np.int64) @ msg.astype(np.int64)
    pts = orc.decrypt_to_points(sk, C_c)
    p, b, gx, gy, q = orc.curve_params()
    G = orc.generator()
    for (i, j), v in np.ndenumerate(AB):
        assert _pt(pts[i, j]) == orc.ladder_big(int(v) % q, G)
    # a transposed operand would not match
    if shape.m == shape.n:
        assert not (orc.pcmm_cussen(np.ascontiguousarray(A.T), B) == C_c).all()


@pytest.mark.parametrize("bits,signed", [(12, True), (16, False), (16, True)])
def test_wide_plaintexts_closed_form_and_decryption(orc, bits, signed):
    """t up to 16 (Tab. A1/A2 and the vector experiments use t in 4..16):
    schoolbook = Cussen = the closed form, and decryption gives (A.B) G."""
    shape = W.PCMMShape(4, 5, 2, bits, signed, 8, seed=40 + bits + signed)
    A, msg = W.make_inputs(shape)
    assert A.dtype == (np.int16 if signed else np.uint16)
    sk, pk = orc.keygen(shape.seed)
    B = orc.encrypt(pk, msg, shape.seed)
    C_c = orc.pcmm_cussen(A, B)
    assert (orc.pcmm_schoolbook(A, B) == C_c).all()
    ii, jj = np.meshgrid(np.arange(shape.m), np.arange(shape.l), indexing="ij")
    C_f = orc.pcmm_closed_form(A, shape.l, sk, msg, shape.seed, ii.ravel(), jj.ravel())
    assert (C_f.reshape(C_c.shape) == C_c).all()
    AB = A.astype(np.int64) @ msg.astype(np.int64)
    pts = orc.decrypt_to_points(sk, C_c)
    p, b, gx, gy, q = orc.curve_params()
    G = orc.generator()
    for (i, j), v in np.ndenumerate(AB):
        assert _pt(pts[i, j]) == orc.ladder_big(int(v) % q, G)


def test_schoolbook_equals_cussen_every_round_count(orc):
    rnd = random.Random(31)
    rng = np.random.default_rng(31)
    B = _random_cts(orc, 20, 2, rnd)
    A = rng.integers(0, 16, size=(12, 20)).astype(np.uint8)
    ref = orc.pcmm_schoolbook(A, B)
    for N in (1, 2, 3, 4, 5):
        assert (orc.pcmm_cussen(A, B, N=N) == ref).all()
    # a subset of output columns computes only those columns
    part = orc.pcmm_cussen(A, B, cols=[1])
    assert (part[:, 1] == ref[:, 1]).all() and (part[:, 0] == 0).all()
