"""Pins of the Paillier oracle (Sec. 2 scheme, Alg. 4 ladder, Alg. 2 / Alg. 3
over ciphertext multiplication) against what the mathematics fixes:

* Alg. 4 returns g^k: checked against Python's built-in modular
  exponentiation, which the oracle's ladder does not use;
* with g = n + 1, g^m = 1 + m n (mod n^2) by the binomial theorem;
* decryption inverts encryption, and a product of ciphertext powers decrypts
  to the sum of the scaled plaintexts (Eq. ahe_6_paillier);
* Alg. 2 reconstruction returns base^v for every vector over {0..2^t-1}^n at
  tiny n, t (exhaustive), with the operation counts of the compression levels;
* schoolbook and Cussen PC-MM agree, and both decrypt to the plaintext
  product A msg mod n (independent of either method).
"""
import itertools
import random

import numpy as np
import pytest

from oracle import paillier as P
from paper_2504_14497_amd import workloads as W


@pytest.fixture(scope="module")
def key():
    return W.paillier_key(11)


@pytest.fixture(scope="module")
def small_key():
    return W.paillier_key(5, bits=256)


def test_key_shape(key):
    n, p, q = key
    assert n == p * q and n.bit_length() == 3072
    assert p.bit_length() == q.bit_length() == 1536 and p != q
    # Fermat witnesses for the factors (the generator used Miller-Rabin)
    for a in (2, 3, 5, 7):
        assert pow(a, p - 1, p) == 1 and pow(a, q - 1, q) == 1


def test_ladder_is_exponentiation(small_key):
    n, _, _ = small_key
    n2 = n * n
    rnd = random.Random(3)
    for t in range(0, 17):
        for _ in range(6):
            k = rnd.randrange(1 << t) if t else 0
            g = rnd.randrange(n2)
            assert P.ladder(g, k, t, n2) == pow(g, k, n2)
    k = rnd.getrandbits(256)
    g = rnd.randrange(n2)
    assert P.ladder(g, k, 256, n2) == pow(g, k, n2)


def test_generator_power_closed_form(small_key):
    n, _, _ = small_key
    n2 = n * n
    for m in (0, 1, 2, 12345, n - 1):
        assert pow(n + 1, m, n2) == (1 + m * n) % n2


def test_encrypt_decrypt_round_trip(key):
    n, p, q = key
    for idx, m in enumerate([0, 1, 2, 255, 65535, 2**31 - 1, n - 1]):
        c = P.encrypt(n, m, seed=9, idx=idx)
        assert 0 < c < n * n
        assert P.decrypt(p, q, c) == m % n
    r = P.nonce(n, 9, 4)
    assert 1 <= r < n and r == P.nonce(n, 9, 4) and r != P.nonce(n, 9, 5)


def test_homomorphic_property(key):
    n, p, q = key
    n2 = n * n
    rnd = random.Random(4)
    ms = [rnd.randrange(1 << 20) for _ in range(5)]
    ss = [rnd.randrange(1 << 8) for _ in range(5)]
    cs = [P.encrypt(n, m, 21, i) for i, m in enumerate(ms)]
    prod = 1
    for c, s in zip(cs, ss):
        prod = prod * pow(c, s, n2) % n2
    assert P.decrypt(p, q, prod) == sum(s * m for s, m in zip(ss, ms)) % n


def test_alg2_reconstruction_exhaustive():
    mod = 1000003  # a prime: the multiplicative group is cyclic of order mod - 1
    base = 5
    mul = lambda x, y: x * y % mod  # noqa: E731
    power = lambda g, s: pow(g, s, mod)  # noqa: E731
    for nvals in range(0, 5):
        for t in range(1, 4):
            for vec in itertools.product(range(1 << t), repeat=nvals):
                for N in (1, 2, 3, 4):
                    out, powers, products = P.alg2_reconstruct(list(vec), N, base, mul, power)
                    assert out == [pow(base, v, mod) for v in vec]
                    # level-N multiplications: the distinct values left after
                    # N - 1 rounds of differencing (zeros dropped each round)
                    cur = sorted(set(v for v in vec if v))
                    lens = [len(cur)]
                    for _ in range(N - 1):
                        d = [cur[0]] + [cur[i] - cur[i - 1] for i in range(1, len(cur))] if cur else []
                        cur = sorted(set(d))
                        lens.append(len(cur))
                    assert powers == lens[-1]
                    assert products == sum(max(x - 1, 0) for x in lens[:-1])


def test_pcmm_methods_agree_and_decrypt_to_the_product(key):
    n, p, q = key
    n2 = n * n
    rng = np.random.default_rng(6)
    A = rng.integers(0, 16, size=(3, 5)).tolist()
    A[1] = [0] * 5          # an all-zero row: the identity ciphertext 1
    A[2][0] = 15
    msg = rng.integers(0, 1 << 16, size=(5, 2)).tolist()
    B = [[P.encrypt(n, msg[k][j], 17, k * 2 + j) for j in range(2)] for k in range(5)]
    Cs = P.pcmm_schoolbook(A, B, n2, 4)
    Cc = P.pcmm_cussen(A, B, n2, 4)
    assert Cs == Cc
    assert Cs[1] == [1, 1]
    want = P.closed_form(A, msg, n)
    for i in range(3):
        for j in range(2):
            assert P.decrypt(p, q, Cs[i][j]) == want[i][j]


def test_pcmm_rejects_out_of_range_plaintexts(small_key):
    n, _, _ = small_key
    with pytest.raises(ValueError):
        P.pcmm_schoolbook([[16]], [[2]], n * n, 4)
    with pytest.raises(ValueError):
        P.pcmm_cussen([[-1]], [[2]], n * n, 4)
