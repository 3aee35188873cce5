"""Paillier PC-MM on the GPU (Sec. "Extension to Paillier Encryption") against
the Python-integer oracle, bit for bit:

* the wavefront arithmetic mod n^2 (Montgomery product with R = 2^6148, the
  full product, Alg. 4 powers with 32-bit and 3072-bit exponents);
* encryption with the counter-derived nonces;
* schoolbook and Cussen PC-MM (N = 1..4 rounds, column groups 1..4, 2- to
  16-bit plaintexts, zero rows and columns, an empty inner dimension) equal
  the oracle's schoolbook result, and decrypt to A msg mod n.
"""
import random

import numpy as np
import pytest

from gpu_helpers import log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pl():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_14497_amd import paillier, workloads as W
    n, p, q = W.paillier_key(11)
    ctx = paillier.Paillier(n)
    return paillier, ctx, (n, p, q)


def test_arithmetic_mod_n2(pl):
    paillier, ctx, (n, p, q) = pl
    N = n * n
    R = 1 << 6148
    rnd = random.Random(5)
    a = [rnd.randrange(N) for _ in range(37)] + [0, 1, N - 1]
    b = [rnd.randrange(N) for _ in range(37)] + [N - 1, N - 1, N - 1]
    log("paillier diag 0/1", len(a))
    assert ctx.diag(0, a, b) == [x * y * pow(R, -1, N) % N for x, y in zip(a, b)]
    assert ctx.diag(1, a, b) == [x * y % N for x, y in zip(a, b)]
    e = [rnd.randrange(1 << 32) for _ in range(len(a))]
    e[0], e[1] = 0, 1
    log("paillier diag 2")
    assert ctx.diag(2, a, e) == [pow(x, k, N) for x, k in zip(a, e)]
    log("paillier diag 3")
    assert ctx.diag(3, a[:6], b[:6]) == [pow(x, n, N) for x in a[:6]]


def test_encrypt_matches_oracle(pl):
    import torch
    from oracle import paillier as P
    paillier, ctx, (n, p, q) = pl
    msg = np.array([[0, 1, 2, 255], [65535, 2**31 - 1, 12345, 7]], dtype=np.int32)
    log("paillier encrypt", msg.size)
    ct = ctx.encrypt(torch.from_numpy(msg), seed=21, idx0=5)
    torch.cuda.synchronize()
    got = paillier.download(ct)
    want = [P.encrypt(n, int(m), 21, 5 + e) for e, m in enumerate(msg.ravel())]
    assert got == want
    assert [P.decrypt(p, q, c) for c in got] == [int(m) for m in msg.ravel()]


def _case(rng, m, k, l, bits, zero_row=False, zero_col=False):
    A = rng.integers(0, 1 << bits, size=(m, k), dtype=np.int64)
    if zero_row and m > 1:
        A[1] = 0
    if zero_col and k > 1:
        A[:, 0] = 0
    return A.astype(np.uint16 if bits > 8 else np.uint8)


@pytest.mark.parametrize("m,k,l,bits,N,g", [(3, 5, 2, 4, 4, 1), (7, 6, 3, 8, 4, 1), (5, 9, 2, 4, 2, 2),
                                            (4, 7, 2, 2, 1, 3), (6, 4, 2, 12, 3, 1), (9, 11, 1, 4, 4, 2),
                                            (5, 6, 2, 16, 4, 1), (6, 5, 2, 3, 4, 4)])
def test_pcmm_vs_oracle(pl, m, k, l, bits, N, g):
    import torch
    from oracle import paillier as P
    paillier, ctx, (n, p, q) = pl
    n2 = n * n
    rng = np.random.default_rng(m * 100 + k)
    A = _case(rng, m, k, l, bits, zero_row=True, zero_col=True)
    msg = rng.integers(0, 1 << 16, size=(k, l)).astype(np.int32)
    B = ctx.encrypt(torch.from_numpy(msg), seed=31, idx0=0)
    cfg = paillier.pcmm.cussen_cfg(N, g)
    log("paillier pcmm", m, k, l, bits, N, g)
    Cc, st = ctx.cussen(A, bits, B, cfg=cfg)
    Cs = ctx.schoolbook(A, bits, B)
    torch.cuda.synchronize()
    Bi = paillier.download(B)
    Bmat = [Bi[r * l:(r + 1) * l] for r in range(k)]
    want = P.pcmm_schoolbook(A.tolist(), Bmat, n2, bits)
    flat = [x for row in want for x in row]
    assert paillier.download(Cs) == flat
    assert paillier.download(Cc) == flat
    assert st["group"] == g
    # the closed form: every output decrypts to (A msg)_ij mod n
    closed = P.closed_form(A.tolist(), msg.tolist(), n)
    for (i, j) in [(0, 0), (1, l - 1), (m - 1, 0)]:
        assert P.decrypt(p, q, want[i][j]) == closed[i][j]


def test_pcmm_degenerate_shapes(pl):
    import torch
    paillier, ctx, (n, p, q) = pl
    # empty inner dimension: every output is the identity ciphertext 1
    B = torch.empty((0, 3, 192), dtype=torch.int32, device="cuda")
    A = np.zeros((2, 0), dtype=np.uint8)
    Cc, _ = ctx.cussen(A, 4, B)
    Cs = ctx.schoolbook(A, 4, B)
    torch.cuda.synchronize()
    assert paillier.download(Cc) == [1] * 6 and paillier.download(Cs) == [1] * 6
    # an all-zero A: identity outputs through the kernels
    msg = np.arange(6, dtype=np.int32).reshape(2, 3)
    B = ctx.encrypt(torch.from_numpy(msg), seed=3)
    A = np.zeros((4, 2), dtype=np.uint8)
    Cc, _ = ctx.cussen(A, 4, B)
    Cs = ctx.schoolbook(A, 4, B)
    torch.cuda.synchronize()
    assert paillier.download(Cc) == [1] * 12 and paillier.download(Cs) == [1] * 12
    # out-of-range plaintexts are rejected on the host
    with pytest.raises(paillier.PCMMError) as ei:
        ctx.cussen(np.array([[16]], dtype=np.uint8), 4, B[:1, :1].contiguous())
    assert ei.value.code == -2


def test_pcmm_benchmark_shape_sampled(pl):
    """The benchmark's 64 x 64 x 64 4-bit shape: Cussen equals schoolbook on
    every output; sampled outputs equal the oracle's and decrypt to A msg."""
    import torch
    from oracle import paillier as P
    from paper_2504_14497_amd import workloads as W
    paillier, ctx, (n, p, q) = pl
    n2 = n * n
    rng = W.rng_for(43)
    A = W.gen_plain_matrix(rng, 64, 64, 4, False)
    msg = W.paillier_messages(rng, 64, 64, 16)
    B = ctx.encrypt(torch.from_numpy(msg), seed=43)
    log("paillier pcmm 64^3")
    Cc, _ = ctx.cussen(A, 4, B)
    Cs = ctx.schoolbook(A, 4, B)
    torch.cuda.synchronize()
    assert torch.equal(Cc, Cs)
    Bi = paillier.download(B)
    Ci = paillier.download(Cc)
    for (i, j) in [(0, 0), (63, 63), (5, 40), (31, 7), (62, 1)]:
        col = [[Bi[k * 64 + j]] for k in range(64)]
        want = P.pcmm_schoolbook(A[i:i + 1].tolist(), col, n2, 4)[0][0]
        assert Ci[i * 64 + j] == want
        assert P.decrypt(p, q, want) == int(A[i].astype(np.int64) @ msg[:, j].astype(np.int64)) % n
