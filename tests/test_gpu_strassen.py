"""GPU parity of Strassen PC-MM (Sec. 3.1): the block recursion (ciphertext
block sums on the GPU, plaintext block sums exact on the host, schoolbook
leaves) equals the oracle bit-exactly, on padded ragged shapes, at several
depths, signed and unsigned, affine and Jacobian output."""
import numpy as np
import pytest

from gpu_helpers import log, random_cts

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_14497_amd import pcmm
    pcmm.lib()
    return pcmm


@pytest.mark.parametrize("m,n,l,bits,signed,depth", [
    (8, 8, 8, 4, False, 1),
    (16, 12, 10, 4, False, 2),
    (37, 23, 19, 3, True, 2),     # ragged: padded to multiples of 4
    (20, 20, 20, 8, True, 3),
    (9, 30, 5, 12, True, 1),      # 12-bit plaintexts, one level
])
def test_strassen_vs_oracle(dev, orc, m, n, l, bits, signed, depth):
    import torch
    rng = np.random.default_rng(m * 131 + n)
    lo, hi = (-(1 << (bits - 1)), 1 << (bits - 1)) if signed else (0, 1 << bits)
    dt = (np.int8 if signed else np.uint8) if bits <= 8 else (np.int16 if signed else np.uint16)
    A = rng.integers(lo, hi, size=(m, n)).astype(dt)
    A[0, :] = hi - 1
    B = random_cts(orc, n, l, 1400 + m)
    Bd = dev.DevPoints.from_host(B.reshape(-1, 128), n, l, 2)
    ref = orc.pcmm_cussen(A, B)
    log("strassen", m, n, l, bits, signed, depth)
    C, st = dev.strassen(A, bits, Bd, depth=depth)
    torch.cuda.synchronize()
    assert st["depth"] == depth and st["leaves"] == 7 ** depth
    assert (C.to_host() == ref).all()
    Cj, _ = dev.strassen(A, bits, Bd, c_form=dev.JACOBIAN, depth=depth)
    assert (dev.normalize(Cj).to_host() == ref).all()


def test_strassen_auto_depth_and_errors(dev, orc):
    import torch
    rng = np.random.default_rng(5)
    A = rng.integers(0, 16, size=(10, 6)).astype(np.uint8)
    B = random_cts(orc, 6, 4, 1500)
    Bd = dev.DevPoints.from_host(B.reshape(-1, 128), 6, 4, 2)
    C, st = dev.strassen(A, 4, Bd)           # small: no levels, schoolbook
    torch.cuda.synchronize()
    assert st["depth"] == 0 and (C.to_host() == orc.pcmm_cussen(A, B)).all()
    W = np.full((4, 6), 65535, dtype=np.uint16)   # leaf sums would exceed 16-bit signed
    with pytest.raises(dev.PCMMError) as ei:
        dev.strassen(W, 16, Bd, depth=1)
    assert ei.value.code == -2
