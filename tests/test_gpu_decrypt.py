"""Full decryption on the GPU (Sec. 2.4): the bounded discrete logarithm by
baby-step giant-step returns exactly the encrypted integers within the
bound, and INT64_MIN outside it; an encrypted linear layer decrypts to the
exact integer product."""
import numpy as np
import pytest

from gpu_helpers import log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_14497_amd import pcmm
    pcmm.lib()
    return pcmm


def test_decrypt_boundaries(dev):
    import torch
    log2 = 10
    s = 1 << log2
    stride = 2 * s - 1
    bound = 5 * stride + 17
    table = dev.DlogTable(log2)
    vals = [0, 1, -1, 2, -2, s - 1, -(s - 1), s, -s, stride, -stride, stride + 1, -(stride + 1),
            bound, -bound, bound - 1, 3 * stride - s + 1, -(3 * stride) + s - 1, 12345 % bound, -777]
    rng = np.random.default_rng(1)
    vals += [int(x) for x in rng.integers(-bound, bound + 1, size=60)]
    out_of_range = [bound + 1, -(bound + 1), 10 * bound, -(10 * bound)]
    msg = np.array(vals + out_of_range, dtype=np.int32).reshape(1, -1)
    sk, pk = dev.keygen(77)
    C = dev.encrypt(pk, msg, 77)
    log("decrypt", msg.size)
    m = dev.decrypt(sk, C, bound, table)
    torch.cuda.synchronize()
    got = m.cpu().numpy().ravel()
    want = np.array(vals + [np.iinfo(np.int64).min] * len(out_of_range), dtype=np.int64)
    assert (got == want).all(), [(int(a), int(b)) for a, b in zip(got, want) if a != b][:5]


def test_encrypted_linear_layer_decrypts_to_integer_product(dev):
    import torch
    rng = np.random.default_rng(3)
    W = rng.integers(-128, 128, size=(24, 40)).astype(np.int8)
    msg = rng.integers(0, 256, size=(40, 3)).astype(np.int32)
    sk, pk = dev.keygen(78)
    X = dev.encrypt(pk, msg, 78)
    C, _ = dev.cussen(W, 8, X, cfg=dev.cussen_cfg(4, dev.GROUP_AUTO))
    bound = 40 * 128 * 255
    table = dev.DlogTable(14)
    log("linear layer decrypt")
    m = dev.decrypt(sk, C, bound, table)
    torch.cuda.synchronize()
    want = W.astype(np.int64) @ msg.astype(np.int64)
    assert (m.cpu().numpy() == want).all()
    # the schoolbook result decrypts the same way
    Cs = dev.schoolbook(W, 8, X)
    assert (dev.decrypt(sk, Cs, bound, table).cpu().numpy() == want).all()


def test_decrypt_rejects_bad_arguments(dev):
    sk, pk = dev.keygen(79)
    C = dev.encrypt(pk, np.zeros((1, 2), dtype=np.int32), 79)
    table = dev.DlogTable(6)
    with pytest.raises(dev.PCMMError):
        dev.decrypt(sk, C, 1 << 45, table)  # giant multiples would exceed 32 bits
    with pytest.raises(dev.PCMMError):
        dev.DlogTable(30)
