"""GPU parity of KeyGen / Encrypt / Decrypt-to-point / normalise (Sec. 2.4)."""
import numpy as np
import pytest

from gpu_helpers import log, random_points

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_14497_amd import pcmm
    pcmm.lib()
    return pcmm


def test_keygen_matches_oracle(dev, orc):
    for seed in (1, 34, 2**63 + 5):
        log("keygen seed", seed)
        sk, pk = dev.keygen(seed)
        osk, opk = orc.keygen(seed)
        assert int.from_bytes(sk, "big") == osk == orc.scalar_from_seed(seed, 0, 0)
        assert pk == opk


def test_encrypt_matches_oracle(dev, orc):
    osk, opk = orc.keygen(7)
    msg = np.array([[0, 1, 2, 3, 15, 16, 255, -1, -255, 2**31 - 1, -2**31]] * 6, dtype=np.int32)
    msg[1] += 3
    for seed, idx0 in ((7, 0), (8, 1000)):
        log("encrypt", msg.shape, seed, idx0)
        ct = dev.encrypt(opk, msg, seed, idx0=idx0).to_host()
        want = orc.encrypt(opk, msg, seed, idx0=idx0)
        assert (ct == want).all()


def test_encrypt_ragged_sizes(dev, orc):
    osk, opk = orc.keygen(3)
    for rows, cols in ((1, 1), (1, 65), (17, 15)):
        msg = np.random.default_rng(rows * cols).integers(0, 256, size=(rows, cols)).astype(np.int32)
        log("encrypt ragged", rows, cols)
        ct = dev.encrypt(opk, msg, 11).to_host()
        assert (ct == orc.encrypt(opk, msg, 11)).all()


def test_encrypt_rejects_bad_public_key(dev, orc):
    osk, opk = orc.keygen(3)
    bad = bytearray(opk)
    bad[63] ^= 1
    with pytest.raises(dev.PCMMError) as ei:
        dev.encrypt(bytes(bad), np.zeros((1, 1), np.int32), 1)
    assert ei.value.code == -5
    with pytest.raises(dev.PCMMError) as ei:
        dev.encrypt(bytes(64), np.zeros((1, 1), np.int32), 1)  # infinity is not a key
    assert ei.value.code == -5


def test_decrypt_to_points_matches_oracle(dev, orc):
    osk, opk = orc.keygen(5)
    msg = np.arange(-20, 44, dtype=np.int32).reshape(8, 8)
    ct = orc.encrypt(opk, msg, 5)
    log("decrypt", msg.shape)
    C = dev.DevPoints.from_host(ct.reshape(-1, 128), 8, 8, 2)
    M = dev.decrypt_to_points(osk.to_bytes(32, "big"), C).to_host()
    want = orc.decrypt_to_points(osk, ct)
    assert (M == want).all()
    G = orc.generator()
    assert bytes(M[2, 4]) == orc.INF  # m = 0 -> infinity
    assert bytes(M[2, 5]) == G  # m = 1


def test_normalize_matches_affine_path(dev, orc):
    # Jacobian points from the GPU schoolbook, normalised by pcmm_normalize,
    # must equal the affine output of the same call; both equal the oracle.
    pts = random_points(orc, 2 * 5 * 3, 13)
    B = np.frombuffer(b"".join(pts), dtype=np.uint8).reshape(5, 3, 128)
    A = np.random.default_rng(13).integers(0, 16, size=(4, 5)).astype(np.uint8)
    A[2] = 0  # a row of identities
    Bd = dev.DevPoints.from_host(B.reshape(-1, 128), 5, 3, 2)
    log("normalize")
    Cj = dev.schoolbook(A, 4, Bd, c_form=dev.JACOBIAN)
    Ca = dev.schoolbook(A, 4, Bd, c_form=dev.AFFINE).to_host()
    Cn = dev.normalize(Cj).to_host()
    assert (Cn == Ca).all()
    Ci = dev.normalize(Cj, inplace=True).to_host()
    assert (Ci == Ca).all()
    assert (Ca == orc.pcmm_schoolbook(A, B)).all()
    assert (Ca[2] == 0).all()
