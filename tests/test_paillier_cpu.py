"""Host-side checks of the Paillier PC-MM library (no GPU): the constants the
library derives from a modulus n (n^2, R mod n^2, R^2 mod n^2 for R = 2^6148,
and -(n^2)^-1 mod 2^32, as 29-bit limbs) equal those computed with Python
integers, and bad moduli and arguments are rejected before any device work."""
import ctypes

import numpy as np
import pytest

from paper_2504_14497_amd import pcmm, workloads as W

_VP = ctypes.c_void_p


def _constants(n: int):
    arrs = [np.zeros(256, dtype=np.uint32) for _ in range(3)]
    n0 = ctypes.c_uint32()
    rc = pcmm.lib().pcmm_paillier_diag_constants(n.to_bytes(384, "big"),
                                                 *[a.ctypes.data_as(_VP) for a in arrs], ctypes.byref(n0))
    return rc, arrs, n0.value


def _value(limbs):
    return sum(int(x) << (29 * i) for i, x in enumerate(limbs))


@pytest.mark.parametrize("seed", [11, 12])
def test_modulus_constants(seed):
    n, _, _ = W.paillier_key(seed)
    N = n * n
    rc, (Nl, one, r2), n0 = _constants(n)
    assert rc == 0
    R = 1 << 6148
    assert _value(Nl) == N
    assert _value(one) == R % N
    assert _value(r2) == R * R % N
    assert (N * n0 + 1) % (1 << 32) == 0
    assert all(int(x) < (1 << 29) for a in (Nl, one, r2) for x in a)


def test_bad_moduli_rejected():
    n, _, _ = W.paillier_key(11)
    assert _constants(n + 1)[0] == -1          # even
    assert _constants(n >> 1 | 1)[0] == -1     # 3071 bits
    h = _VP()
    assert pcmm.lib().pcmm_paillier_create((n + 1).to_bytes(384, "big"), ctypes.byref(h)) == -1
    assert pcmm.lib().pcmm_paillier_create(None, ctypes.byref(h)) == -1


def test_workspace_and_argument_checks():
    L = pcmm.lib()
    size = ctypes.c_size_t()
    A = np.array([[1, 2, 3], [0, 0, 15]], dtype=np.uint8)
    assert L.pcmm_paillier_cussen_workspace(A.ctypes.data_as(_VP), 2, 3, 4, 4, None, ctypes.byref(size)) == 0
    assert size.value >= 3 * 4 * 1024                     # B in internal form
    bad = np.array([[16]], dtype=np.uint8)
    assert L.pcmm_paillier_cussen_workspace(bad.ctypes.data_as(_VP), 1, 1, 1, 4, None, ctypes.byref(size)) == -2
    assert L.pcmm_paillier_cussen_workspace(A.ctypes.data_as(_VP), 2, 3, 4, 17, None, ctypes.byref(size)) == -1
    assert L.pcmm_paillier_schoolbook_workspace(2, 3, 4, ctypes.byref(size)) == 0
    assert size.value >= 3 * 4 * 1024 + 2 * 3 * 2
    # null context
    assert L.pcmm_paillier_schoolbook(None, A.ctypes.data_as(_VP), 2, 3, 4, 4, None, None, None, 0, None) == -1
    assert L.pcmm_paillier_encrypt(None, None, 1, 0, 0, None, None) == -1
