"""Paillier PC-MM through the C-ABI (argument marshalling only).

Ciphertexts are residues mod n^2 for a 3072-bit n (Sec. 2, Sec. "Extension
to Paillier Encryption"); on the device a ciphertext is 192 little-endian
32-bit words, matrices row-major, held here in int32 torch tensors of shape
(rows, cols, 192) (the bits of the uint32 words).  Every step runs in the
HIP library; the library must be built (no fallback).
"""
import ctypes

import numpy as np

from . import pcmm
from .pcmm import CussenCfg, CussenStats, PCMMError, _call, _tensor_ptr, _workspace, stream_ptr

_VP = ctypes.c_void_p
WORDS = 192
MODULUS_BYTES = 384


def ints_to_words(vals) -> np.ndarray:
    """Python ints (< 2^6144) -> uint32 array (len, 192), little-endian words."""
    out = np.zeros((len(vals), WORDS), dtype=np.uint32)
    for i, v in enumerate(vals):
        out[i] = np.frombuffer(int(v).to_bytes(4 * WORDS, "little"), dtype=np.uint32)
    return out


def words_to_ints(arr) -> list:
    arr = np.ascontiguousarray(np.asarray(arr).reshape(-1, WORDS)).view(np.uint32)
    return [int.from_bytes(row.tobytes(), "little") for row in arr]


def upload(vals, rows: int, cols: int, device="cuda"):
    import torch
    w = ints_to_words(vals).view(np.int32).reshape(rows, cols, WORDS)
    return torch.from_numpy(w.copy()).to(device)


def download(t) -> list:
    return words_to_ints(t.detach().cpu().numpy().view(np.uint32))


def _plain_A(A, bits: int):
    """A as the library reads it: unsigned, uint8 up to 8 bits, uint16 for 9..16."""
    A = np.ascontiguousarray(A)
    if A.dtype not in (np.uint8, np.uint16):
        raise TypeError("A must be uint8 or uint16 (unsigned plaintexts)")
    if bits > 8 and A.dtype == np.uint8:
        A = A.astype(np.uint16)
    elif bits <= 8 and A.dtype == np.uint16:
        if A.size and A.max() > 255:
            raise PCMMError(-2, "plaintext entries outside the declared bit-width")
        A = A.astype(np.uint8)
    return A


class Paillier:
    """Context of a public modulus n (3072-bit, odd)."""

    def __init__(self, n: int):
        if n.bit_length() != 8 * MODULUS_BYTES:
            raise PCMMError(-1, "pcmm_paillier_create (n must have 3072 bits)")
        self.n = n
        self.n2 = n * n
        h = _VP()
        _call("pcmm_paillier_create", ctypes.c_char_p(n.to_bytes(MODULUS_BYTES, "big")), ctypes.byref(h))
        self._h = h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            pcmm.lib().pcmm_paillier_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def encrypt(self, msg, seed: int, idx0: int = 0, stream=None):
        """Ciphertexts of the int32 messages `msg` (a device tensor or array of
        shape (rows, cols), values in [0, 2^31)); returns (rows, cols, 192)."""
        import torch
        m = torch.as_tensor(msg, dtype=torch.int32).to("cuda").contiguous()
        rows, cols = m.shape
        out = torch.empty((rows, cols, WORDS), dtype=torch.int32, device="cuda")
        _call("pcmm_paillier_encrypt", self._h, _tensor_ptr(m), rows * cols, seed, idx0, _tensor_ptr(out),
              stream_ptr(stream))
        out._keep = (m,)
        return out

    def schoolbook(self, A, bits: int, B, stream=None, workspace=None):
        import torch
        A = _plain_A(A, bits)
        m, n = A.shape
        l = B.shape[1]
        if B.shape[0] != n:
            raise PCMMError(-1, "pcmm_paillier_schoolbook (B rows != A cols)")
        need = ctypes.c_size_t()
        _call("pcmm_paillier_schoolbook_workspace", m, n, l, ctypes.byref(need))
        ws = workspace if workspace is not None else _workspace(need.value)
        C = torch.empty((m, l, WORDS), dtype=torch.int32, device="cuda")
        _call("pcmm_paillier_schoolbook", self._h, A.ctypes.data_as(_VP), m, n, l, bits, _tensor_ptr(B),
              _tensor_ptr(C), _tensor_ptr(ws), ws.numel(), stream_ptr(stream))
        C._keep = (ws,)
        return C

    def cussen_workspace_bytes(self, A, bits: int, l: int, cfg: CussenCfg = None) -> int:
        A = _plain_A(A, bits)
        m, n = A.shape
        need = ctypes.c_size_t()
        _call("pcmm_paillier_cussen_workspace", A.ctypes.data_as(_VP), m, n, l, bits,
              ctypes.byref(cfg) if cfg is not None else None, ctypes.byref(need))
        return need.value

    def cussen(self, A, bits: int, B, cfg: CussenCfg = None, stream=None, workspace=None, out=None):
        """Cussen PC-MM; returns (C, stats dict)."""
        import torch
        A = _plain_A(A, bits)
        m, n = A.shape
        l = B.shape[1]
        if B.shape[0] != n:
            raise PCMMError(-1, "pcmm_paillier_cussen (B rows != A cols)")
        ws = workspace if workspace is not None else _workspace(self.cussen_workspace_bytes(A, bits, l, cfg))
        C = out if out is not None else torch.empty((m, l, WORDS), dtype=torch.int32, device="cuda")
        st = CussenStats()
        _call("pcmm_paillier_cussen", self._h, A.ctypes.data_as(_VP), m, n, l, bits, _tensor_ptr(B),
              _tensor_ptr(C), ctypes.byref(cfg) if cfg is not None else None, _tensor_ptr(ws), ws.numel(),
              ctypes.byref(st), stream_ptr(stream))
        C._keep = (ws,)
        return C, st.as_dict()

    def diag(self, op: int, a_vals, b_vals, stream=None) -> list:
        """Element-wise op (0 raw Montgomery product, 1 product, 2 a^(b mod
        2^32), 3 a^n) on lists of ints; returns ints."""
        import torch
        cnt = len(a_vals)
        a = upload(a_vals, cnt, 1)
        b = upload(b_vals, cnt, 1)
        out = torch.empty_like(a)
        _call("pcmm_paillier_diag", self._h, op, _tensor_ptr(a), _tensor_ptr(b), _tensor_ptr(out), cnt,
              stream_ptr(stream))
        torch.cuda.synchronize()
        return download(out)
