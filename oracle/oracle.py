"""ctypes wrapper around the C oracle (``liboracle.so``).

TEST INFRASTRUCTURE ONLY.  Byte conventions: scalars and field elements are
32-byte big-endian; points are 64 bytes x || y (affine, infinity = 64 zero
bytes); ciphertexts are 128 bytes C1 || C2.  Arrays are numpy uint8 arrays of
shape (..., 64) or (..., 128).
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

INF = bytes(64)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(_LIB_PATH)
        u8p = ctypes.c_char_p
        vp = ctypes.c_void_p
        L.oracle_mod_op.argtypes = [ctypes.c_int, ctypes.c_int, u8p, u8p, vp]
        L.oracle_curve_params.argtypes = [vp]
        L.oracle_curve_params.restype = None
        L.oracle_pt_add.argtypes = [u8p, u8p, vp]
        L.oracle_pt_dbl.argtypes = [u8p, vp]
        L.oracle_pt_neg.argtypes = [u8p, vp]
        L.oracle_on_curve.argtypes = [u8p]
        L.oracle_ladder_small.argtypes = [ctypes.c_uint64, ctypes.c_int, u8p, vp]
        L.oracle_ladder_big.argtypes = [u8p, u8p, vp]
        L.oracle_repeated_add.argtypes = [ctypes.c_uint64, u8p, vp]
        L.oracle_scalar_from_seed.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64, vp]
        L.oracle_scalar_from_seed.restype = None
        L.oracle_keygen.argtypes = [ctypes.c_uint64, vp, vp]
        L.oracle_encrypt.argtypes = [u8p, vp, ctypes.c_int64, ctypes.c_uint64, ctypes.c_int64, vp,
                                     ctypes.c_int]
        L.oracle_encrypt_indexed.argtypes = [u8p, vp, vp, ctypes.c_int64, ctypes.c_uint64, vp,
                                             ctypes.c_int]
        L.oracle_decrypt_to_points.argtypes = [u8p, vp, ctypes.c_int64, vp, ctypes.c_int]
        L.oracle_alg2_plain.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int64, vp, vp, vp,
                                        vp]
        L.oracle_alg2_point.argtypes = [vp, ctypes.c_int, ctypes.c_int, u8p, vp]
        L.oracle_pcmm_schoolbook.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                             vp, vp, vp, ctypes.c_int, ctypes.c_int]
        L.oracle_pcmm_cussen.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                         vp, vp, vp, ctypes.c_int, ctypes.c_int]
        L.oracle_pcmm_closed_form.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                              u8p, vp, ctypes.c_uint64, vp, vp,
                                              ctypes.c_int, vp, ctypes.c_int]
        _lib = L
    return _lib


def default_threads():
    return max(1, min(os.cpu_count() or 1, 16))


def _ptr(arr):
    return arr.ctypes.data_as(ctypes.c_void_p)


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"oracle {what} failed with code {rc}")


def _b32(x: int) -> bytes:
    return int(x).to_bytes(32, "big")


# ---------------------------------------------------------------- arithmetic

MOD_P, MOD_Q = 0, 1
OP_ADD, OP_SUB, OP_MUL, OP_INV, OP_NEG = range(5)


def mod_op(mod: int, op: int, a: int, b: int = 0) -> int:
    out = ctypes.create_string_buffer(32)
    _check(lib().oracle_mod_op(mod, op, _b32(a), _b32(b), out), "mod_op")
    return int.from_bytes(out.raw, "big")


def curve_params():
    """(p, b, Gx, Gy, q) as Python ints."""
    out = ctypes.create_string_buffer(160)
    lib().oracle_curve_params(out)
    raw = out.raw
    return tuple(int.from_bytes(raw[32 * i:32 * i + 32], "big") for i in range(5))


def generator() -> bytes:
    _, _, gx, gy, _ = curve_params()
    return _b32(gx) + _b32(gy)


def point(x: int, y: int) -> bytes:
    return _b32(x) + _b32(y)


def coords(P: bytes):
    """(x, y) as ints, or None for infinity."""
    if P == INF:
        return None
    return int.from_bytes(P[:32], "big"), int.from_bytes(P[32:], "big")


def pt_add(P: bytes, Q: bytes) -> bytes:
    out = ctypes.create_string_buffer(64)
    _check(lib().oracle_pt_add(P, Q, out), "pt_add")
    return out.raw


def pt_dbl(P: bytes) -> bytes:
    out = ctypes.create_string_buffer(64)
    _check(lib().oracle_pt_dbl(P, out), "pt_dbl")
    return out.raw


def pt_neg(P: bytes) -> bytes:
    out = ctypes.create_string_buffer(64)
    _check(lib().oracle_pt_neg(P, out), "pt_neg")
    return out.raw


def on_curve(P: bytes) -> bool:
    return bool(lib().oracle_on_curve(P))


def ladder_small(k: int, t: int, P: bytes) -> bytes:
    out = ctypes.create_string_buffer(64)
    _check(lib().oracle_ladder_small(k, t, P, out), "ladder_small")
    return out.raw


def ladder_big(k: int, P: bytes) -> bytes:
    out = ctypes.create_string_buffer(64)
    _check(lib().oracle_ladder_big(_b32(k % (1 << 256)), P, out), "ladder_big")
    return out.raw


def repeated_add(k: int, P: bytes) -> bytes:
    out = ctypes.create_string_buffer(64)
    _check(lib().oracle_repeated_add(k, P, out), "repeated_add")
    return out.raw


def scalar_from_seed(seed: int, domain: int, idx: int) -> int:
    out = ctypes.create_string_buffer(32)
    lib().oracle_scalar_from_seed(seed, domain, idx, out)
    return int.from_bytes(out.raw, "big")


# ---------------------------------------------------------------- ElGamal

def keygen(seed: int):
    """(sk as int, pk as 64 bytes)."""
    sk = ctypes.create_string_buffer(32)
    pk = ctypes.create_string_buffer(64)
    _check(lib().oracle_keygen(seed, sk, pk), "keygen")
    return int.from_bytes(sk.raw, "big"), pk.raw


def encrypt(pk: bytes, msg, seed: int, idx0: int = 0, nthreads=None) -> np.ndarray:
    m = np.ascontiguousarray(np.asarray(msg, dtype=np.int32).reshape(-1))
    out = np.zeros((m.size, 128), dtype=np.uint8)
    _check(lib().oracle_encrypt(pk, _ptr(m), m.size, seed, idx0, _ptr(out),
                                nthreads or default_threads()), "encrypt")
    return out.reshape(tuple(np.shape(msg)) + (128,))


def encrypt_indexed(pk: bytes, msg, idx, seed: int, nthreads=None) -> np.ndarray:
    """Element e encrypted with the nonce of index idx[e] (flat arrays)."""
    m = np.ascontiguousarray(np.asarray(msg, dtype=np.int32).reshape(-1))
    ix = np.ascontiguousarray(np.asarray(idx, dtype=np.int64).reshape(-1))
    if m.size != ix.size:
        raise ValueError("msg and idx differ in length")
    out = np.zeros((m.size, 128), dtype=np.uint8)
    _check(lib().oracle_encrypt_indexed(pk, _ptr(m), _ptr(ix), m.size, seed, _ptr(out),
                                        nthreads or default_threads()), "encrypt_indexed")
    return out


def encrypt_columns(pk: bytes, msg, cols, seed: int, nthreads=None) -> np.ndarray:
    """Ciphertexts of msg[:, j] for j in cols with the nonces of their
    positions in the full n x l matrix (index k * l + j); returns an n x l
    array with only those columns filled."""
    msg = np.asarray(msg, dtype=np.int32)
    n, l = msg.shape
    cols = list(cols)
    kk, jj = np.meshgrid(np.arange(n), np.asarray(cols, dtype=np.int64), indexing="ij")
    cts = encrypt_indexed(pk, msg[:, cols].reshape(-1), (kk * l + jj).reshape(-1), seed, nthreads)
    B = np.zeros((n, l, 128), dtype=np.uint8)
    B[:, cols] = cts.reshape(n, len(cols), 128)
    return B


def decrypt_to_points(sk: int, ct: np.ndarray, nthreads=None) -> np.ndarray:
    c = np.ascontiguousarray(ct, dtype=np.uint8).reshape(-1, 128)
    out = np.zeros((c.shape[0], 64), dtype=np.uint8)
    _check(lib().oracle_decrypt_to_points(_b32(sk), _ptr(c), c.shape[0], _ptr(out),
                                          nthreads or default_threads()), "decrypt")
    return out.reshape(ct.shape[:-1] + (64,))


# ---------------------------------------------------------------- Alg. 2

def alg2_plain(a, N: int, Cs: int):
    """(C*a as int64 array, muls, adds, lens) by Alg. 2 on integers."""
    v = np.ascontiguousarray(np.asarray(a, dtype=np.int64))
    out = np.zeros(v.size, dtype=np.int64)
    muls = np.zeros(1, dtype=np.int64)
    adds = np.zeros(1, dtype=np.int64)
    lens = np.zeros(N + 1, dtype=np.int32)
    _check(lib().oracle_alg2_plain(_ptr(v), v.size, N, Cs, _ptr(out), _ptr(muls), _ptr(adds),
                                   _ptr(lens)), "alg2_plain")
    return out, int(muls[0]), int(adds[0]), [int(x) for x in lens]


def alg2_point(a, N: int, P: bytes) -> np.ndarray:
    v = np.ascontiguousarray(np.asarray(a, dtype=np.int64))
    out = np.zeros((v.size, 64), dtype=np.uint8)
    _check(lib().oracle_alg2_point(_ptr(v), v.size, N, P, _ptr(out)), "alg2_point")
    return out


# ---------------------------------------------------------------- PC-MM

def _plain(A):
    """A as int32 values (the oracle takes the plaintexts themselves)."""
    A = np.asarray(A)
    if A.dtype not in (np.int8, np.uint8, np.int16, np.uint16, np.int32):
        raise TypeError("A must be an integer matrix")
    return np.ascontiguousarray(A, dtype=np.int32)


def _mm_args(A, B, cols):
    A32 = _plain(A)
    B = np.ascontiguousarray(B, dtype=np.uint8)
    m, n = A32.shape
    n2, l, w = B.shape
    if n2 != n or w != 128:
        raise ValueError("shape mismatch")
    colarr = None if cols is None else np.ascontiguousarray(np.asarray(cols, dtype=np.int32))
    return A32, m, n, l, B, colarr


def pcmm_schoolbook(A, B, cols=None, nthreads=None, out=None) -> np.ndarray:
    A32, m, n, l, B, colarr = _mm_args(A, B, cols)
    C = out if out is not None else np.zeros((m, l, 128), dtype=np.uint8)
    _check(lib().oracle_pcmm_schoolbook(_ptr(A32), m, n, l, _ptr(B), _ptr(C),
                                        None if colarr is None else _ptr(colarr),
                                        -1 if colarr is None else colarr.size,
                                        nthreads or default_threads()), "schoolbook")
    return C


def pcmm_cussen(A, B, N: int = 4, cols=None, nthreads=None, out=None) -> np.ndarray:
    A32, m, n, l, B, colarr = _mm_args(A, B, cols)
    C = out if out is not None else np.zeros((m, l, 128), dtype=np.uint8)
    _check(lib().oracle_pcmm_cussen(_ptr(A32), m, n, l, N, _ptr(B), _ptr(C),
                                    None if colarr is None else _ptr(colarr),
                                    -1 if colarr is None else colarr.size,
                                    nthreads or default_threads()), "cussen")
    return C


def pcmm_closed_form(A, l: int, sk: int, msg, seed: int, ii, jj, nthreads=None) -> np.ndarray:
    A32 = _plain(A)
    m, n = A32.shape
    msg = np.ascontiguousarray(np.asarray(msg, dtype=np.int32))
    if msg.shape != (n, l):
        raise ValueError("msg must be n x l")
    ii = np.ascontiguousarray(np.asarray(ii, dtype=np.int32))
    jj = np.ascontiguousarray(np.asarray(jj, dtype=np.int32))
    out = np.zeros((ii.size, 128), dtype=np.uint8)
    _check(lib().oracle_pcmm_closed_form(_ptr(A32), m, n, l, _b32(sk), _ptr(msg), seed,
                                         _ptr(ii), _ptr(jj), ii.size, _ptr(out),
                                         nthreads or default_threads()), "closed_form")
    return out
