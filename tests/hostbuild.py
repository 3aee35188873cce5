"""Builds the host (CPU) compile of the library's device field and point
arithmetic (tests/hostshim) with g++ and the undefined-behaviour sanitizer,
once per test session, and wraps its entry points.  Test infrastructure."""
import ctypes
import os
import shutil
import subprocess
import tempfile

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SHIM = os.path.join(HERE, "hostshim")
SRC = os.path.join(SHIM, "device_math_check.cpp")

_lib = None


def build(outdir=None) -> str:
    outdir = outdir or tempfile.mkdtemp(prefix="pcmm_hostshim_")
    so = os.path.join(outdir, "libdevice_math_check.so")
    gxx = shutil.which("g++") or "g++"
    cmd = [gxx, "-O1", "-std=c++17", "-shared", "-fPIC", "-fsanitize=undefined",
           "-fno-sanitize-recover=undefined", "-I", SHIM, "-o", so, SRC]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("host build of the device arithmetic failed:\n" + r.stderr)
    return so


def lib():
    global _lib
    if _lib is None:
        L = ctypes.CDLL(build())
        vp = ctypes.c_void_p
        L.hs_field_raw_n.argtypes = [ctypes.c_int, vp, vp, vp, ctypes.c_int64]
        L.hs_point.argtypes = [ctypes.c_int, vp, vp, vp, vp, ctypes.c_uint32, ctypes.c_int, vp]
        L.hs_accumulate.argtypes = [vp, vp, ctypes.c_int, vp]
        _lib = L
    return _lib


def field_raw(op, a_limbs, b_limbs=None):
    """Raw-limb field op on (count, 9) limb arrays; returns (count, 9) uint32
    (the host counterpart of the library's raw-limb diagnostic)."""
    a = np.ascontiguousarray(np.asarray(a_limbs, dtype=np.int64).astype(np.uint32))
    b = a if b_limbs is None else np.ascontiguousarray(np.asarray(b_limbs, dtype=np.int64).astype(np.uint32))
    out = np.zeros_like(a)
    rc = lib().hs_field_raw_n(op, a.ctypes.data, b.ctypes.data, out.ctypes.data, a.shape[0])
    assert rc == 0, rc
    return out


def _words(P):
    """64-byte big-endian x || y -> 16 little-endian words (x then y)."""
    x = int.from_bytes(P[:32], "big")
    y = int.from_bytes(P[32:], "big")
    return (ctypes.c_uint32 * 16)(*[(x >> (32 * i)) & 0xFFFFFFFF for i in range(8)],
                                  *[(y >> (32 * i)) & 0xFFFFFFFF for i in range(8)])


def _w8(v):
    return (ctypes.c_uint32 * 8)(*[(v >> (32 * i)) & 0xFFFFFFFF for i in range(8)])


def point(op, P, Q=None, zp=None, zq=None, k=0, t=0):
    """Point op (see device_math_check.cpp) on 64-byte affine points; z values
    are Python ints (Jacobian coordinates of P and Q) or None for Z = 1.
    Returns the 64-byte canonical affine result (zeros for the identity)."""
    out = (ctypes.c_uint32 * 16)()
    rc = lib().hs_point(op, _words(P), _w8(zp) if zp is not None else None,
                        _words(Q) if Q is not None else None, _w8(zq) if zq is not None else None,
                        k, t, out)
    if rc:
        raise AssertionError(f"host point op {op} reported {rc}")
    x = sum(out[i] << (32 * i) for i in range(8))
    y = sum(out[8 + i] << (32 * i) for i in range(8))
    return x.to_bytes(32, "big") + y.to_bytes(32, "big")


def accumulate(points, negs):
    """The accumulation's loop (XYZZ form, identity flag carried) over
    64-byte affine points, each negated where negs says; returns the 64-byte
    canonical affine sum."""
    n = len(points)
    words = (ctypes.c_uint32 * (16 * max(n, 1)))()
    for i, P in enumerate(points):
        w = _words(P)
        for k in range(16):
            words[16 * i + k] = w[k]
    neg = (ctypes.c_uint8 * max(n, 1))(*[1 if v else 0 for v in negs])
    out = (ctypes.c_uint32 * 16)()
    rc = lib().hs_accumulate(words, neg, n, out)
    assert rc == 0, rc
    x = sum(out[i] << (32 * i) for i in range(8))
    y = sum(out[8 + i] << (32 * i) for i in range(8))
    return x.to_bytes(32, "big") + y.to_bytes(32, "big")
