"""Seeded synthetic workloads for PC-MM (inputs only, no group arithmetic).

The paper measures uniform random square matrices with element bit-widths
t in {4, 8, 12, 16} and sizes n in {8, ..., 512} (Sec. 4.2; Appendix A).  The
workloads below follow that recipe and add the rectangular, signed, batched and
serving shapes of this library's benchmark set.  Everything is drawn with
numpy's PCG64 from a fixed seed; encryption nonces and the secret key are not
drawn here: they are derived from the same seed by the counter-based scalar
derivation that both the library and the CPU reference implement.

This module is shared by the tests, the benchmark and the CPU reference; it
holds no curve, field or compression arithmetic.
"""
import math
from dataclasses import dataclass, field
from typing import List

import numpy as np


@dataclass(frozen=True)
class PCMMShape:
    m: int
    n: int
    l: int
    bits: int          # plaintext bit-width t of A
    signed: bool       # A entries in [-2^(t-1), 2^(t-1)) instead of [0, 2^t)
    msg_bits: int      # plaintext bit-width of the encrypted matrix
    seed: int
    name: str = ""


@dataclass
class BatchWorkload:
    shapes: List[PCMMShape] = field(default_factory=list)
    seed: int = 4


# The named workloads (sizes and seeds are fixed so every run sees the same
# inputs).  "tiny" is the 16x16 case the CPU reference finishes in seconds.
TINY = PCMMShape(16, 16, 16, 4, False, 4, seed=1, name="tiny16_t4")
SIGNED128 = PCMMShape(128, 128, 128, 8, True, 8, seed=2, name="signed128_t8")
LARGE_T2 = PCMMShape(512, 512, 512, 2, False, 4, seed=32, name="large512_t2")
LARGE_T4 = PCMMShape(512, 512, 512, 4, False, 4, seed=34, name="large512_t4")
SERVE_LAYER = PCMMShape(256, 1024, 8, 8, True, 8, seed=5, name="serve256x1024x8_t8")

NAMED = {s.name: s for s in (TINY, SIGNED128, LARGE_T2, LARGE_T4, SERVE_LAYER)}


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def gen_plain_matrix(rng: np.random.Generator, rows: int, cols: int, bits: int,
                     signed: bool) -> np.ndarray:
    """Uniform t-bit plaintext matrix: int8 / uint8 for t <= 8, int16 / uint16
    for 9 <= t <= 16 (signed: [-2^(t-1), 2^(t-1)), unsigned: [0, 2^t))."""
    if not (1 <= bits <= 16):
        raise ValueError("bits must be in 1..16")
    wide = bits > 8
    if signed:
        lo, hi = -(1 << (bits - 1)), (1 << (bits - 1))
        return rng.integers(lo, hi, size=(rows, cols), dtype=np.int64).astype(np.int16 if wide else np.int8)
    return rng.integers(0, 1 << bits, size=(rows, cols), dtype=np.int64).astype(np.uint16 if wide else np.uint8)


def gen_messages(rng: np.random.Generator, rows: int, cols: int, bits: int) -> np.ndarray:
    """Uniform unsigned messages of `bits` bits (the encrypted matrix B)."""
    return rng.integers(0, 1 << bits, size=(rows, cols), dtype=np.int64).astype(np.int32)


def make_inputs(shape: PCMMShape):
    """(A, msg) for one PC-MM: A is m x n, msg is n x l (drawn in that order)."""
    rng = rng_for(shape.seed)
    A = gen_plain_matrix(rng, shape.m, shape.n, shape.bits, shape.signed)
    msg = gen_messages(rng, shape.n, shape.l, shape.msg_bits)
    return A, msg


def batch_workload(count: int = 64, seed: int = 4, lo: int = 32, hi: int = 512,
                   bit_choices=(1, 2, 4, 8), msg_bits: int = 8) -> BatchWorkload:
    """Uneven batch: m, n, l uniform in {lo..hi}, A bit-width uniform over
    `bit_choices` (unsigned), uniform `msg_bits`-bit messages."""
    rng = rng_for(seed)
    shapes = []
    for b in range(count):
        m, n, l = (int(x) for x in rng.integers(lo, hi + 1, size=3))
        bits = int(rng.choice(np.asarray(bit_choices)))
        shapes.append(PCMMShape(m, n, l, bits, False, msg_bits, seed=seed * 1000003 + b,
                                name=f"batch{b}"))
    return BatchWorkload(shapes=shapes, seed=seed)


# ---------------------------------------------------------------------------
# Paillier key material (inputs of the Paillier PC-MM; no PC-MM arithmetic)
# ---------------------------------------------------------------------------
_SMALL_PRIMES = [p for p in range(3, 2000, 2) if all(p % d for d in range(3, int(p ** 0.5) + 1, 2))]
_KEY_CACHE = {}


def _probable_prime(x: int, rng: np.random.Generator, rounds: int = 40) -> bool:
    """Trial division by small primes, then Miller-Rabin with seeded bases."""
    if x < 2 or x % 2 == 0:
        return x == 2
    for p in _SMALL_PRIMES:
        if x % p == 0:
            return x == p
    d, s = x - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for _ in range(rounds):
        a = 2 + int.from_bytes(rng.bytes((x.bit_length() + 7) // 8), "little") % (x - 3)
        y = pow(a, d, x)
        if y in (1, x - 1):
            continue
        for _ in range(s - 1):
            y = y * y % x
            if y == x - 1:
                break
        else:
            return False
    return True


def paillier_key(seed: int, bits: int = 3072):
    """(n, p, q) for a Paillier key of `bits`-bit modulus n = p q: p and q are
    distinct bits/2-bit primes with their top two bits set (so n has exactly
    `bits` bits) and gcd(n, (p-1)(q-1)) = 1.  Candidates come from PCG64(seed);
    cached per (seed, bits)."""
    key = (seed, bits)
    if key in _KEY_CACHE:
        return _KEY_CACHE[key]
    rng = rng_for(seed)
    half = bits // 2

    def prime():
        while True:
            x = int.from_bytes(rng.bytes(half // 8), "little")
            x |= (3 << (half - 2)) | 1
            x &= (1 << half) - 1
            if _probable_prime(x, rng):
                return x

    while True:
        p, q = prime(), prime()
        n = p * q
        if p != q and n.bit_length() == bits and math.gcd(n, (p - 1) * (q - 1)) == 1:
            break
    _KEY_CACHE[key] = (n, p, q)
    return n, p, q


def paillier_messages(rng: np.random.Generator, rows: int, cols: int, bits: int) -> np.ndarray:
    """Uniform unsigned `bits`-bit messages (int32) for Paillier encryption."""
    return rng.integers(0, 1 << bits, size=(rows, cols), dtype=np.int64).astype(np.int32)
