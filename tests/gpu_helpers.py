"""Helpers shared by the GPU tests (inputs from the oracle, comparisons)."""
import random
import sys

import numpy as np


def log(*args):
    print(*args, flush=True)
    sys.stdout.flush()


def random_points(orc, count, seed):
    """`count` pseudo-random curve points from the oracle (chained additions)."""
    rnd = random.Random(seed)
    p_, b_, gx, gy, q = orc.curve_params()
    G = orc.generator()
    base = [orc.ladder_big(rnd.randrange(1, q), G) for _ in range(min(count, 6))]
    pts = list(base)
    i = 0
    while len(pts) < count:
        pts.append(orc.pt_add(pts[-1], base[i % len(base)]))
        i += 1
    return pts[:count]


def random_cts(orc, rows, cols, seed):
    """rows x cols 'ciphertexts' made of arbitrary curve points (oracle-made)."""
    pts = random_points(orc, max(1, 2 * rows * cols), seed)
    arr = np.frombuffer(b"".join(pts), dtype=np.uint8)[:rows * cols * 128]
    return arr.reshape(rows, cols, 128).copy()


def sample_positions(m, l, count, seed):
    rng = np.random.default_rng(seed)
    pos = {(0, 0), (m - 1, l - 1), (0, l - 1), (m - 1, 0)}
    while len(pos) < min(count, m * l):
        pos.add((int(rng.integers(m)), int(rng.integers(l))))
    ii = np.array([p[0] for p in sorted(pos)], dtype=np.int32)
    jj = np.array([p[1] for p in sorted(pos)], dtype=np.int32)
    return ii, jj
