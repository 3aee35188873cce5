"""Pins of the oracle's Alg. 2 (Cussen compression-reconstruction).

* exactness: reconstruction returns exactly C * a for every vector over
  {0..2^t-1}^n at tiny n, t (exhaustive) and for random longer vectors, on
  integers and on curve points (against repeated addition);
* operation counts: averages over random vectors reproduce the paper's
  Tab. A1 (multiplications) and Tab. A2 (additions) of Appendix A.1, while the
  two plausible alternative counting conventions do not;
* the toy example of Sec. 3.2 / Sec. 3.3 (8 elements, 8-bit, N = 4: 3
  multiplications and 15 additions; encrypted: 6 ECSMs, 30 point additions,
  saving 130 equivalent additions) is realisable under the same convention.
"""
import itertools
import math
import random

import numpy as np
import pytest

from helpers import load_golden


def test_exhaustive_tiny_vectors(orc):
    for n in range(0, 5):
        for t in range(1, 4):
            for vec in itertools.product(range(1 << t), repeat=n):
                for N in (1, 2, 3, 4):
                    out, muls, adds, lens = orc.alg2_plain(list(vec), N, 7)
                    assert list(out) == [7 * v for v in vec]
                    assert lens[0] == n


@pytest.mark.parametrize("N", [1, 2, 3, 4, 6])
def test_random_vectors_exact(orc, N):
    rng = np.random.default_rng(N)
    for n in (1, 5, 64, 300):
        for t in (1, 4, 8, 12, 16, 20):
            a = rng.integers(0, 1 << t, size=n)
            C = int(rng.integers(-1000, 1000))
            out, muls, adds, lens = orc.alg2_plain(a, N, C)
            assert (out == C * a).all()
            # lengths never grow; the last level holds n_N multiplications
            assert all(lens[w + 1] <= max(lens[w], 0) for w in range(N))
            assert muls == lens[N]
            assert adds == sum(lens[1:N])


def test_point_reconstruction_matches_repeated_addition(orc):
    rnd = random.Random(11)
    p, b, gx, gy, q = orc.curve_params()
    B = orc.ladder_big(rnd.randrange(1, q), orc.generator())
    vecs = [[1, 2], [3, 3, 0, 1], [0, 0, 0], [15, 1, 7, 7, 2, 9, 0, 14], [1, 2, 4, 8, 16, 31]]
    for a in vecs:
        for N in (1, 2, 4):
            out = orc.alg2_point(a, N, B)
            for i, ai in enumerate(a):
                assert bytes(out[i]) == orc.repeated_add(ai, B), (a, N, i)


def _stats(orc, n, t, trials, rng):
    mu = np.empty(trials)
    ad = np.empty(trials)
    alt_adds = np.empty(trials)   # n_w - 1 additions per level
    zero_muls = np.empty(trials)  # zeros kept as an element of the last level
    for r in range(trials):
        a = rng.integers(0, 1 << t, size=n)
        _, m_, a_, lens = orc.alg2_plain(a, 4, 1)
        mu[r] = m_
        ad[r] = a_
        alt_adds[r] = sum(max(x - 1, 0) for x in lens[1:4])
        zero_muls[r] = m_ + (1 if (a == 0).any() else 0)
    return mu, ad, alt_adds, zero_muls


def _within(mean_ours, sd, table_value, trials_ours, trials_paper=1000):
    # the table prints a rounded average over 1000 random trials
    tol = 0.5 + 4.0 * sd * math.sqrt(1.0 / trials_ours + 1.0 / trials_paper) + 1e-9
    return abs(mean_ours - table_value) <= tol


# Tab. A2's averages scatter around the expectation of this convention by up to
# about 1.2 in both directions (e.g. +1.15 at n = 16, t = 8; -0.62 at n = 128,
# t = 12), more than the Monte-Carlo error of a 1000-trial average allows, so
# its cells are pinned to +-1.5 rather than to rounding.
A2_TOL = 1.5


def test_tables_a1_a2_operation_counts(orc):
    muls = load_golden("tab_a1_vector_plain_muls.csv")
    adds = load_golden("tab_a2_vector_plain_adds.csv")
    rng = np.random.default_rng(2504)
    trials = 3000
    rejected_alt_adds = rejected_zero = 0
    for rm, ra in zip(muls, adds):
        n = rm["n"]
        assert rm["schoolbook"] == n and ra["schoolbook"] == 0
        for t in (4, 8, 12, 16):
            mu, ad, alt, zm = _stats(orc, n, t, trials, rng)
            assert _within(mu.mean(), mu.std(), rm[f"t{t}"], trials), (n, t, mu.mean())
            assert abs(ad.mean() - ra[f"t{t}"]) <= A2_TOL, (n, t, ad.mean())
            rejected_alt_adds += abs(alt.mean() - ra[f"t{t}"]) > A2_TOL
            rejected_zero += not _within(zm.mean(), zm.std(), rm[f"t{t}"], trials)
    # the alternative conventions are contradicted by the tables: n_w - 1
    # additions per level, or a zero kept as an element of the last level
    assert rejected_alt_adds >= 20
    assert rejected_zero >= 5


def test_toy_example_counts_realisable(orc):
    # 8 elements of 8 bits compressed to length 3 with 15 reconstruction
    # additions (Sec. 3.2); encrypted: 2 * 3 ECSMs and 2 * 15 point additions,
    # i.e. 6 * 16 + 30 = 126 equivalent additions against 16 * 16 (Sec. 3.3).
    rng = np.random.default_rng(0)
    found = None
    for _ in range(200000):
        a = rng.integers(0, 256, size=8)
        _, muls, adds, lens = orc.alg2_plain(a, 4, 1)
        if muls == 3 and adds == 15:
            found = a
            break
    assert found is not None
    t = 8
    schoolbook = 2 * 8 * (2 * t)
    proposed = 2 * 3 * (2 * t) + 2 * 15
    assert schoolbook - proposed == 130
