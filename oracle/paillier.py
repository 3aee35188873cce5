"""CPU oracle for PC-MM over Paillier ciphertexts (Python integers).

TEST INFRASTRUCTURE ONLY: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may use it; the product library never
does.  It shares nothing with the GPU path: arbitrary-precision integers,
``%`` for reduction, no Montgomery form, no limbs.

What it follows:
* the Paillier scheme of Sec. 2 (KeyGen / Encrypt / Decrypt with the quotient
  function L(x) = (x - 1) / n) and its homomorphic property, Eq.
  (ahe_6_paillier): a product of ciphertext powers prod c_i^{s_i} mod n^2
  decrypts to sum s_i m_i;
* the PC-MM of Sec. "Extension to Paillier Encryption": C_ij = prod_k
  B_kj^{a_ik} mod n^2, i.e. ciphertext multiplication in place of point
  addition and exponentiation in place of scalar multiplication;
* exponentiation by the Montgomery powering ladder of Alg. 4;
* the compression-reconstruction of Alg. 2 inside Alg. 3, with the group
  operation a multiplication mod n^2.

Readings (the paper is silent): g = n + 1 (a valid generator choice: g^m =
1 + m n mod n^2); the nonce r of element ``idx`` under ``seed`` is derived
counter-style with SplitMix64 (domain 2) as 48 64-bit words, X mod n, with 0
mapped to 1.  A holds unsigned plaintexts (negative exponents would need
inverses mod n^2).
"""
from typing import List, Sequence

MASK64 = (1 << 64) - 1
GOLDEN_GAMMA = 0x9E3779B97F4A7C15
DOMAIN_PAILLIER_NONCE = 2
NONCE_WORDS = 48  # 3072 bits


# ---------------------------------------------------------------------------
# Scheme (Sec. 2)
# ---------------------------------------------------------------------------
def splitmix64_mix(z: int) -> int:
    """The SplitMix64 finaliser (public-domain reference mixing function)."""
    z &= MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def nonce(n: int, seed: int, idx: int) -> int:
    """r in [1, n - 1] for element idx: w_i = mix(mix(seed ^ (2 << 56) ^ idx) +
    (i + 1) * golden gamma), X = sum_i w_i 2^(64 i), r = X mod n (0 -> 1)."""
    base = splitmix64_mix((seed ^ (DOMAIN_PAILLIER_NONCE << 56) ^ idx) & MASK64)
    X = 0
    for i in range(NONCE_WORDS):
        X |= splitmix64_mix((base + (i + 1) * GOLDEN_GAMMA) & MASK64) << (64 * i)
    r = X % n
    return r if r else 1


def lcm(a: int, b: int) -> int:
    x, y = a, b
    while y:
        x, y = y, x % y
    return a // x * b


def L(x: int, n: int) -> int:
    """The quotient function L(x) = (x - 1) / n (exact for x = 1 mod n)."""
    assert (x - 1) % n == 0
    return (x - 1) // n


def keys(p: int, q: int):
    """Public (n, g) and secret (lambda, mu) for primes p, q (g = n + 1)."""
    n = p * q
    n2 = n * n
    g = n + 1
    lam = lcm(p - 1, q - 1)
    mu = pow(L(pow(g, lam, n2), n), -1, n)
    return (n, g), (lam, mu)


def encrypt(n: int, m: int, seed: int, idx: int) -> int:
    """c = g^m r^n mod n^2 with g = n + 1 and r = nonce(n, seed, idx)."""
    n2 = n * n
    g = n + 1
    r = nonce(n, seed, idx)
    return pow(g, m % n, n2) * pow(r, n, n2) % n2


def decrypt(p: int, q: int, c: int) -> int:
    """m = L(c^lambda mod n^2) mu mod n."""
    (n, _g), (lam, mu) = keys(p, q)
    return L(pow(c, lam, n * n), n) * mu % n


# ---------------------------------------------------------------------------
# Alg. 4: Montgomery powering ladder
# ---------------------------------------------------------------------------
def ladder(g: int, k: int, t: int, mod: int) -> int:
    """g^k mod `mod` for a t-bit exponent k, step by step as Alg. 4: r0 = 1,
    r1 = g; for bits k_{t-1} .. k_0: r_{1-b} = r1 r0, r_b = r_b^2."""
    assert 0 <= k < (1 << t) or (k == 0 and t == 0)
    r = [1 % mod, g % mod]
    for i in range(t - 1, -1, -1):
        b = (k >> i) & 1
        r[1 - b] = r[1] * r[0] % mod
        r[b] = r[b] * r[b] % mod
    return r[0]


# ---------------------------------------------------------------------------
# PC-MM (Sec. "Extension to Paillier Encryption")
# ---------------------------------------------------------------------------
def _check_plain(A: Sequence[Sequence[int]], bits: int):
    for row in A:
        for a in row:
            if not 0 <= a < (1 << bits):
                raise ValueError("A holds unsigned %d-bit plaintexts" % bits)


def pcmm_schoolbook(A, B, n2: int, bits: int, cols=None) -> List[List[int]]:
    """C_ij = prod_k B_kj^{a_ik} mod n^2, each power by Alg. 4 (t = bits);
    returns the m x len(cols) block of columns `cols` (default: all)."""
    _check_plain(A, bits)
    m, nk = len(A), len(A[0]) if A else 0
    l = len(B[0]) if B else 0
    cols = list(range(l)) if cols is None else list(cols)
    C = [[1 % n2] * len(cols) for _ in range(m)]
    for i in range(m):
        for jj, j in enumerate(cols):
            acc = 1 % n2
            for k in range(nk):
                acc = acc * ladder(B[k][j], A[i][k], bits, n2) % n2
            C[i][jj] = acc
    return C


def alg2_reconstruct(vals: Sequence[int], N: int, base: int, mul, power):
    """Reconstruction of Alg. 2 over a multiplicative group: returns
    [base^v for v in vals] (1 for v = 0) computed as Alg. 2 does: the level-N
    values by `power`, then prefix products down to level 1, un-sorting with
    the rank pointers.  Counts (powers, products) are returned too."""
    # compression: per level, the sorted distinct nonzero values, each one's
    # rank (the tracking pointer), and for levels below N their differences
    lev_vals = [None] * (N + 1)  # distinct sorted values per level (pre-difference)
    diffs = [None] * (N + 1)
    ptrs = [None] * (N + 1)
    cur = list(vals)
    row_rank = None
    for w in range(1, N + 1):
        u = sorted(set(x for x in cur if x != 0))
        pos = {x: i for i, x in enumerate(u)}
        rank = [pos[x] if x != 0 else -1 for x in cur]
        if w == 1:
            row_rank = rank
        else:
            ptrs[w] = rank
        lev_vals[w] = u
        if w < N:
            d = [u[0]] + [u[i] - u[i - 1] for i in range(1, len(u))] if u else []
            diffs[w] = d
            cur = d
    powers = products = 0
    # level N: base^s for each distinct value
    top = []
    for s in lev_vals[N]:
        top.append(power(base, s))
        powers += 1
    cur_pts = top
    for w in range(N - 1, 0, -1):
        # element i of level w (a difference d_i) is base^{d_i}: un-sort from
        # level w + 1 through its rank there (zero differences are the identity)
        b = [cur_pts[ptrs[w + 1][i]] if ptrs[w + 1][i] >= 0 else 1 for i in range(len(diffs[w]))]
        # prefix products give base^{u_i} for the sorted distinct values u
        S = []
        for i, x in enumerate(b):
            if i == 0:
                S.append(x)
            else:
                S.append(mul(S[-1], x))
                products += 1
        cur_pts = S
    out = [cur_pts[r] if r >= 0 else 1 for r in row_rank]
    return out, powers, products


def pcmm_cussen(A, B, n2: int, bits: int, N: int = 4, cols=None) -> List[List[int]]:
    """Alg. 3 over Paillier ciphertexts: for every column k of A and output
    column j, the table of B_kj^u for the distinct values u of the column by
    Alg. 2 (powers by Alg. 4), then C_ij = prod_k table[a_ik] mod n^2."""
    _check_plain(A, bits)
    m, nk = len(A), len(A[0]) if A else 0
    l = len(B[0]) if B else 0
    cols = list(range(l)) if cols is None else list(cols)
    mul = lambda x, y: x * y % n2  # noqa: E731
    power = lambda g, s: ladder(g, s, max(s.bit_length(), 1), n2)  # noqa: E731
    C = [[1 % n2] * len(cols) for _ in range(m)]
    for jj, j in enumerate(cols):
        for k in range(nk):
            col = [A[i][k] for i in range(m)]
            T, _, _ = alg2_reconstruct(col, N, B[k][j], mul, power)
            for i in range(m):
                C[i][jj] = C[i][jj] * T[i] % n2
    return C


def closed_form(A, msg, n: int) -> List[List[int]]:
    """The plaintext product A msg mod n that every correct PC-MM result
    decrypts to (Eq. ahe_6_paillier)."""
    m, nk = len(A), len(A[0]) if A else 0
    l = len(msg[0]) if msg else 0
    return [[sum(A[i][k] * msg[k][j] for k in range(nk)) % n for j in range(l)] for i in range(m)]
