"""The paper's operation-count model for PC-MM (no group arithmetic here).

Sec. 3.1: one plaintext-ciphertext multiplication is two ECSMs, each of t
doublings and t additions by Alg. 1 (so 4t equivalent point additions, taking a
doubling as one addition, Sec. 3.3); one ciphertext-ciphertext addition is two
point additions.  Sec. 3.3 / Appendix A.1: Cussen's method spends n_N
multiplications per compressed column and its reconstruction counts n_w
additions at every level w < N.  These formulas regenerate every cell of the
appendix's equivalent-addition tables from its multiplication/addition tables.
"""


def schoolbook_equiv_adds(m: int, n: int, l: int, t: int) -> int:
    """m n l pt-ct multiplications and m l (n - 1) ct-ct additions."""
    return 4 * t * m * n * l + 2 * m * l * (n - 1)


def cussen_equiv_adds_from_plan(m: int, n: int, l: int, t: int, level_n_muls, level_adds) -> int:
    """Alg. 3 with per-column compression results: column k costs
    2 l n_N(k) ECSMs of t bits and 2 l sum_{w<N} n_w(k) point additions for
    reconstruction; accumulation costs 2 m l (n - 1) point additions."""
    recon = sum(4 * t * l * int(mk) + 2 * l * int(ak) for mk, ak in zip(level_n_muls, level_adds))
    return recon + 2 * m * l * (n - 1)


def cussen_equiv_adds_square(n: int, t: int, mul_v: float, add_v: float) -> float:
    """Square case m = n = l with average per-column counts mul_v, add_v."""
    return 4 * t * n * n * mul_v + 2 * (n * n * add_v + n * n * (n - 1))


def vector_schoolbook_equiv_adds(n: int, t: int) -> int:
    """Plaintext vector of length n times one ciphertext: 2n ECSMs."""
    return 4 * t * n


def vector_cussen_equiv_adds(t: int, mul_v: float, add_v: float) -> float:
    return 4 * t * mul_v + 2 * add_v


def plain_matrix_counts_cussen(n: int, mul_v: float, add_v: float):
    """(multiplications, additions) of plaintext n x n Cussen MatMul."""
    return n * n * mul_v, n * n * add_v + n * n * (n - 1)


def plain_matrix_counts_schoolbook(n: int):
    return n ** 3, n * n * (n - 1)


def _strassen_block_elems(n: int) -> int:
    """Sum over recursion levels d of 7^d (n / 2^(d+1))^2: block elements per
    block addition, with the recursion down to 1 x 1 blocks (n a power of 2)."""
    k = n.bit_length() - 1
    return sum(7 ** d * (n >> (d + 1)) ** 2 for d in range(k))


def strassen_plain_counts(n: int):
    """Plaintext n x n Strassen (Sec. 3.1): 7^log2(n) scalar multiplications
    and 18 block additions per recursion node (Tab. A3, A4)."""
    k = n.bit_length() - 1
    return 7 ** k, 18 * _strassen_block_elems(n)


def strassen_equiv_adds(n: int, t: int) -> int:
    """Equivalent point additions of Strassen PC-MM (Tab. A6): every scalar x
    ciphertext product costs 2 ECSMs of 2t additions each, and each recursion
    node adds 13 ciphertext blocks (2 points per ciphertext); the 5 plaintext
    block additions are free."""
    k = n.bit_length() - 1
    return 4 * t * 7 ** k + 26 * _strassen_block_elems(n)
