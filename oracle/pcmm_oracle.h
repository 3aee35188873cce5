/*
 * pcmm_oracle.h -- plain, slow CPU reference for plaintext-ciphertext matrix
 * multiplication (PC-MM) over EC-ElGamal on NIST P-256.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this code; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no source, header, table or constant
 * generator with the GPU library: its own bignum (4 x 64-bit limbs, fold
 * reduction with 2^256 mod M, binary extended-Euclid inversion), affine points
 * with the textbook group law, and its own compression code.
 *
 * Byte conventions at this interface (chosen for easy comparison):
 *   field elements / scalars : 32 bytes, big-endian
 *   points                   : 64 bytes, x || y big-endian, affine;
 *                              the point at infinity is 64 zero bytes
 *                              (not on the curve because b != 0)
 *   ciphertexts              : 128 bytes, C1 || C2
 * All functions return 0 on success and a negative value on bad arguments.
 */
#ifndef PCMM_ORACLE_H
#define PCMM_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Field / scalar arithmetic, exposed so that tests can pin them against an
 * independent big-integer implementation.  op: 0 add, 1 sub, 2 mul, 3 inv,
 * 4 neg.  mod: 0 = p (field), 1 = q (group order). */
int oracle_mod_op(int mod, int op, const uint8_t a[32], const uint8_t b[32], uint8_t out[32]);

/* Curve constants in big-endian: p, b, Gx, Gy, q (5 x 32 bytes). */
void oracle_curve_params(uint8_t out[160]);

/* Group law (Sec. 2.3). */
int oracle_pt_add(const uint8_t P[64], const uint8_t Q[64], uint8_t R[64]);
int oracle_pt_dbl(const uint8_t P[64], uint8_t R[64]);
int oracle_pt_neg(const uint8_t P[64], uint8_t R[64]);
int oracle_on_curve(const uint8_t P[64]); /* 1 on curve, 0 not; infinity -> 1 */

/* Alg. 1 (Montgomery ladder) over t bits of k (t <= 64); R = k P. */
int oracle_ladder_small(uint64_t k, int t, const uint8_t P[64], uint8_t R[64]);
/* Alg. 1 with a 256-bit big-endian scalar (t = 256). */
int oracle_ladder_big(const uint8_t k[32], const uint8_t P[64], uint8_t R[64]);
/* k P computed as P + P + ... + P (k - 1 additions): the textbook definition. */
int oracle_repeated_add(uint64_t k, const uint8_t P[64], uint8_t R[64]);

/* Scalar derivation for keys and nonces (counter-based, SplitMix64 mixing).
 * domain 0 = secret key, 1 = encryption nonce; idx = element index.
 * Result in [1, q-1], big-endian.  Parity unpinned: this is a project
 * convention (the paper only says "uniform in [1, q-1]"); the tests check its
 * range and spread, and that the GPU library derives the same scalars. */
void oracle_scalar_from_seed(uint64_t seed, uint64_t domain, uint64_t idx, uint8_t out[32]);

/* EC-ElGamal (Sec. 2.4).  keygen: x from (seed, 0, 0), H = xG.
 * encrypt: element e gets r = scalar(seed, 1, idx0 + e); C = (rG, rH + mG).
 * decrypt_to_points: C2 - x C1 (the message point mG). */
int oracle_keygen(uint64_t seed, uint8_t sk[32], uint8_t pk[64]);
int oracle_encrypt(const uint8_t pk[64], const int32_t *msg, int64_t count, uint64_t seed,
                   int64_t idx0, uint8_t *ct_out, int nthreads);
/* Encrypt with explicit nonce indices: element e uses r = scalar(seed, 1, idx[e]). */
int oracle_encrypt_indexed(const uint8_t pk[64], const int32_t *msg, const int64_t *idx, int64_t count,
                           uint64_t seed, uint8_t *ct_out, int nthreads);
int oracle_decrypt_to_points(const uint8_t sk[32], const uint8_t *ct, int64_t count,
                             uint8_t *pt_out, int nthreads);

/* Alg. 2 on plain integers (compression + reconstruction).
 * a: n non-negative integers; N rounds; Cs: the scalar.  out: n values C*a_i.
 * muls/adds: operation counts under the counting convention of the paper's
 * tables (N-level multiplications = n_N; each reconstruction level w < N
 * counts n_w additions).  lens (optional, N+1 ints): n_0..n_N. */
int oracle_alg2_plain(const int64_t *a, int n, int N, int64_t Cs, int64_t *out,
                      int64_t *muls, int64_t *adds, int *lens);

/* Alg. 2 with a ciphertext point as the scalar: out[i] = a_i P (n points). */
int oracle_alg2_point(const int64_t *a, int n, int N, const uint8_t P[64], uint8_t *out);

/* PC-MM.  A: m x n row-major plaintext values (int32; any sign and size).
 * B: n x l ciphertexts row-major
 * (128 bytes each).  C: m x l ciphertexts row-major.  Only the output columns
 * listed in cols[0..ncols) are computed (ncols < 0: all columns); other
 * columns of C are left untouched. */
int oracle_pcmm_schoolbook(const int32_t *A, int m, int n, int l,
                           const uint8_t *B, uint8_t *C, const int32_t *cols, int ncols,
                           int nthreads);
int oracle_pcmm_cussen(const int32_t *A, int m, int n, int l, int N,
                       const uint8_t *B, uint8_t *C, const int32_t *cols, int ncols,
                       int nthreads);

/* Closed form of Eq. (ahe_5): for the listed output positions (i, j),
 * e1 = sum_k a_ik r_kj, e2 = sum_k a_ik (x r_kj + msg_kj)  (mod q),
 * C_ij = (e1 G, e2 G).  Nonces r_kj = scalar(seed, 1, k*l + j).
 * ii/jj: npos positions; out: npos ciphertexts. */
int oracle_pcmm_closed_form(const int32_t *A, int m, int n, int l,
                            const uint8_t sk[32], const int32_t *msg, uint64_t seed,
                            const int32_t *ii, const int32_t *jj, int npos, uint8_t *out,
                            int nthreads);

#ifdef __cplusplus
}
#endif
#endif
