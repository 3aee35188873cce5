/* pcmm_paillier.h -- PC-MM over Paillier ciphertexts on one MI355X (gfx950).
 *
 * The extension of Sec. "Extension to Paillier Encryption": for the
 * additively homomorphic Paillier scheme (Sec. 2: n = p q, ciphertexts in
 * Z*_{n^2}, Eq. (ahe_6_paillier)), ciphertext multiplication mod n^2 adds
 * plaintexts and a plaintext power multiplies them, so the product of an
 * m x n plaintext matrix A with an n x l matrix of ciphertexts B is
 *     C_ij = prod_k B_kj^{a_ik} mod n^2,
 * an encryption of sum_k a_ik b_kj.  Powers use the Montgomery powering
 * ladder of Alg. 4; the Cussen form builds, per column of A and output
 * column, the table of powers of B_kj for the column's distinct values by
 * Alg. 2 (prefix products) and then multiplies one table entry per nonzero
 * a_ik (Alg. 3), exactly as the EC-ElGamal path does with points.
 *
 * Parameters: n has exactly 3072 bits (384 bytes), so a ciphertext is a
 * residue mod n^2 of 6144 bits.  Generator g = n + 1 (g^m = 1 + m n mod n^2).
 *
 * Layout: a ciphertext is 192 little-endian 32-bit words (768 bytes), value
 * below n^2.  A ciphertext matrix is row-major, element e = row * cols + col
 * at words [192 e, 192 e + 192).  A is a host array, row-major, of unsigned
 * t-bit plaintexts (1 <= t <= 16): uint8 for t <= 8, uint16 for 9..16
 * (negative plaintexts would need inverses mod n^2 and are not supported).
 *
 * Ownership: device buffers (messages, ciphertexts, workspace) belong to the
 * caller.  A context owns a small device block with the modulus constants
 * (allocated on the device current at creation) until it is destroyed; its
 * calls must run with that device current (PCMM_EINVAL otherwise).
 * Calls enqueue their kernels on `stream` (a hipStream_t; NULL = default)
 * and return without waiting for them, except that the PC-MM calls copy their
 * host-side plan (and A) to the workspace first and wait for that copy.
 *
 * Errors (pcmm_status of pcmm.h): PCMM_EINVAL for null pointers, bad shapes
 * or bit-widths, a modulus that is even or not 3072 bits long; PCMM_ERANGE
 * for an A entry outside [0, 2^t); PCMM_ENOMEM for a workspace smaller than
 * the matching *_workspace call reports; PCMM_EDEVICE for HIP errors.
 */
#ifndef PCMM_PAILLIER_H
#define PCMM_PAILLIER_H

#include <stddef.h>
#include <stdint.h>

#include "pcmm.h"

#ifdef __cplusplus
extern "C" {
#endif

#define PCMM_PAILLIER_MODULUS_BYTES 384
#define PCMM_PAILLIER_CT_WORDS 192

typedef struct pcmm_paillier_s *pcmm_paillier;

/* Context of the public modulus n (n_be: 384 big-endian bytes, odd, top bit
 * set).  Derives n^2 and its Montgomery constants on the host. */
pcmm_status pcmm_paillier_create(const uint8_t *n_be, pcmm_paillier *out);
pcmm_status pcmm_paillier_destroy(pcmm_paillier ctx);

/* Encrypt (Sec. 2) count messages msg_dev[e] in [0, 2^31) (device int32):
 * ct[e] = g^m r^n mod n^2 = (1 + m n) r^n mod n^2, where the nonce of element
 * e is r = X mod n (0 -> 1) for X = sum_i w_i 2^(64 i), i = 0..47, and
 * w_i = mix(mix(seed ^ (2 << 56) ^ (idx0 + e)) + (i + 1) 0x9E3779B97F4A7C15)
 * with mix the SplitMix64 finaliser.  ct_dev: count x 192 words. */
pcmm_status pcmm_paillier_encrypt(pcmm_paillier ctx, const int32_t *msg_dev, int64_t count, uint64_t seed,
                                  int64_t idx0, uint32_t *ct_dev, void *stream);

/* Schoolbook PC-MM: C_ij = prod_k B_kj^{a_ik} mod n^2, one Alg. 4 power of
 * t = bits steps per nonzero a_ik.  B: n x l ciphertexts, C: m x l
 * ciphertexts (device, must not overlap B).  Workspace: B in internal form
 * and A (pcmm_paillier_schoolbook_workspace). */
pcmm_status pcmm_paillier_schoolbook_workspace(int32_t m, int32_t n, int32_t l, size_t *bytes);
pcmm_status pcmm_paillier_schoolbook(pcmm_paillier ctx, const void *A, int32_t m, int32_t n, int32_t l,
                                     int32_t bits, const uint32_t *B, uint32_t *C, void *workspace,
                                     size_t ws_bytes, void *stream);

/* Cussen PC-MM (Alg. 2 in Alg. 3 over ciphertext multiplication): the same
 * result as the schoolbook call, bit for bit.  cfg: rounds N (<= 0: 4) and
 * column group g (1..4, <= 0: 1; a group's table holds the products of
 * powers of g ciphertexts); the other fields are ignored.  stats (optional)
 * receives the plan's operation counts in the EC path's units: level_mults
 * = Alg. 4 powers per output column, table_adds = table products per output
 * column, accum_adds = accumulation products per output column.  Workspace:
 * B in internal form, the table registers (1 KiB each) and the plan
 * (pcmm_paillier_cussen_workspace). */
pcmm_status pcmm_paillier_cussen_workspace(const void *A, int32_t m, int32_t n, int32_t l, int32_t bits,
                                           const pcmm_cussen_cfg *cfg, size_t *bytes);
pcmm_status pcmm_paillier_cussen(pcmm_paillier ctx, const void *A, int32_t m, int32_t n, int32_t l, int32_t bits,
                                 const uint32_t *B, uint32_t *C, const pcmm_cussen_cfg *cfg, void *workspace,
                                 size_t ws_bytes, pcmm_cussen_stats *stats, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* PCMM_PAILLIER_H */
