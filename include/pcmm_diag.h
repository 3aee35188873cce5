/*
 * pcmm_diag.h -- self-test and measurement entry points of libpcmm.
 *
 * These expose the device building blocks one operation at a time so that the
 * field arithmetic, the point formulas and the ladder of Alg. 1 can be checked
 * element by element against an independent implementation, and they measure
 * the instruction rates that bound the PC-MM kernels (the 32 x 32 -> 64-bit
 * multiply-add that dominates prime-field multiplication, plain 32-bit
 * additions, the field multiplication and the mixed point addition).
 * Conventions (errors, streams, ownership, canonical limbs) as in pcmm.h.
 */
#ifndef PCMM_DIAG_H
#define PCMM_DIAG_H
#include <stddef.h>
#include <stdint.h>

#include "pcmm.h"
#include "pcmm_paillier.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Field operations on `count` elements in [0, p).  Operands and result are
 * structure-of-arrays: limb w of element e at x[w * count + e].
 * op: 0 a+b, 1 a-b, 2 a*b, 3 a^2, 4 a^-1 (0 -> 0), 5 -a, 6 Montgomery
 * round trip of a (to and from Montgomery form).  b is ignored by unary ops. */
pcmm_status pcmm_diag_field(int32_t op, const uint32_t *a, const uint32_t *b, uint32_t *out,
                            int64_t count, void *stream);

/* The same on the internal representation: operands and result are nine
 * 29-bit limbs per element (Montgomery limbs, normal form: value < 2p, limbs
 * 0..7 < 2^29, limb 8 < 2^25), limb w of element e at x[w * count + e], with
 * no conversion.  op: 0 a+b, 1 a-b, 2 a*b (Montgomery), 3 a^2, 4 2(a-b),
 * 5 3a, 6 4a, 7 -a, 8 full reduction (value < p), 9 2a, 10 normal form of
 * arbitrary signed limbs a (|limb| < 2^30, 0 <= value < 2^259),
 * 11 equality flag a = b (mod p) in limb 0, 12 zero flag a = 0 (mod p);
 * lazy forms (carry-only results: limbs 0..7 < 2^29, the rest in limb 8):
 * 13 a-b+2p in (0, 4p), 14 4a in [0, 8p), 15 a-3b (mod p, normal form, one
 * limb pass adding 6p), 16 a-2b (likewise, adding 4p),
 * 17 (a-b+2p) * 4b with both operands carry-only (normal form);
 * products that absorb an addition: 18 a*b + (2p - b) with the addend above
 * R (carry-only, in (0, 4p)), 20 (2a)*b - 2 b'*b' with one reduction, for a
 * and b carry-only (value < 4p) and b' the normal form of b (normal form);
 * 19 4a-3b (mod p, normal form, one limb pass adding 6p); the split
 * (latency) forms 21 a*b and 22 a^2, 23 the inverse of a below 4p (0 -> 0,
 * Montgomery form: x^-1 R for a = x R, by divsteps); products with
 * loose quotient digits, for operand bounds multiplying to at most
 * 31.99 p^2 (normal form): 24 a*b, 25 a^2, 26 a*b + (2p - b) as 18,
 * 27 a*(2b) with b carry-only (limbs of 2b below 2^30, no carry), 28 as 20,
 * 29 a*b - b'*b' with one reduction, a, b and b' as in 20 (normal form),
 * 30 the inverse of a by Fermat's little theorem (must agree with 23). */
pcmm_status pcmm_diag_field_raw(int32_t op, const uint32_t *a, const uint32_t *b, uint32_t *out,
                                int64_t count, void *stream);

/* Host-only check of the compression plan of A (m x n, row-major, elements as
 * for pcmm_cussen, bits 1..16) with `rounds` rounds (1..8) and column group
 * `group` (1..4): each group's table-build program is run on integer
 * coefficient vectors over its base points B_t (Alg. 2 reconstruction as
 * exact integer arithmetic, no GPU), and *result receives 0 when every row's
 * code names the table entry equal to its signed row segment and the table's
 * register entries follow the order of their producing ops, else 1 (entry
 * order), 2 (code outside its table), 3 (entry and row segment differ) or 4
 * (malformed program).  Errors: PCMM_EINVAL (arguments, unsupported shape),
 * PCMM_ERANGE (an entry of A outside the bit-width). */
pcmm_status pcmm_diag_plan_check(const void *A, int32_t m, int32_t n, int32_t bits, int32_t is_signed,
                                 int32_t rounds, int32_t group, int32_t *result);

/* Point operations, element-wise over count = P->rows * P->cols elements.
 * P, Q: affine npts 1.  k: device uint32 scalars (op 3).  R: Jacobian npts 1.
 * op: 0 P + Q by the mixed addition (P lifted to Z = 1);
 *     1 P + Q by the general addition, both operands first given Z != 1
 *       (Z_P = x_Q + 2, Z_Q = y_P + 3 when nonzero);
 *     2 2P; 3 k P by Alg. 1 over the low `t` bits of k; 4 -P. */
pcmm_status pcmm_diag_point(int32_t op, const pcmm_mat *P, const pcmm_mat *Q, const uint32_t *k,
                            int32_t t, pcmm_mat *R, void *stream);

/* Throughput probes.  kind: 0 v_mad_u64_u32 (32x32+64 -> 64-bit multiply-add),
 * 1 v_add3_u32 (32-bit three-input add), 2 field multiplication,
 * 3 mixed point addition, 4 v_fma_f64, 5 v_xor_b32 (lane-dependent operands,
 * so the work stays on the vector unit).  Launches `blocks` x 256 threads that
 * each run `iters` iterations; returns the kernel time (HIP events) and the
 * number of operations of that kind executed. */
pcmm_status pcmm_diag_probe(int32_t kind, int64_t iters, int32_t blocks, double *seconds,
                            double *ops);

/* Copy `words` 32-bit words from src to dst (device).  A kernel of known
 * traffic (4 * words bytes read and written once) used to calibrate hardware
 * memory-traffic counters. */
pcmm_status pcmm_diag_copy(const uint32_t *src, uint32_t *dst, int64_t words, void *stream);

/* Device properties used for roofline figures. */
pcmm_status pcmm_diag_device(int32_t *cus, int32_t *clock_khz, int64_t *lds_per_block,
                             char name[64]);

/* Paillier arithmetic mod n^2 of a context (pcmm_paillier.h), element-wise
 * over count residues given as canonical 192-word values (below n^2):
 * op 0 the raw Montgomery product a b R^-1 with R = 2^6148, 1 the product
 * a b, 2 the power a^k by Alg. 4 with k = word 0 of b (32-bit exponent),
 * 3 the power a^n (the encryption's 3072-bit exponent); all results
 * canonical (mod n^2). */
pcmm_status pcmm_paillier_diag(pcmm_paillier ctx, int32_t op, const uint32_t *a, const uint32_t *b,
                               uint32_t *out, int64_t count, void *stream);

/* The host-side constants of a Paillier modulus n (384 big-endian bytes), as
 * 256 limbs of 29 bits each: n^2, R mod n^2 and R^2 mod n^2 for R = 2^6148,
 * and n0 = -(n^2)^-1 mod 2^32.  No device work; EINVAL unless n is odd with
 * 3072 bits. */
pcmm_status pcmm_paillier_diag_constants(const uint8_t *n_be, uint32_t *N_limbs, uint32_t *one_limbs,
                                         uint32_t *r2_limbs, uint32_t *n0);

#ifdef __cplusplus
}
#endif
#endif
