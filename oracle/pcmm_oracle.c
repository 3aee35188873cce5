/*
 * pcmm_oracle.c -- plain, slow CPU reference for PC-MM over EC-ElGamal on
 * NIST P-256 (TEST INFRASTRUCTURE ONLY; see pcmm_oracle.h).
 *
 * What it follows:
 *   - prime field and curve: Sec. 4.1 (P-256, y^2 = x^3 - 3x + b over F_p,
 *     p = 2^256 - 2^224 + 2^192 + 2^96 - 1, prime order q); the constants b,
 *     G, q are the standard P-256 domain parameters (cross-checked by the tests
 *     against the system's OpenSSL);
 *   - group law with the point at infinity as identity: Sec. 2.3;
 *   - scalar multiplication: Alg. 1 (Montgomery ladder), Sec. 2.3;
 *   - EC-ElGamal KeyGen / Encrypt / Decrypt with phi(m) = mG: Sec. 2.4;
 *   - schoolbook PC-MM (n pt-ct multiplications, n-1 ct-ct additions per
 *     output): Sec. 3.1;
 *   - Cussen compression-reconstruction for one vector: Alg. 2, Sec. 3.2;
 *   - the proposed PC-MM, one column of A at a time: Alg. 3, Sec. 3.3;
 *   - closed form of the homomorphic inner product: Eq. (ahe_5_elgamal).
 *
 * Readings where the paper is silent (each is listed in the design notes):
 *   - zeros are dropped when a vector is sorted and de-duplicated (0 * C needs
 *     no operation), and the first element of a difference vector is kept;
 *   - signed plaintext entries a < 0 act as |a| (-P);
 *   - the point at infinity serialises as 64 zero bytes;
 *   - keys and nonces come from a counter-based SplitMix64 derivation.
 *
 * Deliberate independence from the GPU library: 4 x 64-bit limbs; products
 * reduced by folding with c = 2^256 mod M (no Montgomery form); inversion by
 * the binary extended Euclidean algorithm (no Fermat power); affine points.
 */
#include "pcmm_oracle.h"

#include <pthread.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;
typedef struct { uint64_t w[4]; } u256; /* little-endian 64-bit limbs */

/* ------------------------------------------------------------------------ */
/* 256-bit unsigned integers                                                */
/* ------------------------------------------------------------------------ */

static int u256_cmp(const u256 *a, const u256 *b) {
    for (int i = 3; i >= 0; --i) {
        if (a->w[i] != b->w[i]) return a->w[i] < b->w[i] ? -1 : 1;
    }
    return 0;
}

static int u256_is_zero(const u256 *a) { return (a->w[0] | a->w[1] | a->w[2] | a->w[3]) == 0; }

static int u256_is_one(const u256 *a) { return a->w[0] == 1 && (a->w[1] | a->w[2] | a->w[3]) == 0; }

static uint64_t u256_add(u256 *r, const u256 *a, const u256 *b) {
    u128 c = 0;
    for (int i = 0; i < 4; ++i) {
        c += (u128)a->w[i] + b->w[i];
        r->w[i] = (uint64_t)c;
        c >>= 64;
    }
    return (uint64_t)c;
}

static uint64_t u256_sub(u256 *r, const u256 *a, const u256 *b) {
    uint64_t borrow = 0;
    for (int i = 0; i < 4; ++i) {
        uint64_t ai = a->w[i], bi = b->w[i];
        uint64_t d = ai - bi - borrow;
        borrow = (ai < bi) || (ai == bi && borrow) ? 1 : 0;
        r->w[i] = d;
    }
    return borrow;
}

/* shift right by one bit, shifting `top` in as bit 255 */
static void u256_shr1(u256 *a, uint64_t top) {
    for (int i = 0; i < 3; ++i) a->w[i] = (a->w[i] >> 1) | (a->w[i + 1] << 63);
    a->w[3] = (a->w[3] >> 1) | (top << 63);
}

static void u256_from_be(u256 *r, const uint8_t b[32]) {
    for (int i = 0; i < 4; ++i) {
        uint64_t v = 0;
        for (int k = 0; k < 8; ++k) v = (v << 8) | b[(3 - i) * 8 + k];
        r->w[i] = v;
    }
}

static void u256_to_be(uint8_t b[32], const u256 *a) {
    for (int i = 0; i < 4; ++i) {
        uint64_t v = a->w[i];
        for (int k = 7; k >= 0; --k) { b[(3 - i) * 8 + k] = (uint8_t)v; v >>= 8; }
    }
}

static void u256_from_hex(u256 *r, const char *hex) {
    /* 64 hex digits, most significant first */
    memset(r, 0, sizeof *r);
    for (int i = 0; i < 64; ++i) {
        char ch = hex[i];
        uint64_t d = (ch >= '0' && ch <= '9') ? (uint64_t)(ch - '0')
                   : (ch >= 'a' && ch <= 'f') ? (uint64_t)(ch - 'a' + 10)
                                              : (uint64_t)(ch - 'A' + 10);
        int bit = (63 - i) * 4;
        r->w[bit / 64] |= d << (bit % 64);
    }
}

/* ------------------------------------------------------------------------ */
/* Residues modulo M, 2^255 < M < 2^256                                     */
/* ------------------------------------------------------------------------ */

typedef struct {
    u256 m; /* the modulus */
    u256 c; /* 2^256 - m = 2^256 mod m */
} modulus;

static void mod_init(modulus *M, const u256 *m) {
    u256 zero = {{0, 0, 0, 0}};
    M->m = *m;
    u256_sub(&M->c, &zero, m); /* two's complement: 2^256 - m */
}

/* r = x mod M for an (8-limb, 512-bit) x.  Writing x = hi 2^256 + lo, the
 * identity 2^256 = c (mod M) gives x = hi c + lo; repeat until hi = 0, then
 * subtract M while the value is at least M. */
static void mod_reduce_wide(u256 *r, const uint64_t xin[8], const modulus *M) {
    uint64_t x[8];
    memcpy(x, xin, sizeof x);
    while (x[4] | x[5] | x[6] | x[7]) {
        uint64_t t[8] = {0};
        for (int i = 0; i < 4; ++i) { /* t = hi * c */
            u128 carry = 0;
            for (int j = 0; j < 4; ++j) {
                carry += (u128)x[4 + i] * M->c.w[j] + t[i + j];
                t[i + j] = (uint64_t)carry;
                carry >>= 64;
            }
            t[i + 4] = (uint64_t)carry;
        }
        u128 carry = 0; /* t += lo */
        for (int i = 0; i < 8; ++i) {
            carry += (u128)t[i] + (i < 4 ? x[i] : 0);
            t[i] = (uint64_t)carry;
            carry >>= 64;
        }
        memcpy(x, t, sizeof x);
    }
    u256 v = {{x[0], x[1], x[2], x[3]}};
    while (u256_cmp(&v, &M->m) >= 0) u256_sub(&v, &v, &M->m);
    *r = v;
}

static void mod_add(u256 *r, const u256 *a, const u256 *b, const modulus *M) {
    uint64_t x[8] = {0};
    u256 s;
    uint64_t carry = u256_add(&s, a, b);
    memcpy(x, s.w, sizeof s.w);
    x[4] = carry;
    mod_reduce_wide(r, x, M);
}

static void mod_sub(u256 *r, const u256 *a, const u256 *b, const modulus *M) {
    u256 d;
    if (u256_sub(&d, a, b)) u256_add(&d, &d, &M->m); /* went negative: add M */
    *r = d;
}

static void mod_neg(u256 *r, const u256 *a, const modulus *M) {
    u256 zero = {{0, 0, 0, 0}};
    mod_sub(r, &zero, a, M);
}

static void mod_mul(u256 *r, const u256 *a, const u256 *b, const modulus *M) {
    uint64_t x[8] = {0};
    for (int i = 0; i < 4; ++i) {
        u128 carry = 0;
        for (int j = 0; j < 4; ++j) {
            carry += (u128)a->w[i] * b->w[j] + x[i + j];
            x[i + j] = (uint64_t)carry;
            carry >>= 64;
        }
        x[i + 4] = (uint64_t)carry;
    }
    mod_reduce_wide(r, x, M);
}

/* x / 2 mod M for odd M: if x is odd, x + M is even (257-bit sum). */
static void mod_half(u256 *x, const modulus *M) {
    if (x->w[0] & 1) {
        uint64_t carry = u256_add(x, x, &M->m);
        u256_shr1(x, carry);
    } else {
        u256_shr1(x, 0);
    }
}

/* Binary extended Euclidean inversion (odd modulus, a != 0 mod M).
 * Invariants: x1 a = u and x2 a = v (mod M); gcd(u, v) = 1 throughout. */
static int mod_inv(u256 *r, const u256 *ain, const modulus *M) {
    u256 a;
    {
        uint64_t x[8] = {ain->w[0], ain->w[1], ain->w[2], ain->w[3], 0, 0, 0, 0};
        mod_reduce_wide(&a, x, M);
    }
    if (u256_is_zero(&a)) return -1;
    u256 u = a, v = M->m;
    u256 x1 = {{1, 0, 0, 0}}, x2 = {{0, 0, 0, 0}};
    while (!u256_is_one(&u) && !u256_is_one(&v)) {
        while (!(u.w[0] & 1)) { u256_shr1(&u, 0); mod_half(&x1, M); }
        while (!(v.w[0] & 1)) { u256_shr1(&v, 0); mod_half(&x2, M); }
        if (u256_cmp(&u, &v) >= 0) {
            u256_sub(&u, &u, &v);
            mod_sub(&x1, &x1, &x2, M);
        } else {
            u256_sub(&v, &v, &u);
            mod_sub(&x2, &x2, &x1, M);
        }
    }
    *r = u256_is_one(&u) ? x1 : x2;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* P-256 domain parameters                                                  */
/* ------------------------------------------------------------------------ */

static modulus FP, FQ;       /* field prime p, group order q */
static u256 CURVE_B, GX, GY; /* y^2 = x^3 - 3x + b, generator G */
static pthread_once_t params_once = PTHREAD_ONCE_INIT;

static void params_init(void) {
    u256 p, q;
    u256_from_hex(&p, "ffffffff00000001000000000000000000000000ffffffffffffffffffffffff");
    u256_from_hex(&q, "ffffffff00000000ffffffffffffffffbce6faada7179e84f3b9cac2fc632551");
    u256_from_hex(&CURVE_B, "5ac635d8aa3a93e7b3ebbd55769886bc651d06b0cc53b0f63bce3c3e27d2604b");
    u256_from_hex(&GX, "6b17d1f2e12c4247f8bce6e563a440f277037d812deb33a0f4a13945d898c296");
    u256_from_hex(&GY, "4fe342e2fe1a7f9b8ee7eb4a7c0f9e162bce33576b315ececbb6406837bf51f5");
    mod_init(&FP, &p);
    mod_init(&FQ, &q);
}

static void params(void) { pthread_once(&params_once, params_init); }

/* ------------------------------------------------------------------------ */
/* Affine points and the group law (Sec. 2.3)                               */
/* ------------------------------------------------------------------------ */

typedef struct {
    u256 x, y;
    int inf; /* 1: the point at infinity (identity) */
} apt;

static apt pt_infinity(void) {
    apt r;
    memset(&r, 0, sizeof r);
    r.inf = 1;
    return r;
}

static apt pt_generator(void) {
    apt g;
    g.x = GX;
    g.y = GY;
    g.inf = 0;
    return g;
}

static apt pt_neg(const apt *P) {
    apt r = *P;
    if (!P->inf) mod_neg(&r.y, &P->y, &FP);
    return r;
}

/* The chord-and-tangent rule with every case written out:
 *   inf + Q = Q, P + inf = P;
 *   x1 = x2, y1 = -y2 (includes y = 0)  -> inf;
 *   P = Q: lambda = (3 x1^2 + a) / (2 y1), a = -3;
 *   otherwise lambda = (y2 - y1) / (x2 - x1);
 *   x3 = lambda^2 - x1 - x2, y3 = lambda (x1 - x3) - y1. */
static apt pt_add(const apt *P, const apt *Q) {
    if (P->inf) return *Q;
    if (Q->inf) return *P;
    u256 lam, num, den, t;
    if (u256_cmp(&P->x, &Q->x) == 0) {
        u256 sum;
        mod_add(&sum, &P->y, &Q->y, &FP);
        if (u256_is_zero(&sum)) return pt_infinity();
        /* here y1 = y2 != 0: tangent */
        mod_mul(&num, &P->x, &P->x, &FP);        /* x^2 */
        u256 three = {{3, 0, 0, 0}};
        mod_mul(&num, &num, &three, &FP);        /* 3 x^2 */
        mod_sub(&num, &num, &three, &FP);        /* 3 x^2 - 3 */
        mod_add(&den, &P->y, &P->y, &FP);        /* 2 y */
    } else {
        mod_sub(&num, &Q->y, &P->y, &FP);
        mod_sub(&den, &Q->x, &P->x, &FP);
    }
    mod_inv(&t, &den, &FP);
    mod_mul(&lam, &num, &t, &FP);
    apt R;
    R.inf = 0;
    mod_mul(&R.x, &lam, &lam, &FP);
    mod_sub(&R.x, &R.x, &P->x, &FP);
    mod_sub(&R.x, &R.x, &Q->x, &FP);
    mod_sub(&t, &P->x, &R.x, &FP);
    mod_mul(&R.y, &lam, &t, &FP);
    mod_sub(&R.y, &R.y, &P->y, &FP);
    return R;
}

static apt pt_dbl(const apt *P) { return pt_add(P, P); }

static int pt_on_curve(const apt *P) {
    if (P->inf) return 1;
    if (u256_cmp(&P->x, &FP.m) >= 0 || u256_cmp(&P->y, &FP.m) >= 0) return 0;
    u256 lhs, rhs, t;
    mod_mul(&lhs, &P->y, &P->y, &FP);
    mod_mul(&rhs, &P->x, &P->x, &FP);
    mod_mul(&rhs, &rhs, &P->x, &FP); /* x^3 */
    u256 three = {{3, 0, 0, 0}};
    mod_mul(&t, &P->x, &three, &FP);
    mod_sub(&rhs, &rhs, &t, &FP);
    mod_add(&rhs, &rhs, &CURVE_B, &FP);
    return u256_cmp(&lhs, &rhs) == 0;
}


static void pt_to_bytes(uint8_t out[64], const apt *P) {
    if (P->inf) { memset(out, 0, 64); return; }
    u256_to_be(out, &P->x);
    u256_to_be(out + 32, &P->y);
}

static apt pt_from_bytes(const uint8_t in[64]) {
    apt P;
    int allzero = 1;
    for (int i = 0; i < 64; ++i) allzero &= in[i] == 0;
    if (allzero) return pt_infinity();
    u256_from_be(&P.x, in);
    u256_from_be(&P.y, in + 32);
    P.inf = 0;
    return P;
}

/* ------------------------------------------------------------------------ */
/* Scalar multiplication: Alg. 1, Montgomery ladder                          */
/* ------------------------------------------------------------------------ */

/* bit(i) of the scalar is supplied by a callback so that one ladder serves
 * small (uint64) and 256-bit scalars. */
typedef int (*bit_fn)(const void *k, int i);

static int bit_u64(const void *k, int i) { return (int)((*(const uint64_t *)k >> i) & 1); }
static int bit_u256(const void *k, int i) { return (int)((((const u256 *)k)->w[i / 64] >> (i % 64)) & 1); }

static apt ladder(const void *k, bit_fn bit, int t, const apt *P) {
    apt R[2];
    R[0] = pt_infinity();
    R[1] = *P;
    for (int i = t - 1; i >= 0; --i) {
        int b = bit(k, i);
        apt sum = pt_add(&R[1], &R[0]); /* R_{1-b} <- R_1 + R_0 */
        apt dbl = pt_dbl(&R[b]);        /* R_b     <- 2 R_b     */
        R[1 - b] = sum;
        R[b] = dbl;
    }
    return R[0];
}

static int bitlen_u64(uint64_t k) {
    int t = 0;
    while (k) { ++t; k >>= 1; }
    return t;
}

/* k P for a small non-negative k, by Alg. 1 over the bit length of k */
static apt smul_small(uint64_t k, const apt *P) { return ladder(&k, bit_u64, bitlen_u64(k), P); }

/* s P for a signed small s: |s| (-P) when s < 0 */
static apt smul_signed(int64_t s, const apt *P) {
    if (s < 0) {
        apt n = pt_neg(P);
        return smul_small((uint64_t)(-s), &n);
    }
    return smul_small((uint64_t)s, P);
}

static apt smul_big(const u256 *k, const apt *P) { return ladder(k, bit_u256, 256, P); }

/* ------------------------------------------------------------------------ */
/* Key and nonce derivation (counter-based SplitMix64 mixing)               */
/* ------------------------------------------------------------------------ */

/* SplitMix64 output function (Steele, Lea, Flood 2014; public domain
 * reference code by S. Vigna). */
static uint64_t mix64(uint64_t z) {
    z ^= z >> 30;
    z *= 0xBF58476D1CE4E5B9ULL;
    z ^= z >> 27;
    z *= 0x94D049BB133111EBULL;
    z ^= z >> 31;
    return z;
}

/* 320 pseudo-random bits w_0..w_4 from (seed, domain, idx); the scalar is
 * X mod (q - 1) + 1, which lies in [1, q - 1]. */
static u256 scalar_from_seed(uint64_t seed, uint64_t domain, uint64_t idx) {
    params();
    uint64_t base = mix64(seed ^ (domain << 56) ^ idx);
    uint64_t X[8] = {0};
    for (int i = 0; i < 5; ++i) X[i] = mix64(base + (uint64_t)(i + 1) * 0x9E3779B97F4A7C15ULL);
    u256 qm1 = FQ.m;
    qm1.w[0] -= 1; /* q is odd, no borrow */
    modulus Mq1;
    mod_init(&Mq1, &qm1);
    u256 r;
    mod_reduce_wide(&r, X, &Mq1);
    u256 one = {{1, 0, 0, 0}};
    u256_add(&r, &r, &one);
    return r;
}

/* a mod q for a signed machine integer */
static u256 scalar_from_int(int64_t a) {
    u256 r = {{0, 0, 0, 0}};
    if (a >= 0) {
        r.w[0] = (uint64_t)a;
    } else {
        u256 t = {{(uint64_t)(-a), 0, 0, 0}};
        mod_neg(&r, &t, &FQ);
    }
    return r;
}

/* ------------------------------------------------------------------------ */
/* Small thread pool helper: run f(ctx, item) for item in [0, count)         */
/* ------------------------------------------------------------------------ */

typedef void (*item_fn)(void *ctx, int64_t item);

typedef struct {
    item_fn f;
    void *ctx;
    int64_t count;
    int64_t next;
    pthread_mutex_t lock;
} pool_job;

static void *pool_worker(void *arg) {
    pool_job *job = (pool_job *)arg;
    for (;;) {
        pthread_mutex_lock(&job->lock);
        int64_t it = job->next++;
        pthread_mutex_unlock(&job->lock);
        if (it >= job->count) break;
        job->f(job->ctx, it);
    }
    return NULL;
}

static void run_parallel(item_fn f, void *ctx, int64_t count, int nthreads) {
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    pool_job job;
    job.f = f;
    job.ctx = ctx;
    job.count = count;
    job.next = 0;
    pthread_mutex_init(&job.lock, NULL);
    if (nthreads == 1 || count <= 1) {
        pool_worker(&job);
    } else {
        pthread_t th[256];
        int started = 0;
        for (int i = 0; i < nthreads; ++i) {
            if (pthread_create(&th[i], NULL, pool_worker, &job) == 0) ++started;
        }
        if (started == 0) pool_worker(&job);
        for (int i = 0; i < started; ++i) pthread_join(th[i], NULL);
    }
    pthread_mutex_destroy(&job.lock);
}

/* ------------------------------------------------------------------------ */
/* Alg. 2: Cussen compression-reconstruction for one vector                  */
/* ------------------------------------------------------------------------ */

#define ALG2_MAX_ROUNDS 16

typedef struct {
    int N;
    int len[ALG2_MAX_ROUNDS + 1];        /* n_0 .. n_N */
    int64_t *val[ALG2_MAX_ROUNDS + 1];   /* a^(w): after the difference step for w < N */
    int *ptr[ALG2_MAX_ROUNDS + 1];       /* ptr[w][i], i < n_{w-1}: position in a^(w) of
                                            element i of a^(w-1), or -1 for a zero */
} alg2_plan;

static int cmp_i64(const void *a, const void *b) {
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return (x > y) - (x < y);
}

static void alg2_free(alg2_plan *P) {
    for (int w = 0; w <= P->N; ++w) {
        free(P->val[w]);
        free(P->ptr[w]);
        P->val[w] = NULL;
        P->ptr[w] = NULL;
    }
}

/* Compression phase.  a: n values >= 0. */
static int alg2_compress(alg2_plan *P, const int64_t *a, int n, int N) {
    if (N < 1 || N > ALG2_MAX_ROUNDS || n < 0) return -1;
    memset(P, 0, sizeof *P);
    P->N = N;
    P->len[0] = n;
    P->val[0] = (int64_t *)malloc(sizeof(int64_t) * (n > 0 ? n : 1));
    if (n > 0) memcpy(P->val[0], a, sizeof(int64_t) * n);
    for (int w = 1; w <= N; ++w) {
        int prev = P->len[w - 1];
        const int64_t *src = P->val[w - 1];
        /* sort, drop zeros, eliminate duplicates */
        int64_t *tmp = (int64_t *)malloc(sizeof(int64_t) * (prev > 0 ? prev : 1));
        int cnt = 0;
        for (int i = 0; i < prev; ++i) if (src[i] != 0) tmp[cnt++] = src[i];
        qsort(tmp, cnt, sizeof(int64_t), cmp_i64);
        int u = 0;
        for (int i = 0; i < cnt; ++i) if (u == 0 || tmp[i] != tmp[u - 1]) tmp[u++] = tmp[i];
        P->len[w] = u;
        P->val[w] = tmp;
        /* tracking pointers: where each element of a^(w-1) went */
        P->ptr[w] = (int *)malloc(sizeof(int) * (prev > 0 ? prev : 1));
        for (int i = 0; i < prev; ++i) {
            if (src[i] == 0) { P->ptr[w][i] = -1; continue; }
            int lo = 0, hi = u - 1;
            while (lo < hi) {
                int mid = (lo + hi) / 2;
                if (tmp[mid] < src[i]) lo = mid + 1; else hi = mid;
            }
            P->ptr[w][i] = lo;
        }
        /* differences of consecutive elements, except in the last round */
        if (w != N) {
            for (int i = u - 1; i >= 1; --i) tmp[i] -= tmp[i - 1];
        }
    }
    return 0;
}

/* Reconstruction on plain integers. */
static void alg2_reconstruct_int(const alg2_plan *P, int64_t Cs, int64_t *out, int64_t *muls,
                                 int64_t *adds) {
    int N = P->N;
    int64_t nm = 0, na = 0;
    int cur_len = P->len[N];
    int64_t *cur = (int64_t *)malloc(sizeof(int64_t) * (cur_len > 0 ? cur_len : 1));
    for (int i = 0; i < cur_len; ++i) cur[i] = Cs * P->val[N][i];
    nm += cur_len;
    for (int w = N; w >= 1; --w) {
        if (w != N) {
            for (int i = 0; i + 1 < cur_len; ++i) cur[i + 1] += cur[i];
            na += cur_len; /* counting convention: n_w additions at level w */
        }
        int prev = P->len[w - 1];
        int64_t *nxt = (int64_t *)malloc(sizeof(int64_t) * (prev > 0 ? prev : 1));
        for (int i = 0; i < prev; ++i) nxt[i] = P->ptr[w][i] < 0 ? 0 : cur[P->ptr[w][i]];
        free(cur);
        cur = nxt;
        cur_len = prev;
    }
    memcpy(out, cur, sizeof(int64_t) * P->len[0]);
    free(cur);
    if (muls) *muls = nm;
    if (adds) *adds = na;
}

/* Reconstruction with a point as the scalar: ECSMs at level N (Alg. 1),
 * prefix sums by point additions, un-sorting by the tracking pointers. */
static void alg2_reconstruct_point(const alg2_plan *P, const apt *B, apt *out) {
    int N = P->N;
    int cur_len = P->len[N];
    apt *cur = (apt *)malloc(sizeof(apt) * (cur_len > 0 ? cur_len : 1));
    for (int i = 0; i < cur_len; ++i) cur[i] = smul_small((uint64_t)P->val[N][i], B);
    for (int w = N; w >= 1; --w) {
        if (w != N) {
            for (int i = 0; i + 1 < cur_len; ++i) cur[i + 1] = pt_add(&cur[i + 1], &cur[i]);
        }
        int prev = P->len[w - 1];
        apt *nxt = (apt *)malloc(sizeof(apt) * (prev > 0 ? prev : 1));
        for (int i = 0; i < prev; ++i) nxt[i] = P->ptr[w][i] < 0 ? pt_infinity() : cur[P->ptr[w][i]];
        free(cur);
        cur = nxt;
        cur_len = prev;
    }
    memcpy(out, cur, sizeof(apt) * P->len[0]);
    free(cur);
}

/* ------------------------------------------------------------------------ */
/* Exported: arithmetic and curve                                           */
/* ------------------------------------------------------------------------ */

int oracle_mod_op(int mod, int op, const uint8_t a[32], const uint8_t b[32], uint8_t out[32]) {
    params();
    const modulus *M = mod == 0 ? &FP : mod == 1 ? &FQ : NULL;
    if (!M) return -1;
    u256 x, y, r;
    u256_from_be(&x, a);
    u256_from_be(&y, b);
    /* inputs may be any 256-bit value: reduce first */
    uint64_t wx[8] = {x.w[0], x.w[1], x.w[2], x.w[3], 0, 0, 0, 0};
    uint64_t wy[8] = {y.w[0], y.w[1], y.w[2], y.w[3], 0, 0, 0, 0};
    mod_reduce_wide(&x, wx, M);
    mod_reduce_wide(&y, wy, M);
    switch (op) {
        case 0: mod_add(&r, &x, &y, M); break;
        case 1: mod_sub(&r, &x, &y, M); break;
        case 2: mod_mul(&r, &x, &y, M); break;
        case 3: if (mod_inv(&r, &x, M)) return -2; break;
        case 4: mod_neg(&r, &x, M); break;
        default: return -1;
    }
    u256_to_be(out, &r);
    return 0;
}

void oracle_curve_params(uint8_t out[160]) {
    params();
    u256_to_be(out, &FP.m);
    u256_to_be(out + 32, &CURVE_B);
    u256_to_be(out + 64, &GX);
    u256_to_be(out + 96, &GY);
    u256_to_be(out + 128, &FQ.m);
}

int oracle_pt_add(const uint8_t P[64], const uint8_t Q[64], uint8_t R[64]) {
    params();
    apt a = pt_from_bytes(P), b = pt_from_bytes(Q);
    apt r = pt_add(&a, &b);
    pt_to_bytes(R, &r);
    return 0;
}

int oracle_pt_dbl(const uint8_t P[64], uint8_t R[64]) {
    params();
    apt a = pt_from_bytes(P);
    apt r = pt_dbl(&a);
    pt_to_bytes(R, &r);
    return 0;
}

int oracle_pt_neg(const uint8_t P[64], uint8_t R[64]) {
    params();
    apt a = pt_from_bytes(P);
    apt r = pt_neg(&a);
    pt_to_bytes(R, &r);
    return 0;
}

int oracle_on_curve(const uint8_t P[64]) {
    params();
    apt a = pt_from_bytes(P);
    return pt_on_curve(&a);
}

int oracle_ladder_small(uint64_t k, int t, const uint8_t P[64], uint8_t R[64]) {
    params();
    if (t < 0 || t > 64) return -1;
    apt a = pt_from_bytes(P);
    apt r = ladder(&k, bit_u64, t, &a);
    pt_to_bytes(R, &r);
    return 0;
}

int oracle_ladder_big(const uint8_t k[32], const uint8_t P[64], uint8_t R[64]) {
    params();
    u256 s;
    u256_from_be(&s, k);
    apt a = pt_from_bytes(P);
    apt r = smul_big(&s, &a);
    pt_to_bytes(R, &r);
    return 0;
}

int oracle_repeated_add(uint64_t k, const uint8_t P[64], uint8_t R[64]) {
    params();
    apt a = pt_from_bytes(P);
    apt r = pt_infinity();
    if (k > 0) {
        r = a;
        for (uint64_t i = 1; i < k; ++i) r = pt_add(&r, &a);
    }
    pt_to_bytes(R, &r);
    return 0;
}

void oracle_scalar_from_seed(uint64_t seed, uint64_t domain, uint64_t idx, uint8_t out[32]) {
    u256 s = scalar_from_seed(seed, domain, idx);
    u256_to_be(out, &s);
}

/* ------------------------------------------------------------------------ */
/* Exported: EC-ElGamal (Sec. 2.4)                                          */
/* ------------------------------------------------------------------------ */

int oracle_keygen(uint64_t seed, uint8_t sk[32], uint8_t pk[64]) {
    params();
    u256 x = scalar_from_seed(seed, 0, 0);
    apt G = pt_generator();
    apt H = smul_big(&x, &G);
    u256_to_be(sk, &x);
    pt_to_bytes(pk, &H);
    return 0;
}

typedef struct {
    apt H;
    const int32_t *msg;
    uint64_t seed;
    int64_t idx0;
    const int64_t *idx; /* optional explicit nonce indices */
    uint8_t *out;
} enc_ctx;

static void enc_item(void *vctx, int64_t e) {
    enc_ctx *c = (enc_ctx *)vctx;
    apt G = pt_generator();
    u256 r = scalar_from_seed(c->seed, 1, (uint64_t)(c->idx ? c->idx[e] : c->idx0 + e));
    u256 mq = scalar_from_int(c->msg[e]);
    apt C1 = smul_big(&r, &G);
    apt rH = smul_big(&r, &c->H);
    apt mG = smul_big(&mq, &G);
    apt C2 = pt_add(&rH, &mG);
    pt_to_bytes(c->out + e * 128, &C1);
    pt_to_bytes(c->out + e * 128 + 64, &C2);
}

int oracle_encrypt(const uint8_t pk[64], const int32_t *msg, int64_t count, uint64_t seed,
                   int64_t idx0, uint8_t *ct_out, int nthreads) {
    params();
    if (count < 0) return -1;
    enc_ctx c;
    c.H = pt_from_bytes(pk);
    c.msg = msg;
    c.seed = seed;
    c.idx0 = idx0;
    c.idx = NULL;
    c.out = ct_out;
    run_parallel(enc_item, &c, count, nthreads);
    return 0;
}

int oracle_encrypt_indexed(const uint8_t pk[64], const int32_t *msg, const int64_t *idx, int64_t count,
                           uint64_t seed, uint8_t *ct_out, int nthreads) {
    params();
    if (count < 0 || (count > 0 && !idx)) return -1;
    enc_ctx c;
    c.H = pt_from_bytes(pk);
    c.msg = msg;
    c.seed = seed;
    c.idx0 = 0;
    c.idx = idx;
    c.out = ct_out;
    run_parallel(enc_item, &c, count, nthreads);
    return 0;
}

typedef struct {
    u256 x;
    const uint8_t *ct;
    uint8_t *out;
} dec_ctx;

static void dec_item(void *vctx, int64_t e) {
    dec_ctx *c = (dec_ctx *)vctx;
    apt C1 = pt_from_bytes(c->ct + e * 128);
    apt C2 = pt_from_bytes(c->ct + e * 128 + 64);
    apt xC1 = smul_big(&c->x, &C1);
    apt neg = pt_neg(&xC1);
    apt M = pt_add(&C2, &neg);
    pt_to_bytes(c->out + e * 64, &M);
}

int oracle_decrypt_to_points(const uint8_t sk[32], const uint8_t *ct, int64_t count,
                             uint8_t *pt_out, int nthreads) {
    params();
    if (count < 0) return -1;
    dec_ctx c;
    u256_from_be(&c.x, sk);
    c.ct = ct;
    c.out = pt_out;
    run_parallel(dec_item, &c, count, nthreads);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Exported: Alg. 2                                                          */
/* ------------------------------------------------------------------------ */

int oracle_alg2_plain(const int64_t *a, int n, int N, int64_t Cs, int64_t *out, int64_t *muls,
                      int64_t *adds, int *lens) {
    for (int i = 0; i < n; ++i) if (a[i] < 0) return -1;
    alg2_plan P;
    if (alg2_compress(&P, a, n, N)) return -1;
    alg2_reconstruct_int(&P, Cs, out, muls, adds);
    if (lens) for (int w = 0; w <= N; ++w) lens[w] = P.len[w];
    alg2_free(&P);
    return 0;
}

int oracle_alg2_point(const int64_t *a, int n, int N, const uint8_t Pb[64], uint8_t *out) {
    params();
    for (int i = 0; i < n; ++i) if (a[i] < 0) return -1;
    alg2_plan P;
    if (alg2_compress(&P, a, n, N)) return -1;
    apt B = pt_from_bytes(Pb);
    apt *res = (apt *)malloc(sizeof(apt) * (n > 0 ? n : 1));
    alg2_reconstruct_point(&P, &B, res);
    for (int i = 0; i < n; ++i) pt_to_bytes(out + (int64_t)i * 64, &res[i]);
    free(res);
    alg2_free(&P);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Exported: PC-MM                                                           */
/* ------------------------------------------------------------------------ */

/* A holds the plaintext values themselves (int32), row-major m x n */
static int64_t a_at(const int32_t *A, int64_t idx) { return (int64_t)A[idx]; }

typedef struct {
    const int32_t *A;
    int m, n, l, N;
    const uint8_t *B;
    uint8_t *C;
    const int32_t *cols;
    alg2_plan *plans; /* Cussen: one compressed column of A per k */
} mm_ctx;

static int mm_col(const mm_ctx *c, int64_t item) { return c->cols ? c->cols[item] : (int)item; }

/* Sec. 3.1: c_ij = sum_k a_ik Enc(b_kj), each product by Alg. 1 */
static void school_item(void *vctx, int64_t item) {
    mm_ctx *c = (mm_ctx *)vctx;
    int j = mm_col(c, item);
    for (int i = 0; i < c->m; ++i) {
        for (int pt = 0; pt < 2; ++pt) {
            apt acc = pt_infinity();
            for (int k = 0; k < c->n; ++k) {
                apt Bk = pt_from_bytes(c->B + ((int64_t)k * c->l + j) * 128 + pt * 64);
                apt term = smul_signed(a_at(c->A, (int64_t)i * c->n + k), &Bk);
                acc = pt_add(&acc, &term);
            }
            pt_to_bytes(c->C + ((int64_t)i * c->l + j) * 128 + pt * 64, &acc);
        }
    }
}

/* Alg. 3 for one output column j: for every k, reconstruct the column of the
 * k-th outer product from the compressed k-th column of A and accumulate. */
static void cussen_item(void *vctx, int64_t item) {
    mm_ctx *c = (mm_ctx *)vctx;
    int j = mm_col(c, item);
    int m = c->m;
    apt *acc = (apt *)malloc(sizeof(apt) * 2 * (m > 0 ? m : 1));
    apt *col = (apt *)malloc(sizeof(apt) * (m > 0 ? m : 1));
    for (int i = 0; i < 2 * m; ++i) acc[i] = pt_infinity();
    for (int k = 0; k < c->n; ++k) {
        for (int pt = 0; pt < 2; ++pt) {
            apt Bk = pt_from_bytes(c->B + ((int64_t)k * c->l + j) * 128 + pt * 64);
            alg2_reconstruct_point(&c->plans[k], &Bk, col); /* |a_ik| B_kj */
            for (int i = 0; i < m; ++i) {
                apt term = col[i];
                if (a_at(c->A, (int64_t)i * c->n + k) < 0) term = pt_neg(&term);
                acc[2 * i + pt] = pt_add(&acc[2 * i + pt], &term);
            }
        }
    }
    for (int i = 0; i < m; ++i)
        for (int pt = 0; pt < 2; ++pt)
            pt_to_bytes(c->C + ((int64_t)i * c->l + j) * 128 + pt * 64, &acc[2 * i + pt]);
    free(acc);
    free(col);
}

static int mm_check(int m, int n, int l, const int32_t *cols, int ncols) {
    if (m < 0 || n < 0 || l < 0) return -1;
    if (cols && ncols >= 0)
        for (int i = 0; i < ncols; ++i) if (cols[i] < 0 || cols[i] >= l) return -1;
    return 0;
}

int oracle_pcmm_schoolbook(const int32_t *A, int m, int n, int l,
                           const uint8_t *B, uint8_t *C, const int32_t *cols, int ncols,
                           int nthreads) {
    params();
    if (mm_check(m, n, l, cols, ncols)) return -1;
    mm_ctx c = {A, m, n, l, 0, B, C, ncols >= 0 ? cols : NULL, NULL};
    run_parallel(school_item, &c, ncols >= 0 ? ncols : l, nthreads);
    return 0;
}

int oracle_pcmm_cussen(const int32_t *A, int m, int n, int l, int N,
                       const uint8_t *B, uint8_t *C, const int32_t *cols, int ncols,
                       int nthreads) {
    params();
    if (mm_check(m, n, l, cols, ncols) || N < 1 || N > ALG2_MAX_ROUNDS) return -1;
    /* compression of every column of A, shared by all output columns (Sec. 3.3) */
    alg2_plan *plans = (alg2_plan *)calloc(n > 0 ? n : 1, sizeof(alg2_plan));
    int64_t *colv = (int64_t *)malloc(sizeof(int64_t) * (m > 0 ? m : 1));
    for (int k = 0; k < n; ++k) {
        for (int i = 0; i < m; ++i) {
            int64_t a = a_at(A, (int64_t)i * n + k);
            colv[i] = a < 0 ? -a : a;
        }
        alg2_compress(&plans[k], colv, m, N);
    }
    free(colv);
    mm_ctx c = {A, m, n, l, N, B, C, ncols >= 0 ? cols : NULL, plans};
    run_parallel(cussen_item, &c, ncols >= 0 ? ncols : l, nthreads);
    for (int k = 0; k < n; ++k) alg2_free(&plans[k]);
    free(plans);
    return 0;
}

typedef struct {
    const int32_t *A;
    int m, n, l;
    u256 x;
    const int32_t *msg;
    uint64_t seed;
    const int32_t *ii, *jj;
    uint8_t *out;
} cf_ctx;

static void cf_item(void *vctx, int64_t p) {
    cf_ctx *c = (cf_ctx *)vctx;
    int i = c->ii[p], j = c->jj[p];
    u256 e1 = {{0, 0, 0, 0}}, e2 = {{0, 0, 0, 0}}, t, u;
    for (int k = 0; k < c->n; ++k) {
        u256 a = scalar_from_int(a_at(c->A, (int64_t)i * c->n + k));
        u256 r = scalar_from_seed(c->seed, 1, (uint64_t)k * (uint64_t)c->l + (uint64_t)j);
        u256 mk = scalar_from_int(c->msg[(int64_t)k * c->l + j]);
        mod_mul(&t, &a, &r, &FQ);
        mod_add(&e1, &e1, &t, &FQ);          /* e1 += a r            */
        mod_mul(&u, &c->x, &r, &FQ);
        mod_add(&u, &u, &mk, &FQ);           /* x r + m              */
        mod_mul(&u, &a, &u, &FQ);
        mod_add(&e2, &e2, &u, &FQ);          /* e2 += a (x r + m)    */
    }
    apt G = pt_generator();
    apt C1 = smul_big(&e1, &G);
    apt C2 = smul_big(&e2, &G);
    pt_to_bytes(c->out + p * 128, &C1);
    pt_to_bytes(c->out + p * 128 + 64, &C2);
}

int oracle_pcmm_closed_form(const int32_t *A, int m, int n, int l,
                            const uint8_t sk[32], const int32_t *msg, uint64_t seed,
                            const int32_t *ii, const int32_t *jj, int npos, uint8_t *out,
                            int nthreads) {
    params();
    if (m < 0 || n < 0 || l < 0 || npos < 0) return -1;
    for (int p = 0; p < npos; ++p)
        if (ii[p] < 0 || ii[p] >= m || jj[p] < 0 || jj[p] >= l) return -1;
    cf_ctx c;
    c.A = A;
    c.m = m;
    c.n = n;
    c.l = l;
    u256_from_be(&c.x, sk);
    c.msg = msg;
    c.seed = seed;
    c.ii = ii;
    c.jj = jj;
    c.out = out;
    run_parallel(cf_item, &c, npos, nthreads);
    return 0;
}
