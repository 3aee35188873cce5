// k_elgamal.hip -- EC-ElGamal KeyGen / Encrypt / Decrypt-to-point (Sec. 2.4).
//
// Fixed-base scalar multiplication by 4-bit windows: for a base point B the
// table holds d 2^(4w) B for w = 0..63, d = 1..15 (affine, Montgomery form),
// so k B = sum_w T[w][digit_w(k)] costs at most 64 mixed additions and no
// doublings.  The generator's table is built once per device and kept; the
// public key's table is built per pcmm_encrypt call in the caller's
// workspace.  Decryption multiplies each C1 by the secret scalar with a plain
// left-to-right double-and-add (the scalar is the same on every lane, so the
// control flow is uniform).
#include <mutex>

#include "common.hpp"
#include "elgamal.hpp"
#include "normalize.hpp"

using namespace pcmm;

namespace {

constexpr int WINDOWS = 64;
constexpr int DIGITS = 15;
constexpr int TABLE_POINTS = WINDOWS * DIGITS;  // 960

// ---------------------------------------------------------------------------
// Scalar derivation: SplitMix64 output function (Steele, Lea, Flood 2014),
// 320 bits, reduced mod (q - 1), plus one.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z ^= z >> 30;
    z *= 0xBF58476D1CE4E5B9ull;
    z ^= z >> 27;
    z *= 0x94D049BB133111EBull;
    z ^= z >> 31;
    return z;
}

constexpr fe_const QM1 = c_sub(ORDER_Q, ONE_PLAIN);                      // q - 1
constexpr fe_const ZERO_C = {{0, 0, 0, 0, 0, 0, 0, 0}};
constexpr fe_const FOLD_QM1 = c_sub(ZERO_C, QM1);                         // 2^256 - (q - 1)

__device__ bool geq8(const uint32_t a[8], const fe_const &m) {
    for (int i = 7; i >= 0; --i) {
        if (a[i] != m.v[i]) return a[i] > m.v[i];
    }
    return true;
}

__device__ void derive_scalar(uint64_t seed, uint64_t domain, uint64_t idx, uint32_t out[8]) {
    uint64_t base = mix64(seed ^ (domain << 56) ^ idx);
    uint32_t x[10];
    for (int i = 0; i < 5; ++i) {
        uint64_t w = mix64(base + (uint64_t)(i + 1) * 0x9E3779B97F4A7C15ull);
        x[2 * i] = (uint32_t)w;
        x[2 * i + 1] = (uint32_t)(w >> 32);
    }
    // x = hi 2^256 + lo = hi (2^256 - M) + lo (mod M), repeated while hi != 0
    for (int round = 0; round < 16 && (x[8] | x[9]); ++round) {
        uint32_t hi[2] = {x[8], x[9]};
        uint32_t y[10];
        for (int i = 0; i < 10; ++i) y[i] = i < 8 ? x[i] : 0;
        for (int i = 0; i < 2; ++i) {
            uint64_t carry = 0;
            for (int j = 0; j < 8; ++j) {
                uint64_t s = (uint64_t)hi[i] * FOLD_QM1.v[j] + y[i + j] + carry;
                y[i + j] = (uint32_t)s;
                carry = s >> 32;
            }
            for (int j = i + 8; j < 10 && carry; ++j) {
                uint64_t s = (uint64_t)y[j] + carry;
                y[j] = (uint32_t)s;
                carry = s >> 32;
            }
        }
        for (int i = 0; i < 10; ++i) x[i] = y[i];
    }
    while (geq8(x, QM1)) {
        uint64_t bw = 0;
        for (int i = 0; i < 8; ++i) {
            uint64_t d = (uint64_t)x[i] - QM1.v[i] - bw;
            x[i] = (uint32_t)d;
            bw = d >> 63;
        }
    }
    uint64_t c = 1;
    for (int i = 0; i < 8; ++i) {
        c += x[i];
        x[i] = (uint32_t)c;
        c >>= 32;
    }
    for (int i = 0; i < 8; ++i) out[i] = x[i];
}

__device__ __forceinline__ apt table_entry(const uint32_t *__restrict__ tab, int idx) {
    return load_aff_m(tab, TABLE_POINTS, 0, idx);
}

// k B from the 4-bit window table of B (k as 8 little-endian words)
__device__ jpt fixed_base_mul(const uint32_t *__restrict__ tab, const uint32_t k[8]) {
    jpt acc = jpt_infinity();
    for (int w = 0; w < WINDOWS; ++w) {
        uint32_t d = (k[w >> 3] >> ((w & 7) * 4)) & 15u;
        if (d) acc = jpt_add_affine(acc, table_entry(tab, w * DIGITS + (int)d - 1));
    }
    return acc;
}

struct point16 {
    uint32_t w[16];  // canonical affine x (8 words) then y (8 words)
};

__device__ __forceinline__ apt point16_mont(const point16 &p) {
    apt a;
    a.x = fe_to_mont(fe_from_words(p.w));
    a.y = fe_to_mont(fe_from_words(p.w + 8));
    return a;
}

// 2^(4w) B and its multiples for window w = thread index (Jacobian, Montgomery)
__global__ void __launch_bounds__(64) fixed_base_table_kernel(point16 base, uint32_t *__restrict__ jac_tmp) {
    int w = threadIdx.x;
    if (w >= WINDOWS) return;
    apt b = point16_mont(base);
    jpt P = jpt_from_affine(b);
    for (int i = 0; i < 4 * w; ++i) P = jpt_dbl(P);
    jpt T = P;
    store_jac_m(jac_tmp, TABLE_POINTS, 0, w * DIGITS, T);
    for (int d = 2; d <= DIGITS; ++d) {
        T = jpt_add(T, P);
        store_jac_m(jac_tmp, TABLE_POINTS, 0, w * DIGITS + d - 1, T);
    }
}

// flag = 1 if the canonical affine point is a finite point on the curve
__global__ void on_curve_kernel(point16 p, uint32_t *flag) {
    if (threadIdx.x != 0) return;
    fe xc = fe_from_words(p.w), yc = fe_from_words(p.w + 8);
    // reject non-canonical coordinates (>= p): the round trip would change them
    fe x = fe_to_mont(xc), y = fe_to_mont(yc);
    bool canon = fe_raw_eq(fe_from_mont(x), xc) && fe_raw_eq(fe_from_mont(y), yc);
    fe b = fe_to_mont(fe_from_const(CURVE_B_PLAIN));
    fe rhs = fe_mul(fe_sqr(x), x);
    fe x3 = fe_add(fe_dbl(x), x);
    rhs = fe_add(fe_sub(rhs, x3), b);
    bool ok = canon && fe_eq(fe_sqr(y), rhs) && !(fe_is_raw_zero(xc) && fe_is_raw_zero(yc));
    *flag = ok ? 1u : 0u;
}

__global__ void __launch_bounds__(256) encrypt_kernel(const uint32_t *__restrict__ tabG,
                                                      const uint32_t *__restrict__ tabH,
                                                      const int32_t *__restrict__ msg, int64_t n,
                                                      uint64_t seed, int64_t idx0,
                                                      uint32_t *__restrict__ out, int64_t ld) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    uint32_t r[8];
    derive_scalar(seed, 1, (uint64_t)(idx0 + e), r);
    jpt C1 = fixed_base_mul(tabG, r);
    jpt rH = fixed_base_mul(tabH, r);
    int32_t m = msg[e];
    uint32_t am = m < 0 ? 0u - (uint32_t)m : (uint32_t)m;
    jpt mG = jpt_infinity();
    for (int w = 0; w < 8; ++w) {
        uint32_t d = (am >> (4 * w)) & 15u;
        if (d) mG = jpt_add_affine(mG, table_entry(tabG, w * DIGITS + (int)d - 1));
    }
    if (m < 0) mG = jpt_neg(mG);
    jpt C2 = jpt_add(rH, mG);
    // one inversion for both points (Montgomery's trick on two values)
    bool inf1 = jpt_is_inf(C1), inf2 = jpt_is_inf(C2);
    fe z1 = inf1 ? fe_one_mont() : C1.Z;
    fe z2 = inf2 ? fe_one_mont() : C2.Z;
    fe inv = fe_inv(fe_mul(z1, z2));
    apt A1 = jpt_to_affine_with(C1, fe_mul(inv, z2));
    apt A2 = jpt_to_affine_with(C2, fe_mul(inv, z1));
    if (inf1) A1.x = A1.y = fe_zero();
    if (inf2) A2.x = A2.y = fe_zero();
    store_affine(out, ld, 0, e, A1);
    store_affine(out, ld, 1, e, A2);
}

struct scalar8 {
    uint32_t w[8];
};

__global__ void __launch_bounds__(256) decrypt_kernel(scalar8 x, const uint32_t *__restrict__ C, int64_t ldc,
                                                      uint32_t *__restrict__ M, int64_t ldm, int64_t n) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    apt c1 = load_affine(C, ldc, 0, e);
    apt c2 = load_affine(C, ldc, 1, e);
    jpt acc = jpt_infinity();
    int top = 255;
    while (top >= 0 && !((x.w[top >> 5] >> (top & 31)) & 1u)) --top;
    // few lanes per call and one long dependent chain each: the split
    // product form (lower latency per product) suits this kernel
    for (int i = top; i >= 0; --i) {
        acc = jpt_dbl<false>(acc);
        if ((x.w[i >> 5] >> (i & 31)) & 1u) acc = jpt_add_affine<false>(acc, c1);
    }
    jpt R = jpt_add<false>(jpt_from_affine(c2), jpt_neg(acc));
    apt A;
    if (jpt_is_inf(R)) {
        A.x = A.y = fe_zero();
    } else {
        A = jpt_to_affine_with(R, fe_inv(R.Z));
    }
    store_affine(M, ldm, 0, e, A);
}

// keygen: x = scalar(seed, 0, 0), H = xG; out = [x canonical (8) | Hx (8) | Hy (8)]
__global__ void keygen_kernel(const uint32_t *__restrict__ tabG, uint64_t seed, uint32_t *out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    uint32_t x[8];
    derive_scalar(seed, 0, 0, x);
    jpt H = fixed_base_mul(tabG, x);
    apt A = jpt_to_affine_with(H, fe_inv(H.Z));
    for (int i = 0; i < 8; ++i) out[i] = x[i];
    fe_to_words(fe_from_mont(A.x), out + 8);
    fe_to_words(fe_from_mont(A.y), out + 16);
}

// --- per-device generator table ---------------------------------------------
std::mutex g_table_lock;
uint32_t *g_table[64] = {nullptr};

pcmm_status build_table(const point16 &base, uint32_t *table_out, void *tmp, size_t tmp_bytes, hipStream_t s) {
    // tmp layout: [jacobian 960 x 24 words][normalize scratch]
    size_t jac_bytes = (size_t)TABLE_POINTS * 3 * NL * sizeof(uint32_t);
    size_t need = jac_bytes + normalize_scratch_bytes(TABLE_POINTS, 1);
    if (tmp_bytes < need) return PCMM_ENOMEM;
    uint32_t *jac = (uint32_t *)tmp;
    void *scratch = (char *)tmp + jac_bytes;
    hipLaunchKernelGGL(fixed_base_table_kernel, dim3(1), dim3(64), 0, s, base, jac);
    PCMM_LAUNCH_CHECK();
    return launch_normalize(jac, TABLE_POINTS, true, table_out, TABLE_POINTS, true, TABLE_POINTS, 1, scratch,
                            tmp_bytes - jac_bytes, s);
}

size_t table_tmp_bytes() {
    return (size_t)TABLE_POINTS * 3 * NL * sizeof(uint32_t) + normalize_scratch_bytes(TABLE_POINTS, 1);
}

size_t table_bytes() { return (size_t)TABLE_POINTS * 2 * NL * sizeof(uint32_t); }

void be32_to_words(const uint8_t be[32], uint32_t w[8]) {
    for (int i = 0; i < 8; ++i) {
        const uint8_t *p = be + (7 - i) * 4;
        w[i] = ((uint32_t)p[0] << 24) | ((uint32_t)p[1] << 16) | ((uint32_t)p[2] << 8) | p[3];
    }
}

void words_to_be32(const uint32_t w[8], uint8_t be[32]) {
    for (int i = 0; i < 8; ++i) {
        uint8_t *p = be + (7 - i) * 4;
        p[0] = (uint8_t)(w[i] >> 24);
        p[1] = (uint8_t)(w[i] >> 16);
        p[2] = (uint8_t)(w[i] >> 8);
        p[3] = (uint8_t)w[i];
    }
}

}  // namespace

namespace pcmm {

// generator table of the current device, built on first use (blocking)
pcmm_status generator_table(const uint32_t **out) {
    int dev = 0;
    PCMM_HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return PCMM_EDEVICE;
    std::lock_guard<std::mutex> guard(g_table_lock);
    if (!g_table[dev]) {
        point16 base;
        for (int i = 0; i < 8; ++i) {
            base.w[i] = GX_PLAIN.v[i];
            base.w[8 + i] = GY_PLAIN.v[i];
        }
        uint32_t *tab = nullptr;
        void *tmp = nullptr;
        PCMM_HIP_TRY(hipMalloc(&tab, table_bytes()));
        // on the error paths the frees' own status adds nothing: PCMM_EDEVICE either way
        if (hipMalloc(&tmp, table_tmp_bytes()) != hipSuccess) {
            (void)hipFree(tab);
            return PCMM_EDEVICE;
        }
        hipStream_t s;
        if (hipStreamCreate(&s) != hipSuccess) {
            (void)hipFree(tab);
            (void)hipFree(tmp);
            return PCMM_EDEVICE;
        }
        pcmm_status st = build_table(base, tab, tmp, table_tmp_bytes(), s);
        hipError_t e = hipStreamSynchronize(s);
        if (e == hipSuccess) e = hipStreamDestroy(s);
        else (void)hipStreamDestroy(s);
        if (e == hipSuccess) e = hipFree(tmp);
        else (void)hipFree(tmp);
        if (st != PCMM_OK || e != hipSuccess) {
            (void)hipFree(tab);
            return st != PCMM_OK ? st : PCMM_EDEVICE;
        }
        g_table[dev] = tab;
    }
    *out = g_table[dev];
    return PCMM_OK;
}

}  // namespace pcmm

extern "C" size_t pcmm_encrypt_workspace(void) {
    return 256 + table_bytes() + table_tmp_bytes();
}

extern "C" pcmm_status pcmm_keygen(uint64_t seed, uint8_t sk_be[32], pcmm_point_be *pk) {
    if (!sk_be || !pk) return PCMM_EINVAL;
    const uint32_t *tabG = nullptr;
    pcmm_status st = generator_table(&tabG);
    if (st != PCMM_OK) return st;
    uint32_t *dout = nullptr;
    PCMM_HIP_TRY(hipMalloc(&dout, 24 * sizeof(uint32_t)));
    hipLaunchKernelGGL(keygen_kernel, dim3(1), dim3(64), 0, 0, tabG, seed, dout);
    uint32_t h[24];
    hipError_t le = hipGetLastError();
    hipError_t ce = hipMemcpy(h, dout, sizeof h, hipMemcpyDeviceToHost);
    hipError_t fe = hipFree(dout);
    if (le != hipSuccess || ce != hipSuccess || fe != hipSuccess) return PCMM_EDEVICE;
    words_to_be32(h, sk_be);
    words_to_be32(h + 8, pk->x);
    words_to_be32(h + 16, pk->y);
    return PCMM_OK;
}

extern "C" pcmm_status pcmm_encrypt(const pcmm_point_be *pk, const int32_t *msg_dev, int32_t rows,
                                    int32_t cols, uint64_t seed, int64_t idx0, pcmm_mat *ct_out,
                                    void *workspace, size_t ws_bytes, void *stream) {
    if (!pk || !ct_out || rows < 0 || cols < 0 || idx0 < 0) return PCMM_EINVAL;
    int64_t n = (int64_t)rows * cols;
    if (ct_out->rows != rows || ct_out->cols != cols || ct_out->npts != 2 || ct_out->form != PCMM_AFFINE ||
        ct_out->ld < n || (n > 0 && (!msg_dev || !ct_out->d)))
        return PCMM_EINVAL;
    if (!workspace || ws_bytes < pcmm_encrypt_workspace()) return PCMM_ENOMEM;
    hipStream_t s = (hipStream_t)stream;
    const uint32_t *tabG = nullptr;
    pcmm_status st = generator_table(&tabG);
    if (st != PCMM_OK) return st;
    point16 base;
    be32_to_words(pk->x, base.w);
    be32_to_words(pk->y, base.w + 8);
    // synchronous validation of the public point
    uint32_t *flag = (uint32_t *)workspace;               // 256 B header
    uint32_t *tabH = (uint32_t *)((char *)workspace + 256);
    void *tmp = (char *)workspace + 256 + table_bytes();
    hipLaunchKernelGGL(on_curve_kernel, dim3(1), dim3(64), 0, s, base, flag);
    PCMM_LAUNCH_CHECK();
    uint32_t ok = 0;
    PCMM_HIP_TRY(hipMemcpyAsync(&ok, flag, sizeof ok, hipMemcpyDeviceToHost, s));
    PCMM_HIP_TRY(hipStreamSynchronize(s));
    if (!ok) return PCMM_ENOTONCURVE;
    st = build_table(base, tabH, tmp, table_tmp_bytes(), s);
    if (st != PCMM_OK) return st;
    if (n == 0) return PCMM_OK;
    int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(encrypt_kernel, dim3((unsigned)blocks), dim3(256), 0, s, tabG, tabH, msg_dev, n, seed,
                       idx0, ct_out->d, ct_out->ld);
    PCMM_LAUNCH_CHECK();
    return PCMM_OK;
}

extern "C" pcmm_status pcmm_decrypt_to_points(const uint8_t sk_be[32], const pcmm_mat *C, pcmm_mat *M,
                                              void *stream) {
    if (!sk_be || !C || !M) return PCMM_EINVAL;
    int64_t n = (int64_t)C->rows * C->cols;
    if (C->rows < 0 || C->cols < 0 || C->npts != 2 || C->form != PCMM_AFFINE || C->ld < n) return PCMM_EINVAL;
    if (M->rows != C->rows || M->cols != C->cols || M->npts != 1 || M->form != PCMM_AFFINE || M->ld < n)
        return PCMM_EINVAL;
    scalar8 x;
    be32_to_words(sk_be, x.w);
    bool zero = true;
    for (int i = 0; i < 8; ++i) zero &= x.w[i] == 0;
    bool below_q = false;  // x < q
    for (int i = 7; i >= 0; --i) {
        if (x.w[i] != ORDER_Q.v[i]) {
            below_q = x.w[i] < ORDER_Q.v[i];
            break;
        }
    }
    if (zero || !below_q) return PCMM_EINVAL;
    if (n == 0) return PCMM_OK;
    int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(decrypt_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, x, C->d, C->ld,
                       M->d, M->ld, n);
    PCMM_LAUNCH_CHECK();
    return PCMM_OK;
}
