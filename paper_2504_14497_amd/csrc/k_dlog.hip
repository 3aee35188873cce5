// k_dlog.hip -- full decryption (Sec. 2.4): the bounded discrete logarithm
// of M = C2 - x C1 = m G by baby-step giant-step, on gfx950.
//
// Baby steps: the points j G for 0 <= j < s = 2^k (computed once, one ladder
// per lane and a batched normalisation) in canonical affine form, indexed by
// an open-addressing hash table on the low 64 bits of x (inserted with a
// compare-and-swap).  A point and its negation share x, so one table serves
// +-j: every integer m with |m| <= bound is uniquely m = i (2s - 1) + k with
// |i| <= I = ceil(bound / (2s - 1)) and |k| < s.  Giant steps: for every
// target M and every i, one lane forms M - i S (S = (2s - 1) G; the affine
// multiples -i S are computed per call), all of them are normalised in one
// batch, and one lane per (target, i) looks the x-coordinate up; a hit whose
// full x matches gives k = +-j from y, and m = i (2s - 1) + k.  Only the
// matching i writes its target's result; targets outside the bound keep
// INT64_MIN.
#include <algorithm>
#include <cstring>

#include "common.hpp"
#include "normalize.hpp"

using namespace pcmm;

extern "C" pcmm_status pcmm_decrypt_to_points(const uint8_t sk_be[32], const pcmm_mat *C, pcmm_mat *M,
                                              void *stream);

namespace {

constexpr int AFF1_WORDS = 16;  // canonical affine point: x (8 words), y (8 words)

__device__ __forceinline__ apt generator_mont() {
    apt G;
    G.x = fe_to_mont(fe_from_const(GX_PLAIN));
    G.y = fe_to_mont(fe_from_const(GY_PLAIN));
    return G;
}

__device__ __forceinline__ uint64_t x_key(const uint32_t *x) { return (uint64_t)x[0] | ((uint64_t)x[1] << 32); }

__device__ __forceinline__ uint64_t slot_of(uint64_t key, int log2cap) {
    return (key * 0x9E3779B97F4A7C15ull) >> (64 - log2cap);
}

// j G for j = t (one lane per baby step), Jacobian internal, one point per element
__global__ void __launch_bounds__(256) baby_kernel(int64_t s, int log2s, uint32_t *__restrict__ out, int64_t ld) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= s) return;
    jpt R = ladder_small((uint32_t)j, log2s + 1, generator_mont());
    store_jac_m(out, ld, 0, j, R);
}

// hash insertion of the baby steps j >= 1 (j = 0 is the identity, recognised
// directly); slot = (high 32 bits of the key) << 32 | (j + 1)
__global__ void __launch_bounds__(256) insert_kernel(const uint32_t *__restrict__ baby, int64_t ld, int64_t s,
                                                     unsigned long long *__restrict__ slots, int log2cap) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < 1 || j >= s) return;
    uint32_t x[2];
    x[0] = baby[0 * ld + j];
    x[1] = baby[1 * ld + j];
    const uint64_t key = x_key(x);
    const unsigned long long v = ((unsigned long long)(key >> 32) << 32) | (unsigned long long)(j + 1);
    const uint64_t mask = (1ull << log2cap) - 1;
    uint64_t h = slot_of(key, log2cap);
    for (uint64_t probe = 0; probe <= mask; ++probe) {  // the table is at most half full: this ends early
        if (atomicCAS(&slots[h], 0ull, v) == 0ull) return;
        h = (h + 1) & mask;
    }
}

// the giant multiples -i S for i = k - I, k = 0..2I (Jacobian internal)
__global__ void __launch_bounds__(256) giant_kernel(int64_t I, int64_t stride, uint32_t *__restrict__ out, int64_t ld) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k > 2 * I) return;
    const int64_t i = k - I;
    const uint64_t mag = (uint64_t)(i < 0 ? -i : i) * (uint64_t)stride;  // < 2^32 (checked by the host)
    jpt R = ladder_small((uint32_t)mag, 32, generator_mont());
    if (i > 0) R = jpt_neg(R);
    store_jac_m(out, ld, 0, k, R);
}

// lane (target e, k): M_e + (-i S), Jacobian internal
__global__ void __launch_bounds__(256) step_kernel(const uint32_t *__restrict__ M, int64_t ldm, int64_t targets,
                                                   const uint32_t *__restrict__ giants, int64_t ldg, int64_t steps,
                                                   uint32_t *__restrict__ out, int64_t ld_out) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= targets * steps) return;
    const int64_t e = t / steps, k = t - e * steps;
    const apt Y = load_affine(M, ldm, 0, e);
    const apt Gk = load_aff_m(giants, ldg, 0, k);
    store_jac_m(out, ld_out, 0, t, jpt_add_affine(jpt_from_affine(Y), Gk));
}

__global__ void fill_i64_kernel(int64_t *out, int64_t n, int64_t v) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) out[e] = v;
}

// lane (target e, k): look up the normalised point (canonical affine, boundary layout)
__global__ void __launch_bounds__(256) lookup_kernel(const uint32_t *__restrict__ P, int64_t ldp, int64_t targets,
                                                     int64_t steps, int64_t I, int64_t stride,
                                                     const unsigned long long *__restrict__ slots, int log2cap,
                                                     const uint32_t *__restrict__ baby, int64_t ldb,
                                                     int64_t bound, int64_t *__restrict__ out) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= targets * steps) return;
    const int64_t e = t / steps, k = t - e * steps;
    const int64_t i = k - I;
    uint32_t x[8], y[8];
    uint32_t any = 0;
#pragma unroll
    for (int w = 0; w < 8; ++w) {
        x[w] = P[(0 * 8 + w) * ldp + t];
        y[w] = P[(1 * 8 + w) * ldp + t];
        any |= x[w] | y[w];
    }
    // the giant steps cover a little more than [-bound, bound]; results
    // beyond the bound are not reported
    if (any == 0) {  // M_e - i S is the identity: k = 0
        const int64_t m = i * stride;
        if (m <= bound && m >= -bound) out[e] = m;
        return;
    }
    const uint64_t key = x_key(x);
    const uint64_t mask = (1ull << log2cap) - 1;
    uint64_t h = slot_of(key, log2cap);
    for (uint64_t probe = 0; probe <= mask; ++probe) {
        const unsigned long long v = slots[h];
        if (v == 0ull) return;  // empty slot: not a baby step
        if ((v >> 32) == (key >> 32)) {
            const int64_t j = (int64_t)(v & 0xffffffffull) - 1;
            bool same_x = true, same_y = true;
#pragma unroll
            for (int w = 0; w < 8; ++w) {
                same_x &= baby[(0 * 8 + w) * ldb + j] == x[w];
                same_y &= baby[(1 * 8 + w) * ldb + j] == y[w];
            }
            if (same_x) {
                const int64_t m = i * stride + (same_y ? j : -j);
                if (m <= bound && m >= -bound) out[e] = m;
                return;
            }
        }
        h = (h + 1) & mask;
    }
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
int64_t ld64(int64_t n) { return std::max<int64_t>(64, (n + 63) / 64 * 64); }

struct table_layout {
    int64_t s, ldb;
    int log2cap;
    size_t off_slots, off_baby, total;
};

table_layout table_geom(int log2s) {
    table_layout T;
    T.s = (int64_t)1 << log2s;
    T.ldb = ld64(T.s);
    T.log2cap = log2s + 1;  // at most half full
    T.off_slots = 0;
    T.off_baby = align256(((size_t)1 << T.log2cap) * 8);
    T.total = T.off_baby + align256((size_t)AFF1_WORDS * T.ldb * 4);
    return T;
}

struct decrypt_layout {
    int64_t I, steps, stride, ldm, ldg, ldj;
    size_t off_m, off_g, off_gjac, off_jac, off_aff, off_norm, norm_bytes, total;
};

decrypt_layout decrypt_geom(int64_t elements, int64_t bound, int log2s) {
    decrypt_layout L;
    const int64_t s = (int64_t)1 << log2s;
    L.stride = 2 * s - 1;
    L.I = (bound + L.stride - 1) / L.stride;
    L.steps = 2 * L.I + 1;
    L.ldm = ld64(elements);
    L.ldg = ld64(L.steps);
    L.ldj = ld64(elements * L.steps);
    size_t off = 0;
    L.off_m = off;
    off += align256((size_t)AFF1_WORDS * L.ldm * 4);          // decrypted points (canonical affine)
    L.off_gjac = off;
    off += align256((size_t)3 * NL * L.ldg * 4);              // giant multiples (Jacobian)
    L.off_g = off;
    off += align256((size_t)2 * NL * L.ldg * 4);              // giant multiples (affine internal)
    L.off_jac = off;
    off += align256((size_t)3 * NL * L.ldj * 4);              // steps (Jacobian)
    L.off_aff = off;
    off += align256((size_t)AFF1_WORDS * L.ldj * 4);          // steps (canonical affine)
    L.norm_bytes = normalize_scratch_bytes(std::max<int64_t>(elements * L.steps, L.steps), 1);
    L.off_norm = off;
    off += align256(L.norm_bytes);
    L.total = off + 256;
    return L;
}

bool valid_dlog(int log2s, int64_t bound) {
    if (log2s < 4 || log2s > 24 || bound < 0) return false;
    const int64_t s = (int64_t)1 << log2s;
    const int64_t stride = 2 * s - 1;
    const int64_t I = (bound + stride - 1) / stride;
    return I * stride < ((int64_t)1 << 32);  // giant multiples fit the 32-bit ladder
}

}  // namespace

extern "C" pcmm_status pcmm_dlog_table_bytes(int32_t log2_baby, size_t *bytes) {
    if (!bytes || log2_baby < 4 || log2_baby > 24) return PCMM_EINVAL;
    *bytes = table_geom(log2_baby).total;
    return PCMM_OK;
}

extern "C" pcmm_status pcmm_dlog_table_build(int32_t log2_baby, void *table, size_t bytes, void *workspace,
                                             size_t ws_bytes, void *stream) {
    if (log2_baby < 4 || log2_baby > 24 || !table) return PCMM_EINVAL;
    const table_layout T = table_geom(log2_baby);
    if (bytes < T.total) return PCMM_ENOMEM;
    const size_t need = align256((size_t)3 * NL * T.ldb * 4) + normalize_scratch_bytes(T.s, 1) + 256;
    if (!workspace || ws_bytes < need) return PCMM_ENOMEM;
    hipStream_t s = (hipStream_t)stream;
    char *tb = (char *)table;
    char *ws = (char *)workspace;
    uint32_t *jac = (uint32_t *)ws;
    const int64_t blocks = (T.s + 255) / 256;
    hipLaunchKernelGGL(baby_kernel, dim3((unsigned)blocks), dim3(256), 0, s, T.s, log2_baby, jac, T.ldb);
    PCMM_LAUNCH_CHECK();
    uint32_t *baby = (uint32_t *)(tb + T.off_baby);
    const size_t off_norm = align256((size_t)3 * NL * T.ldb * 4);
    pcmm_status st = launch_normalize(jac, T.ldb, true, baby, T.ldb, false, T.s, 1, ws + off_norm,
                                      ws_bytes - off_norm, s);
    if (st != PCMM_OK) return st;
    // clear the slots with a kernel (no memset node if the caller captures this)
    const int64_t nslots = (int64_t)1 << T.log2cap;
    hipLaunchKernelGGL(fill_i64_kernel, dim3((unsigned)((nslots + 255) / 256)), dim3(256), 0, s,
                       (int64_t *)(tb + T.off_slots), nslots, (int64_t)0);
    PCMM_LAUNCH_CHECK();
    hipLaunchKernelGGL(insert_kernel, dim3((unsigned)blocks), dim3(256), 0, s, (const uint32_t *)baby, T.ldb, T.s,
                       (unsigned long long *)(tb + T.off_slots), T.log2cap);
    PCMM_LAUNCH_CHECK();
    return PCMM_OK;
}

extern "C" pcmm_status pcmm_dlog_table_workspace(int32_t log2_baby, size_t *bytes) {
    if (!bytes || log2_baby < 4 || log2_baby > 24) return PCMM_EINVAL;
    const table_layout T = table_geom(log2_baby);
    *bytes = align256((size_t)3 * NL * T.ldb * 4) + normalize_scratch_bytes(T.s, 1) + 256;
    return PCMM_OK;
}

extern "C" pcmm_status pcmm_decrypt_workspace(int64_t elements, int64_t bound, int32_t log2_baby, size_t *bytes) {
    if (!bytes || elements < 0 || !valid_dlog(log2_baby, bound)) return PCMM_EINVAL;
    *bytes = decrypt_geom(elements, bound, log2_baby).total;
    return PCMM_OK;
}

extern "C" pcmm_status pcmm_decrypt(const uint8_t sk_be[32], const pcmm_mat *C, int64_t bound, const void *table,
                                    size_t table_bytes, int32_t log2_baby, int64_t *out, void *workspace,
                                    size_t ws_bytes, void *stream) {
    if (!sk_be || !C || !valid_dlog(log2_baby, bound)) return PCMM_EINVAL;
    if (C->rows < 0 || C->cols < 0 || C->npts != 2 || C->form != PCMM_AFFINE) return PCMM_EINVAL;
    const int64_t n = (int64_t)C->rows * C->cols;
    if (n > 0 && (!out || !table)) return PCMM_EINVAL;
    const table_layout T = table_geom(log2_baby);
    if (table_bytes < T.total) return PCMM_EINVAL;
    const decrypt_layout L = decrypt_geom(n, bound, log2_baby);
    if (n == 0) return PCMM_OK;
    if (!workspace || ws_bytes < L.total) return PCMM_ENOMEM;
    if (n * L.steps > ((int64_t)1 << 40)) return PCMM_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    char *ws = (char *)workspace;
    // M = C2 - x C1 (canonical affine, one point per element)
    pcmm_mat M{C->rows, C->cols, 1, PCMM_AFFINE, L.ldm, (uint32_t *)(ws + L.off_m)};
    pcmm_status st = pcmm_decrypt_to_points(sk_be, C, &M, stream);
    if (st != PCMM_OK) return st;
    // giant multiples -i S
    hipLaunchKernelGGL(giant_kernel, dim3((unsigned)((L.steps + 255) / 256)), dim3(256), 0, s, L.I, L.stride,
                       (uint32_t *)(ws + L.off_gjac), L.ldg);
    PCMM_LAUNCH_CHECK();
    st = launch_normalize((uint32_t *)(ws + L.off_gjac), L.ldg, true, (uint32_t *)(ws + L.off_g), L.ldg, true,
                          L.steps, 1, ws + L.off_norm, L.norm_bytes, s);
    if (st != PCMM_OK) return st;
    // every (target, i): M - i S, normalised together
    const int64_t lanes = n * L.steps;
    const unsigned blocks = (unsigned)((lanes + 255) / 256);
    hipLaunchKernelGGL(step_kernel, dim3(blocks), dim3(256), 0, s, (const uint32_t *)M.d, L.ldm, n,
                       (const uint32_t *)(ws + L.off_g), L.ldg, L.steps, (uint32_t *)(ws + L.off_jac), L.ldj);
    PCMM_LAUNCH_CHECK();
    st = launch_normalize((uint32_t *)(ws + L.off_jac), L.ldj, true, (uint32_t *)(ws + L.off_aff), L.ldj, false,
                          lanes, 1, ws + L.off_norm, L.norm_bytes, s);
    if (st != PCMM_OK) return st;
    hipLaunchKernelGGL(fill_i64_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, out, n, INT64_MIN);
    PCMM_LAUNCH_CHECK();
    const char *tb = (const char *)table;
    hipLaunchKernelGGL(lookup_kernel, dim3(blocks), dim3(256), 0, s, (const uint32_t *)(ws + L.off_aff), L.ldj, n,
                       L.steps, L.I, L.stride, (const unsigned long long *)(tb + T.off_slots), T.log2cap,
                       (const uint32_t *)(tb + T.off_baby), T.ldb, bound, out);
    PCMM_LAUNCH_CHECK();
    return PCMM_OK;
}
