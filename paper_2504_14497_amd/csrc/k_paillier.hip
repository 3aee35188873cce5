// k_paillier.hip -- PC-MM over Paillier ciphertexts (Sec. "Extension to
// Paillier Encryption"): C_ij = prod_k B_kj^{a_ik} mod n^2, schoolbook (one
// Alg. 4 power per term) and Cussen (Alg. 2 tables of powers built by the
// same straight-line plans as the EC-ElGamal path, then one product per
// nonzero code), plus encryption c = (1 + m n) r^n mod n^2 (g = n + 1).
//
// One residue per wavefront (bn.hpp); blocks of 256 threads hold 4
// independent wavefronts.  Internal residues are Montgomery limbs (256 x 29
// bits, 1 KiB); at the boundary they are 192 canonical 32-bit words.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "../../include/pcmm.h"
#include "../../include/pcmm_paillier.h"
#include "bn.hpp"
#include "plan.hpp"

#define PCMM_HIP_TRY(expr)                        \
    do {                                           \
        hipError_t _e = (expr);                    \
        if (_e != hipSuccess) return PCMM_EDEVICE; \
    } while (0)

#define PCMM_LAUNCH_CHECK()                        \
    do {                                           \
        hipError_t _e = hipGetLastError();         \
        if (_e != hipSuccess) return PCMM_EDEVICE; \
    } while (0)

namespace pcmm {
namespace {

constexpr int WAVES_PER_BLOCK = 4;
constexpr size_t BN_BYTES = BN_LIMBS * 4;   // one residue in limb form

// device constants of one modulus (limb arrays are BN_LIMBS long)
struct paillier_consts {
    uint32_t N[BN_LIMBS];     // n^2
    uint32_t one[BN_LIMBS];   // R mod n^2 (Montgomery form of 1)
    uint32_t r2[BN_LIMBS];    // R^2 mod n^2
    uint32_t nl[BN_LIMBS];    // n
    uint32_t nw[BN_NWORDS];   // n as 32-bit words (the encryption exponent)
};

struct wave_ctx {
    int lane, wave;
    int64_t inst;
    uint32_t *lds;
};

__device__ __forceinline__ wave_ctx wave_of(uint32_t *lds_all) {
    wave_ctx w;
    w.lane = (int)(threadIdx.x & 63);
    w.wave = (int)(threadIdx.x >> 6);
    w.inst = (int64_t)blockIdx.x * WAVES_PER_BLOCK + w.wave;
    w.lds = lds_all + w.wave * BN_LIMBS;
    return w;
}

// canonical words of a residue (< n^2) -> Montgomery limbs
__device__ __forceinline__ bn to_mont(const uint32_t *__restrict__ words, const paillier_consts &K, const bn &N,
                                      uint32_t n0, uint32_t *lds) {
    const bn x = bn_from_words(words, BN_WORDS, lds);
    return bn_mont(x, bn_load(K.r2), N, n0);
}

// Montgomery limbs -> canonical words
__device__ __forceinline__ void from_mont(const bn &x, uint32_t *__restrict__ words, const bn &N, uint32_t n0,
                                          uint32_t *lds) {
    bn one_plain;
#pragma unroll
    for (int t = 0; t < BN_W; ++t) one_plain.v[t] = (bn_lane() == 0 && t == 0) ? 1u : 0u;
    const bn y = bn_canon(bn_mont(x, one_plain, N, n0), N);
    bn_to_words(y, words, BN_WORDS, lds);
}

// --------------------------------------------------------------------------
// Kernels
// --------------------------------------------------------------------------
// canonical ciphertexts -> Montgomery limbs
__global__ void __launch_bounds__(256) paillier_to_mont_kernel(const paillier_consts *__restrict__ K, uint32_t n0,
                                                      const uint32_t *__restrict__ in, uint32_t *__restrict__ out,
                                                      int64_t count) {
    __shared__ uint32_t lds[WAVES_PER_BLOCK * BN_LIMBS];
    const wave_ctx w = wave_of(lds);
    if (w.inst >= count) return;
    const bn N = bn_load(K->N);
    bn_store(out + w.inst * BN_LIMBS, to_mont(in + w.inst * BN_WORDS, *K, N, n0, w.lds));
}

// the identity ciphertext 1 (canonical words) in `count` elements
__global__ void __launch_bounds__(256) paillier_identity_kernel(uint32_t *__restrict__ out, int64_t count) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= count * BN_WORDS) return;
    out[x] = (x % BN_WORDS) == 0 ? 1u : 0u;
}

// SplitMix64 finaliser
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// c = (1 + m n) r^n mod n^2 for element e: r from 48 SplitMix64 words of
// (seed, domain 2, idx0 + e), reduced mod n (0 -> 1)
__global__ void __launch_bounds__(256) paillier_encrypt_kernel(const paillier_consts *__restrict__ K, uint32_t n0,
                                                      const int32_t *__restrict__ msg, int64_t count,
                                                      uint64_t seed, int64_t idx0, uint32_t *__restrict__ ct) {
    __shared__ uint32_t lds[WAVES_PER_BLOCK * BN_LIMBS];
    const wave_ctx w = wave_of(lds);
    if (w.inst >= count) return;
    const bn N = bn_load(K->N), one = bn_load(K->one), nl = bn_load(K->nl);
    // nonce words: lane L < 48 holds 64-bit word L (32-bit words 2L, 2L + 1)
    const uint64_t base = mix64(seed ^ (2ull << 56) ^ (uint64_t)(idx0 + w.inst));
    const uint64_t word = mix64(base + (uint64_t)(w.lane + 1) * 0x9E3779B97F4A7C15ull);
    __shared__ uint32_t nonce_words[WAVES_PER_BLOCK * BN_NWORDS];
    uint32_t *nw = nonce_words + w.wave * BN_NWORDS;
    if (w.lane < BN_NWORDS / 2) {
        nw[2 * w.lane] = (uint32_t)word;
        nw[2 * w.lane + 1] = (uint32_t)(word >> 32);
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    bn r = bn_from_words(nw, BN_NWORDS, w.lds);
    // X < 2^3072 <= 2n (n has 3072 bits): one conditional subtraction
    bool ge;
    r = bn_sub_if_ge(r, nl, &ge);
    if (bn_is_zero(r)) {
#pragma unroll
        for (int t = 0; t < BN_W; ++t) r.v[t] = (w.lane == 0 && t == 0) ? 1u : 0u;
    }
    const bn r2 = bn_load(K->r2);
    const bn rn = bn_pow_words(bn_mont(r, r2, N, n0), K->nw, 32 * BN_NWORDS, one, N, n0);
    // 1 + m n (below n^2 for 0 <= m < 2^31), then three carry rounds
    const uint32_t m = (uint32_t)msg[w.inst];
    uint64_t acc[BN_W];
#pragma unroll
    for (int t = 0; t < BN_W; ++t) acc[t] = (uint64_t)m * nl.v[t];
    if (w.lane == 0) acc[0] += 1;
#pragma unroll
    for (int rr = 0; rr < 3; ++rr) {
        uint64_t c[BN_W];
#pragma unroll
        for (int t = 0; t < BN_W; ++t) {
            c[t] = acc[t] >> BN_LB;
            acc[t] &= BN_MASK;
        }
        acc[0] += lane_from_below(c[BN_W - 1]);
#pragma unroll
        for (int t = 1; t < BN_W; ++t) acc[t] += c[t - 1];
    }
    bn gm;
#pragma unroll
    for (int t = 0; t < BN_W; ++t) gm.v[t] = (uint32_t)acc[t];
    const bn c = bn_mont(bn_mont(gm, r2, N, n0), rn, N, n0);
    from_mont(c, ct + w.inst * BN_WORDS, N, n0, w.lds);
}

// schoolbook: one wavefront per output (i, j), i fastest
__global__ void __launch_bounds__(256) paillier_schoolbook_kernel(const paillier_consts *__restrict__ K, uint32_t n0,
                                                         const uint16_t *__restrict__ A, int m, int n, int l,
                                                         int bits, const uint32_t *__restrict__ Bm,
                                                         uint32_t *__restrict__ C) {
    __shared__ uint32_t lds[WAVES_PER_BLOCK * BN_LIMBS];
    const wave_ctx w = wave_of(lds);
    if (w.inst >= (int64_t)m * l) return;
    const int i = (int)(w.inst % m), j = (int)(w.inst / m);
    const bn N = bn_load(K->N), one = bn_load(K->one);
    bn acc = one;
    for (int k = 0; k < n; ++k) {
        const uint32_t a = A[(int64_t)i * n + k];
        if (a == 0) continue;
        const bn p = bn_pow_small(bn_load(Bm + ((int64_t)k * l + j) * BN_LIMBS), a, bits, one, N, n0);
        acc = bn_mont(acc, p, N, n0);
    }
    from_mont(acc, C + ((int64_t)i * l + j) * BN_WORDS, N, n0, w.lds);
}

// Cussen digit tables: one wavefront per (unit = column k of A, output
// column j) runs the column's straight-line program (MUL: an Alg. 4 power of
// the base B_kj; ADD: a product of two operands) into its register file, then
// copies the column's digit-table entries into its group's table
__global__ void __launch_bounds__(256) paillier_table_kernel(const paillier_consts *__restrict__ K, uint32_t n0,
                                                   const plan_op *__restrict__ ops,
                                                   const int32_t *__restrict__ op_begin,
                                                   const int32_t *__restrict__ entry_begin,
                                                   const int16_t *__restrict__ entries,
                                                   const int32_t *__restrict__ unit_col,
                                                   const int32_t *__restrict__ unit_grp,
                                                   const int32_t *__restrict__ unit_off, int nunits, int l,
                                                   int rmax, int emax, const uint32_t *__restrict__ Bm,
                                                   uint32_t *__restrict__ regs, uint32_t *__restrict__ table) {
    __shared__ uint32_t lds[WAVES_PER_BLOCK * BN_LIMBS];
    const wave_ctx w = wave_of(lds);
    if (w.inst >= (int64_t)nunits * l) return;
    const int u = (int)(w.inst / l), j = (int)(w.inst % l);
    const int k = unit_col[u];
    const bn N = bn_load(K->N), one = bn_load(K->one);
    uint32_t *R = regs + w.inst * rmax * BN_LIMBS;
    const uint32_t *base = Bm + ((int64_t)k * l + j) * BN_LIMBS;
    auto operand = [&](int o) -> bn { return o >= 0 ? bn_load(R + (int64_t)o * BN_LIMBS) : bn_load(base); };
    for (int o = op_begin[u]; o < op_begin[u + 1]; ++o) {
        const plan_op op = ops[o];
        bn r;
        if (op.kind == OP_MUL) {
            const uint32_t s = (uint32_t)op.s;
            r = bn_pow_small(operand(op.a), s, 32 - __builtin_clz(s), one, N, n0);
        } else {
            r = bn_mont(operand(op.a), operand(op.b), N, n0);
        }
        bn_store(R + (int64_t)op.dst * BN_LIMBS, r);
    }
    uint32_t *T = table + (((int64_t)unit_grp[u] * l + j) * emax + unit_off[u]) * BN_LIMBS;
    for (int e = 0; e < entry_begin[u + 1] - entry_begin[u]; ++e)
        bn_store(T + (int64_t)e * BN_LIMBS, operand(entries[entry_begin[u] + e]));
}

// Cussen digit combinations (column groups g > 1): one wavefront per (group,
// output column j); each combination is the product of two entries of the
// group's table (plaintexts are unsigned here, so no entry is inverted),
// level by level
__global__ void __launch_bounds__(256) paillier_combo_kernel(const paillier_consts *__restrict__ K, uint32_t n0,
                                                   const plan_combo *__restrict__ combos,
                                                   const int32_t *__restrict__ combo_begin, int ngroups, int l,
                                                   int emax, uint32_t *__restrict__ table) {
    __shared__ uint32_t lds[WAVES_PER_BLOCK * BN_LIMBS];
    const wave_ctx w = wave_of(lds);
    if (w.inst >= (int64_t)ngroups * l) return;
    const int grp = (int)(w.inst / l);
    const bn N = bn_load(K->N);
    uint32_t *T = table + w.inst * emax * BN_LIMBS;
    for (int c = combo_begin[grp]; c < combo_begin[grp + 1]; ++c) {
        const plan_combo cm = combos[c];
        bn_store(T + (int64_t)cm.dst * BN_LIMBS,
                 bn_mont(bn_load(T + (int64_t)cm.a * BN_LIMBS), bn_load(T + (int64_t)cm.b * BN_LIMBS), N, n0));
    }
}

// Cussen accumulation: one wavefront per output (i, j), i fastest; the
// product over the groups of the table entry each row segment's code names
__global__ void __launch_bounds__(256) paillier_accumulate_kernel(const paillier_consts *__restrict__ K, uint32_t n0,
                                                         const int16_t *__restrict__ codes, int m, int ngroups,
                                                         int l, int emax, const uint32_t *__restrict__ table,
                                                         uint32_t *__restrict__ C) {
    __shared__ uint32_t lds[WAVES_PER_BLOCK * BN_LIMBS];
    const wave_ctx w = wave_of(lds);
    if (w.inst >= (int64_t)m * l) return;
    const int i = (int)(w.inst % m), j = (int)(w.inst / m);
    const bn N = bn_load(K->N);
    bn acc = bn_load(K->one);
    for (int grp = 0; grp < ngroups; ++grp) {
        const int code = codes[(int64_t)grp * m + i];
        if (code == 0) continue;
        const uint32_t *src = table + (((int64_t)grp * l + j) * emax + code - 1) * BN_LIMBS;
        acc = bn_mont(acc, bn_load(src), N, n0);
    }
    from_mont(acc, C + ((int64_t)i * l + j) * BN_WORDS, N, n0, w.lds);
}

// diagnostics: 0 raw Montgomery product a b R^-1, 1 a b, 2 a^(b word 0) by
// Alg. 4, 3 a^n (all mod n^2; canonical words in and out)
__global__ void __launch_bounds__(256) paillier_diag_kernel(const paillier_consts *__restrict__ K, uint32_t n0, int op,
                                                   const uint32_t *__restrict__ a, const uint32_t *__restrict__ b,
                                                   uint32_t *__restrict__ out, int64_t count) {
    __shared__ uint32_t lds[WAVES_PER_BLOCK * BN_LIMBS];
    const wave_ctx w = wave_of(lds);
    if (w.inst >= count) return;
    const bn N = bn_load(K->N), one = bn_load(K->one);
    const uint32_t *aw = a + w.inst * BN_WORDS, *bw = b + w.inst * BN_WORDS;
    uint32_t *ow = out + w.inst * BN_WORDS;
    if (op == 0) {
        const bn x = bn_from_words(aw, BN_WORDS, w.lds);
        const bn y = bn_from_words(bw, BN_WORDS, w.lds);
        bn_to_words(bn_canon(bn_mont(x, y, N, n0), N), ow, BN_WORDS, w.lds);
        return;
    }
    const bn x = to_mont(aw, *K, N, n0, w.lds);
    bn r;
    if (op == 1) {
        r = bn_mont(x, to_mont(bw, *K, N, n0, w.lds), N, n0);
    } else if (op == 2) {
        r = bn_pow_small(x, bw[0], 32, one, N, n0);
    } else {
        r = bn_pow_words(x, K->nw, 32 * BN_NWORDS, one, N, n0);
    }
    from_mont(r, ow, N, n0, w.lds);
}

// --------------------------------------------------------------------------
// Host: the modulus, its constants and the plan upload
// --------------------------------------------------------------------------
using words = std::vector<uint32_t>;

// a >= b over equal lengths
bool w_ge(const words &a, const words &b) {
    for (size_t i = a.size(); i-- > 0;) {
        if (a[i] != b[i]) return a[i] > b[i];
    }
    return true;
}

void w_sub(words &a, const words &b) {
    uint64_t borrow = 0;
    for (size_t i = 0; i < a.size(); ++i) {
        const uint64_t d = (uint64_t)a[i] - b[i] - borrow;
        a[i] = (uint32_t)d;
        borrow = (d >> 63) & 1;
    }
}

// 2^e mod M for e >= 0 (M of `len` words, top bit set somewhere), by doubling
words pow2_mod(const words &M, int e) {
    const size_t len = M.size();
    words x(len + 1, 0), Mx(M);
    Mx.push_back(0);
    x[0] = 1;
    for (int i = 0; i < e; ++i) {
        uint32_t carry = 0;
        for (size_t k = 0; k < len + 1; ++k) {
            const uint32_t nc = x[k] >> 31;
            x[k] = (x[k] << 1) | carry;
            carry = nc;
        }
        if (w_ge(x, Mx)) w_sub(x, Mx);
    }
    x.pop_back();
    return x;
}

void to_limbs(const words &x, uint32_t *limbs) {
    for (int i = 0; i < BN_LIMBS; ++i) {
        const int bit = BN_LB * i, k = bit / 32, o = bit % 32;
        uint64_t v = k < (int)x.size() ? x[k] : 0u;
        if (k + 1 < (int)x.size()) v |= (uint64_t)x[k + 1] << 32;
        limbs[i] = (uint32_t)(v >> o) & BN_MASK;
    }
}

}  // namespace
}  // namespace pcmm

using namespace pcmm;

struct pcmm_paillier_s {
    int device = 0;
    uint32_t n0 = 0;
    paillier_consts *d_consts = nullptr;
    ~pcmm_paillier_s() {
        if (d_consts) (void)hipFree(d_consts);  // destructors report nothing
    }
};

namespace {

// A (host, unsigned 8- or 16-bit) as 16-bit values; validates the bit-width
pcmm_status plain_u16(const void *A, int m, int n, int bits, std::vector<uint16_t> &out) {
    out.resize((size_t)m * n);
    for (int64_t x = 0; x < (int64_t)m * n; ++x) {
        const int v = plain_at(A, x, bits, false);
        if (v < 0 || v >= (1 << bits)) return PCMM_ERANGE;
        out[x] = (uint16_t)v;
    }
    return PCMM_OK;
}

// the context's constants live on the device it was created on
bool on_ctx_device(const pcmm_paillier_s *ctx) {
    int dev = -1;
    return hipGetDevice(&dev) == hipSuccess && dev == ctx->device;
}

bool shapes_ok(const void *A, int m, int n, int l, int bits, const uint32_t *B, const uint32_t *C) {
    if (m < 0 || n < 0 || l < 0 || bits < 1 || bits > 16) return false;
    if ((int64_t)m * n > 0 && !A) return false;
    if ((int64_t)n * l > 0 && !B) return false;
    if ((int64_t)m * l > 0 && !C) return false;
    return true;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

unsigned blocks_for(int64_t waves) { return (unsigned)((waves + WAVES_PER_BLOCK - 1) / WAVES_PER_BLOCK); }

// copies host bytes to device memory on the stream and waits for the copy
pcmm_status upload(void *dst, const void *src, size_t bytes, hipStream_t s) {
    if (!bytes) return PCMM_OK;
    PCMM_HIP_TRY(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s));
    PCMM_HIP_TRY(hipStreamSynchronize(s));
    return PCMM_OK;
}

// the identity ciphertext 1 into every element of C (canonical words)
pcmm_status fill_identity(uint32_t *C, int64_t count, hipStream_t s) {
    if (!count) return PCMM_OK;
    const int64_t words = count * BN_WORDS;
    hipLaunchKernelGGL(paillier_identity_kernel, dim3((unsigned)((words + 255) / 256)), dim3(256), 0, s, C, count);
    PCMM_LAUNCH_CHECK();
    return PCMM_OK;
}

struct cussen_layout {
    size_t off_bm, off_regs, off_table, off_ops, off_opb, off_entb, off_ent, off_ucol, off_ugrp, off_uoff, off_cbeg,
        off_combos, off_codes, total;
};

cussen_layout cussen_geom(const cussen_plan &P, int n, int l) {
    cussen_layout L;
    size_t o = 0;
    L.off_bm = o;
    o = align256(o + (size_t)n * l * BN_BYTES);
    L.off_regs = o;
    o = align256(o + (size_t)P.nunits * l * std::max(P.max_regs, 1) * BN_BYTES);
    L.off_table = o;
    o = align256(o + (size_t)P.ngroups * l * std::max(P.max_entries, 1) * BN_BYTES);
    auto arr = [&](size_t &off, size_t bytes) {
        off = o;
        o = align256(o + bytes);
    };
    arr(L.off_ops, P.ops.size() * sizeof(plan_op));
    arr(L.off_opb, P.op_begin.size() * 4);
    arr(L.off_entb, P.entry_begin.size() * 4);
    arr(L.off_ent, P.entries.size() * 2);
    arr(L.off_ucol, P.unit_col.size() * 4);
    arr(L.off_ugrp, P.unit_grp.size() * 4);
    arr(L.off_uoff, P.unit_off.size() * 4);
    arr(L.off_cbeg, P.combo_begin.size() * 4);
    arr(L.off_combos, P.combos.size() * sizeof(plan_combo));
    arr(L.off_codes, P.codes.size() * 2);
    L.total = o;
    return L;
}

int cfg_rounds(const pcmm_cussen_cfg *cfg) { return cfg && cfg->rounds > 0 ? cfg->rounds : 4; }
int cfg_group(const pcmm_cussen_cfg *cfg) { return cfg && cfg->group > 0 ? cfg->group : 1; }

// the modulus constants of n (n_be: 384 big-endian bytes); EINVAL unless n
// is odd with exactly 3072 bits.  Host only.
pcmm_status host_constants(const uint8_t *n_be, paillier_consts &host, uint32_t *n0) {
    words n(BN_NWORDS, 0u);
    for (int i = 0; i < 4 * BN_NWORDS; ++i)
        n[i / 4] |= (uint32_t)n_be[4 * BN_NWORDS - 1 - i] << (8 * (i % 4));
    if (!(n[0] & 1u) || !(n[BN_NWORDS - 1] >> 31)) return PCMM_EINVAL;
    // N = n^2
    words N(BN_WORDS, 0u);
    for (int i = 0; i < BN_NWORDS; ++i) {
        uint64_t carry = 0;
        for (int k = 0; k < BN_NWORDS; ++k) {
            const uint64_t t = (uint64_t)n[i] * n[k] + N[i + k] + carry;
            N[i + k] = (uint32_t)t;
            carry = t >> 32;
        }
        N[i + BN_NWORDS] = (uint32_t)carry;
    }
    // -N^-1 mod 2^32 by Newton's iteration (x <- x (2 - N x) doubles the
    // correct low bits; N x = 1 mod 8 for x = N)
    uint32_t inv = N[0];
    for (int it = 0; it < 5; ++it) inv *= 2u - N[0] * inv;
    *n0 = 0u - inv;
    memset(&host, 0, sizeof(host));
    to_limbs(N, host.N);
    to_limbs(pow2_mod(N, BN_LB * BN_K), host.one);
    to_limbs(pow2_mod(N, 2 * BN_LB * BN_K), host.r2);
    to_limbs(n, host.nl);
    memcpy(host.nw, n.data(), sizeof(host.nw));
    return PCMM_OK;
}

}  // namespace

extern "C" {

pcmm_status pcmm_paillier_create(const uint8_t *n_be, pcmm_paillier *out) {
    if (!n_be || !out) return PCMM_EINVAL;
    *out = nullptr;
    paillier_consts host;
    uint32_t n0 = 0;
    pcmm_status st = host_constants(n_be, host, &n0);
    if (st) return st;
    auto *ctx = new (std::nothrow) pcmm_paillier_s();
    if (!ctx) return PCMM_ENOMEM;
    ctx->n0 = n0;
    if (hipGetDevice(&ctx->device) != hipSuccess ||
        hipMalloc((void **)&ctx->d_consts, sizeof(paillier_consts)) != hipSuccess ||
        hipMemcpy(ctx->d_consts, &host, sizeof(host), hipMemcpyHostToDevice) != hipSuccess) {
        delete ctx;
        return PCMM_EDEVICE;
    }
    *out = ctx;
    return PCMM_OK;
}

pcmm_status pcmm_paillier_diag_constants(const uint8_t *n_be, uint32_t *N_limbs, uint32_t *one_limbs,
                                         uint32_t *r2_limbs, uint32_t *n0) {
    if (!n_be || !N_limbs || !one_limbs || !r2_limbs || !n0) return PCMM_EINVAL;
    paillier_consts host;
    pcmm_status st = host_constants(n_be, host, n0);
    if (st) return st;
    memcpy(N_limbs, host.N, sizeof(host.N));
    memcpy(one_limbs, host.one, sizeof(host.one));
    memcpy(r2_limbs, host.r2, sizeof(host.r2));
    return PCMM_OK;
}

pcmm_status pcmm_paillier_destroy(pcmm_paillier ctx) {
    delete ctx;
    return PCMM_OK;
}

pcmm_status pcmm_paillier_encrypt(pcmm_paillier ctx, const int32_t *msg_dev, int64_t count, uint64_t seed,
                                  int64_t idx0, uint32_t *ct_dev, void *stream) {
    if (!ctx || count < 0 || (count > 0 && (!msg_dev || !ct_dev))) return PCMM_EINVAL;
    if (!on_ctx_device(ctx)) return PCMM_EINVAL;
    if (!count) return PCMM_OK;
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(paillier_encrypt_kernel, dim3(blocks_for(count)), dim3(256), 0, s, ctx->d_consts, ctx->n0, msg_dev,
                       count, seed, idx0, ct_dev);
    PCMM_LAUNCH_CHECK();
    return PCMM_OK;
}

pcmm_status pcmm_paillier_schoolbook_workspace(int32_t m, int32_t n, int32_t l, size_t *bytes) {
    if (!bytes || m < 0 || n < 0 || l < 0) return PCMM_EINVAL;
    *bytes = align256((size_t)n * l * BN_BYTES) + align256((size_t)m * n * 2);
    return PCMM_OK;
}

pcmm_status pcmm_paillier_schoolbook(pcmm_paillier ctx, const void *A, int32_t m, int32_t n, int32_t l,
                                     int32_t bits, const uint32_t *B, uint32_t *C, void *workspace,
                                     size_t ws_bytes, void *stream) {
    if (!ctx || !shapes_ok(A, m, n, l, bits, B, C)) return PCMM_EINVAL;
    if (!on_ctx_device(ctx)) return PCMM_EINVAL;
    std::vector<uint16_t> a16;
    pcmm_status st = plain_u16(A, m, n, bits, a16);
    if (st) return st;
    size_t need;
    pcmm_paillier_schoolbook_workspace(m, n, l, &need);
    if ((int64_t)m * l == 0) return PCMM_OK;
    hipStream_t s = (hipStream_t)stream;
    if (n == 0) return fill_identity(C, (int64_t)m * l, s);
    if (!workspace || ws_bytes < need) return PCMM_ENOMEM;
    char *ws = (char *)workspace;
    uint32_t *Bm = (uint32_t *)ws;
    uint16_t *Ad = (uint16_t *)(ws + align256((size_t)n * l * BN_BYTES));
    st = upload(Ad, a16.data(), a16.size() * 2, s);
    if (st) return st;
    hipLaunchKernelGGL(paillier_to_mont_kernel, dim3(blocks_for((int64_t)n * l)), dim3(256), 0, s, ctx->d_consts, ctx->n0, B,
                       Bm, (int64_t)n * l);
    PCMM_LAUNCH_CHECK();
    hipLaunchKernelGGL(paillier_schoolbook_kernel, dim3(blocks_for((int64_t)m * l)), dim3(256), 0, s, ctx->d_consts,
                       ctx->n0, Ad, m, n, l, bits, Bm, C);
    PCMM_LAUNCH_CHECK();
    return PCMM_OK;
}

pcmm_status pcmm_paillier_cussen_workspace(const void *A, int32_t m, int32_t n, int32_t l, int32_t bits,
                                           const pcmm_cussen_cfg *cfg, size_t *bytes) {
    if (!bytes || !shapes_ok(A, m, n, l, bits, (const uint32_t *)1, (uint32_t *)1)) return PCMM_EINVAL;
    cussen_plan P;
    const int rc = build_cussen_plan(A, m, n, bits, false, cfg_rounds(cfg), cfg_group(cfg), &P);
    if (rc) return rc == -2 ? PCMM_ERANGE : PCMM_EINVAL;
    *bytes = cussen_geom(P, n, l).total;
    return PCMM_OK;
}

pcmm_status pcmm_paillier_cussen(pcmm_paillier ctx, const void *A, int32_t m, int32_t n, int32_t l, int32_t bits,
                                 const uint32_t *B, uint32_t *C, const pcmm_cussen_cfg *cfg, void *workspace,
                                 size_t ws_bytes, pcmm_cussen_stats *stats, void *stream) {
    if (!ctx || !shapes_ok(A, m, n, l, bits, B, C)) return PCMM_EINVAL;
    if (!on_ctx_device(ctx)) return PCMM_EINVAL;
    cussen_plan P;
    const int rc = build_cussen_plan(A, m, n, bits, false, cfg_rounds(cfg), cfg_group(cfg), &P);
    if (rc) return rc == -2 ? PCMM_ERANGE : PCMM_EINVAL;
    const cussen_layout L = cussen_geom(P, n, l);
    if (stats) {
        memset(stats, 0, sizeof(*stats));
        stats->level_mults = P.level_mults;
        stats->level_adds = P.level_adds;
        stats->table_entries = P.table_entries;
        stats->table_adds = P.table_adds;
        stats->combo_adds = P.combo_adds;
        stats->digit_entries = P.digit_entries;
        stats->accum_adds = P.accum_adds;
        stats->max_entries = P.max_entries;
        stats->workspace_bytes = (int64_t)L.total;
        stats->group = P.g;
    }
    if ((int64_t)m * l == 0) return PCMM_OK;
    hipStream_t s = (hipStream_t)stream;
    if (n == 0) return fill_identity(C, (int64_t)m * l, s);
    if (!workspace || ws_bytes < L.total) return PCMM_ENOMEM;
    char *ws = (char *)workspace;
    // the plan arrays, packed once on the host
    std::vector<char> blob(L.total - L.off_ops, 0);
    auto put = [&](size_t off, const void *src, size_t bytes) {
        if (bytes) memcpy(blob.data() + (off - L.off_ops), src, bytes);
    };
    put(L.off_ops, P.ops.data(), P.ops.size() * sizeof(plan_op));
    put(L.off_opb, P.op_begin.data(), P.op_begin.size() * 4);
    put(L.off_entb, P.entry_begin.data(), P.entry_begin.size() * 4);
    put(L.off_ent, P.entries.data(), P.entries.size() * 2);
    put(L.off_ucol, P.unit_col.data(), P.unit_col.size() * 4);
    put(L.off_ugrp, P.unit_grp.data(), P.unit_grp.size() * 4);
    put(L.off_uoff, P.unit_off.data(), P.unit_off.size() * 4);
    put(L.off_cbeg, P.combo_begin.data(), P.combo_begin.size() * 4);
    put(L.off_combos, P.combos.data(), P.combos.size() * sizeof(plan_combo));
    put(L.off_codes, P.codes.data(), P.codes.size() * 2);
    pcmm_status st = upload(ws + L.off_ops, blob.data(), blob.size(), s);
    if (st) return st;
    uint32_t *Bm = (uint32_t *)(ws + L.off_bm);
    uint32_t *regs = (uint32_t *)(ws + L.off_regs);
    uint32_t *table = (uint32_t *)(ws + L.off_table);
    const int rmax = std::max(P.max_regs, 1);
    const int emax = std::max(P.max_entries, 1);
    hipLaunchKernelGGL(paillier_to_mont_kernel, dim3(blocks_for((int64_t)n * l)), dim3(256), 0, s, ctx->d_consts, ctx->n0, B,
                       Bm, (int64_t)n * l);
    PCMM_LAUNCH_CHECK();
    hipLaunchKernelGGL(paillier_table_kernel, dim3(blocks_for((int64_t)P.nunits * l)), dim3(256), 0, s, ctx->d_consts,
                       ctx->n0, (const plan_op *)(ws + L.off_ops), (const int32_t *)(ws + L.off_opb),
                       (const int32_t *)(ws + L.off_entb), (const int16_t *)(ws + L.off_ent),
                       (const int32_t *)(ws + L.off_ucol), (const int32_t *)(ws + L.off_ugrp),
                       (const int32_t *)(ws + L.off_uoff), P.nunits, l, rmax, emax, (const uint32_t *)Bm, regs, table);
    PCMM_LAUNCH_CHECK();
    if (!P.combos.empty()) {
        hipLaunchKernelGGL(paillier_combo_kernel, dim3(blocks_for((int64_t)P.ngroups * l)), dim3(256), 0, s,
                           ctx->d_consts, ctx->n0, (const plan_combo *)(ws + L.off_combos),
                           (const int32_t *)(ws + L.off_cbeg), P.ngroups, l, emax, table);
        PCMM_LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(paillier_accumulate_kernel, dim3(blocks_for((int64_t)m * l)), dim3(256), 0, s, ctx->d_consts, ctx->n0,
                       (const int16_t *)(ws + L.off_codes), m, P.ngroups, l, emax, (const uint32_t *)table, C);
    PCMM_LAUNCH_CHECK();
    return PCMM_OK;
}

pcmm_status pcmm_paillier_diag(pcmm_paillier ctx, int32_t op, const uint32_t *a, const uint32_t *b,
                               uint32_t *out, int64_t count, void *stream) {
    if (!ctx || op < 0 || op > 3 || count < 0) return PCMM_EINVAL;
    if (!on_ctx_device(ctx)) return PCMM_EINVAL;
    if (count > 0 && (!a || !b || !out)) return PCMM_EINVAL;
    if (!count) return PCMM_OK;
    hipLaunchKernelGGL(paillier_diag_kernel, dim3(blocks_for(count)), dim3(256), 0, (hipStream_t)stream, ctx->d_consts,
                       ctx->n0, op, a, b, out, count);
    PCMM_LAUNCH_CHECK();
    return PCMM_OK;
}

}  // extern "C"
