// k_schoolbook.hip -- schoolbook PC-MM (Sec. 3.1) and the public normaliser.
//
// One lane per output point (i, j, pt): for k = 0..n-1 it computes
// |a_ik| (+-B_kj) with the Montgomery ladder of Alg. 1 over the declared t
// bits (t doublings and t additions, branch-free per lane) and adds it into a
// Jacobian accumulator held in VGPRs.  Lanes are ordered with j fastest so the
// loads of B[k, :] coalesce.
#include "common.hpp"
#include "normalize.hpp"
#include "plan.hpp"

using namespace pcmm;

namespace {

// plaintext element x: int8 / uint8 up to 8 bits, int16 / uint16 beyond
__device__ __forceinline__ int plain_at_dev(const void *A, int64_t x, int bits, int is_signed) {
    if (bits <= 8) return is_signed ? (int)((const int8_t *)A)[x] : (int)((const uint8_t *)A)[x];
    return is_signed ? (int)((const int16_t *)A)[x] : (int)((const uint16_t *)A)[x];
}

__global__ void __launch_bounds__(256) schoolbook_kernel(const void *__restrict__ A, int m, int n, int l, int bits,
                                                         int is_signed, const uint32_t *__restrict__ B, int64_t ldb,
                                                         uint32_t *__restrict__ out, int64_t ld_out,
                                                         int out_canonical) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t total = (int64_t)m * l * 2;
    if (t >= total) return;
    const int j = (int)(t % l);
    const int pt = (int)((t / l) & 1);
    const int i = (int)(t / (2 * (int64_t)l));
    jpt acc = jpt_infinity();
    for (int k = 0; k < n; ++k) {
        const int a = plain_at_dev(A, (int64_t)i * n + k, bits, is_signed);
        if (a == 0) continue;
        apt b = load_affine(B, ldb, pt, (int64_t)k * l + j);
        if (a < 0) b = apt_neg(b);
        jpt term = ladder_small((uint32_t)(a < 0 ? -a : a), bits, b);
        acc = jpt_add(acc, term);
    }
    const int64_t e = (int64_t)i * l + j;
    if (out_canonical) store_jac(out, ld_out, pt, e, acc);
    else store_jac_m(out, ld_out, pt, e, acc);
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

bool a_in_range(const void *A, int64_t count, int bits, bool is_signed) {
    const int lo = is_signed ? -(1 << (bits - 1)) : 0;
    const int hi = is_signed ? (1 << (bits - 1)) - 1 : (1 << bits) - 1;
    for (int64_t x = 0; x < count; ++x) {
        const int v = plain_at(A, x, bits, is_signed);
        if (v < lo || v > hi) return false;
    }
    return true;
}

// device bytes of A: 2 per element, enough for either element width
size_t a_bytes(int32_t m, int32_t n) { return align256((size_t)m * n * 2); }

}  // namespace

extern "C" size_t pcmm_schoolbook_workspace(int32_t m, int32_t n, int32_t l, int32_t c_form) {
    if (m < 0 || n < 0 || l < 0) return 0;
    int64_t n_out = (int64_t)m * l;
    int64_t ldc = std::max<int64_t>(64, (n_out + 63) / 64 * 64);
    size_t bytes = a_bytes(m, n);
    if (c_form == PCMM_AFFINE) bytes += align256((size_t)JAC2_PLANES * ldc * 4) + align256(normalize_scratch_bytes(n_out, 2));
    return bytes + 256;
}

extern "C" pcmm_status pcmm_schoolbook(const void *A, int32_t m, int32_t n, int32_t bits, int32_t is_signed,
                                       const pcmm_mat *B, pcmm_mat *C, void *workspace, size_t ws_bytes,
                                       void *stream) {
    if (!B || !C || m < 0 || n < 0 || bits < 1 || bits > 16) return PCMM_EINVAL;
    if (B->rows != n || B->cols < 0 || B->npts != 2 || B->form != PCMM_AFFINE) return PCMM_EINVAL;
    const int l = B->cols;
    const int64_t n_out = (int64_t)m * l;
    if (B->ld < (int64_t)n * l || ((int64_t)n * l > 0 && !B->d)) return PCMM_EINVAL;
    if (C->rows != m || C->cols != l || C->npts != 2 || (C->form != PCMM_AFFINE && C->form != PCMM_JACOBIAN))
        return PCMM_EINVAL;
    if (C->ld < n_out || (n_out > 0 && !C->d)) return PCMM_EINVAL;
    if ((int64_t)m * n > 0 && !A) return PCMM_EINVAL;
    if (!a_in_range(A, (int64_t)m * n, bits, is_signed != 0)) return PCMM_ERANGE;
    if (n_out == 0) return PCMM_OK;
    if (!workspace || ws_bytes < pcmm_schoolbook_workspace(m, n, l, C->form)) return PCMM_ENOMEM;
    hipStream_t s = (hipStream_t)stream;
    char *ws = (char *)workspace;
    void *dA = ws;
    const size_t elem = bits <= 8 ? 1 : 2;
    if ((int64_t)m * n > 0) PCMM_HIP_TRY(hipMemcpyAsync(dA, A, (size_t)m * n * elem, hipMemcpyHostToDevice, s));
    const bool affine_out = C->form == PCMM_AFFINE;
    const int64_t ldc = std::max<int64_t>(64, (n_out + 63) / 64 * 64);
    uint32_t *jac = affine_out ? (uint32_t *)(ws + a_bytes(m, n)) : C->d;
    const int64_t ld_jac = affine_out ? ldc : C->ld;
    int64_t blocks = (2 * n_out + 255) / 256;
    hipLaunchKernelGGL(schoolbook_kernel, dim3((unsigned)blocks), dim3(256), 0, s, dA, m, n, l, bits, is_signed, B->d,
                       B->ld, jac, ld_jac, affine_out ? 0 : 1);
    PCMM_LAUNCH_CHECK();
    if (affine_out) {
        size_t off = a_bytes(m, n) + align256((size_t)JAC2_PLANES * ldc * 4);
        return launch_normalize(jac, ld_jac, true, C->d, C->ld, false, n_out, 2, ws + off, ws_bytes - off, s);
    }
    return PCMM_OK;
}

extern "C" size_t pcmm_normalize_workspace(int64_t elements, int32_t npts) {
    if (elements < 0 || npts < 1 || npts > 2) return 0;
    return normalize_scratch_bytes(elements, npts) + 256;
}

extern "C" pcmm_status pcmm_normalize(const pcmm_mat *in, pcmm_mat *out, void *workspace, size_t ws_bytes,
                                      void *stream) {
    if (!in || !out) return PCMM_EINVAL;
    const int64_t n = (int64_t)in->rows * in->cols;
    if (in->rows < 0 || in->cols < 0 || in->form != PCMM_JACOBIAN || (in->npts != 1 && in->npts != 2) ||
        in->ld < n || (n > 0 && !in->d))
        return PCMM_EINVAL;
    if (out->rows != in->rows || out->cols != in->cols || out->npts != in->npts || out->form != PCMM_AFFINE ||
        out->ld < n || (n > 0 && !out->d))
        return PCMM_EINVAL;
    if (out->d == in->d && out->ld != in->ld) return PCMM_EINVAL;
    if (n == 0) return PCMM_OK;
    if (!workspace || ws_bytes < normalize_scratch_bytes(n, in->npts)) return PCMM_ENOMEM;
    return launch_normalize(in->d, in->ld, false, out->d, out->ld, false, n, in->npts, workspace, ws_bytes,
                            (hipStream_t)stream);
}

extern "C" const char *pcmm_strerror(pcmm_status s) {
    switch (s) {
        case PCMM_OK: return "success";
        case PCMM_EINVAL: return "invalid argument (shape, form, bit-width, pointer or configuration)";
        case PCMM_ERANGE: return "an entry of A is outside its declared bit-width";
        case PCMM_ENOMEM: return "workspace too small";
        case PCMM_EDEVICE: return "HIP runtime or launch error";
        case PCMM_ENOTONCURVE: return "point is not a finite point of P-256";
        case PCMM_ETOOLARGE: return "problem needs more than the library's static scratch (PCMM_STATIC_SCRATCH_BYTES)";
        default: return "unknown status";
    }
}
