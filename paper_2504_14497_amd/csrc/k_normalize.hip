// k_normalize.hip -- Jacobian -> canonical affine with batched inversion.
//
// Montgomery's simultaneous-inversion trick: one thread walks its batch of
// points forward keeping the running product of the nonzero Z values (and
// storing each prefix), inverts the total once (Fermat, 255 S + 12 M), then
// walks backward: Z_j^-1 = inv * prefix_{j-1}, inv <- inv * Z_j.  Per point
// that is 3 multiplications plus the affine conversion (x = X Z^-2,
// y = Y Z^-3), with one inversion per batch.  Z = 0 (the identity) maps to
// (0, 0) and is skipped in the product.
#include "common.hpp"
#include "normalize.hpp"

using namespace pcmm;

namespace {

// Thread t handles elements e = t + j * T (j < per_thread); both points of an
// element are handled by the same thread, and an element is written only after
// all of its inputs were read, so `out` may alias `in`.
template <bool IN_MONT, bool OUT_MONT>
__global__ void __launch_bounds__(256) normalize_kernel(const uint32_t *in, int64_t ld_in, uint32_t *out,
                                                        int64_t ld_out, int64_t n_elem, int npts,
                                                        uint32_t *__restrict__ prefix, int64_t ld_pre,
                                                        int per_thread) {
    int64_t T = (int64_t)gridDim.x * blockDim.x;
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    fe acc = fe_one_mont();
    int slot = 0;
    for (int j = 0; j < per_thread; ++j) {
        int64_t e = t + (int64_t)j * T;
        if (e >= n_elem) break;
        for (int pt = 0; pt < npts; ++pt, ++slot) {
            fe z = IN_MONT ? soa_load_m(in, ld_in, pt * 3 + 2, e) : soa_load_mont(in, ld_in, pt * 3 + 2, e);
            soa_store_m(prefix, ld_pre, 0, t + (int64_t)slot * T, acc);
            if (!fe_is_zero(z)) acc = fe_mul(acc, z);
        }
    }
    if (slot == 0) return;
    fe inv = fe_inv(acc);
    for (int j = per_thread - 1; j >= 0; --j) {
        int64_t e = t + (int64_t)j * T;
        if (e >= n_elem) continue;
        // npts is 1 or 2; the fixed-size loops keep P and A in registers
        jpt P[2];
        apt A[2];
#pragma unroll
        for (int pt = 0; pt < 2; ++pt) {
            if (pt < npts) P[pt] = IN_MONT ? load_jac_m(in, ld_in, pt, e) : load_jac(in, ld_in, pt, e);
        }
#pragma unroll
        for (int pt = 1; pt >= 0; --pt) {
            if (pt >= npts) continue;
            --slot;
            bool inf = fe_is_zero(P[pt].Z);
            fe pre = soa_load_m(prefix, ld_pre, 0, t + (int64_t)slot * T);
            fe zinv = fe_mul(inv, pre);
            if (!inf) inv = fe_mul(inv, P[pt].Z);
            A[pt] = jpt_to_affine_with(P[pt], zinv);
            if (inf) {
                A[pt].x = fe_zero();
                A[pt].y = fe_zero();
            }
        }
#pragma unroll
        for (int pt = 0; pt < 2; ++pt) {
            if (pt >= npts) continue;
            if (OUT_MONT) {
                store_aff_m(out, ld_out, pt, e, A[pt]);
            } else {
                store_affine(out, ld_out, pt, e, A[pt]);
            }
        }
    }
}

}  // namespace

namespace pcmm {

// number of threads and batch length for n_elem elements
void normalize_geometry(int64_t n_elem, int64_t *threads, int *per_thread) {
    const int64_t target_batch = 24;  // points per thread (inversion amortised over them)
    int64_t th = (n_elem + target_batch - 1) / target_batch;
    if (th < 1) th = 1;
    th = (th + 255) / 256 * 256;
    *threads = th;
    *per_thread = (int)((n_elem + th - 1) / th);
}

size_t normalize_scratch_bytes(int64_t n_elem, int npts) {
    int64_t th;
    int per;
    normalize_geometry(n_elem, &th, &per);
    return (size_t)th * (size_t)per * (size_t)npts * NL * sizeof(uint32_t);
}

pcmm_status launch_normalize(const uint32_t *in, int64_t ld_in, bool in_mont, uint32_t *out,
                             int64_t ld_out, bool out_mont, int64_t n_elem, int npts, void *scratch,
                             size_t scratch_bytes, hipStream_t s) {
    if (n_elem == 0) return PCMM_OK;
    int64_t th;
    int per;
    normalize_geometry(n_elem, &th, &per);
    int64_t ld_pre = th * per * npts;
    if (scratch_bytes < (size_t)ld_pre * NL * sizeof(uint32_t)) return PCMM_ENOMEM;
    // prefix slot s of thread t lives at column t + s * th (slots < per * npts)
    unsigned blocks = (unsigned)(th / 256);
void (*kern)(const uint32_t *, int64_t, uint32_t *, int64_t, int64_t, int, uint32_t *, int64_t, int) =
        in_mont ? (out_mont ? normalize_kernel<true, true> : normalize_kernel<true, false>)
                : (out_mont ? normalize_kernel<false, true> : normalize_kernel<false, false>);
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(256), 0, s, in, ld_in, out, ld_out, n_elem, npts,
                       (uint32_t *)scratch, ld_pre, per);
    PCMM_LAUNCH_CHECK();
    return PCMM_OK;
}

}  // namespace pcmm
