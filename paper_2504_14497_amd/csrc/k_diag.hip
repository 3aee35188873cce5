// k_diag.hip -- element-wise self-test kernels and throughput probes.
#include "../../include/pcmm_diag.h"
#include "common.hpp"

using namespace pcmm;

namespace {

__global__ void __launch_bounds__(256) field_op_kernel(int op, const uint32_t *__restrict__ a,
                                                        const uint32_t *__restrict__ b,
                                                        uint32_t *__restrict__ out, int64_t n) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    fe x = soa_load_mont(a, n, 0, e);
    fe y = (op <= 2) ? soa_load_mont(b, n, 0, e) : fe_zero();
    fe r;
    switch (op) {
        case 0: r = fe_add(x, y); break;
        case 1: r = fe_sub(x, y); break;
        case 2: r = fe_mul(x, y); break;
        case 3: r = fe_sqr(x); break;
        case 4: r = fe_inv(x); break;
        case 5: r = fe_neg(x); break;
        default: r = x; break;
    }
    soa_store_canon(out, n, 0, e, r);
}

__global__ void __launch_bounds__(256) field_raw_kernel(int op, const uint32_t *__restrict__ a,
                                                         const uint32_t *__restrict__ b,
                                                         uint32_t *__restrict__ out, int64_t n) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    fe x = soa_load_m(a, n, 0, e);
    fe y = soa_load_m(b, n, 0, e);
    fe r = fe_zero();
    switch (op) {
        case 0: r = fe_add(x, y); break;
        case 1: r = fe_sub(x, y); break;
        case 2: r = fe_mul(x, y); break;
        case 3: r = fe_sqr(x); break;
        case 4: r = fe_sub2(x, y); break;
        case 5: r = fe_mul3(x); break;
        case 6: r = fe_mul4(x); break;
        case 7: r = fe_neg(x); break;
        case 8: r = fe_canon(x); break;
        case 9: r = fe_dbl(x); break;
        case 10: r = fe_norm(x); break;
        case 11: r.v[0] = fe_eq(x, y) ? 1u : 0u; break;
        case 12: r.v[0] = fe_is_zero(x) ? 1u : 0u; break;
        case 13: r = fe_sub_w(x, y); break;
        case 14: r = fe_mul4_w(x); break;
        case 15: r = fe_sub_sub2(x, y, y); break;
        case 16: r = fe_sub2x(x, y); break;
        case 17: r = fe_mul(fe_sub_w(x, y), fe_mul4_w(y)); break;
        case 18: r = fe_mul_plus_t<true>(x, y, fe_2p_minus(y)); break;
        case 19: r = fe_4sub_sub2(x, y, y); break;
        case 20: r = fe_mul_sub2_t<true>(fe_x2(x), y, fe_norm(y), fe_norm(y)); break;
        case 21: r = fe_mul_ilp(x, y); break;
        case 22: r = fe_sqr_ilp(x); break;
        case 23: r = fe_inv(x); break;
        case 24: r = fe_mul_t<true, true>(x, y); break;
        case 25: r = fe_sqr_t<true, true>(x); break;
        case 26: r = fe_mul_plus_t<true, true>(x, y, fe_2p_minus(y)); break;
        case 27: r = fe_mul_t<true, true>(x, fe_x2(y)); break;
        case 28: r = fe_mul_sub2_t<true, true>(fe_x2(x), y, fe_norm(y), fe_norm(y)); break;
        case 29: r = fe_mul_sub_t<true, true>(x, y, fe_norm(y), fe_norm(y)); break;
        default: r = fe_inv_fermat(x); break;
    }
    soa_store_m(out, n, 0, e, r);
}

__global__ void __launch_bounds__(256) point_op_kernel(int op, const uint32_t *__restrict__ P,
                                                        int64_t ldp, const uint32_t *__restrict__ Q,
                                                        int64_t ldq, const uint32_t *__restrict__ K,
                                                        int t, uint32_t *__restrict__ R,
                                                        int64_t ldr, int64_t n) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    apt p = load_affine(P, ldp, 0, e);
    jpt r;
    switch (op) {
        case 0: {
            apt q = load_affine(Q, ldq, 0, e);
            r = jpt_add_affine(jpt_from_affine(p), q);
            break;
        }
        case 1: {
            apt q = load_affine(Q, ldq, 0, e);
            jpt jp = jpt_from_affine(p), jq = jpt_from_affine(q);
            // rescale to Z != 1: (X z^2, Y z^3, z) represents the same point
            fe zp = fe_add(q.x, fe_dbl(fe_one_mont()));
            fe zq = fe_add(p.y, fe_add(fe_dbl(fe_one_mont()), fe_one_mont()));
            if (!fe_is_zero(zp) && !jpt_is_inf(jp)) {
                fe z2 = fe_sqr(zp);
                jp.X = fe_mul(jp.X, z2);
                jp.Y = fe_mul(jp.Y, fe_mul(z2, zp));
                jp.Z = zp;
            }
            if (!fe_is_zero(zq) && !jpt_is_inf(jq)) {
                fe z2 = fe_sqr(zq);
                jq.X = fe_mul(jq.X, z2);
                jq.Y = fe_mul(jq.Y, fe_mul(z2, zq));
                jq.Z = zq;
            }
            r = jpt_add(jp, jq);
            break;
        }
        case 2: r = jpt_dbl(jpt_from_affine(p)); break;
        case 3: r = ladder_small(K[e], t, p); break;
        default: r = jpt_neg(jpt_from_affine(p)); break;
    }
    store_jac(R, ldr, 0, e, r);
}

// --- probes -----------------------------------------------------------------

__global__ void __launch_bounds__(256) probe_mad_kernel(uint32_t *out, uint32_t seed, int64_t iters) {
    uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t acc[8];
    uint32_t y[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        acc[i] = seed + tid + i;
        y[i] = (0x9E3779B9u * (i + 1)) ^ tid;
    }
    for (int64_t it = 0; it < iters; ++it) {
#pragma unroll
        for (int i = 0; i < 8; ++i) acc[i] = (uint64_t)(uint32_t)acc[i] * y[i] + acc[i];
    }
    uint64_t s = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) s ^= acc[i];
    if ((uint32_t)s == 0x12345678u) out[tid] = (uint32_t)(s >> 32);
}

__global__ void __launch_bounds__(256) probe_add3_kernel(uint32_t *out, uint32_t seed, int64_t iters) {
    uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t acc[8];
    uint32_t y[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        acc[i] = seed + tid * 7 + i;
        y[i] = (0x9E3779B9u * (i + 1)) ^ tid;
    }
    for (int64_t it = 0; it < iters; ++it) {
#pragma unroll
        for (int i = 0; i < 8; ++i) acc[i] = acc[i] + acc[(i + 3) & 7] + y[i];
    }
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) s ^= acc[i];
    if (s == 0x12345678u) out[tid] = s;
}

// 32-bit exclusive-or: 8 chains per lane, each reading another chain's value,
// with lane-dependent operands (so the compiler can neither fold the loop nor
// move the work to the scalar unit)
__global__ void __launch_bounds__(256) probe_xor_kernel(uint32_t *out, uint32_t seed, int64_t iters) {
    uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t acc[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) acc[i] = (seed + tid * 0x9E3779B9u) ^ (0x85EBCA6Bu * (i + 1));
    for (int64_t it = 0; it < iters; ++it) {
#pragma unroll
        for (int i = 0; i < 8; ++i) acc[i] ^= acc[(i + 1) & 7];
    }
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) s += acc[i];
    if (s == 0x12345678u) out[tid] = s;
}

__global__ void __launch_bounds__(256) probe_fma64_kernel(uint32_t *out, uint32_t seed, int64_t iters) {
    uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    double acc[8], y[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        acc[i] = (double)(seed + tid + i) * 1e-9;
        y[i] = 0.999999 + 1e-7 * i;
    }
    for (int64_t it = 0; it < iters; ++it) {
#pragma unroll
        for (int i = 0; i < 8; ++i) acc[i] = __builtin_fma(acc[i], y[i], 1e-12);
    }
    double s = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) s += acc[i];
    if (s == 12345.0) out[tid] = 1;
}

__global__ void __launch_bounds__(256) probe_femul_kernel(uint32_t *out, uint32_t seed, int64_t iters) {
    uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    fe x, y;
#pragma unroll
    for (int i = 0; i < NL; ++i) {
        x.v[i] = ((seed ^ (tid * 2654435761u)) + i * 77u) & LMASK;
        y.v[i] = (0x9E3779B9u * (i + 3) + tid) & LMASK;
    }
    x.v[NL - 1] &= 0xFFFFFFu;
    y.v[NL - 1] &= 0xFFFFFFu;
    for (int64_t it = 0; it < iters; ++it) x = fe_mul(x, y);
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < NL; ++i) s ^= x.v[i];
    if (s == 0x12345678u) out[tid] = s;
}

__global__ void __launch_bounds__(256) probe_madd_kernel(uint32_t *out, uint32_t seed, int64_t iters) {
    uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    // a fixed valid affine point (the generator) added over and over
    apt g;
    g.x = fe_to_mont(fe_from_const(GX_PLAIN));
    g.y = fe_to_mont(fe_from_const(GY_PLAIN));
    jpt acc = jpt_from_affine(g);
    acc = jpt_dbl(acc);
    for (int64_t it = 0; it < iters; ++it) acc = jpt_add_affine(acc, g);
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < NL; ++i) s ^= acc.X.v[i] ^ acc.Z.v[i];
    if (s == (0x12345678u ^ tid ^ seed)) out[tid] = s;
}

__global__ void __launch_bounds__(256) copy_kernel(const uint4 *__restrict__ src, uint4 *__restrict__ dst,
                                                   int64_t n4) {
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n4; x += (int64_t)gridDim.x * blockDim.x)
        dst[x] = src[x];
}

}  // namespace

extern "C" pcmm_status pcmm_diag_copy(const uint32_t *src, uint32_t *dst, int64_t words, void *stream) {
    if (words < 0 || (words > 0 && (!src || !dst)) || (words & 3) || (((uintptr_t)src | (uintptr_t)dst) & 15))
        return PCMM_EINVAL;
    if (words == 0) return PCMM_OK;
    int64_t n4 = words / 4;
    int64_t blocks = std::min<int64_t>((n4 + 255) / 256, 256 * 64);
    hipLaunchKernelGGL(copy_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, (const uint4 *)src,
                       (uint4 *)dst, n4);
    PCMM_LAUNCH_CHECK();
    return PCMM_OK;
}

extern "C" pcmm_status pcmm_diag_field(int32_t op, const uint32_t *a, const uint32_t *b,
                                       uint32_t *out, int64_t count, void *stream) {
    if (op < 0 || op > 6 || count < 0) return PCMM_EINVAL;
    if (count == 0) return PCMM_OK;
    if (!a || !out || (op <= 2 && !b)) return PCMM_EINVAL;
    int64_t blocks = (count + 255) / 256;
    if (blocks > 0x7FFFFFFF) return PCMM_EINVAL;
    hipLaunchKernelGGL(field_op_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, op,
                       a, b, out, count);
    PCMM_LAUNCH_CHECK();
    return PCMM_OK;
}

extern "C" pcmm_status pcmm_diag_field_raw(int32_t op, const uint32_t *a, const uint32_t *b, uint32_t *out,
                                           int64_t count, void *stream) {
    if (op < 0 || op > 30 || count < 0) return PCMM_EINVAL;
    if (count == 0) return PCMM_OK;
    if (!a || !b || !out) return PCMM_EINVAL;
    int64_t blocks = (count + 255) / 256;
    hipLaunchKernelGGL(field_raw_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, op, a, b, out,
                       count);
    PCMM_LAUNCH_CHECK();
    return PCMM_OK;
}

extern "C" pcmm_status pcmm_diag_point(int32_t op, const pcmm_mat *P, const pcmm_mat *Q,
                                       const uint32_t *k, int32_t t, pcmm_mat *R, void *stream) {
    if (op < 0 || op > 4 || !P || !R) return PCMM_EINVAL;
    int64_t n = (int64_t)P->rows * P->cols;
    if (P->rows < 0 || P->cols < 0 || P->form != PCMM_AFFINE || P->npts != 1 || P->ld < n) return PCMM_EINVAL;
    if (R->form != PCMM_JACOBIAN || R->npts != 1 || R->rows != P->rows || R->cols != P->cols || R->ld < n)
        return PCMM_EINVAL;
    if (op <= 1) {
        if (!Q || Q->form != PCMM_AFFINE || Q->npts != 1 || Q->rows != P->rows || Q->cols != P->cols ||
            Q->ld < n)
            return PCMM_EINVAL;
    }
    if (op == 3 && (!k || t < 0 || t > 32)) return PCMM_EINVAL;
    if (n == 0) return PCMM_OK;
    int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(point_op_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, op,
                       P->d, P->ld, Q ? Q->d : nullptr, Q ? Q->ld : 0, k, t, R->d, R->ld, n);
    PCMM_LAUNCH_CHECK();
    return PCMM_OK;
}

extern "C" pcmm_status pcmm_diag_probe(int32_t kind, int64_t iters, int32_t blocks, double *seconds,
                                       double *ops) {
    if (kind < 0 || kind > 5 || iters <= 0 || blocks <= 0 || !seconds || !ops) return PCMM_EINVAL;
    uint32_t *scratch = nullptr;
    PCMM_HIP_TRY(hipMalloc(&scratch, (size_t)blocks * 256 * sizeof(uint32_t)));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t err = hipEventCreate(&e0);
    auto keep = [&](hipError_t e) {  // the first error is the one reported
        if (err == hipSuccess) err = e;
    };
    keep(hipEventCreate(&e1));
    float ms = 0.f;
    if (err == hipSuccess) {
        keep(hipEventRecord(e0, 0));
        switch (kind) {
            case 0: hipLaunchKernelGGL(probe_mad_kernel, dim3(blocks), dim3(256), 0, 0, scratch, 1u, iters); break;
            case 1: hipLaunchKernelGGL(probe_add3_kernel, dim3(blocks), dim3(256), 0, 0, scratch, 1u, iters); break;
            case 2: hipLaunchKernelGGL(probe_femul_kernel, dim3(blocks), dim3(256), 0, 0, scratch, 1u, iters); break;
            case 3: hipLaunchKernelGGL(probe_madd_kernel, dim3(blocks), dim3(256), 0, 0, scratch, 1u, iters); break;
            case 4: hipLaunchKernelGGL(probe_fma64_kernel, dim3(blocks), dim3(256), 0, 0, scratch, 1u, iters); break;
            default: hipLaunchKernelGGL(probe_xor_kernel, dim3(blocks), dim3(256), 0, 0, scratch, 1u, iters); break;
        }
        keep(hipGetLastError());
        keep(hipEventRecord(e1, 0));
        keep(hipEventSynchronize(e1));
        keep(hipEventElapsedTime(&ms, e0, e1));
    }
    if (e0) keep(hipEventDestroy(e0));
    if (e1) keep(hipEventDestroy(e1));
    keep(hipFree(scratch));
    if (err != hipSuccess) return PCMM_EDEVICE;
    double per_thread = (kind <= 1 || kind >= 4) ? 8.0 * (double)iters : (double)iters;
    *seconds = ms * 1e-3;
    *ops = per_thread * (double)blocks * 256.0;
    return PCMM_OK;
}

extern "C" pcmm_status pcmm_diag_device(int32_t *cus, int32_t *clock_khz, int64_t *lds_per_block,
                                        char name[64]) {
    int dev = 0;
    PCMM_HIP_TRY(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    PCMM_HIP_TRY(hipGetDeviceProperties(&prop, dev));
    if (cus) *cus = prop.multiProcessorCount;
    if (clock_khz) *clock_khz = prop.clockRate;
    if (lds_per_block) *lds_per_block = (int64_t)prop.sharedMemPerBlock;
    if (name) {
        int i = 0;
        for (; i < 63 && prop.gcnArchName[i]; ++i) name[i] = prop.gcnArchName[i];
        name[i] = 0;
    }
    return PCMM_OK;
}
