// k_normalize.hip -- Jacobian -> canonical affine with batched inversion
// (pcmm_normalize and the internal launcher; the per-thread algorithm is in
// normalize_dev.hpp).
#include "normalize.hpp"
#include "normalize_dev.hpp"

using namespace pcmm;

namespace {

template <bool IN_MONT, bool OUT_MONT>
__global__ void __launch_bounds__(256) normalize_kernel(const uint32_t *in, int64_t ld_in, uint32_t *out,
                                                        int64_t ld_out, int64_t n_elem, int npts,
                                                        uint32_t *__restrict__ prefix, int64_t ld_pre,
                                                        int per_thread) {
    const int64_t T = (int64_t)gridDim.x * blockDim.x;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    normalize_points<IN_MONT, OUT_MONT>(in, ld_in, out, ld_out, n_elem, npts, prefix, ld_pre, per_thread, t, T);
}

}  // namespace

namespace pcmm {

// number of threads and batch length for n_elem elements
void normalize_geometry(int64_t n_elem, int64_t *threads, int *per_thread) {
    // elements per thread: one inversion is amortised over them, but each
    // thread is one serial chain (prefix products, the inversion, the way
    // back).  One element per thread while the chains fit one wavefront per
    // SIMD (65536 threads: latency is then one inversion), two up to twice
    // that, batches of 4 until there are enough chains for 4 wavefronts per
    // SIMD (262144 threads), larger batches (up to 24) beyond that.
    constexpr int64_t enough_threads = 262144;
    const int64_t target_batch =
        n_elem <= 65536    ? 1
        : n_elem <= 131072 ? 2
                           : std::min<int64_t>(24, std::max<int64_t>(4, (n_elem + enough_threads - 1) / enough_threads));
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
