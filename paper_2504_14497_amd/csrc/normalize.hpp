// normalize.hpp -- batched Jacobian -> affine conversion (internal launcher).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/pcmm.h"

namespace pcmm {

// Threads (a multiple of 256) and points per thread used to normalise n_elem
// elements: about 24 elements per thread, so that one inversion serves them.
void normalize_geometry(int64_t n_elem, int64_t *threads, int *per_thread);

// Scratch bytes needed by launch_normalize for n_elem elements of npts points.
size_t normalize_scratch_bytes(int64_t n_elem, int npts);

// in: Jacobian planes (3 coordinates per point), out: affine planes (2 per
// point); in_mont / out_mont select Montgomery or canonical limbs on each side.
// out may alias in.  Queues one kernel on s.
pcmm_status launch_normalize(const uint32_t *in, int64_t ld_in, bool in_mont, uint32_t *out,
                             int64_t ld_out, bool out_mont, int64_t n_elem, int npts, void *scratch,
                             size_t scratch_bytes, hipStream_t s);

}  // namespace pcmm
