// Test-side stand-in for <hip/hip_runtime.h>: lets the library's device
// headers (field and point arithmetic) compile as plain host C++ with g++, so
// that their formulas can be checked on the CPU against the oracle.  One
// lane per call: a wavefront vote is the lane's own predicate, and register
// constraints that only steer the GPU compiler's scheduling vanish.
//
// Test infrastructure only; nothing in the library includes this file.
#pragma once
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <cmath>

#define __device__
#define __host__
#define __global__
#define __shared__
#define __forceinline__ inline __attribute__((always_inline))
#define __noinline__ __attribute__((noinline))
#define __launch_bounds__(...)

typedef int hipError_t;
typedef void *hipStream_t;
typedef void *hipEvent_t;
enum { hipSuccess = 0 };
static inline hipError_t hipGetLastError() { return hipSuccess; }

// a single lane: the vote over the wavefront is the lane's own predicate
static inline unsigned long long __ballot(int pred) { return pred ? 1ull : 0ull; }

// empty register constraints (scheduling hints for the GPU compiler) drop out
#define asm(...) ((void)0)
