// Host-side launch interface of the FP64 arithmetic check (hx_arith.hip).
#pragma once
#include <hip/hip_runtime.h>

namespace hx {

// q[i] = div_rn(a[i], b[i]) and s[i] = sqrt_rn(|a[i]|), n elements (device pointers)
hipError_t launch_arith_check(const double* a, const double* b, long long n, double* q, double* s, hipStream_t st);

}  // namespace hx
