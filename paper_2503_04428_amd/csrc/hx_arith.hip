// The FP64 division and square root the sweeps use (div_rn, sqrt_rn in hx_device.h), applied to
// arrays, so that they can be checked against IEEE results computed elsewhere.
#include "hx_arith.h"
#include "hx_device.h"

namespace hx {

__global__ void __launch_bounds__(256) arith_check_kernel(const double* __restrict__ a, const double* __restrict__ b,
                                                         long long n, double* __restrict__ q, double* __restrict__ s)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const double x = a[i];
        q[i] = div_rn(x, b[i]);
        s[i] = sqrt_rn(fabs(x));
    }
}

hipError_t launch_arith_check(const double* a, const double* b, long long n, double* q, double* s, hipStream_t st)
{
    const long long blocks = (n + 255) / 256;
    const unsigned grid = (unsigned)(blocks < 65536 ? blocks : 65536);
    hipLaunchKernelGGL(arith_check_kernel, dim3(grid), dim3(256), 0, st, a, b, n, q, s);
    return hipGetLastError();
}

}  // namespace hx
