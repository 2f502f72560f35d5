// Host-side launch interface of the persistent one-workgroup 1D run (kernel in hx_run1d_kernel.h;
// FP64 instantiations in hx_run1d_fp64.hip, FP32 in hx_run1d_fp32.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "hx_params.h"

namespace hx {

// persistent 1D run (one workgroup): Cartesian, one row, ideal gas, no sources
struct Run1dParams {
    void* U;             // the current state [nvar][n] (FP64 or FP32), advanced in place
    int n, ng;
    long long plane;     // cells per field (= n)
    double gamma, cfl;
    int limiter, riemann;
    int bc0[2];          // boundary kinds of axis 0
    Geo geo;
    int* flag;           // set to 1 when a non-physical state is met
    double* out;         // out[0] = final time, out[1] = steps taken
    double t0, t_end;
    int max_steps;
};
constexpr int RUN1D_MAX_CELLS = 2046;  // one workgroup: 1024 threads x 2 cells (FP32), 512 x 4 (FP64)
// LDS bytes of the field arrays: primitives (then face fluxes) and the two half-step face states
// of cells -2 .. n+1, 3 nvar (n + 4) values
inline size_t run1d_lds_bytes(int n, int nvar, bool fp32)
{
    return (size_t)3 * nvar * (n + 4) * (fp32 ? 4 : 8);
}
hipError_t launch_run1d_fp64(const Run1dParams& p, int nvar, hipStream_t s);
hipError_t launch_run1d_fp32(const Run1dParams& p, int nvar, hipStream_t s);
inline hipError_t launch_run1d(const Run1dParams& p, int nvar, bool fp32, hipStream_t s)
{
    return fp32 ? launch_run1d_fp32(p, nvar, s) : launch_run1d_fp64(p, nvar, s);
}

}  // namespace hx
