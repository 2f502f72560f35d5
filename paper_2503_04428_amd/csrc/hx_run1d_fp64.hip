// FP64 instantiations of the persistent 1D run, built like the FP64 sweep (no contraction), so
// that each step rounds as the sweep's 1D path and the oracle do.
#include "hx_run1d_kernel.h"

namespace hx {

hipError_t launch_run1d_fp64(const Run1dParams& p, int nvar, hipStream_t s)
{
    return run1d_launch<double>(p, nvar, s);
}

}  // namespace hx
