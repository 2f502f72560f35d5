// FP32-form instantiations of the persistent 1D run, built with the FP32 sweep's flags
// (contraction allowed), like the FP32 sweep's 1D path.
#include "hx_run1d_kernel.h"

namespace hx {

hipError_t launch_run1d_fp32(const Run1dParams& p, int nvar, hipStream_t s)
{
    return run1d_launch<float>(p, nvar, s);
}

}  // namespace hx
