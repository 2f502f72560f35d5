// FP32-form instantiations of the fused sweep (FP32 storage and bulk arithmetic; FP64 for
// the internal-energy recovery at high Mach, the positivity test, the time step and the source
// terms).
// HLLC + van Leer, fixed at compile time.
#include "hx_sweep_inst.h"

namespace hx {

hipError_t launch_sweep_fp32_hllc_vl(const SweepParams& p, int ndim, int nvar, int geom, hipStream_t s, int* occ)
{
    return launch_sweep_t<float, 1>(p, ndim, nvar, geom, s, occ);
}

}  // namespace hx
