// FP32-form instantiations of the fused sweep with the learned slope limiter (BF16 matrix-core
// network, HLLC), for 5 to 7 fields.
#include "hx_sweep_inst.h"

namespace hx {

hipError_t launch_sweep_fp32_mlp(const SweepParams& p, int ndim, int nvar, int geom, hipStream_t s, int* occ)
{
    return launch_sweep_mlp_t<float>(p, ndim, nvar, geom, s, occ);
}

}  // namespace hx
