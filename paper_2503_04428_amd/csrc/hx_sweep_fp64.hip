// FP64 instantiations of the fused sweep.  Built with -ffp-contract=off so that every
// expression rounds exactly like the FP64 CPU oracle's.
// Limiter and Riemann solver chosen at run time.
#include "hx_sweep_inst.h"

namespace hx {

hipError_t launch_sweep_fp64_generic(const SweepParams& p, int ndim, int nvar, int geom, hipStream_t s, int* occ)
{
    return launch_sweep_t<double, 0>(p, ndim, nvar, geom, s, occ);
}

}  // namespace hx
