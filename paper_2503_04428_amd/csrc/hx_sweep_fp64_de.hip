// FP64 instantiations of the fused sweep with the internal-energy monitor (variant 3: the last
// field is the internal energy e; HLLC, limiter chosen at run time), for 6 to 9 fields.  Built
// with -ffp-contract=off like the other FP64 units.
#include "hx_sweep_inst.h"

namespace hx {

hipError_t launch_sweep_fp64_de(const SweepParams& p, int ndim, int nvar, int geom, hipStream_t s, int* occ)
{
    switch (nvar) {
    case 6: return go_nv<double, 6, 3>(p, ndim, geom, s, occ);
    case 7: return go_nv<double, 7, 3>(p, ndim, geom, s, occ);
    case 8: return go_nv<double, 8, 3>(p, ndim, geom, s, occ);
    case 9: return go_nv<double, 9, 3>(p, ndim, geom, s, occ);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace hx
