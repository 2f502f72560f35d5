// FP64 instantiations of the fused sweep with the internal-energy monitor and the gas + radiation
// EoS together (variant 5: the monitor's pressure through the EoS; HLLC, limiter chosen at run
// time), for 6 to 9 fields.  Built with -ffp-contract=off like the other FP64 units.
#include "hx_sweep_inst.h"

namespace hx {

hipError_t launch_sweep_fp64_de_rad(const SweepParams& p, int ndim, int nvar, int geom, hipStream_t s, int* occ)
{
    switch (nvar) {
    case 6: return go_nv<double, 6, 5>(p, ndim, geom, s, occ);
    case 7: return go_nv<double, 7, 5>(p, ndim, geom, s, occ);
    case 8: return go_nv<double, 8, 5>(p, ndim, geom, s, occ);
    case 9: return go_nv<double, 9, 5>(p, ndim, geom, s, occ);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace hx
