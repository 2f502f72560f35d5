// FP64 instantiations of the fused sweep with the gas + radiation EoS (variant 4: temperature by
// Newton's method in every primitive <-> conserved conversion, sound speed of the mixture; limiter
// and Riemann solver chosen at run time), for 5 to 9 fields.  Built with -ffp-contract=off like the
// other FP64 units.
#include "hx_sweep_inst.h"

namespace hx {

hipError_t launch_sweep_fp64_rad(const SweepParams& p, int ndim, int nvar, int geom, hipStream_t s, int* occ)
{
    switch (nvar) {
    case 5: return go_nv<double, 5, 4>(p, ndim, geom, s, occ);
    case 6: return go_nv<double, 6, 4>(p, ndim, geom, s, occ);
    case 7: return go_nv<double, 7, 4>(p, ndim, geom, s, occ);
    case 8: return go_nv<double, 8, 4>(p, ndim, geom, s, occ);
    case 9: return go_nv<double, 9, 4>(p, ndim, geom, s, occ);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace hx
