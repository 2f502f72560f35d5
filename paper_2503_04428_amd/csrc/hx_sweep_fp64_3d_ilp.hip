// FP64 3D instantiations that run one wave per SIMD (HLLC + van Leer with 6 to 9 fields, and the
// gas + radiation EoS with 5 to 9 fields), built with the instruction-level-parallelism machine
// scheduler: with a single wave per SIMD nothing hides a dependent instruction's latency, and
// that scheduler interleaves independent chains (e.g. the two Newton solves of a face pair).
// Measured: Sedov 256^3 2.46 -> 2.39 ms (ideal gas, 7 fields), 8.43 -> 8.03 ms (gas + radiation
// with ten fixed Newton steps); 6 fields on 256x128x128 0.689 -> 0.676 ms (Cartesian), 0.778 ->
// 0.738 ms (spherical).  The same schedule on the two-waves-per-SIMD 5-field sweeps spills more and
// is slower (1.24 -> 1.60 ms), so those stay in the default units.  Built with -ffp-contract=off:
// the arithmetic is the same as the default units', only the order of independent instructions
// differs.
#include "hx_sweep_inst.h"

namespace hx {

hipError_t launch_sweep_fp64_3d_ilp(const SweepParams& p, int spec, int nvar, int geom, hipStream_t s, int* occ)
{
    if (spec == 1) {
        switch (nvar) {
        case 6: return go<double, 6, 3, 1, 1>(p, geom, s, occ);
        case 7: return go<double, 7, 3, 1, 1>(p, geom, s, occ);
        case 8: return go<double, 8, 3, 1, 1>(p, geom, s, occ);
        case 9: return go<double, 9, 3, 1, 1>(p, geom, s, occ);
        default: return hipErrorInvalidValue;
        }
    }
    if (spec == 4) {
        switch (nvar) {
        case 5: return go<double, 5, 3, 4, 1>(p, geom, s, occ);
        case 6: return go<double, 6, 3, 4, 1>(p, geom, s, occ);
        case 7: return go<double, 7, 3, 4, 1>(p, geom, s, occ);
        case 8: return go<double, 8, 3, 4, 1>(p, geom, s, occ);
        case 9: return go<double, 9, 3, 4, 1>(p, geom, s, occ);
        default: return hipErrorInvalidValue;
        }
    }
    return hipErrorInvalidValue;
}

}  // namespace hx
