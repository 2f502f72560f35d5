// FP64 instantiations of the fused sweep.  Built with -ffp-contract=off so that every
// expression rounds exactly like the FP64 CPU oracle's.
#include "hx_launch.h"
#include "hx_sweep.h"

namespace hx {

template <typename R, int NV, int NDIM>
static hipError_t go(const SweepParams& p, int geom, hipStream_t s)
{
    dim3 grid = sweep_grid(NDIM, p.n, p.kz), block = sweep_block(NDIM);
    if (geom == HX_SPH)
        sweep_kernel<R, NV, NDIM, HX_SPH><<<grid, block, 0, s>>>(p);
    else
        sweep_kernel<R, NV, NDIM, HX_CART><<<grid, block, 0, s>>>(p);
    return hipGetLastError();
}

template <typename R, int NV>
static hipError_t go_nv(const SweepParams& p, int ndim, int geom, hipStream_t s)
{
    switch (ndim) {
    case 1: return go<R, NV, 1>(p, geom, s);
    case 2: return go<R, NV, 2>(p, geom, s);
    default: return go<R, NV, 3>(p, geom, s);
    }
}

hipError_t launch_sweep_fp64(const SweepParams& p, int ndim, int nvar, int geom, hipStream_t s)
{
    switch (nvar) {
    case 5: return go_nv<double, 5>(p, ndim, geom, s);
    case 6: return go_nv<double, 6>(p, ndim, geom, s);
    case 7: return go_nv<double, 7>(p, ndim, geom, s);
    case 8: return go_nv<double, 8>(p, ndim, geom, s);
    case 9: return go_nv<double, 9>(p, ndim, geom, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace hx
