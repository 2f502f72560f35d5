// Dispatch of the fused sweep over the compile-time shapes (dimension, field count, geometry).
#pragma once
#include "hx_launch.h"
#include "hx_sweep.h"

namespace hx {

// Launches the instantiation that matches the run-time shape, or, with occ != nullptr, only
// reports how many of its workgroups fit on one compute unit.
template <typename R, int NV, int NDIM, int SPEC, int TAG = 0>
static hipError_t go(const SweepParams& p, int geom, hipStream_t s, int* occ)
{
    const dim3 grid = sweep_grid(NDIM, p.n, p.kz), block = sweep_block(NDIM);
    auto run = [&](auto kern) -> hipError_t {
        if (occ)
            return hipOccupancyMaxActiveBlocksPerMultiprocessor(occ, kern, (int)(block.x * block.y), 0);
        hipLaunchKernelGGL(kern, grid, block, 0, s, p);
        return hipGetLastError();
    };
    if (geom == HX_SPH)
        return run(sweep_kernel<R, NV, NDIM, HX_SPH, SPEC, TAG>);
    // 3D Cartesian configurations without gravity or heating: the instantiation without sources
    if constexpr (NDIM == 3) {
        if (p.gravity == HX_GRAV_NONE && p.ni < 0)
            return run(sweep_kernel<R, NV, NDIM, HX_CART, SPEC, TAG, 0>);
    }
    return run(sweep_kernel<R, NV, NDIM, HX_CART, SPEC, TAG>);
}

template <typename R, int NV, int SPEC>
static hipError_t go_nv(const SweepParams& p, int ndim, int geom, hipStream_t s, int* occ)
{
    switch (ndim) {
    case 1: return go<R, NV, 1, SPEC>(p, geom, s, occ);
    case 2: return go<R, NV, 2, SPEC>(p, geom, s, occ);
    default: return go<R, NV, 3, SPEC>(p, geom, s, occ);
    }
}

template <typename R, int SPEC>
static hipError_t launch_sweep_t(const SweepParams& p, int ndim, int nvar, int geom, hipStream_t s, int* occ)
{
    switch (nvar) {
    case 5: return go_nv<R, 5, SPEC>(p, ndim, geom, s, occ);
    case 6: return go_nv<R, 6, SPEC>(p, ndim, geom, s, occ);
    case 7: return go_nv<R, 7, SPEC>(p, ndim, geom, s, occ);
    case 8: return go_nv<R, 8, SPEC>(p, ndim, geom, s, occ);
    case 9: return go_nv<R, 9, SPEC>(p, ndim, geom, s, occ);
    default: return hipErrorInvalidValue;
    }
}

// learned-limiter form: FP32, 5..7 fields
template <typename R>
static hipError_t launch_sweep_mlp_t(const SweepParams& p, int ndim, int nvar, int geom, hipStream_t s, int* occ)
{
    switch (nvar) {
    case 5: return go_nv<R, 5, 2>(p, ndim, geom, s, occ);
    case 6: return go_nv<R, 6, 2>(p, ndim, geom, s, occ);
    case 7: return go_nv<R, 7, 2>(p, ndim, geom, s, occ);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace hx
