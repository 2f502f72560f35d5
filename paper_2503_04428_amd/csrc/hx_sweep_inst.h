// Dispatch of the fused sweep over the compile-time shapes (dimension, field count, geometry).
#pragma once
#include "hx_launch.h"
#include "hx_sweep.h"

namespace hx {

template <typename R, int NV, int NDIM, int SPEC>
static hipError_t go(const SweepParams& p, int geom, hipStream_t s)
{
    dim3 grid = sweep_grid(NDIM, p.n, p.kz), block = sweep_block(NDIM);
    if (geom == HX_SPH)
        sweep_kernel<R, NV, NDIM, HX_SPH, SPEC><<<grid, block, 0, s>>>(p);
    else
        sweep_kernel<R, NV, NDIM, HX_CART, SPEC><<<grid, block, 0, s>>>(p);
    return hipGetLastError();
}

template <typename R, int NV, int SPEC>
static hipError_t go_nv(const SweepParams& p, int ndim, int geom, hipStream_t s)
{
    switch (ndim) {
    case 1: return go<R, NV, 1, SPEC>(p, geom, s);
    case 2: return go<R, NV, 2, SPEC>(p, geom, s);
    default: return go<R, NV, 3, SPEC>(p, geom, s);
    }
}

template <typename R, int SPEC>
static hipError_t launch_sweep_t(const SweepParams& p, int ndim, int nvar, int geom, hipStream_t s)
{
    switch (nvar) {
    case 5: return go_nv<R, 5, SPEC>(p, ndim, geom, s);
    case 6: return go_nv<R, 6, SPEC>(p, ndim, geom, s);
    case 7: return go_nv<R, 7, SPEC>(p, ndim, geom, s);
    case 8: return go_nv<R, 8, SPEC>(p, ndim, geom, s);
    case 9: return go_nv<R, 9, SPEC>(p, ndim, geom, s);
    default: return hipErrorInvalidValue;
    }
}

// learned-limiter form: FP32, 5..7 fields
template <typename R>
static hipError_t launch_sweep_mlp_t(const SweepParams& p, int ndim, int nvar, int geom, hipStream_t s)
{
    switch (nvar) {
    case 5: return go_nv<R, 5, 2>(p, ndim, geom, s);
    case 6: return go_nv<R, 6, 2>(p, ndim, geom, s);
    case 7: return go_nv<R, 7, 2>(p, ndim, geom, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace hx
