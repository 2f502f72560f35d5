// Grid shift along axis 0 (moving grid, Sect. 3.1.1): every face of axis 0 moves by delta and the
// state is carried over conservatively.  Each old cell holds the minmod-limited linear profile of
// its conserved variables about its volume centroid; a new cell takes the integral of the
// profiles over its overlap with the old cells (at most two, |delta| being at most the narrowest
// cell), with the measure dx (Cartesian) or r^2 dr (spherical; the angular factor is common to the
// row), over its new volume.  Beyond the grid the boundary images supply the state.  A cell whose
// result is not physical takes the piecewise-constant remap, a convex combination of old cells.
// One thread per new cell; FP64 arithmetic (the FP32 form converts on load and store), built with
// -ffp-contract=off.  Spherical measures are taken without their common factor 1/3 (b^3 - a^3 and
// (3/4)(b^4 - a^4)), which cancels in content / volume and in the centroids; the slopes and the
// final average multiply by reciprocals formed once per cell (the centroid spacings are common to
// every field), so a cell costs 8 FP64 divisions.
#include <hip/hip_runtime.h>

#include "hx_launch.h"

namespace hx {

namespace {

constexpr int SB = 256;

// measure of [a, b] up to a factor common to the grid (only ratios of measures enter the remap):
// b - a (Cartesian), b^3 - a^3 = 3 x the integral of r^2 dr (spherical)
__device__ __forceinline__ double m0_of(int sph, double a, double b)
{
    return sph ? b * b * b - a * a * a : b - a;
}

// first moment of [a, b] in the same scale as m0_of
__device__ __forceinline__ double m1_of(int sph, double a, double b)
{
    return sph ? 0.75 * (b * b * b * b - a * a * a * a) : 0.5 * (b * b - a * a);
}

__device__ __forceinline__ double minmod_d(double a, double b)
{
    if (a * b <= 0.0)
        return 0.0;
    return fabs(a) < fabs(b) ? a : b;
}

// image of index i on axis 0 (periodic, null gradient, reflective with the normal momentum negated)
__device__ __forceinline__ int image0(int i, int n, int lo, int hi, bool& flip)
{
    flip = false;
    if (i < 0) {
        if (lo == HX_BC_PERIODIC)
            return i + n;
        if (lo == HX_BC_TRANSMISSIVE)
            return 0;
        flip = true;
        return -1 - i;
    }
    if (i >= n) {
        if (hi == HX_BC_PERIODIC)
            return i - n;
        if (hi == HX_BC_TRANSMISSIVE)
            return n - 1;
        flip = true;
        return 2 * n - 1 - i;
    }
    return i;
}

// The grid holds bpr = ceil(n0 / SB) workgroups per (j, k) row of axis 0, so a thread's row and
// index follow from one wave-uniform division of the workgroup index (no per-thread 64-bit modulo).
template <typename R, int NV>
__global__ void __launch_bounds__(SB) shift_kernel(const ShiftParams p, unsigned bpr)
{
    const long long ncell = p.plane;
    const unsigned row = blockIdx.x / bpr;
    const int i = (int)((blockIdx.x - row * bpr) * SB + threadIdx.x);
    const int n = p.n0;
    if (i >= n)
        return;
    const long long rowoff = (long long)row * n;  // first cell of this (j, k) row
    const long long c = rowoff + i;
    const R* __restrict__ U = (const R*)p.U;
    R* __restrict__ Un = (R*)p.Unew;
    const double* xf = p.xf + p.ng;  // xf[i]: face i of axis 0, ghost faces at negative indices
    const double a = xf[i] + p.delta, b = xf[i + 1] + p.delta;
    const double vnew = m0_of(p.sph, a, b);
    // the two old cells under the new one are m0 and m0 + 1; their slope stencils span m0 - 1 .. m0 + 2
    const int m0 = p.delta > 0.0 ? i : i - 1;
    long long src[4];
    double sgn[4];  // -1 for the normal momentum of a reflected image
#pragma unroll
    for (int s = 0; s < 4; s++) {
        bool fl;
        src[s] = rowoff + image0(m0 - 1 + s, n, p.bc0[0], p.bc0[1], fl);
        sgn[s] = fl ? -1.0 : 1.0;
    }
    double q[4][NV], cm[4];
#pragma unroll
    for (int v = 0; v < NV; v++)
#pragma unroll
        for (int s = 0; s < 4; s++)
            q[s][v] = (double)U[(long long)v * ncell + src[s]];
#pragma unroll
    for (int s = 0; s < 4; s++)
        q[s][1] = sgn[s] * q[s][1];
#pragma unroll
    for (int s = 0; s < 4; s++) {
        const double fa = xf[m0 - 1 + s], fb = xf[m0 + s];
        cm[s] = m1_of(p.sph, fa, fb) / m0_of(p.sph, fa, fb);
    }
    // overlaps of the new cell with the old cells m0 and m0 + 1 (an empty one adds zeros: the same
    // sums as skipping it, since the sums start at +0)
    double w0[2], w1[2];
#pragma unroll
    for (int j = 0; j < 2; j++) {
        const double lo = fmax(a, xf[m0 + j]), hi = fmin(b, xf[m0 + j + 1]);
        const bool has = hi > lo;
        w0[j] = has ? m0_of(p.sph, lo, hi) : 0.0;
        w1[j] = has ? m1_of(p.sph, lo, hi) : 0.0;
    }
    // reciprocal centroid spacings of the slope stencils, common to every field
    double idc[3];
#pragma unroll
    for (int s = 0; s < 3; s++)
        idc[s] = 1.0 / (cm[s + 1] - cm[s]);
    // content of field v under the new cell: with the linear profiles, and with constant ones
    auto content = [&](int v, double& lin, double& con) {
        lin = 0.0;
        con = 0.0;
#pragma unroll
        for (int j = 0; j < 2; j++) {
            const double sl = minmod_d((q[j + 1][v] - q[j][v]) * idc[j],
                                       (q[j + 2][v] - q[j + 1][v]) * idc[j + 1]);
            lin += q[j + 1][v] * w0[j] + sl * (w1[j] - cm[j + 1] * w0[j]);
            con += q[j + 1][v] * w0[j];
        }
    };
    // physical check on the linear result (rho, E, momenta and the monitored e)
    double h[5], c5;
#pragma unroll
    for (int v = 0; v < 5; v++)
        content(v, h[v], c5);
    double el = 1.0;
    if (p.de)
        content(NV - 1, el, c5);
    const double m2 = h[1] * h[1] + h[2] * h[2] + h[3] * h[3];
    const bool ok = h[0] > 0.0 && 2.0 * h[0] * h[4] - m2 > 0.0 && el > 0.0;
    const double ivnew = 1.0 / vnew;
#pragma unroll
    for (int v = 0; v < NV; v++) {
        double lin, con;
        content(v, lin, con);
        Un[(long long)v * ncell + c] = (R)((ok ? lin : con) * ivnew);
    }
}

template <typename R>
hipError_t go_shift(const ShiftParams& p, hipStream_t s)
{
    if (p.n0 < 1 || p.plane % p.n0 != 0)
        return hipErrorInvalidValue;
    const unsigned bpr = (unsigned)((p.n0 + SB - 1) / SB);
    const long long rows = p.plane / p.n0;
    if (rows * bpr > 0x7fffffffLL)
        return hipErrorInvalidValue;
    const unsigned nb = (unsigned)(rows * bpr);
    switch (p.nvar) {
    case 5: shift_kernel<R, 5><<<nb, SB, 0, s>>>(p, bpr); break;
    case 6: shift_kernel<R, 6><<<nb, SB, 0, s>>>(p, bpr); break;
    case 7: shift_kernel<R, 7><<<nb, SB, 0, s>>>(p, bpr); break;
    case 8: shift_kernel<R, 8><<<nb, SB, 0, s>>>(p, bpr); break;
    case 9: shift_kernel<R, 9><<<nb, SB, 0, s>>>(p, bpr); break;
    case 10: shift_kernel<R, 10><<<nb, SB, 0, s>>>(p, bpr); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_shift(const ShiftParams& p, bool fp32, hipStream_t s)
{
    return fp32 ? go_shift<float>(p, s) : go_shift<double>(p, s);
}

}  // namespace hx
