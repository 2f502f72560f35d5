// Grid shift along axis 0 (moving grid, Sect. 3.1.1): every face of axis 0 moves by delta and the
// state is carried over conservatively.  Each old cell holds the minmod-limited linear profile of
// its conserved variables about its volume centroid; a new cell takes the integral of the
// profiles over its overlap with the old cells (at most two, |delta| being at most the narrowest
// cell), with the measure dx (Cartesian) or r^2 dr (spherical; the angular factor is common to the
// row), over its new volume.  Beyond the grid the boundary images supply the state.  A cell whose
// result is not physical takes the piecewise-constant remap, a convex combination of old cells.
// One thread per new cell; FP64 arithmetic in the oracle's order (the FP32 form converts on load
// and store).  Built with -ffp-contract=off.
#include <hip/hip_runtime.h>

#include "hx_launch.h"

namespace hx {

namespace {

constexpr int SB = 256;
constexpr int SMAXV = 10;

__device__ __forceinline__ double m0_of(int sph, double a, double b)
{
    return sph ? (b * b * b - a * a * a) / 3.0 : b - a;
}

__device__ __forceinline__ double m1_of(int sph, double a, double b)
{
    return sph ? (b * b * b * b - a * a * a * a) / 4.0 : 0.5 * (b * b - a * a);
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

template <typename R>
__global__ void __launch_bounds__(SB) shift_kernel(const ShiftParams p)
{
    const long long ncell = p.plane;
    const long long c = (long long)blockIdx.x * SB + threadIdx.x;
    if (c >= ncell)
        return;
    const R* __restrict__ U = (const R*)p.U;
    R* __restrict__ Un = (R*)p.Unew;
    const int n = p.n0, nv = p.nvar;
    const int i = (int)(c % n);
    const long long row = c / n;  // (j, k) row: its cells are row * n + i
    const double* xf = p.xf + p.ng;  // xf[i]: face i of axis 0, ghost faces at negative indices
    const double a = xf[i] + p.delta, b = xf[i + 1] + p.delta;
    const double vnew = m0_of(p.sph, a, b);
    const int mfirst = p.delta > 0.0 ? i : i - 1;
    double lin[SMAXV], con[SMAXV];
#pragma unroll
    for (int v = 0; v < SMAXV; v++)
        lin[v] = con[v] = 0.0;
    for (int m = mfirst; m <= mfirst + 1; m++) {
        const double lo = fmax(a, xf[m]), hi = fmin(b, xf[m + 1]);
        if (!(hi > lo))
            continue;
        double cm[3];
        int src[3];
        bool fl[3];
#pragma unroll
        for (int s = 0; s < 3; s++) {
            const double fa = xf[m - 1 + s], fb = xf[m + s];
            cm[s] = m1_of(p.sph, fa, fb) / m0_of(p.sph, fa, fb);
            src[s] = image0(m - 1 + s, n, p.bc0[0], p.bc0[1], fl[s]);
        }
        const double w0 = m0_of(p.sph, lo, hi), w1 = m1_of(p.sph, lo, hi);
#pragma unroll
        for (int v = 0; v < SMAXV; v++) {
            if (v < nv) {
                double q[3];
#pragma unroll
                for (int s = 0; s < 3; s++) {
                    q[s] = (double)U[(long long)v * ncell + row * n + src[s]];
                    if (v == 1 && fl[s])
                        q[s] = -q[s];
                }
                const double sl = minmod_d((q[1] - q[0]) / (cm[1] - cm[0]), (q[2] - q[1]) / (cm[2] - cm[1]));
                lin[v] += q[1] * w0 + sl * (w1 - cm[1] * w0);
                con[v] += q[1] * w0;
            }
        }
    }
    const double m2 = lin[1] * lin[1] + lin[2] * lin[2] + lin[3] * lin[3];
    double elast = 0.0;
#pragma unroll
    for (int v = 0; v < SMAXV; v++)
        if (v == nv - 1)
            elast = lin[v];
    const bool ok = lin[0] > 0.0 && 2.0 * lin[0] * lin[4] - m2 > 0.0 && (!p.de || elast > 0.0);
#pragma unroll
    for (int v = 0; v < SMAXV; v++)
        if (v < nv)
            Un[(long long)v * ncell + c] = (R)((ok ? lin[v] : con[v]) / vnew);
}

}  // namespace

hipError_t launch_shift(const ShiftParams& p, bool fp32, hipStream_t s)
{
    const long long nb = (p.plane + SB - 1) / SB;
    if (fp32)
        shift_kernel<float><<<(unsigned)nb, SB, 0, s>>>(p);
    else
        shift_kernel<double><<<(unsigned)nb, SB, 0, s>>>(p);
    return hipGetLastError();
}

}  // namespace hx
