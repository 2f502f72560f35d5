// Persistent 1D run: a whole 1D Cartesian problem advanced to t_end inside one workgroup.
//
// A 1D problem of a thousand cells (the Sod tube of App. C.1) gives the fused sweep four
// workgroups of work per step, so a host-driven time loop is bound by launch latency (two launches
// per step: CFL maximum and sweep).  Here one workgroup keeps the conserved state in registers
// (FP32: 1024 threads x 2 cells; FP64: 512 x 4), the primitives and the exchanged face states in LDS,
// and runs the CFL step, the clip to t_end and the MUSCL-Hancock step (Sect. 3.2) in a device-side
// loop: no launch and no host synchronisation per step.  Every cell takes the operations of the
// fused sweep's 1D path in the same order (the same device functions), so in FP64 (built without
// contraction, hx_run1d_fp64.hip) the results equal a host loop of hx_compute_dt / hx_step bit for
// bit; the FP32 form (hx_run1d_fp32.hip, the FP32 sweep's flags) agrees with its host loop to FP32
// rounding, as the compiler may fuse FP32 products and sums differently in the two kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "hx_run1d.h"
#include "hx_sweep.h"

namespace hx {

// threads of the workgroup and cells per thread: FP32 1024 x 2 (four waves per SIMD), FP64 512 x 4
// (two waves per SIMD: the FP64 Riemann solve needs more than the 128 registers of four)
template <typename R>
struct Run1dShape {
    static constexpr int threads = sizeof(R) == 8 ? 512 : 1024;
    static constexpr int cpt = sizeof(R) == 8 ? 4 : 2;
};

// LDS: primitives W[v][c + 2] of cells c = -2 .. n+1 (then, in the same storage, the flux of face
// f at f + 2), and the -x and +x half-step states of the predictor cells c = -1 .. n: 3 NV (n + 4)
// values.  The conserved state stays in registers.
template <typename R, int NV>
__global__ void __launch_bounds__(Run1dShape<R>::threads) run1d_kernel(const Run1dParams p)
{
    constexpr int R1_THREADS = Run1dShape<R>::threads;
    constexpr int R1_CPT = Run1dShape<R>::cpt;
    extern __shared__ __align__(16) unsigned char smem[];
    R* sW = reinterpret_cast<R*>(smem);           // [NV][n + 4]: primitives, then face fluxes
    R* sQp = sW + (size_t)NV * (p.n + 4);         // [NV][n + 4]: +x half-step states
    R* sQm = sQp + (size_t)NV * (p.n + 4);        // [NV][n + 4]: -x half-step states
    __shared__ double sRed[R1_THREADS / 64];
    __shared__ double sDt;
    __shared__ int sStop;

    using N = Num<R>;
    const int n = p.n, ng = p.ng, tid = threadIdx.x;
    const int ld = n + 4;
    R* const Ug = (R*)p.U;
    Gas<R> gas;
    gas.gamma = N::from_d(p.gamma);
    gas.gm1 = N::from_d(p.gamma - 1.0);
    gas.inv_gm1 = N::from_d(1.0 / (p.gamma - 1.0));
    const int lim = p.limiter, solver = p.riemann;

    // interior cells i = tid + T m; predictor cells c = tid - 1 + T m (c = -1 .. n), T threads
    R U[R1_CPT][NV];
#pragma unroll
    for (int m = 0; m < R1_CPT; m++) {
        const int i = tid + R1_THREADS * m;
#pragma unroll
        for (int v = 0; v < NV; v++)
            U[m][v] = i < n ? Ug[(long long)v * p.plane + i] : R(0);
    }
    double t = p.t0;
    int steps = 0;
    bool bad_state = false;

    // the CFL rate of the state held by this thread (the sweep's rate of a stored cell)
    auto rate = [&]() {
        double s = 0.0;
#pragma unroll
        for (int m = 0; m < R1_CPT; m++) {
            const int i = tid + R1_THREADS * m;
            if (i < n) {
                const double wx = p.geo.w[0][i + ng];
                double sr;
                if constexpr (sizeof(R) == 4) {
                    const float rw[3] = {(float)(1.0 / wx), 0.0f, 0.0f};
                    sr = cfl_rate_f32<NV, 1>(U[m], gas, rw);
                } else {
                    const double wd[3] = {wx, 0.0, 0.0};
                    sr = cfl_rate<R, NV, 1>(U[m], p.gamma, wd, gas);
                }
                if (sr < 0.0)
                    bad_state = true;
                s = fmax(s, sr);
            }
        }
        return s;
    };
    // time step of the held states: cfl / max rate (FP64), clipped to t_end; sets sStop
    auto next_dt = [&](double s) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1)
            s = fmax(s, __shfl_xor(s, o, 64));
        if ((tid & 63) == 0)
            sRed[tid >> 6] = s;
        __syncthreads();
        if (tid == 0) {
            double m = sRed[0];
            for (int w = 1; w < R1_THREADS / 64; w++)
                m = fmax(m, sRed[w]);
            double dt = p.cfl / m;
            dt = fmin(dt, p.t_end - t);
            sDt = dt;
            sStop = (t < p.t_end * (1.0 - 1e-14) && steps < p.max_steps) ? 0 : 1;
        }
        __syncthreads();
    };

    next_dt(rate());
    while (!sStop) {
        const double dtd = sDt;
        // primitives of the interior cells, then of the ghost cells (images with the normal
        // momentum flipped behind a reflective end)
#pragma unroll
        for (int m = 0; m < R1_CPT; m++) {
            const int i = tid + R1_THREADS * m;
            if (i < n) {
                R w[NV];
                to_prim<R, NV>(gas, U[m], w);
#pragma unroll
                for (int v = 0; v < NV; v++)
                    sW[v * ld + i + 2] = w[v];
            }
        }
        __syncthreads();
        if (tid < 4) {
            const int c = tid < 2 ? tid - 2 : n + tid - 2;  // -2, -1, n, n+1
            bool fl;
            const int im = bc_image(c, n, ng, p.bc0[0], p.bc0[1], fl);
#pragma unroll
            for (int v = 0; v < NV; v++) {
                const R x = sW[v * ld + im + 2];
                sW[v * ld + c + 2] = (v == 1 && fl) ? -x : x;
            }
        }
        __syncthreads();
        // Hancock half step of the predictor cells c = -1 .. n; both half-step states go to LDS
        // (one cell at a time: nothing of it stays in registers)
#pragma unroll 1
        for (int m = 0; m < R1_CPT; m++) {
            const int c = tid - 1 + R1_THREADS * m;
            if (c > n)
                continue;
            // (the tables hold every cell's own slope factors and its image's width)
            const int gx = c + ng;
            const R cmx = N::from_d(p.geo.cm[0][gx]), cpx = N::from_d(p.geo.cp[0][gx]);
            const R lamx = N::from_d(div_rn(dtd, 2.0 * p.geo.w[0][gx]));
            R w[NV], dl[NV], a[NV], b[NV];
#pragma unroll
            for (int v = 0; v < NV; v++) {
                const R w1 = sW[v * ld + c + 1], w2 = sW[v * ld + c + 2], w3 = sW[v * ld + c + 3];
                w[v] = w2;
                a[v] = cmx * (w2 - w1);
                b[v] = cpx * (w3 - w2);
            }
#pragma unroll
            for (int v = 0; v < NV; v++)
                dl[v] = limit<R>(lim, a[v], b[v]);
            R wm[NV], wp[NV], um[NV], up[NV], fm[NV], fp[NV], du[NV];
#pragma unroll
            for (int v = 0; v < NV; v++) {
                wm[v] = w[v] - dl[v];
                wp[v] = w[v] + dl[v];
            }
            to_cons<R, NV>(gas, wm, um);
            to_cons<R, NV>(gas, wp, up);
            phys_flux<R, NV, 0>(wm, um, fm);
            phys_flux<R, NV, 0>(wp, up, fp);
#pragma unroll
            for (int v = 0; v < NV; v++)
                du[v] = R(0) + lamx * (fm[v] - fp[v]);
            // positivity of both half-step face states; otherwise first order for this cell
            R qs[2][NV];
            bool bad = false;
#pragma unroll
            for (int side = 0; side < 2; side++) {
                R ws[NV];
#pragma unroll
                for (int v = 0; v < NV; v++)
                    ws[v] = side ? w[v] + dl[v] : w[v] - dl[v];
                to_cons<R, NV>(gas, ws, qs[side]);
#pragma unroll
                for (int v = 0; v < NV; v++)
                    qs[side][v] += du[v];
                bad = bad || !positive_state<R>(qs[side]);
            }
            if (bad) {
#pragma unroll
                for (int side = 0; side < 2; side++) {
                    R ws[NV];
#pragma unroll
                    for (int v = 0; v < NV; v++)
                        ws[v] = side ? w[v] + R(0) : w[v] - R(0);
                    to_cons<R, NV>(gas, ws, qs[side]);
                }
            }
#pragma unroll
            for (int v = 0; v < NV; v++) {
                sQm[v * ld + c + 2] = qs[0][v];
                sQp[v * ld + c + 2] = qs[1][v];
            }
        }
        __syncthreads();
        // flux through the lower face of the cells c = 0 .. n (face c), from the +x state of cell
        // c-1 and the -x state of cell c; the fluxes replace the primitives in LDS (last read
        // before the barrier above)
#pragma unroll 1
        for (int m = 0; m < R1_CPT; m++) {
            const int c = tid - 1 + R1_THREADS * m;
            if (c < 0 || c > n)
                continue;
            R L[NV], Rr[NV];
#pragma unroll
            for (int v = 0; v < NV; v++) {
                L[v] = sQp[v * ld + c + 1];
                Rr[v] = sQm[v * ld + c + 2];
            }
            R F[NV];
            riemann<R, NV, 0>(solver, gas, L, Rr, F);
#pragma unroll
            for (int v = 0; v < NV; v++)
                sW[v * ld + c + 2] = F[v];
        }
        __syncthreads();
        // update of the interior cells: U + dt/dx (F_lower - F_upper), then the CFL rate of the new
        // state (the time step of the next step)
#pragma unroll
        for (int m = 0; m < R1_CPT; m++) {
            const int i = tid + R1_THREADS * m;
            if (i < n) {
                const R mu = N::from_d(div_rn(dtd, p.geo.w[0][i + ng]));
#pragma unroll
                for (int v = 0; v < NV; v++)
                    U[m][v] += mu * (sW[v * ld + i + 2] - sW[v * ld + i + 3]);
            }
        }
        t += dtd;
        steps++;
        next_dt(rate());
    }
#pragma unroll
    for (int m = 0; m < R1_CPT; m++) {
        const int i = tid + R1_THREADS * m;
        if (i < n)
#pragma unroll
            for (int v = 0; v < NV; v++)
                Ug[(long long)v * p.plane + i] = U[m][v];
    }
    if (bad_state)
        p.flag[0] = 1;
    if (tid == 0) {
        p.out[0] = t;
        p.out[1] = (double)steps;
    }
}

// launch of the R instantiations (one workgroup, dynamic LDS for the field arrays)
template <typename R>
hipError_t run1d_launch(const Run1dParams& p, int nvar, hipStream_t s)
{
    const size_t lds = run1d_lds_bytes(p.n, nvar, sizeof(R) == 4);
    auto go = [&](auto kern) -> hipError_t {
        hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess)
            return e;
        hipLaunchKernelGGL(kern, dim3(1), dim3(Run1dShape<R>::threads), lds, s, p);
        return hipGetLastError();
    };
    switch (nvar) {
    case 5: return go(run1d_kernel<R, 5>);
    case 6: return go(run1d_kernel<R, 6>);
    case 7: return go(run1d_kernel<R, 7>);
    case 8: return go(run1d_kernel<R, 8>);
    case 9: return go(run1d_kernel<R, 9>);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace hx
