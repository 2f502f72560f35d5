// Reductions of the step: CFL time step, conserved totals, enclosed-mass gravity; and the
// FP32 <-> FP64 state conversions of the FP32 form.
#include <hip/hip_runtime.h>

#include "hx_device.h"
#include "hx_launch.h"

namespace hx {

constexpr int RB = 256;  // threads per reduction block

__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        v += __shfl_xor(v, o, 64);
    return v;
}

// CFL signal rate of every interior cell, sum_d (|u_d| + c_s) / dx_d, maximised per block.
// FP64 throughout (the FP32 form converts its state on load), in the oracle's operation order;
// P and c_s from the ideal-gas or the gas + radiation EoS (Sect. 2.3).
template <typename R>
__global__ void __launch_bounds__(RB) dt_partial_kernel(const DtParams p)
{
    __shared__ double red[RB / 64];
    const R* __restrict__ U = (const R*)p.U;
    const long long ncell = p.plane;
    double smax = 0.0;
    int bad = 0;
    for (long long c = (long long)blockIdx.x * RB + threadIdx.x; c < ncell; c += (long long)gridDim.x * RB) {
        const int i = (int)(c % p.n[0]);
        const long long r = c / p.n[0];
        const int j = (int)(r % p.n[1]);
        const int k = (int)(r / p.n[1]);
        if constexpr (sizeof(R) == 4) {
            // the FP32 form's rate, as the sweep forms it when it stores a cell
            if (p.eos == 0) {
                float qf[5];
                bool fin = true;
#pragma unroll
                for (int v = 0; v < 5; v++)
                    qf[v] = (float)U[(long long)v * ncell + c];
                for (int v = 5; v < p.nvar; v++)
                    fin = fin && isfinite((double)U[(long long)v * ncell + c]);
                Gas<float> g;
                g.gamma = (float)p.gamma;
                g.gm1 = (float)p.gm1;
                g.inv_gm1 = (float)(1.0 / p.gm1);
                float rw[3] = {0.0f, 0.0f, 0.0f};
                for (int d = 0; d < p.ndim; d++) {
                    double w;
                    if (p.geom == HX_CART) {
                        const int id = d == 0 ? i : (d == 1 ? j : k);
                        w = p.geo.w[d][id + p.ng];
                    } else if (d == 0) {
                        w = p.geo.w[0][i + p.ng];
                    } else if (d == 1) {
                        w = p.geo.rabs[i + p.ng] * p.geo.w[1][j + p.ng];
                    } else {
                        w = p.geo.rabs[i + p.ng] * p.geo.sabs[j + p.ng] * p.geo.w[2][k + p.ng];
                    }
                    rw[d] = (float)(1.0 / w);
                }
                const double s = cfl_rate_f32<5, 3>(qf, g, rw);
                if (!fin || s < 0.0) {
                    bad = 1;
                    continue;
                }
                smax = fmax(smax, s);
                continue;
            }
        }
        double q[5];
#pragma unroll
        for (int v = 0; v < 5; v++)
            q[v] = (double)U[(long long)v * ncell + c];
        bool fin = isfinite(q[0]) && isfinite(q[1]) && isfinite(q[2]) && isfinite(q[3]) && isfinite(q[4]);
        for (int v = 5; v < p.nvar; v++)
            fin = fin && isfinite((double)U[(long long)v * ncell + c]);
        double rho = q[0];
        double inv = 1.0 / rho;
        double u1 = q[1] * inv, u2 = q[2] * inv, u3 = q[3] * inv;
        double ke = 0.5 * (q[1] * u1 + q[2] * u2 + q[3] * u3);
        double pr, cs;
        if (p.eos == 1) {
            Gas<double> g;
            g.gamma = p.gamma;
            g.gm1 = p.gm1;
            g.inv_gm1 = 1.0 / p.gm1;
            g.Rg = p.eos_R;
            g.arad = p.eos_arad;
            const double T = temp_from_e(g, rho, q[4] - ke);
            pr = (rho * g.Rg) * T + (g.arad * t4(T)) / 3.0;
            if (!fin || !(rho > 0.0) || !(pr > 0.0)) {
                bad = 1;
                continue;
            }
            const double w[5] = {rho, u1, u2, u3, pr};
            cs = sound_speed<double, 1>(g, w, inv, T);
        } else {
            pr = p.gm1 * (q[4] - ke);
            if (!fin || !(rho > 0.0) || !(pr > 0.0)) {
                bad = 1;
                continue;
            }
            cs = sqrt(p.gamma * pr * inv);
        }
        double u[3] = {u1, u2, u3};
        double s = 0.0;
        for (int d = 0; d < p.ndim; d++) {
            double w;
            if (p.geom == HX_CART) {
                const int id = d == 0 ? i : (d == 1 ? j : k);
                w = p.geo.w[d][id + p.ng];
            } else if (d == 0) {
                w = p.geo.w[0][i + p.ng];
            } else if (d == 1) {
                w = p.geo.rabs[i + p.ng] * p.geo.w[1][j + p.ng];
            } else {
                w = p.geo.rabs[i + p.ng] * p.geo.sabs[j + p.ng] * p.geo.w[2][k + p.ng];
            }
            s += (fabs(u[d]) + cs) / w;
        }
        smax = fmax(smax, s);
    }
    if (bad)
        p.flag[0] = 1;
    smax = wave_max(smax);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0)
        red[wid] = smax;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = red[0];
        for (int w = 1; w < RB / 64; w++)
            m = fmax(m, red[w]);
        p.partial[blockIdx.x] = m;
    }
}

__global__ void __launch_bounds__(RB) dt_final_kernel(const double* __restrict__ partial, int nb, double cfl,
                                                        double* __restrict__ dt_out)
{
    __shared__ double red[RB / 64];
    double m = 0.0;
    for (int b = threadIdx.x; b < nb; b += RB)
        m = fmax(m, partial[b]);
    m = wave_max(m);
    if ((threadIdx.x & 63) == 0)
        red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        double mm = red[0];
        for (int w = 1; w < RB / 64; w++)
            mm = fmax(mm, red[w]);
        dt_out[0] = cfl / mm;
    }
}

// sum_cells U_v dV per variable, FP64, per-block partials then a final fixed-order pass
template <typename R>
__global__ void __launch_bounds__(RB) totals_partial_kernel(const DtParams p)
{
    __shared__ double red[RB / 64];
    const R* __restrict__ U = (const R*)p.U;
    const long long ncell = p.plane;
    for (int v = 0; v < p.nvar; v++) {
        double s = 0.0;
        for (long long c = (long long)blockIdx.x * RB + threadIdx.x; c < ncell; c += (long long)gridDim.x * RB) {
            const int i = (int)(c % p.n[0]);
            const long long r = c / p.n[0];
            const int j = (int)(r % p.n[1]);
            const int k = (int)(r / p.n[1]);
            double dV;
            if (p.geom == HX_CART)
                dV = p.geo.w[0][i + p.ng] * p.geo.w[1][p.ndim > 1 ? j + p.ng : 0] *
                     p.geo.w[2][p.ndim > 2 ? k + p.ng : 0];
            else
                dV = p.geo.vr[i] * p.geo.ct[j] * p.geo.w[2][k + (p.ndim > 2 ? p.ng : 0)];
            s += (double)U[(long long)v * ncell + c] * dV;
        }
        s = wave_sum(s);
        if ((threadIdx.x & 63) == 0)
            red[threadIdx.x >> 6] = s;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = red[0];
            for (int w = 1; w < RB / 64; w++)
                t += red[w];
            p.partial[(long long)v * gridDim.x + blockIdx.x] = t;
        }
        __syncthreads();
    }
}

__global__ void __launch_bounds__(RB) totals_final_kernel(const double* __restrict__ partial, int nb, int nvar,
                                                            double* __restrict__ out)
{
    __shared__ double red[RB / 64];
    for (int v = 0; v < nvar; v++) {
        double s = 0.0;
        for (int b = threadIdx.x; b < nb; b += RB)
            s += partial[(long long)v * nb + b];
        s = wave_sum(s);
        if ((threadIdx.x & 63) == 0)
            red[threadIdx.x >> 6] = s;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = red[0];
            for (int w = 1; w < RB / 64; w++)
                t += red[w];
            out[v] = t;
        }
        __syncthreads();
    }
}

// Shell masses m_i = sum_{j,k} rho dV for a chunk of (j,k) rows; thread = radial index (coalesced)
template <typename R>
__global__ void __launch_bounds__(RB) shell_partial_kernel(const ShellParams p)
{
    const int i = blockIdx.x * RB + threadIdx.x;
    if (i >= p.n[0])
        return;
    const R* __restrict__ rho = (const R*)p.U;
    const long long rows = (long long)p.n[1] * p.n[2];
    const long long r0 = rows * blockIdx.y / gridDim.y;
    const long long r1 = rows * (blockIdx.y + 1) / gridDim.y;
    double s = 0.0;
    const double vr = p.geo.vr[i];
    const int n1 = p.n[1], kofs = p.ndim > 2 ? p.ng : 0;
    int j = (int)(r0 % n1), k = (int)(r0 / n1);  // row r = k n1 + j, advanced incrementally
    long long r = r0;
    // rows in batches of eight: their loads are issued together, the sum stays in row order
    constexpr int B = 8;
    for (; r + B <= r1; r += B) {
        double x[B], dv[B];
#pragma unroll
        for (int b = 0; b < B; b++) {
            dv[b] = vr * p.geo.ct[j] * p.geo.w[2][k + kofs];
            x[b] = (double)rho[(r + b) * p.n[0] + i];
            if (++j == n1) {
                j = 0;
                k++;
            }
        }
#pragma unroll
        for (int b = 0; b < B; b++)
            s += x[b] * dv[b];
    }
    for (; r < r1; r++) {
        const double dV = vr * p.geo.ct[j] * p.geo.w[2][k + kofs];
        s += (double)rho[r * p.n[0] + i] * dV;
        if (++j == n1) {
            j = 0;
            k++;
        }
    }
    p.partial[(long long)blockIdx.y * p.n[0] + i] = s;
}

// enclosed mass M(r_i) = (4 pi / Omega_w)(sum_{i'<i} m_i' + m_i / 2) and g_r = -G (Mc + M) / r_c^2
__global__ void __launch_bounds__(RB) shell_final_kernel(const ShellParams p, int nchunk)
{
    __shared__ double m[HX_MAX_NR];
    for (int i = threadIdx.x; i < p.n[0]; i += RB) {
        double s = 0.0;
#pragma unroll 8
        for (int c = 0; c < nchunk; c++)
            s += p.partial[(long long)c * p.n[0] + i];
        m[i] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        // the running sum in shell order; the shells go through registers eight at a time, so the
        // LDS loads of a batch overlap instead of each waiting behind the previous shell's store
        constexpr int B = 8;
        double below = 0.0;
        int i = 0;
        for (; i + B <= p.n[0]; i += B) {
            double v[B];
#pragma unroll
            for (int j = 0; j < B; j++)
                v[j] = m[i + j];
#pragma unroll
            for (int j = 0; j < B; j++) {
                m[i + j] = p.scale * (below + 0.5 * v[j]);
                below += v[j];
            }
        }
        for (; i < p.n[0]; i++) {
            const double mi = m[i];
            m[i] = p.scale * (below + 0.5 * mi);
            below += mi;
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < p.n[0]; i += RB) {
        const double rc = 0.5 * (p.geo.rf[i] + p.geo.rf[i + 1]);
        p.gr[i] = -(p.G * (p.Mc + m[i])) / (rc * rc);
        if (p.menc)
            p.menc[i] = m[i];
    }
}

__global__ void f64_to_f32_kernel(const double* __restrict__ a, float* __restrict__ b, long long n)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        b[i] = (float)a[i];
}

__global__ void f32_to_f64_kernel(const float* __restrict__ a, double* __restrict__ b, long long n)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        b[i] = (double)a[i];
}

// ---------------------------------------------------------------------------- launchers

hipError_t launch_dt(const DtParams& p, bool fp32, int nblocks, double cfl, double* dt_out, hipStream_t s)
{
    if (fp32)
        dt_partial_kernel<float><<<nblocks, RB, 0, s>>>(p);
    else
        dt_partial_kernel<double><<<nblocks, RB, 0, s>>>(p);
    dt_final_kernel<<<1, RB, 0, s>>>(p.partial, nblocks, cfl, dt_out);
    return hipGetLastError();
}

hipError_t launch_dt_final(const double* partial, int nb, double cfl, double* dt_out, hipStream_t s)
{
    dt_final_kernel<<<1, RB, 0, s>>>(partial, nb, cfl, dt_out);
    return hipGetLastError();
}

hipError_t launch_totals(const DtParams& p, bool fp32, int nblocks, double* out, hipStream_t s)
{
    if (fp32)
        totals_partial_kernel<float><<<nblocks, RB, 0, s>>>(p);
    else
        totals_partial_kernel<double><<<nblocks, RB, 0, s>>>(p);
    totals_final_kernel<<<1, RB, 0, s>>>(p.partial, nblocks, p.nvar, out);
    return hipGetLastError();
}

hipError_t launch_shell(const ShellParams& p, bool fp32, int nchunk, hipStream_t s)
{
    dim3 grid((p.n[0] + RB - 1) / RB, nchunk);
    if (fp32)
        shell_partial_kernel<float><<<grid, RB, 0, s>>>(p);
    else
        shell_partial_kernel<double><<<grid, RB, 0, s>>>(p);
    shell_final_kernel<<<1, RB, 0, s>>>(p, nchunk);
    return hipGetLastError();
}

hipError_t launch_convert(const void* src, void* dst, long long n, bool to_f32, hipStream_t s)
{
    const int nb = (int)((n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096);
    if (to_f32)
        f64_to_f32_kernel<<<nb, 256, 0, s>>>((const double*)src, (float*)dst, n);
    else
        f32_to_f64_kernel<<<nb, 256, 0, s>>>((const float*)src, (double*)dst, n);
    return hipGetLastError();
}

}  // namespace hx
