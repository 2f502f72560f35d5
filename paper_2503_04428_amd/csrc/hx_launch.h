// Host-side launch interface between the C ABI and the kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "hx_params.h"

#define HX_MAX_NR 4096   // radial shells supported by the enclosed-mass kernel

namespace hx {

struct DtParams {
    const void* U;
    int n[3];
    int ng;
    int ndim;
    int geom;
    int nvar;
    long long plane;
    double gamma, gm1;
    Geo geo;
    double* partial;
    int* flag;
};

struct ShellParams {
    const void* U;       // density field (first variable of the state)
    int n[3];
    int ng;
    int ndim;
    Geo geo;
    double* partial;     // [nchunk][n0]
    double* gr;          // out: radial acceleration per shell
    double* menc;        // optional out: enclosed mass per shell
    double scale;        // 4 pi / Omega_w
    double G, Mc;
};

hipError_t launch_sweep_fp64_generic(const SweepParams& p, int ndim, int nvar, int geom, hipStream_t s);
hipError_t launch_sweep_fp64_hllc_vl(const SweepParams& p, int ndim, int nvar, int geom, hipStream_t s);
hipError_t launch_sweep_fp32_generic(const SweepParams& p, int ndim, int nvar, int geom, hipStream_t s);
hipError_t launch_sweep_fp32_hllc_vl(const SweepParams& p, int ndim, int nvar, int geom, hipStream_t s);
hipError_t launch_sweep_fp32_mlp(const SweepParams& p, int ndim, int nvar, int geom, hipStream_t s);
hipError_t launch_dt_final(const double* partial, int nb, double cfl, double* dt_out, hipStream_t s);
hipError_t launch_dt(const DtParams& p, bool fp32, int nblocks, double cfl, double* dt_out, hipStream_t s);
hipError_t launch_totals(const DtParams& p, bool fp32, int nblocks, double* out, hipStream_t s);
hipError_t launch_shell(const ShellParams& p, bool fp32, int nchunk, hipStream_t s);
hipError_t launch_convert(const void* src, void* dst, long long n, bool to_f32, hipStream_t s);

hipError_t launch_mlp_eval(const float* w, const float* x, long long n, float* phi, hipStream_t s);
hipError_t launch_mlp_features(const double* U, int nrows, int nf, int ratio, double gamma, float* x, float* a,
                               float* t, float* wt, hipStream_t s);
int mlp_grad_blocks(long long n);
hipError_t launch_mlp_grad(const float* w, const float* x, const float* a, const float* t, const float* wt,
                           long long n, float* grad, float* loss, float* part, hipStream_t s);
hipError_t launch_mlp_adam(float* w, const float* g, float* m, float* v, int step, float lr, float b1, float b2,
                           float eps, hipStream_t s);

// grid of the fused sweep for a given shape
inline dim3 sweep_grid(int ndim, const int n[3], int kz)
{
    if (ndim == 1)
        return dim3((n[0] + 61) / 62, n[1], 1);
    if (ndim == 2)
        return dim3((n[0] + 13) / 14, (n[1] + 13) / 14, 1);
    return dim3((n[0] + 13) / 14, (n[1] + 13) / 14, (n[2] + kz - 1) / kz);
}
inline dim3 sweep_block(int ndim) { return ndim == 1 ? dim3(64, 1, 1) : dim3(16, 16, 1); }

inline long long sweep_nblocks(int ndim, const int n[3], int kz)
{
    dim3 g = sweep_grid(ndim, n, kz);
    return (long long)g.x * g.y * g.z;
}

}  // namespace hx
