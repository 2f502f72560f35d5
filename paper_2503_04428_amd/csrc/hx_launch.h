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
    int eos;             // 0 ideal gas, 1 gas + radiation (constants eos_R, eos_arad)
    double eos_R, eos_arad;
    Geo geo;
    double* partial;
    int* flag;
};

struct ShiftParams {
    const void* U;       // state on the old faces
    void* Unew;          // state on the faces moved by delta
    int n0, ng;
    long long plane;     // cells per field
    int nvar;
    int sph;             // 1: measure r^2 dr (spherical), 0: dx
    int de;              // 1: the last field is the monitored internal energy
    int bc0[2];          // boundary kinds of axis 0
    const double* xf;    // the n0 + 1 + 2 ng old faces of axis 0, ghost faces included
    double delta;
};

hipError_t launch_shift(const ShiftParams& p, bool fp32, hipStream_t s);

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

// Fused sweep launchers.  With occ != nullptr nothing is launched: *occ receives how many
// workgroups of the instantiation that would run fit on one compute unit.
hipError_t launch_sweep_fp64_generic(const SweepParams& p, int ndim, int nvar, int geom, hipStream_t s, int* occ);
hipError_t launch_sweep_fp64_hllc_vl(const SweepParams& p, int ndim, int nvar, int geom, hipStream_t s, int* occ);
hipError_t launch_sweep_fp32_generic(const SweepParams& p, int ndim, int nvar, int geom, hipStream_t s, int* occ);
hipError_t launch_sweep_fp32_hllc_vl(const SweepParams& p, int ndim, int nvar, int geom, hipStream_t s, int* occ);
hipError_t launch_sweep_fp32_mlp(const SweepParams& p, int ndim, int nvar, int geom, hipStream_t s, int* occ);
hipError_t launch_sweep_fp64_de(const SweepParams& p, int ndim, int nvar, int geom, hipStream_t s, int* occ);
hipError_t launch_sweep_fp64_rad(const SweepParams& p, int ndim, int nvar, int geom, hipStream_t s, int* occ);
hipError_t launch_sweep_fp64_de_rad(const SweepParams& p, int ndim, int nvar, int geom, hipStream_t s, int* occ);
// 3D one-wave-per-SIMD instantiations of variants 1 (6-9 fields) and 4 (5-9 fields), scheduled for ILP
hipError_t launch_sweep_fp64_3d_ilp(const SweepParams& p, int spec, int nvar, int geom, hipStream_t s, int* occ);
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
// the same with the block partials in the library's static per-device scratch (no allocation)
hipError_t launch_mlp_grad_noalloc(const float* w, const float* x, const float* a, const float* t, const float* wt,
                                   long long n, float* grad, float* loss, hipStream_t s);
size_t mlp_grad_scratch_bytes();
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

// z planes per workgroup of a 3D sweep.  A workgroup marches kz + 2 predictor planes (plus about
// one plane's worth of start-up loads), and the ceil(tiles * ceil(n2 / kz) / slots) dispatch
// rounds of a launch, slots = resident workgroups of the whole chip, run one after the other, so
// the launch costs about rounds * (kz + 3) plane steps.  Tiles differ in cost (the learned
// limiter's network runs where the flow is monotone, divisions are skipped where it is flat), so
// at least min_rounds rounds are kept for the hardware's dynamic dispatch to even them out: 4, and
// 8 for the learned form, whose tiles differ most (quadrants 256^3: kz 16 in 8 rounds 1.42 ms, kz
// 32 in 4 rounds 1.48 ms; the FP32 van Leer sweep takes 0.72 ms with either).  The kz that
// minimises the cost under that constraint (the larger on a tie) is taken.
inline int choose_zchunk(int n2, long long tiles, long long slots, long long min_rounds = 4)
{
    const long long MIN_ROUNDS = min_rounds;
    if (slots < 1)
        slots = 1;
    int best = 0;
    double best_cost = 1e300;
    for (int pass = 0; pass < 2 && best == 0; pass++) {
        for (int kz = 4; kz <= n2; kz++) {
            const long long nch = (n2 + kz - 1) / kz;
            const long long rounds = (tiles * nch + slots - 1) / slots;
            if (pass == 0 && rounds < MIN_ROUNDS)
                continue;  // the second pass drops the constraint when no kz can meet it
            const double cost = (double)rounds * (kz + 3);
            if (cost <= best_cost) {
                best_cost = cost;
                best = kz;
            }
        }
    }
    return best > 0 ? best : (n2 < 32 ? n2 : 32);
}

}  // namespace hx
