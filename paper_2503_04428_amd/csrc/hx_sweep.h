// Fused MUSCL-Hancock step for gfx950: one kernel reads U^n once and writes U^{n+1} once.
//
// The scheme (paper Sect. 3.2) per cell: primitives -> limited slopes along every active axis ->
// Hancock half step summed over the axes (unsplit) -> HLL/HLLC flux on every face ->
// U^{n+1} = U^n + dt/dV (F_L dS_L - F_R dS_R) summed x, y, z -> + dt S (gravity, Sect. 2.2, and the
// spherical momentum sources of Sect. 3.1.2).
//
// Mapping (3D): a 16x16-thread workgroup owns a 14x14 tile of (x, y) columns plus a one-cell
// halo ring of "predictor" cells and marches along z over a chunk of planes.  Per plane:
//   * the U^n plane k+1 is loaded (thread's own column cell into registers, the 18x18 primitive
//     rectangle into LDS), so every plane is read from HBM once per tile;
//   * every thread runs the Hancock predictor for its cell of plane k; x neighbours are exchanged
//     with 16-wide wave shuffles, y neighbours through LDS, z neighbours stay in registers;
//   * x and y fluxes of plane k and the z flux of face k-1/2 are formed; plane k-1 is finished
//     and stored, plane k gets its x and y terms and waits for face k+1/2.
// 1D and 2D use the same code with the inactive axes compiled out.
#pragma once
#include "hx_device.h"
#include "hx_mlp.h"

namespace hx {

// Minimum waves per SIMD the register allocator must allow (launch-bound hint).  More waves hide
// more latency but may force register spills.  FP32 3D sweeps: three waves, two where three would
// spill heavily: spherical sweeps from HX_MINW2_FP32_SPH_NV fields, Cartesian ones from
// HX_MINW2_FP32_CART_NV (256x128x128, fixed and run-time variants: 9 spherical fields 0.82 vs
// 0.47 ms, 9 Cartesian 0.58 vs 0.42 ms, 7 Cartesian 0.35 vs 0.36 ms); the learned form keeps three
// (1.48 vs 1.70 ms); HX_MINW_FP32 overrides the rule.  FP64 3D sweeps: two waves up to
// HX_MINW2_FP64_NV fields in Cartesian sweeps and in spherical sweeps with HLLC + van Leer compiled
// in, one wave otherwise (two vs one, 256x128x128: Cartesian 5 fields 0.50 vs 0.59 ms, 6 fields
// 0.74 vs 0.70 ms, RT 128x128x512 with 6 fields 1.37 vs 1.31 ms; spherical 5 fields 0.64 vs 0.67
// ms fixed, 0.93 vs 0.76 ms run-time variant, 6 fields 1.02 vs 0.78 ms; 7 fields need ~330
// registers); an explicit HX_MINW_FP64 overrides the rule.
#ifndef HX_MINW2_FP32_SPH_NV
#define HX_MINW2_FP32_SPH_NV 6
#endif
#ifndef HX_MINW2_FP32_CART_NV
#define HX_MINW2_FP32_CART_NV 8
#endif
#ifndef HX_MINW2_FP64_NV
#define HX_MINW2_FP64_NV 5
#endif
// face states formed again after the positivity check (rather than kept from it) from this many
// fields on: keeping them is faster where the registers allow (FP64 Sedov, 7 fields, one wave per
// SIMD: 2.312 -> 2.145 ms; boosted Sedov with the monitor, 8 fields: 2.510 -> 2.431 ms; wedge, 9
// fields: 3.280 -> 3.228 ms; FP32 Sedov, 7 fields, three waves: 0.859 -> 0.827 ms), so FP64
// sweeps always keep them and FP32 sweeps up to 7 fields
#ifndef HX_REFORM_FP64_NV
#define HX_REFORM_FP64_NV 10
#endif
#ifndef HX_REFORM_FP32_NV
#define HX_REFORM_FP32_NV 8
#endif
// FP64 sweeps: form the limited slopes again for the face states (1) or hold them (0)
#ifndef HX_RESLOPE_FP64
#define HX_RESLOPE_FP64 0
#endif
template <typename R, int NV, int NDIM, int GEOM, int SPEC>
struct MinWaves {
#ifdef HX_MINW_FP64
    static constexpr int fp64 = HX_MINW_FP64;
#else
    // (the internal-energy monitor's extra state and the gas + radiation EoS's Newton solves spill
    // at two waves even with 5 or 6 fields)
    static constexpr int fp64 =
        NDIM == 3 && NV <= HX_MINW2_FP64_NV && (GEOM == HX_CART ? SPEC < 3 : SPEC == 1) ? 2 : 1;
#endif
#ifdef HX_MINW_FP32
    static constexpr int fp32 = HX_MINW_FP32;
#else
    static constexpr int fp32 =
        NDIM == 3 && SPEC != 2 && NV >= (GEOM == HX_SPH ? HX_MINW2_FP32_SPH_NV : HX_MINW2_FP32_CART_NV) ? 2 : 3;
#endif
    static constexpr int value = sizeof(R) == 8 ? fp64 : fp32;
};

// Two-plane load prefetch: the 3D FP64 sweeps that run one wave per SIMD (their idle issue slots
// are mostly waits on the plane loads); HX_PREFETCH2 = 0 turns it off, 1 forces it everywhere.
template <typename R, int NV, int NDIM, int GEOM, int SPEC>
struct PrefetchTwo {
#ifdef HX_PREFETCH2
    static constexpr bool value = HX_PREFETCH2 != 0;
#else
    static constexpr bool value = sizeof(R) == 8 && MinWaves<R, NV, NDIM, GEOM, SPEC>::value == 1;
#endif
};

template <int NDIM>
struct Tile;
template <>
struct Tile<1> {
    static constexpr int BX = 64, BY = 1;
};
template <>
struct Tile<2> {
    static constexpr int BX = 16, BY = 16;
};
template <>
struct Tile<3> {
    static constexpr int BX = 16, BY = 16;
};


// Load U^n of one (possibly ghost) cell with boundary images applied.
template <typename R, int NV>
__device__ __forceinline__ void fetch_cell(const SweepParams& p, const R* __restrict__ U, int ii, int jj, int kk,
                                           bool f0, bool f1, bool f2, R* q)
{
    const long long off = ((long long)kk * p.n[1] + jj) * p.n[0] + ii;
#pragma unroll
    for (int v = 0; v < NV; v++)
        q[v] = U[(long long)v * p.plane + off];
    if (f0)
        q[1] = -q[1];
    if (f1)
        q[2] = -q[2];
    if (f2)
        q[3] = -q[3];
}

template <typename R, int NV>
__device__ __forceinline__ bool bad_state(const R* q, const R* w)
{
    bool bad = !(q[0] > R(0)) || !(w[4] > R(0));
#pragma unroll
    for (int v = 0; v < NV; v++)
        bad = bad || !isfinite((double)q[v]);
    return bad;
}

// x-neighbour exchange inside 16-lane rows (DPP) or, for 64-wide 1D tiles, across the wave
template <int BX, typename R>
__device__ __forceinline__ R from_left(R v)
{
    if constexpr (BX == 16)
        return row_shift<true>(v);
    else
        return __shfl_up(v, 1, BX);
}
template <int BX, typename R>
__device__ __forceinline__ R from_right(R v)
{
    if constexpr (BX == 16)
        return row_shift<false>(v);
    else
        return __shfl_down(v, 1, BX);
}

// CFL signal rate sum_d (|u_d| + c_s)/dx_d of a conserved state, in FP64, in the operation order
// of the reference definition (EOS = 1: P and c_s of the gas + radiation EoS); returns a negative
// value for a non-physical state.  The FP32 form takes cfl_rate_f32 (hx_device.h) instead.
template <typename R, int NV, int NDIM, int EOS = 0>
__device__ __forceinline__ double cfl_rate(const R* acc, double gamma, const double* wd, const Gas<R>& eg)
{
    double q[NV];
    bool fin = true;
#pragma unroll
    for (int v = 0; v < NV; v++) {
        q[v] = (double)acc[v];
        fin = fin && isfinite(q[v]);
    }
    const double rho = q[0];
    const double inv = div_rn(1.0, rho);
    const double u1 = q[1] * inv, u2 = q[2] * inv, u3 = q[3] * inv;
    const double ke = 0.5 * (q[1] * u1 + q[2] * u2 + q[3] * u3);
    double pr, cs;
    if constexpr (EOS == 1) {
        const double T = temp_from_e(eg, rho, q[4] - ke);
        pr = (rho * eg.Rg) * T + div_rn(eg.arad * t4(T), 3.0);
        if (!fin || !(rho > 0.0) || !(pr > 0.0))
            return -1.0;
        const double w[5] = {rho, u1, u2, u3, pr};
        cs = sound_speed<double, 1>(eg, w, inv, T);
    } else {
        pr = (gamma - 1.0) * (q[4] - ke);
        if (!fin || !(rho > 0.0) || !(pr > 0.0))
            return -1.0;
        cs = sqrt_rn(gamma * pr * inv);
    }
    const double u[3] = {u1, u2, u3};
    double s = 0.0;
#pragma unroll
    for (int d = 0; d < NDIM; d++)
        s += div_rn(fabs(u[d]) + cs, wd[d]);
    return s;
}

// SPEC = 1 compiles the common HLLC + van Leer case with both choices fixed; SPEC = 2 the learned
// limiter with HLLC (slope stencil of half-width 2, BF16 matrix-core network); SPEC = 0 reads the
// limiter and the Riemann solver from the parameters; SPEC = 3 adds the internal-energy monitor
// (Sect. 2.5: the last field is e, with eq. pressure_fix and the alpha blend; HLLC, limiter from
// the parameters); SPEC = 4 the gas + radiation EoS (Sect. 2.3, FP64; limiter and Riemann solver
// from the parameters); SPEC = 5 both (the monitor's P through the EoS; HLLC).
// TAG only separates otherwise identical instantiations built in different units (with different
// code-generation options), so that each unit launches its own.  SRC = 0 compiles out the source
// terms (gravity, 56Ni heating) for Cartesian configurations without them, whose FP64 source
// state would otherwise hold registers through the whole sweep.
template <typename R, int NV, int NDIM, int GEOM, int SPEC, int TAG = 0, int SRC = 1>
__global__ void __launch_bounds__(Tile<NDIM>::BX* Tile<NDIM>::BY, (MinWaves<R, NV, NDIM, GEOM, SPEC>::value))
    sweep_kernel(const SweepParams p)
{
    static_assert(SRC == 1 || GEOM == HX_CART, "spherical sweeps always carry their geometric sources");
    const int grav = SRC ? p.gravity : HX_GRAV_NONE;
    using N = Num<R>;
    constexpr int BX = Tile<NDIM>::BX;
    constexpr int BY = Tile<NDIM>::BY;
    constexpr int NT = BX * BY;
    constexpr bool MLP = SPEC == 2;
    constexpr bool DE = SPEC == 3 || SPEC == 5;  // internal-energy monitor: the last field is e (FP64, HLLC)
    constexpr int EOS = SPEC == 4 || SPEC == 5 ? 1 : 0;  // gas + radiation EoS (FP64)
    constexpr int S = MLP ? 2 : 1;  // half-width of the slope stencil
    constexpr int RX = BX + 2 * S;
    constexpr int RY = NDIM >= 2 ? BY + 2 * S : 1;
    constexpr int NWAVE = NT / 64 > 0 ? NT / 64 : 1;
    constexpr int NSLOT = NDIM == 3 ? 2 : 1;
    constexpr int NYB = NDIM >= 2 ? NT : 1;
    constexpr int TX = BX - 2;
    constexpr int TY = NDIM >= 2 ? BY - 2 : 1;
    // 3D sweeps with one wave per SIMD issue the loads of a plane two iterations before its use
    // (nothing else hides their latency); the others one iteration before
    constexpr bool PF2 = NDIM == 3 && PrefetchTwo<R, NV, NDIM, GEOM, SPEC>::value;
    // reconstruction about volume centroids (spherical r and theta) in the run-time variants
    constexpr bool CEN = GEOM == HX_SPH && (SPEC == 0 || SPEC == 3 || SPEC == 4 || SPEC == 5);

    __shared__ R sW[NSLOT][NV][RY * RX];  // primitives of a plane incl. a 2-cell ring
    __shared__ R sFy[NV][NYB];            // +y half-step state of every predictor cell
    __shared__ R sGy[NV][NYB];            // y flux through the lower face of every cell
    __shared__ R sGu[DE ? NYB : 1];       // and its interface velocity (internal-energy monitor)
    __shared__ double sRed[NWAVE];
    // learned limiter: per-wave queue of the stencils that need the network, and its outputs
    __shared__ unsigned long long sQ[MLP ? NWAVE : 1][MLP ? 2 * 64 * NV : 1];
    __shared__ __align__(16) unsigned char sMlpRaw[MLP ? sizeof(MlpShared) : 16];  // network operands
    MlpShared& sMlp = *reinterpret_cast<MlpShared*>(sMlpRaw);
    const int lim = SPEC == 1 ? HX_LIM_VANLEER : (SPEC == 2 ? HX_LIM_MLP : p.limiter);
    const int solver = SPEC == 0 || SPEC == 4 ? p.riemann : HX_HLLC;
    double smax = 0.0;     // CFL rate of the cells this thread stores

    const R* __restrict__ U = (const R*)p.U;
    R* __restrict__ Un = (R*)p.Unew;
    const int n0 = p.n[0], n1 = p.n[1], n2 = p.n[2], ng = p.ng;
    const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * BX + tx;
    // XCD-aware tile order: workgroups are dealt round-robin to the 8 XCDs by linear id, so the
    // linear id is remapped to give every XCD one contiguous band of tiles (x fastest, then y,
    // then the z chunk); neighbouring tiles then share their halo planes in the same L2.
    int bx, by, bz;
    {
        const unsigned gx = gridDim.x, gy = gridDim.y;
        const unsigned nb = gx * gy * gridDim.z;
        const unsigned b = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
        const unsigned xcd = b % 8u, idx = b / 8u, q = nb / 8u, r = nb % 8u;
        const unsigned L = xcd * q + (xcd < r ? xcd : r) + idx;
        bx = (int)(L % gx);
        by = (int)((L / gx) % gy);
        bz = (int)(L / (gx * gy));
    }
    const int x0 = bx * TX;
    const int y0 = NDIM >= 2 ? by * TY : 0;
    // cell of this thread (clamped into the ghost range for ragged tiles)
    const int ic = clamp_ghost(x0 + tx - 1, n0, ng);
    const int jc = NDIM >= 2 ? clamp_ghost(y0 + ty - 1, n1, ng) : 0;
    const bool interior = tx >= 1 && tx <= TX && (x0 + tx - 1) < n0 &&
                          (NDIM < 2 || (ty >= 1 && ty <= TY && (y0 + ty - 1) < n1));
    int k0 = 0, k1 = 1;
    if (NDIM == 3) {
        k0 = bz * p.kz;
        k1 = min(k0 + p.kz, n2);
    }
    const double dtd = p.dt_dev ? p.dt_dev[0] : p.dt_host;
    const R dt = N::from_d(dtd);
    // 56Ni heating rates at the start and the middle of the step (FP64 forms with the run-time
    // limiter and solver, the internal-energy monitor or the gas + radiation EoS)
    const bool heat = SRC && sizeof(R) == 8 && SPEC != 1 && p.ni >= 0;
    double h_n = 0.0, h_half = 0.0;
    if (heat) {
        const double t = p.t_in[0];
        h_n = uniform_d(ni_rate(p, t));
        h_half = uniform_d(ni_rate(p, t + 0.5 * dtd));
    }
    // rho f_Ni of a state (the field index is a run-time value: select, not index, registers)
    auto ni_of = [&](const R* q) {
        double f = 0.0;
#pragma unroll
        for (int v = 5; v < NV - DE; v++)
            if (v == p.ni)
                f = (double)q[v];
        return f;
    };
    Gas<R> gas;
    gas.gamma = N::from_d(p.gamma);
    gas.gm1 = N::from_d(p.gamma - 1.0);
    gas.inv_gm1 = N::from_d(1.0 / (p.gamma - 1.0));
    gas.Rg = N::from_d(p.eos_R);
    gas.arad = N::from_d(p.eos_arad);

    // images of this thread's x / y indices
    bool fx, fy;
    const int ii = bc_image(ic, n0, ng, p.bc[0][0], p.bc[0][1], fx);
    // 1D: axis 1 indexes independent rows (a batch of 1D problems), one row per workgroup row
    const int jj = NDIM >= 2 ? bc_image(jc, n1, ng, p.bc[1][0], p.bc[1][1], fy) : by;
    if (NDIM < 2)
        fy = false;
    const int gx = NDIM >= 1 ? ic + ng : 0;
    const int gy = NDIM >= 2 ? jc + ng : 0;

    // per-thread geometry that does not change along z
    const R cmx = N::from_d(p.geo.cm[0][gx]), cpx = N::from_d(p.geo.cp[0][gx]);
    R cmy = R(0), cpy = R(0);
    if (NDIM >= 2) {
        cmy = N::from_d(p.geo.cm[1][gy]);
        cpy = N::from_d(p.geo.cp[1][gy]);
    }
    // lower-face over upper-face extrapolation distance of x and y (1 about face midpoints, and
    // always along z); the bound on the increments applies with volume centroids only
    const bool cen = CEN && p.centroid != 0;
    R kpx = R(1), kpy = R(1);
    if constexpr (CEN) {
        kpx = N::from_d(p.geo.kap[0][gx]);
        if (NDIM >= 2)
            kpy = N::from_d(p.geo.kap[1][gy]);
    }
    // predictor coefficients dt / (2 width) for x and y (widths of the image cell)
    R lamx, lamy = R(0);
    double wx = p.geo.w[0][gx], wy = 0.0;
    if (GEOM == HX_CART) {
        lamx = N::from_d(div_rn(dtd, 2.0 * wx));
        if (NDIM >= 2) {
            wy = p.geo.w[1][gy];
            lamy = N::from_d(div_rn(dtd, 2.0 * wy));
        }
    } else {
        lamx = N::from_d(div_rn(dtd, 2.0 * wx));
        if (NDIM >= 2) {
            wy = p.geo.rabs[gx] * p.geo.w[1][gy];
            lamy = N::from_d(div_rn(dtd, 2.0 * wy));
        }
    }
    // FP32 form: reciprocal widths of the CFL rate, rounded once to FP32 (x and y per column)
    const float rwx = sizeof(R) == 4 ? (float)div_rn(1.0, wx) : 0.0f;
    const float rwy = sizeof(R) == 4 && NDIM >= 2 ? (float)div_rn(1.0, wy) : 0.0f;
    // gravity of this column's image (z flips handled per plane)
    double gcol[3] = {0.0, 0.0, 0.0};
    if (grav == HX_GRAV_UNIFORM) {
        gcol[0] = fx ? -p.g0[0] : p.g0[0];
        gcol[1] = fy ? -p.g0[1] : p.g0[1];
        gcol[2] = p.g0[2];
    } else if (grav != HX_GRAV_NONE) {
        gcol[0] = fx ? -p.gr[ii] : p.gr[ii];
    }

    // spherical per-column geometry used in every plane: held in registers by the two-plane
    // prefetch sweeps (for the reason above), read where used by the others
    struct SphCol {
        double rsxy, vrct, hrw, rm, rp, ctj, hrsm, hrsp, smm, spp, dph2;
    } sc = {};
    if constexpr (GEOM == HX_SPH && PF2) {
        sc.rsxy = p.geo.rabs[gx] * p.geo.sabs[gy];
        sc.vrct = p.geo.vr[ii] * p.geo.ct[jj];
        sc.hrw = p.geo.hr[ii] * p.geo.w[1][jj + ng];
        sc.rm = p.geo.rf[ii];
        sc.rp = p.geo.rf[ii + 1];
        sc.ctj = p.geo.ct[jj];
        sc.hrsm = p.geo.hr[ii] * p.geo.sf[jj];
        sc.hrsp = p.geo.hr[ii] * p.geo.sf[jj + 1];
        sc.smm = p.geo.sf[jj];
        sc.spp = p.geo.sf[jj + 1];
        sc.dph2 = p.geo.w[2][0];
    }
    auto g_rsxy = [&]() { return PF2 ? sc.rsxy : p.geo.rabs[gx] * p.geo.sabs[gy]; };
    auto g_vrct = [&]() { return PF2 ? sc.vrct : p.geo.vr[ii] * p.geo.ct[jj]; };
    auto g_hrw = [&]() { return PF2 ? sc.hrw : p.geo.hr[ii] * p.geo.w[1][jj + ng]; };
    auto g_rm = [&]() { return PF2 ? sc.rm : p.geo.rf[ii]; };
    auto g_rp = [&]() { return PF2 ? sc.rp : p.geo.rf[ii + 1]; };
    auto g_ctj = [&]() { return PF2 ? sc.ctj : p.geo.ct[jj]; };
    auto g_hrsm = [&]() { return PF2 ? sc.hrsm : p.geo.hr[ii] * p.geo.sf[jj]; };
    auto g_hrsp = [&]() { return PF2 ? sc.hrsp : p.geo.hr[ii] * p.geo.sf[jj + 1]; };
    auto g_smm = [&]() { return PF2 ? sc.smm : p.geo.sf[jj]; };
    auto g_spp = [&]() { return PF2 ? sc.spp : p.geo.sf[jj + 1]; };
    auto g_dph2 = [&]() { return PF2 ? sc.dph2 : p.geo.w[2][0]; };

    // ------------------------------------------------------------------ plane loader
    // The primitives of the (RX x RY) rectangle of a plane (predictor cells plus an S-wide ring)
    // go to LDS.  Each thread loads its own cell (rectangle position (tx+S, ty+S)); the ring has
    // fewer cells than the block has threads, so a thread loads at most one ring cell.  Loads are
    // split into an issue half (global loads) and a commit half (flips, primitives, LDS stores), so
    // the loads of the next planes are in flight while the x and y predictor of plane k runs.
    // The own column runs S planes ahead of the LDS plane (the z stencil needs k-S .. k+S).
    constexpr int NRING = NDIM >= 2 ? 2 * S * RX + 2 * S * BY : 2 * S;
    static_assert(NRING <= NT, "at most one ring cell per thread");
    const bool has_ring = tid < NRING;
    int ring_lds = 0, ri = 0, rj = 0;
    bool rf0 = false, rf1 = false;
    if (has_ring) {
        int lx, ly;
        if (NDIM >= 2) {
            if (tid < S * RX) {
                lx = tid % RX;
                ly = tid / RX;
            } else if (tid < 2 * S * RX) {
                const int r2 = tid - S * RX;
                lx = r2 % RX;
                ly = RY - S + r2 / RX;
            } else {
                const int r3 = tid - 2 * S * RX;
                const int side = r3 / (S * BY), r4 = r3 % (S * BY);
                ly = S + r4 / S;
                lx = (side == 0 ? 0 : RX - S) + r4 % S;
            }
        } else {
            lx = tid < S ? tid : RX - 2 * S + tid;
            ly = 0;
        }
        ri = bc_image(x0 - 1 - S + lx, n0, ng, p.bc[0][0], p.bc[0][1], rf0);
        if (NDIM >= 2)
            rj = bc_image(y0 - 1 - S + ly, n1, ng, p.bc[1][0], p.bc[1][1], rf1);
        else
            rj = jj;
        ring_lds = ly * RX + lx;
    }
    const int own = (NDIM >= 2 ? (ty + S) * RX : 0) + tx + S;

    auto raw_load = [&](int i0, int j0, int kk, R* q) {
        const long long off = ((long long)kk * n1 + j0) * n0 + i0;
#pragma unroll
        for (int v = 0; v < NV; v++)
            q[v] = U[(long long)v * p.plane + off];
    };
    auto plane_image = [&](int k, bool& fk) {
        fk = false;
        return NDIM == 3 ? bc_image(k, n2, ng, p.bc[2][0], p.bc[2][1], fk) : 0;
    };
    auto issue_own = [&](int k, R* q) {
        bool fk;
        raw_load(ii, jj, plane_image(k, fk), q);
    };
    auto issue_ring = [&](int k, R* q) {
        bool fk;
        const int kk = plane_image(k, fk);
        if (has_ring)
            raw_load(ri, rj, kk, q);
    };
    // flips and primitives of the own cell of plane k (and the non-physical check)
    auto commit_own = [&](int k, R* q, R* w) {
        bool fk;
        (void)plane_image(k, fk);
        if (fx)
            q[1] = -q[1];
        if (fy)
            q[2] = -q[2];
        if (fk)
            q[3] = -q[3];
        to_prim<R, NV, DE, EOS>(gas, q, w);
        const bool kin = NDIM < 3 || (k >= 0 && k < n2);
        if (kin && interior && bad_state<R, NV>(q, w))
            p.flag[0] = 1;
    };
    auto commit_ring = [&](int k, int s, R* q) {
        bool fk;
        (void)plane_image(k, fk);
        if (has_ring) {
            if (rf0)
                q[1] = -q[1];
            if (rf1)
                q[2] = -q[2];
            if (fk)
                q[3] = -q[3];
            R w[NV];
            to_prim<R, NV, DE, EOS>(gas, q, w);
#pragma unroll
            for (int v = 0; v < NV; v++)
                sW[s][v][ring_lds] = w[v];
        }
    };
    auto store_own = [&](int s, const R* w) {
#pragma unroll
        for (int v = 0; v < NV; v++)
            sW[s][v][own] = w[v];
    };

    // ------------------------------------------------------------------ learned limiter
    // The network's operands live once per block in LDS (a barrier follows before the first use).
    // slopes_mlp() handles na axes at once (x and y together, z alone): each monotone (lane, axis,
    // variable) stencil gets a slot of the wave's LDS queue (ordered by axis, variable, lane), the
    // wave evaluates 16 queued stencils per matrix-core tile and writes phi over the low word of
    // the stencil's slot.  A wave without candidates skips all of it.
    if constexpr (MLP)
        mlp_fill_shared(p.mlp, tid, NT, sMlp);
    // limited half increments of one axis; st(j, v) = primitive v at offset j - 2 along the axis
    // (all stencil values are read before the first limiter branch, so that their loads overlap)
    auto slopes = [&](auto&& st, R cm, R cp, R kp, R* dl) {
        R a[NV], b[NV];
#pragma unroll
        for (int v = 0; v < NV; v++) {
            const R w1 = st(1, v), w2 = st(2, v), w3 = st(3, v);
            a[v] = cm * (w2 - w1);
            b[v] = cp * (w3 - w2);
        }
#pragma unroll
        for (int v = 0; v < NV; v++)
            dl[v] = limit<R>(lim, a[v], b[v]);
        // about volume centroids an extrapolation distance can exceed half the distance to the
        // neighbouring centroid: the increment is bounded so that both face values stay between
        // the neighbouring cell values, |dl| <= |w+ - w| and kp |dl| <= |w - w-|
        if constexpr (CEN) {
            if (cen) {
#pragma unroll
                for (int v = 0; v < NV; v++) {
                    if (dl[v] != R(0)) {
                        const R dm = st(2, v) - st(1, v), dp = st(3, v) - st(2, v);
                        const R bound = fmin(N::abs_(dp), N::div(N::abs_(dm), kp));
                        if (N::abs_(dl[v]) > bound)
                            dl[v] = dl[v] > R(0) ? bound : -bound;
                    }
                }
            }
        }
    };
    // learned form of slopes() for the axes a0 .. a0+na-1 (na <= 2); st(a, j, v) = primitive v at
    // offset j - 2 along axis a.  The stencils are read again after the queue fence, so that they
    // are not held in registers across the network tiles.
    auto slopes_mlp = [&](auto&& st, int a0, int na, const R* cmv, const R* cpv, R (*dl)[NV]) {
        const int lane = tid & 63, wv = tid >> 6;
        unsigned long long bal[2][NV];  // candidates: monotone stencils, d1 d2 > 0
        unsigned first[2][NV];          // queue slot of the first candidate of (axis, variable)
        unsigned total = 0;
        // one (axis, variable) at a time: its four differences are queued (d / max|d| as BF16)
        // by the candidate lanes and are dead before the next stencil is read
#pragma unroll
        for (int a = 0; a < na; a++)
#pragma unroll
            for (int v = 0; v < NV; v++) {
                float dd[4];
#pragma unroll
                for (int j = 0; j < 4; j++)
                    dd[j] = st(a0 + a, j + 1, v) - st(a0 + a, j, v);
                bal[a][v] = __builtin_amdgcn_ballot_w64(dd[1] * dd[2] > 0.0f);
                first[a][v] = total;
                if (bal[a][v]) {
                    const float is = __builtin_amdgcn_rcpf(
                        fmaxf(fmaxf(fabsf(dd[0]), fabsf(dd[1])), fmaxf(fabsf(dd[2]), fabsf(dd[3]))));
                    const unsigned long long x = __builtin_bit_cast(
                        unsigned long long, pack_x(dd[0] * is, dd[1] * is, dd[2] * is, dd[3] * is));
                    if ((bal[a][v] >> lane) & 1ull)
                        sQ[wv][total + __builtin_amdgcn_mbcnt_hi((unsigned)(bal[a][v] >> 32),
                                                                 __builtin_amdgcn_mbcnt_lo((unsigned)bal[a][v], 0u))] = x;
                }
                total += (unsigned)__builtin_popcountll(bal[a][v]);
                dl[a][v] = R(0);
            }
        if (total == 0)
            return;
        auto cand = [&](int a, int v) { return ((bal[a][v] >> lane) & 1ull) != 0; };
        auto slot = [&](int a, int v) {
            return (int)(first[a][v] + __builtin_amdgcn_mbcnt_hi((unsigned)(bal[a][v] >> 32),
                                                                 __builtin_amdgcn_mbcnt_lo((unsigned)bal[a][v], 0u)));
        };
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        float* qphi = reinterpret_cast<float*>(sQ[wv]);  // phi of slot e at qphi[2 e]
        // the network's operands, read once for all the tiles of the queue
        MlpLane m;
        mlp_lane_from_shared(sMlp, lane, m);
        for (unsigned t0 = 0; t0 < total; t0 += 16) {
            const unsigned e = t0 + (lane & 15);
            // lanes past the queue's end evaluate a copy of its last entry, which is not stored
            const bf16x4_t xb = __builtin_bit_cast(bf16x4_t, sQ[wv][e < total ? e : total - 1]);
            const float ph = mlp_tile(m, xb);
            if (lane < 16 && e < total)
                qphi[2 * e] = ph;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // phi a inside the TVD region phi <= min(2, 2 b/a), van Leer's slope outside it
        // (a b > 0 here, so phi > 2 b/a is phi |a| > 2 |b|)
        R phv[2][NV];
#pragma unroll
        for (int a = 0; a < na; a++)
#pragma unroll
            for (int v = 0; v < NV; v++)
                phv[a][v] = qphi[2 * (cand(a, v) ? slot(a, v) : 0)];
#pragma unroll
        for (int a = 0; a < na; a++)
#pragma unroll
            for (int v = 0; v < NV; v++) {
                const R phi = phv[a][v];
                const R da = cmv[a] * (st(a0 + a, 2, v) - st(a0 + a, 1, v));
                const R db = cpv[a] * (st(a0 + a, 3, v) - st(a0 + a, 2, v));
                const bool tvd = !(phi > R(2) || phi * fabs(da) > R(2) * fabs(db));
                const R s = tvd ? phi * da : R(2) * da * db * R(__builtin_amdgcn_rcpf((float)(da + db)));
                dl[a][v] = cand(a, v) ? s : R(0);
            }
    };

    // ------------------------------------------------------------------ persistent state
    // own column: wz[S + j] = primitives of plane k + j (j = -S..S), qz[j] = conserved of plane k + j
    R wz[2 * S + 1][NV], qz[S + 1][NV];
    R qpf[PF2 ? NV : 1], rpf[PF2 ? NV : 1];  // two-plane prefetch: own column and ring cell in flight
    // z geometry (cm, cp, width) of the next plane, loaded one iteration ahead by the two-plane
    // prefetch sweeps: a load issued after the plane loads would make its wait (the memory
    // counter is in order) a wait for the plane loads too
    double zgn[3] = {0.0, 0.0, 0.0};
    R acc[NV];     // plane k-1: U^n + x and y flux terms
    R fzlo[NV];    // z flux through the lower face of plane k-1
    R uzp[NV];     // +z half-step state of plane k-1
    double sg[5];  // gravity source of plane k-1 (components 1..4)
    double sph_t[6];  // spherical partial sources of plane k-1: Trt, Trp, Tt, Xt, grg, gtg
    // internal-energy monitor, plane k-1: P of its half-step e, its e^n and blend factor, and the
    // interface velocity of its lower z face
    R pe_prev = R(0), en_prev = R(0), alpha_prev = R(0), ufzlo = R(0);
    // e_new = e^n + alpha d1e + (1 - alpha) d2e: d1e from the updated total energy, d2e from the
    // internal-energy equation (the last field of the updated state a)
    auto de_blend = [&](R* a, R en, R alpha) {
        const R d1 = (a[4] - kinetic_energy<R>(a)) - en;
        const R d2 = a[NV - 1] - en;
        a[NV - 1] = en + alpha * d1 + (R(1) - alpha) * d2;
    };
    double w2prev = 0.0;  // z width of plane k-1 (loaded for its predictor; the kernel's own stores
                          // would force the finish of the plane to load it again from memory)
#pragma unroll
    for (int v = 0; v < NV; v++) {
        acc[v] = R(0);
        fzlo[v] = R(0);
        uzp[v] = R(0);
#pragma unroll
        for (int j = 0; j < 2 * S + 1; j++)
            wz[j][v] = R(0);
    }
#pragma unroll
    for (int v = 0; v < 5; v++)
        sg[v] = 0.0;
#pragma unroll
    for (int v = 0; v < 6; v++)
        sph_t[v] = 0.0;

    int kbeg = k0, kend = k0;  // loop bounds over predictor planes
    if (NDIM == 3) {
        kbeg = k0 - 1;
        kend = k1;
        // own column, planes kbeg-S .. kbeg+S-1, and the LDS rectangle of plane kbeg
#pragma unroll
        for (int j = 0; j < 2 * S; j++) {
            R q[NV];
            issue_own(kbeg - S + j, q);
            commit_own(kbeg - S + j, q, wz[j]);
            if (j >= S) {
#pragma unroll
                for (int v = 0; v < NV; v++)
                    qz[j - S][v] = q[v];
            }
        }
        R qr[NV];
        issue_ring(kbeg, qr);
        commit_ring(kbeg, kbeg & 1, qr);
        store_own(kbeg & 1, wz[S]);
        // a valid state for the (unused) z flux below the first predictor plane
#pragma unroll
        for (int v = 0; v < NV; v++)
            uzp[v] = qz[0][v];
        // two-plane prefetch: the loads the first iteration commits, after the z geometry of its
        // plane
        if constexpr (PF2) {
            const int gz0 = clamp_ghost(kbeg, n2, ng) + ng;
            zgn[0] = p.geo.cm[2][gz0];
            zgn[1] = p.geo.cp[2][gz0];
            zgn[2] = p.geo.w[2][gz0];
            issue_own(kbeg + S, qpf);
            issue_ring(kbeg + 1, rpf);
        }
    } else {
        R qr[NV];
        issue_own(0, qz[0]);
        issue_ring(0, qr);
        commit_own(0, qz[0], wz[S]);
        commit_ring(0, 0, qr);
        store_own(0, wz[S]);
    }
    __syncthreads();

    for (int k = kbeg; k <= kend; ++k) {
        const int slot = NDIM == 3 ? (k & 1) : 0;
        R qring[NV];
        // z geometry of plane k: cm, cp, width
        double zg[3] = {0.0, 0.0, 0.0};
        if (NDIM == 3) {
            const int gzk = clamp_ghost(k, n2, ng) + ng;
            if constexpr (PF2) {
                // the loads of plane k+1 (own column k+S) and this plane's geometry were issued
                // one iteration ago; the next plane's geometry, then the loads of the next planes
                // go out now and have a whole iteration to arrive
#pragma unroll
                for (int t = 0; t < 3; t++)
                    zg[t] = zgn[t];
#pragma unroll
                for (int v = 0; v < NV; v++) {
                    qz[S][v] = qpf[v];
                    qring[v] = rpf[v];
                }
                const int gzn = clamp_ghost(k + 1, n2, ng) + ng;
                zgn[0] = p.geo.cm[2][gzn];
                zgn[1] = p.geo.cp[2][gzn];
                zgn[2] = p.geo.w[2][gzn];
                issue_own(k + S + 1, qpf);
                issue_ring(k + 2, rpf);
            } else {
                // geometry first: its wait then does not include the plane loads
                zg[0] = p.geo.cm[2][gzk];
                zg[1] = p.geo.cp[2][gzk];
                zg[2] = p.geo.w[2][gzk];
                issue_own(k + S, qz[S]);
                issue_ring(k + 1, qring);
            }
        }
        R(&wcur)[NV] = wz[S];
        R(&qcur)[NV] = qz[0];

        // -------------------------------------------------------------- predictor, plane k
        bool fzk = false;
        double w2k = 0.0;  // z width of plane k
        R cmz = R(0), cpz = R(0), lamz = R(0);
        double g[3] = {gcol[0], gcol[1], gcol[2]};
        if (NDIM == 3) {
            const int kc = clamp_ghost(k, n2, ng);
            bc_image(kc, n2, ng, p.bc[2][0], p.bc[2][1], fzk);  // sets the z-mirror flag
            cmz = N::from_d(zg[0]);
            cpz = N::from_d(zg[1]);
            w2k = zg[2];
            double wz = GEOM == HX_CART ? w2k : g_rsxy() * w2k;
            lamz = N::from_d(div_rn(dtd, 2.0 * wz));
            if (fzk && grav == HX_GRAV_UNIFORM)
                g[2] = -g[2];
        }
        // primitive v at offset j - 2 along axis a from the plane in LDS (x, y) or the own column (z)
        auto stv = [&](int a, int j, int v) -> R {
            if (a == 2)
                return wz[S + j - 2][v];
            return j == 2 ? wcur[v] : sW[slot][v][own + (j - 2) * (a == 0 ? 1 : RX)];
        };
        R dlt[3][NV];  // half increments of the limited slopes
        R du[NV];
        // FP64 sweeps form the limited slopes again where the face states are built instead of
        // holding 3 NV of them across the predictor (the register budget of two waves per SIMD)
        constexpr bool RESLOPE = !MLP && sizeof(R) == 8 && HX_RESLOPE_FP64;
        R cm3[3] = {cmx, cmy, cmz}, cp3[3] = {cpx, cpy, cpz};
        const R kp3[3] = {kpx, kpy, R(1)};
        auto slope_of = [&](int d, R* dl) {
            slopes([&](int j, int v) { return stv(d, j, v); }, cm3[d], cp3[d], kp3[d], dl);
        };
        // inputs of slope_of made opaque, so that it is evaluated again rather than kept
        auto reslope_fence = [&]() {
            asm volatile("" ::: "memory");
#pragma unroll
            for (int d = 0; d < 3; d++) {
                opaque(cm3[d]);
                opaque(cp3[d]);
            }
#pragma unroll
            for (int j = 0; j < 2 * S + 1; j++)
#pragma unroll
                for (int v = 0; v < NV; v++)
                    opaque(wz[j][v]);
        };
#pragma unroll
        for (int v = 0; v < NV; v++) {
            du[v] = R(0);
            dlt[0][v] = dlt[1][v] = dlt[2][v] = R(0);
        }
        // internal-energy monitor: P of e^n for the half step's -P div(u) ((gamma - 1) e, or
        // through the gas + radiation EoS, solved once per cell)
        R pen = R(0);
        if constexpr (DE && EOS == 1)
            pen = rad_pressure(gas, qcur[0], temp_from_e(gas, qcur[0], qcur[NV - 1]));
        auto pe_n = [&]() -> R {
            if constexpr (EOS == 1)
                return pen;
            else
                return gas.gm1 * qcur[NV - 1];
        };
        // gas + radiation EoS: internal energies of the six reconstructed face states, solved
        // once here and reused by the positivity check and the final face states
        R ef[EOS ? 3 : 1][2];
        auto pred_cons = [&](int d, const R* wm, const R* wp, R* um, R* up) {
            if constexpr (EOS == 1) {
                rad_energy2(gas, wm, wp, ef[d][0], ef[d][1]);
                to_cons_e<NV, DE>(wm, ef[d][0], um);
                to_cons_e<NV, DE>(wp, ef[d][1], up);
            } else {
                to_cons<R, NV, DE, EOS>(gas, wm, um);
                to_cons<R, NV, DE, EOS>(gas, wp, up);
            }
        };
        {
            // x
            if constexpr (MLP) {
                // the learned form evaluates the network for every axis here, where the least
                // state is live (no half-step increments, no face states): x and y, then, after
                // the commit of the next planes that its five-plane z stencil needs, z
                const R cmv[2] = {cmx, cmy}, cpv[2] = {cpx, cpy};
                slopes_mlp(stv, 0, NDIM >= 2 ? 2 : 1, cmv, cpv, dlt);
                if constexpr (NDIM == 3) {
                    commit_own(k + S, qz[S], wz[2 * S]);
                    commit_ring(k + 1, (k + 1) & 1, qring);
                    store_own((k + 1) & 1, wz[S + 1]);
                    slopes_mlp(stv, 2, 1, &cmz, &cpz, dlt + 2);
                }
            } else {
                slopes([&](int j, int v) { return stv(0, j, v); }, cmx, cpx, kpx, dlt[0]);
            }
            R wm[NV], wp[NV], um[NV], up[NV], fm[NV], fp[NV];
#pragma unroll
            for (int v = 0; v < NV; v++) {
                wm[v] = wcur[v] - kpx * dlt[0][v];
                wp[v] = wcur[v] + dlt[0][v];
            }
            pred_cons(0, wm, wp, um, up);
            phys_flux<R, NV, 0, DE>(wm, um, fm);
            phys_flux<R, NV, 0, DE>(wp, up, fp);
#pragma unroll
            for (int v = 0; v < NV; v++)
                du[v] += lamx * (fm[v] - fp[v]);
            // internal energy: -(dt/2) P div(u) with the reconstructed face velocities, P of e^n
            if constexpr (DE)
                du[NV - 1] += lamx * (pe_n() * (wm[1 + 0] - wp[1 + 0]));
        }
        if (NDIM >= 2) {
            if constexpr (!MLP)
                slopes([&](int j, int v) { return stv(1, j, v); }, cmy, cpy, kpy, dlt[1]);
            R wm[NV], wp[NV], um[NV], up[NV], fm[NV], fp[NV];
#pragma unroll
            for (int v = 0; v < NV; v++) {
                wm[v] = wcur[v] - kpy * dlt[1][v];
                wp[v] = wcur[v] + dlt[1][v];
            }
            pred_cons(1, wm, wp, um, up);
            phys_flux<R, NV, 1, DE>(wm, um, fm);
            phys_flux<R, NV, 1, DE>(wp, up, fp);
#pragma unroll
            for (int v = 0; v < NV; v++)
                du[v] += lamy * (fm[v] - fp[v]);
            // internal energy: -(dt/2) P div(u) with the reconstructed face velocities, P of e^n
            if constexpr (DE)
                du[NV - 1] += lamy * (pe_n() * (wm[1 + 1] - wp[1 + 1]));
        }
        if (NDIM == 3) {
            if constexpr (!MLP) {
                commit_own(k + S, qz[S], wz[2 * S]);
                commit_ring(k + 1, (k + 1) & 1, qring);
                store_own((k + 1) & 1, wz[S + 1]);
                slopes([&](int j, int v) { return stv(2, j, v); }, cmz, cpz, R(1), dlt[2]);
            }
            R wm[NV], wp[NV], um[NV], up[NV], fm[NV], fp[NV];
#pragma unroll
            for (int v = 0; v < NV; v++) {
                wm[v] = wcur[v] - dlt[2][v];
                wp[v] = wcur[v] + dlt[2][v];
            }
            pred_cons(2, wm, wp, um, up);
            phys_flux<R, NV, 2, DE>(wm, um, fm);
            phys_flux<R, NV, 2, DE>(wp, up, fp);
#pragma unroll
            for (int v = 0; v < NV; v++)
                du[v] += lamz * (fm[v] - fp[v]);
            // internal energy: -(dt/2) P div(u) with the reconstructed face velocities, P of e^n
            if constexpr (DE)
                du[NV - 1] += lamz * (pe_n() * (wm[1 + 2] - wp[1 + 2]));
        }
        if (grav != HX_GRAV_NONE) {
            // (dt/2) S(U^n) with S = (0, rho g, m.g, 0)
            R hs = R(0.5) * dt;
            R S[5];
            S[0] = R(0);
            S[1] = qcur[0] * N::from_d(g[0]);
            S[2] = qcur[0] * N::from_d(g[1]);
            S[3] = qcur[0] * N::from_d(g[2]);
            S[4] = qcur[1] * N::from_d(g[0]) + qcur[2] * N::from_d(g[1]) + qcur[3] * N::from_d(g[2]);
#pragma unroll
            for (int v = 0; v < 5; v++)
                du[v] += hs * S[v];
#pragma unroll
            for (int v = 5; v < NV; v++)
                du[v] += hs * R(0);
        }
        // 56Ni decay heating of U^n at t^n over the half step (the monitored e takes it too)
        if (heat) {
            const R hs = R(0.5) * dt;
            const R sh = N::from_d(h_n * ni_of(qcur));
            du[4] += hs * sh;
            if constexpr (DE)
                du[NV - 1] += hs * sh;
        }
        // positivity of all half-step face states; otherwise first order for this cell
        bool bad = false;
        if constexpr (RESLOPE)
            reslope_fence();
#pragma unroll
        for (int d = 0; d < NDIM; d++) {
            R dd[NV];
            if constexpr (RESLOPE) {
                slope_of(d, dd);
            } else {
#pragma unroll
                for (int v = 0; v < NV; v++)
                    dd[v] = dlt[d][v];
            }
#pragma unroll
            for (int side = 0; side < 2; side++) {
                R ws[NV], qs[NV];
#pragma unroll
                for (int v = 0; v < NV; v++)
                    ws[v] = side ? wcur[v] + dd[v] : wcur[v] - kp3[d] * dd[v];
                if constexpr (EOS == 1)
                    to_cons_e<NV, DE>(ws, ef[d][side], qs);
                else
                    to_cons<R, NV, DE, EOS>(gas, ws, qs);
#pragma unroll
                for (int v = 0; v < NV; v++)
                    qs[v] += du[v];
                bad = bad || !positive_state<R>(qs);
            }
        }
        // The face states are formed below one axis at a time, just before their flux.  Where
        // registers allow (HX_REFORM_*_NV) a face state is the check's expression again and the
        // compiler keeps the check's values; otherwise the fallback zeroes du and the slopes first,
        // so the states are recomputed rather than held, which spills less.
        constexpr bool REFORM = RESLOPE || NV >= (sizeof(R) == 8 ? HX_REFORM_FP64_NV : HX_REFORM_FP32_NV);
        if (REFORM && bad) {
#pragma unroll
            for (int v = 0; v < NV; v++) {
                du[v] = R(0);
                dlt[0][v] = dlt[1][v] = dlt[2][v] = R(0);
            }
        }
        if constexpr (RESLOPE) {
#pragma unroll
            for (int v = 0; v < NV; v++)
                opaque(du[v]);
            reslope_fence();
        }
        // limited slopes of axis d for the face states
        auto axis_dl = [&](int d, R* dd) {
            if constexpr (RESLOPE) {
                slope_of(d, dd);
            } else {
#pragma unroll
                for (int v = 0; v < NV; v++)
                    dd[v] = dlt[d][v];
            }
        };
        // gas + radiation EoS, fallback: the internal energy of W itself (rho and P of W -/+ 0)
        R e0 = R(0);
        if constexpr (EOS == 1) {
            if (bad)
                e0 = rad_energy(gas, wcur[0], temp_from_p(gas, wcur[0], wcur[4]));
        }
        // conserved state of face-state primitives ws of axis d, side
        auto face_cons = [&](int d, int side, bool fb, const R* ws, R* out) {
            if constexpr (EOS == 1)
                to_cons_e<NV, DE>(ws, fb ? e0 : ef[d][side], out);
            else
                to_cons<R, NV, DE, EOS>(gas, ws, out);
        };
        // final half-step face states: cons(W -/+ delta) + du, or cons(W -/+ 0) in the fallback
        auto face_state = [&](int d, const R* dd, int side, R* out) {
            R ws[NV];
            if (REFORM) {
                // du and the held slopes are zero in the fallback; recomputed slopes are zeroed here
#pragma unroll
                for (int v = 0; v < NV; v++) {
                    const R dv = RESLOPE && bad ? R(0) : dd[v];
                    ws[v] = side ? wcur[v] + dv : wcur[v] - kp3[d] * dv;
                }
                face_cons(d, side, bad, ws, out);
                if (!bad) {
#pragma unroll
                    for (int v = 0; v < NV; v++)
                        out[v] += du[v];
                }
                return;
            }
#pragma unroll
            for (int v = 0; v < NV; v++)
                ws[v] = side ? wcur[v] + dd[v] : wcur[v] - kp3[d] * dd[v];
            face_cons(d, side, false, ws, out);
#pragma unroll
            for (int v = 0; v < NV; v++)
                out[v] += du[v];
            if (bad) {
#pragma unroll
                for (int v = 0; v < NV; v++)
                    ws[v] = side ? wcur[v] + R(0) : wcur[v] - R(0);
                face_cons(d, side, true, ws, out);
            }
        };
        // sources of the cell half-step state uh = U^n + du (U^n in the fallback): gravity
        // (0, rho g, m.g) now; the spherical terms keep uh for the update
        R uh[GEOM == HX_SPH ? NV : 1];
        double Sg[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
        // internal-energy monitor: P of the half-step e (for -P div(u)), e^n and the blend factor
        R pek = R(0), enk = R(0), alphak = R(0);
        {
            R u[NV];
#pragma unroll
            for (int v = 0; v < NV; v++)
                u[v] = bad ? qcur[v] : qcur[v] + du[v];
            if constexpr (DE) {
                if constexpr (EOS == 1)
                    pek = rad_pressure(gas, u[0], temp_from_e(gas, u[0], u[NV - 1]));
                else
                    pek = gas.gm1 * u[NV - 1];
                enk = qcur[NV - 1];
                alphak = de_alpha<R>(enk, kinetic_energy<R>(qcur), N::from_d(p.de_eps));
            }
            if (grav != HX_GRAV_NONE) {
                Sg[1] = (double)u[0] * g[0];
                Sg[2] = (double)u[0] * g[1];
                Sg[3] = (double)u[0] * g[2];
                Sg[4] = (double)u[1] * g[0] + (double)u[2] * g[1] + (double)u[3] * g[2];
            }
            // 56Ni decay heating of the half-step state at t^n + dt/2; Sg[0] keeps the share of
            // the monitored internal energy
            if (heat) {
                const double sh = h_half * ni_of(u);
                Sg[4] = Sg[4] + sh;
                if constexpr (DE)
                    Sg[0] = sh;
            }
            if constexpr (GEOM == HX_SPH) {
#pragma unroll
                for (int v = 0; v < NV; v++)
                    uh[v] = u[v];
            }
        }

        // -------------------------------------------------------------- fluxes and update
        // Order: (3D) z flux and the end of plane k-1, then the x flux and the x terms of plane k,
        // then the y exchange; every cell still sums U^n + x terms + y terms (+ z terms) and then
        // its sources, as the update equation is written.
        const bool plane_live = NDIM < 3 || (k >= k0 && k < k1);
        if (NDIM == 3) {
            // z: the +z state of plane k-1 is held by the thread; plane k's replaces it
            R Fz[NV], ufz = R(0);
            {
                R dd[NV], qmz[NV];
                axis_dl(2, dd);
                face_state(2, dd, 0, qmz);
                riemann<R, NV, 2, DE, EOS>(solver, gas, uzp, qmz, Fz, DE ? &ufz : nullptr);
                face_state(2, dd, 1, uzp);
            }
            // finish plane k-1 with its z terms and sources, then store it
            if (interior && k - 1 >= k0) {
                const int kp = k - 1;
                if (GEOM == HX_CART) {
                    const R mu = N::from_d(div_rn(dtd, w2prev));
#pragma unroll
                    for (int v = 0; v < NV; v++)
                        acc[v] += mu * (fzlo[v] - Fz[v]);
                    if constexpr (DE)
                        acc[NV - 1] += mu * (pe_prev * (ufzlo - ufz));
                } else {
                    const double dph = w2prev;
                    const double dV = g_vrct() * dph;
                    const R kv = N::from_d(div_rn(dtd, dV));
                    const R dS = N::from_d(g_hrw());
#pragma unroll
                    for (int v = 0; v < NV; v++)
                        acc[v] += kv * (fzlo[v] * dS - Fz[v] * dS);
                    if constexpr (DE)
                        acc[NV - 1] += kv * (pe_prev * (ufzlo * dS - ufz * dS));
                }
                if (grav != HX_GRAV_NONE || GEOM == HX_SPH || heat) {
                    double S[5] = {0.0, sg[1], sg[2], sg[3], sg[4]};
                    if (GEOM == HX_SPH) {
                        const double Xp = 0.5 * ((double)fzlo[3] + (double)Fz[3]);
                        S[1] = S[1] + 0.5 * (sph_t[3] + Xp) * sph_t[4];
                        S[2] = S[2] + (sph_t[0] + Xp * sph_t[5]);
                        S[3] = S[3] + (sph_t[1] + sph_t[2]);
                    }
#pragma unroll
                    for (int v = 1; v < 5; v++)
                        acc[v] = N::from_d((double)acc[v] + dtd * S[v]);
                }
                if constexpr (DE) {
                    if (heat)
                        acc[NV - 1] = acc[NV - 1] + dtd * sg[0];
                    de_blend(acc, en_prev, alpha_prev);
                }
                const long long off = ((long long)kp * n1 + jj) * n0 + ii;
#pragma unroll
                for (int v = 0; v < NV; v++)
                    Un[(long long)v * p.plane + off] = acc[v];
                double sr;
                if constexpr (sizeof(R) == 4) {
                    const float rw[3] = {rwx, rwy, (float)div_rn(1.0, GEOM == HX_CART ? w2prev : g_rsxy() * w2prev)};
                    sr = cfl_rate_f32<NV, NDIM>(acc, gas, rw);
                } else {
                    double wd[3] = {wx, wy, GEOM == HX_CART ? w2prev : g_rsxy() * w2prev};
                    sr = cfl_rate<R, NV, NDIM, EOS>(acc, p.gamma, wd, gas);
                }
                if (sr < 0.0)
                    p.flag[0] = 1;
                smax = fmax(smax, sr);
            }
#pragma unroll
            for (int v = 0; v < NV; v++)
                fzlo[v] = Fz[v];
            if constexpr (DE)
                ufzlo = ufz;
        }
        R Fx[NV], Fxr[NV], ufx = R(0), ufxr = R(0);
        {
            // x: the +x state of the left neighbour arrives by a row shift
            R qmx[NV], L[NV];
            {
                R dd[NV], qpx[NV];
                axis_dl(0, dd);
                face_state(0, dd, 1, qpx);
#pragma unroll
                for (int v = 0; v < NV; v++)
                    L[v] = from_left<BX>(qpx[v]);
                face_state(0, dd, 0, qmx);
            }
            if (tx == 0) {
#pragma unroll
                for (int v = 0; v < NV; v++)
                    L[v] = qmx[v];
            }
            riemann<R, NV, 0, DE, EOS>(solver, gas, L, qmx, Fx, DE ? &ufx : nullptr);
#pragma unroll
            for (int v = 0; v < NV; v++)
                Fxr[v] = from_right<BX>(Fx[v]);
            if constexpr (DE)
                ufxr = from_right<BX>(ufx);
        }
        // x terms of plane k (and the spherical x parts of its sources)
        const bool upd = interior && plane_live;
        double dV = 0.0, dSrm = 0.0, dSrp = 0.0, dStm = 0.0, dStp = 0.0, dph = 1.0, cr = 0.0;
        double Trt = 0.0, Trp = 0.0;
        if (upd) {
#pragma unroll
            for (int v = 0; v < NV; v++)
                acc[v] = qcur[v];
            if (GEOM == HX_CART) {
                const R mu = N::from_d(div_rn(dtd, wx));
#pragma unroll
                for (int v = 0; v < NV; v++)
                    acc[v] += mu * (Fx[v] - Fxr[v]);
                if constexpr (DE)
                    acc[NV - 1] += mu * (pek * (ufx - ufxr));
            } else {
                dph = NDIM == 3 ? w2k : g_dph2();
                const double ctj = g_ctj();
                dV = g_vrct() * dph;
                const double rm = g_rm(), rp = g_rp();
                dSrm = rm * rm * ctj * dph;
                dSrp = rp * rp * ctj * dph;
                const double kvd = div_rn(dtd, dV);
                const R kv = N::from_d(kvd);
                const R sm = N::from_d(dSrm), sp = N::from_d(dSrp);
#pragma unroll
                for (int v = 0; v < NV; v++)
                    acc[v] += kv * (Fx[v] * sm - Fxr[v] * sp);
                if constexpr (DE)
                    acc[NV - 1] += kv * (pek * (ufx * sm - ufxr * sp));
                cr = (rp - rm) / ((rp + rm) * dV);
                Trt = -cr * ((double)Fxr[2] * dSrp + (double)Fx[2] * dSrm);
                Trp = -cr * ((double)Fxr[3] * dSrp + (double)Fx[3] * dSrm);
            }
        }

        // y: +y states through LDS, then the fluxes of the upper faces through LDS
        R Fy[NV], Fyu[NV], ufy = R(0), ufyu = R(0);
        {
            R qmy[NV];
            if (NDIM >= 2) {
                R dd[NV], qpy[NV];
                axis_dl(1, dd);
                face_state(1, dd, 0, qmy);
                face_state(1, dd, 1, qpy);
#pragma unroll
                for (int v = 0; v < NV; v++)
                    sFy[v][tid] = qpy[v];
            }
            __syncthreads();
            if (NDIM >= 2) {
                R L[NV];
#pragma unroll
                for (int v = 0; v < NV; v++)
                    L[v] = ty > 0 ? sFy[v][tid - BX] : qmy[v];
                riemann<R, NV, 1, DE, EOS>(solver, gas, L, qmy, Fy, DE ? &ufy : nullptr);
#pragma unroll
                for (int v = 0; v < NV; v++)
                    sGy[v][tid] = Fy[v];
                if constexpr (DE)
                    sGu[tid] = ufy;
            }
            __syncthreads();
            if (NDIM >= 2) {
#pragma unroll
                for (int v = 0; v < NV; v++)
                    Fyu[v] = ty < BY - 1 ? sGy[v][tid + BX] : Fy[v];
                if constexpr (DE)
                    ufyu = ty < BY - 1 ? sGu[tid + BX] : ufy;
            }
        }

        if (upd) {
            // y terms of plane k
            if (NDIM >= 2) {
                if (GEOM == HX_CART) {
                    const R muy = N::from_d(div_rn(dtd, wy));
#pragma unroll
                    for (int v = 0; v < NV; v++)
                        acc[v] += muy * (Fy[v] - Fyu[v]);
                    if constexpr (DE)
                        acc[NV - 1] += muy * (pek * (ufy - ufyu));
                } else {
                    const double kvd = div_rn(dtd, dV);
                    const R kv = N::from_d(kvd);
                    dStm = g_hrsm() * dph;
                    dStp = g_hrsp() * dph;
                    const R tm = N::from_d(dStm), tp = N::from_d(dStp);
#pragma unroll
                    for (int v = 0; v < NV; v++)
                        acc[v] += kv * (Fy[v] * tm - Fyu[v] * tp);
                    if constexpr (DE)
                        acc[NV - 1] += kv * (pek * (ufy * tm - ufyu * tp));
                }
            }
            // sources of plane k (finished now in 1D/2D, after the z terms in 3D)
            double S[5] = {0.0, Sg[1], Sg[2], Sg[3], Sg[4]};
            if (GEOM == HX_SPH) {
                const double grg = (dSrp - dSrm) / dV;
                double pu = 0.0;
                if (NDIM < 3) {
                    R wu[NV];
                    to_prim<R, NV, DE, EOS>(gas, uh, wu);
                    pu = (double)wu[4];
                }
                double Xt, Tt = 0.0, gtg = 0.0;
                if (NDIM >= 2) {
                    const double smm = g_smm(), spp = g_spp();
                    const double ctc = (spp - smm) / ((spp + smm) * dV);
                    gtg = (dStp - dStm) / dV;
                    Xt = 0.5 * ((double)Fy[2] + (double)Fyu[2]);
                    Tt = -ctc * ((double)Fyu[3] * dStp + (double)Fy[3] * dStm);
                } else {
                    Xt = (double)uh[2] * ((double)uh[2] / (double)uh[0]) + pu;
                }
                if (NDIM == 3) {
                    sph_t[0] = Trt;
                    sph_t[1] = Trp;
                    sph_t[2] = Tt;
                    sph_t[3] = Xt;
                    sph_t[4] = grg;
                    sph_t[5] = gtg;
                } else {
                    const double Xp = (double)uh[3] * ((double)uh[3] / (double)uh[0]) + pu;
                    S[1] = S[1] + 0.5 * (Xt + Xp) * grg;
                    S[2] = S[2] + (Trt + Xp * gtg);
                    S[3] = S[3] + (Trp + Tt);
                }
            }
            if (NDIM == 3) {
#pragma unroll
                for (int v = 1; v < 5; v++)
                    sg[v] = S[v];
                if constexpr (DE)
                    sg[0] = Sg[0];
            } else {
                if (grav != HX_GRAV_NONE || GEOM == HX_SPH || heat) {
#pragma unroll
                    for (int v = 1; v < 5; v++)
                        acc[v] = N::from_d((double)acc[v] + dtd * S[v]);
                }
                if constexpr (DE) {
                    if (heat)
                        acc[NV - 1] = acc[NV - 1] + dtd * Sg[0];
                    de_blend(acc, enk, alphak);
                }
                const long long off = ((long long)jj * n0) + ii;
#pragma unroll
                for (int v = 0; v < NV; v++)
                    Un[(long long)v * p.plane + off] = acc[v];
                double sr;
                if constexpr (sizeof(R) == 4) {
                    const float rw[3] = {rwx, rwy, 0.0f};
                    sr = cfl_rate_f32<NV, NDIM>(acc, gas, rw);
                } else {
                    double wd[3] = {wx, wy, 0.0};
                    sr = cfl_rate<R, NV, NDIM, EOS>(acc, p.gamma, wd, gas);
                }
                if (sr < 0.0)
                    p.flag[0] = 1;
                smax = fmax(smax, sr);
            }
        }
        if (NDIM == 3) {
            w2prev = w2k;
            if constexpr (DE) {
                pe_prev = pek;
                en_prev = enk;
                alpha_prev = alphak;
            }
#pragma unroll
            for (int v = 0; v < NV; v++) {
#pragma unroll
                for (int j = 0; j < 2 * S; j++)
                    wz[j][v] = wz[j + 1][v];
#pragma unroll
                for (int j = 0; j < S; j++)
                    qz[j][v] = qz[j + 1][v];
            }
        }
    }

    // per-block maximum of the CFL rate of the stored cells (the time step of the next step)
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        smax = fmax(smax, __shfl_xor(smax, o, 64));
    if ((tid & 63) == 0)
        sRed[tid >> 6] = smax;
    __syncthreads();
    if (tid == 0) {
        double m = sRed[0];
        for (int w = 1; w < NT / 64; w++)
            m = fmax(m, sRed[w]);
        const long long b = ((long long)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
        p.dtpart[b] = m;
    }
}

}  // namespace hx
