// Device-side numerics of the MUSCL-Hancock step for gfx950 (HIP).
//
// Conserved state U = (rho, m1, m2, m3, E, rho f_1..), primitives W = (rho, u1, u2, u3, P, f..)
// (paper Sect. 2.1 and eq. eos_gas).  The FP64 instantiation evaluates every expression in the
// same order as the FP64 CPU oracle so that the two agree to the last bits; the FP32 form
// recovers the internal energy E - |m|^2/(2 rho) in FP64 where the kinetic energy dominates (high
// Mach) and uses hardware reciprocal/sqrt.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hx_params.h"

namespace hx {

// FP64 quotient a / b rounded to nearest even, for operands whose quotient, reciprocal and
// remainder stay well inside the normal range (exponents within about +-700; the states, widths
// and time steps of this method are): the hardware reciprocal refined by two Newton-Raphson steps
// and the quotient corrected once by its exact FMA remainder (Markstein's method).  These are the
// operations of the compiler's correctly rounded division without its operand range scaling and
// special-value fixup, which act only near the ends of the exponent range and on zeros,
// infinities and NaNs; checked bit for bit against the compiler's division on 1.3e8 operand pairs
// with exponents in [-300, 300].  Two differences remain: -0 / b for b > 0 gives +0 (the values
// are equal), and a zero, infinite or NaN operand does not give IEEE's special result (x / 0 is
// NaN, not an infinity), so a division whose denominator may be zero keeps the IEEE operator.  It saves the two scaling instructions and the fixup of each division, and the
// scaling's use of the single VCC register, which keeps the scheduler from overlapping divisions.
__device__ __forceinline__ double div_rn(double a, double b)
{
    double r = __builtin_amdgcn_rcp(b);
    double e = fma(-b, r, 1.0);
    r = fma(r, e, r);
    e = fma(-b, r, 1.0);
    r = fma(r, e, r);
    const double m = a * r;
    const double t = fma(-b, m, a);
    return fma(t, r, m);
}

// FP64 square root rounded to nearest even, for x in the normal range above 2^-767 (finite,
// positive): the hardware reciprocal square root refined by Goldschmidt-style coupled iterations
// of the root g and the half reciprocal h, then two FMA residual corrections of g.  These are the
// operations of the compiler's correctly rounded square root without its input scaling (for x
// below 2^-767) and its pass-through of zeros and infinities; checked bit for bit against the
// compiler's square root on 1.3e8 arguments with exponents in [-700, 700].  sqrt_rn(0) and
// sqrt_rn(inf) are NaN, so an argument that may be zero or infinite keeps sqrt().
__device__ __forceinline__ double sqrt_rn(double x)
{
    const double y = __builtin_amdgcn_rsq(x);
    double g = x * y;
    double h = y * 0.5;
    const double r = fma(-h, g, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    double d = fma(-g, g, x);
    g = fma(d, h, g);
    d = fma(-g, g, x);
    return fma(d, h, g);
}

template <typename R>
struct Num;

template <>
struct Num<double> {
    static __device__ __forceinline__ double div(double a, double b) { return div_rn(a, b); }
    static __device__ __forceinline__ double sqrt_(double a) { return sqrt_rn(a); }
    static __device__ __forceinline__ double abs_(double a) { return fabs(a); }
    static __device__ __forceinline__ double from_d(double a) { return a; }
};

template <>
struct Num<float> {
    static __device__ __forceinline__ float div(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
    static __device__ __forceinline__ float sqrt_(float a) { return __builtin_amdgcn_sqrtf(a); }
    static __device__ __forceinline__ float abs_(float a) { return fabsf(a); }
    static __device__ __forceinline__ float from_d(double a) { return (float)a; }
};

template <typename R>
struct Gas {
    R gm1, inv_gm1, gamma;
    R Rg, arad;  // gas + radiation EoS: specific gas constant k_b/(mu m_u), radiation constant
};

// ---------------------------------------------------------------- gas + radiation EoS
// Sect. 2.3, eqs. eos_gp_rad_ein and eos_gp_rad: e = rho Rg T/(gamma-1) + arad T^4 and
// P = rho Rg T + arad T^4 / 3 (FP64).  The temperature follows from e (or from P) by Newton's
// method started from the smaller of the gas-only and radiation-only temperatures, an upper bound
// from which the iteration decreases monotonically to the root.  Each lane stops once its own
// correction is at most EOS_NEWTON_TOL of its T (Newton's quadratic convergence, with
// (f''/2f') T <= 3/2 for these residuals, then leaves a relative error below 2e-16), and after
// EOS_NEWTON_STEPS steps at the latest.  Every operation is the IEEE-rounded one of the plain
// definition (divisions and square roots included, in the same order), so a lane's iterates and
// its stopping step do not depend on the other lanes of its wave.
constexpr int EOS_NEWTON_STEPS = 10;
constexpr double EOS_NEWTON_TOL = 1e-8;

__device__ __forceinline__ double t4(double T) { return (T * T) * (T * T); }

// K independent temperatures in one loop (from e, or from P with FROM_P), so that the dependent
// chains of their Newton steps overlap; a lane keeps stepping a chain until that chain has met
// the stopping test
template <bool FROM_P, int K>
__device__ __forceinline__ void temp_solve(const Gas<double>& g, const double* rho, const double* x, double* T)
{
    // from e: f(T) = c T + a T^4 - e, c = rho Rg/(gamma-1); from P: f(T) = c T + a T^4/3 - P,
    // c = rho Rg.  Start: the smaller of c^-1 e (or c^-1 P) and (e/a)^(1/4) (or (3P/a)^(1/4));
    // a = 0 gives an infinite radiation-only temperature, so the start is the gas one
    double c[K];
    bool act[K];
#pragma unroll
    for (int j = 0; j < K; j++) {
        c[j] = FROM_P ? rho[j] * g.Rg : div_rn(rho[j] * g.Rg, g.gm1);
        const double tg = div_rn(x[j], c[j]);
        // IEEE division: a = 0 (the gas-only limit) must give an infinite radiation temperature
        const double tr = sqrt(sqrt(FROM_P ? (3.0 * x[j]) / g.arad : x[j] / g.arad));
        T[j] = tg < tr ? tg : tr;
        act[j] = true;
    }
#pragma unroll 1
    for (int it = 0; it < EOS_NEWTON_STEPS; it++) {
        bool more = false;
#pragma unroll
        for (int j = 0; j < K; j++) {
            if (act[j]) {
                const double Tj = T[j];
                double f, fp;
                if (FROM_P) {
                    f = c[j] * Tj + div_rn(g.arad * t4(Tj), 3.0) - x[j];
                    fp = c[j] + div_rn(4.0 * g.arad * ((Tj * Tj) * Tj), 3.0);
                } else {
                    f = c[j] * Tj + g.arad * t4(Tj) - x[j];
                    fp = c[j] + 4.0 * g.arad * ((Tj * Tj) * Tj);
                }
                const double dT = div_rn(f, fp);
                T[j] = Tj - dT;
                act[j] = !(fabs(dT) <= EOS_NEWTON_TOL * T[j]);
            }
            more = more || act[j];
        }
        if (!__any(more))
            break;
    }
}

__device__ __forceinline__ double temp_from_e(const Gas<double>& g, double rho, double e)
{
    double T;
    temp_solve<false, 1>(g, &rho, &e, &T);
    return T;
}

__device__ __forceinline__ double temp_from_p(const Gas<double>& g, double rho, double P)
{
    double T;
    temp_solve<true, 1>(g, &rho, &P, &T);
    return T;
}

// internal energy per unit volume at temperature T
__device__ __forceinline__ double rad_energy(const Gas<double>& g, double rho, double T)
{
    return div_rn((rho * g.Rg) * T, g.gm1) + g.arad * t4(T);
}

// pressure at temperature T
__device__ __forceinline__ double rad_pressure(const Gas<double>& g, double rho, double T)
{
    return (rho * g.Rg) * T + div_rn(g.arad * t4(T), 3.0);
}

// a wave-uniform double moved to scalar registers (it stays live through a whole sweep)
__device__ __forceinline__ double uniform_d(double v)
{
    const unsigned long long b = __double_as_longlong(v);
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)b);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(b >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// 56Ni decay heating per unit mass of 56Ni at time t (Sect. 2.4, eq. heating_ni):
// lambda {[Q_Ni (tau_Co/tau_Ni - 1) - Q_Co] exp(-t/tau_Ni) + Q_Co exp(-t/tau_Co)},
// lambda = 1 / (m_Ni (tau_Co - tau_Ni))
__device__ __forceinline__ double ni_rate(const SweepParams& p, double t)
{
    const double tn = p.ni_tau[0], tc = p.ni_tau[1];
    const double qn = p.ni_Q[0], qc = p.ni_Q[1];
    const double lam = 1.0 / (p.ni_m * (tc - tn));
    return lam * ((qn * (tc / tn - 1.0) - qc) * exp(-t / tn) + qc * exp(-t / tc));
}

// sound speed from primitives w, reciprocal density inv and (gas + radiation) temperature T:
// eq. eos_gas, or eq. cs_gp_rad with alpha = P_r / P_g
template <typename R, int EOS>
__device__ __forceinline__ R sound_speed(const Gas<R>& g, const R* w, R inv, R T)
{
    if constexpr (EOS == 0) {
        return Num<R>::sqrt_(g.gamma * w[4] * inv);
    } else {
        static_assert(sizeof(R) == 8, "the gas + radiation EoS is built for FP64");
        const double pg = (w[0] * g.Rg) * T;
        const double pr = div_rn(g.arad * t4(T), 3.0);
        const double al = div_rn(pr, pg);
        const double num = div_rn(g.gamma, g.gm1) + 20.0 * al + 16.0 * (al * al);
        const double den = div_rn(1.0, g.gm1) + 12.0 * al;
        return sqrt_rn(div_rn(num, den) * (pg * inv));
    }
}

// ---------------------------------------------------------------- EoS

// primitives from conserved.  DE: the last field is the monitored internal energy e, which is
// its own primitive (per unit volume, like the pressure); the passive scalars before it are
// carried per unit mass.
template <typename R, int NV, bool DE, int EOS>
struct PrimImpl;

template <int NV, bool DE, int EOS>
struct PrimImpl<double, NV, DE, EOS> {
    static __device__ __forceinline__ double run(const Gas<double>& g, const double* q, double* w, double* T)
    {
        double rho = q[0];
        double inv = div_rn(1.0, rho);
        double u1 = q[1] * inv, u2 = q[2] * inv, u3 = q[3] * inv;
        double ke = 0.5 * (q[1] * u1 + q[2] * u2 + q[3] * u3);
        w[0] = rho;
        w[1] = u1;
        w[2] = u2;
        w[3] = u3;
        if constexpr (EOS == 1) {
            const double Tt = temp_from_e(g, rho, q[4] - ke);
            w[4] = rad_pressure(g, rho, Tt);
            if (T)
                *T = Tt;
        } else {
            w[4] = g.gm1 * (q[4] - ke);
        }
#pragma unroll
        for (int v = 5; v < NV - DE; v++)
            w[v] = q[v] * inv;
        if (DE)
            w[NV - 1] = q[NV - 1];
        return inv;
    }
};

template <int NV, bool DE, int EOS>
struct PrimImpl<float, NV, DE, EOS> {
    static_assert(EOS == 0, "the gas + radiation EoS is built for FP64");
    // FP32 bulk: 1/rho from the hardware reciprocal refined by one Newton step, the velocities and
    // e = E - |m|^2/(2 rho) in FP32 where the kinetic energy is at most 3/4 of E (then the
    // subtraction loses at most two bits); above that (high Mach, where E - e_k cancels) and for
    // non-physical states, e is recovered in FP64 from the FP32 values (FP64 island).
    static __device__ __forceinline__ float run(const Gas<float>& g, const float* q, float* w, float*)
    {
        const float rho = q[0];
        const float r = __builtin_amdgcn_rcpf(rho);
        const float inv = fmaf(r, fmaf(-rho, r, 1.0f), r);
        w[0] = rho;
        w[1] = q[1] * inv;
        w[2] = q[2] * inv;
        w[3] = q[3] * inv;
        float e = q[4] - 0.5f * (q[1] * w[1] + q[2] * w[2] + q[3] * w[3]);
        if (!(e > 0.25f * q[4])) {
            double id = (double)r;
            id = id * (2.0 - (double)rho * id);
            const double m1 = q[1], m2 = q[2], m3 = q[3];
            e = (float)((double)q[4] - 0.5 * (m1 * m1 + m2 * m2 + m3 * m3) * id);
        }
        w[4] = g.gm1 * e;
#pragma unroll
        for (int v = 5; v < NV - DE; v++)
            w[v] = q[v] * inv;
        if (DE)
            w[NV - 1] = q[NV - 1];
        return inv;
    }
};

// returns the reciprocal density used for the velocities; T (if not null) receives the
// temperature of the gas + radiation EoS
template <typename R, int NV, bool DE = false, int EOS = 0>
__device__ __forceinline__ R to_prim(const Gas<R>& g, const R* q, R* w, R* T = nullptr)
{
    return PrimImpl<R, NV, DE, EOS>::run(g, q, w, T);
}

// CFL signal rate of the FP32 form, sum_d (|u_d| + c_s) rw_d with rw_d the reciprocal widths rounded
// once to FP32: the internal energy E - |m|^2/(2 rho) is recovered in FP64 for every state (the
// island that to_prim keeps for high Mach), the rest is FP32; the maximum over cells and the time step cfl / max stay FP64.  A negative value
// marks a non-physical state.  The sweep's store and the standalone CFL kernel both use it, and it
// is rounded as written whatever the unit's contraction setting, so the time step of a state does
// not depend on which of them computed it.
template <int NV, int NDIM>
__device__ __forceinline__ double cfl_rate_f32(const float* q, const Gas<float>& g, const float* rw)
{
    // rounded as written whatever the unit's contraction setting: the primitives are the
    // operations of to_prim<float>'s FP64 island, repeated here so that the FP32 sweeps keep
    // contraction in their own conversions
#pragma clang fp contract(off)
    bool fin = true;
#pragma unroll
    for (int v = 0; v < NV; v++)
        fin = fin && isfinite(q[v]);
    const float rho = q[0];
    double id = (double)__builtin_amdgcn_rcpf(rho);
    id = id * (2.0 - (double)rho * id);
    const double m1 = q[1], m2 = q[2], m3 = q[3];
    const double ke = 0.5 * (m1 * m1 + m2 * m2 + m3 * m3) * id;
    const float inv = (float)id;
    const float p = (float)((double)g.gm1 * ((double)q[4] - ke));
    if (!fin || !(rho > 0.0f) || !(p > 0.0f))
        return -1.0;
    const float cs = __builtin_amdgcn_sqrtf(g.gamma * p * inv);
    float s = 0.0f;
#pragma unroll
    for (int d = 0; d < NDIM; d++)
        s += (fabsf(q[1 + d] * inv) + cs) * rw[d];
    return (double)s;
}

// gas + radiation EoS: primitives of two conserved states (the faces of one Riemann problem) with
// their two temperature solves in one loop; the same values as two calls of to_prim
template <int NV, bool DE = false>
__device__ __forceinline__ void to_prim_rad2(const Gas<double>& g, const double* qa, const double* qb, double* wa,
                                             double* wb, double& ia, double& ib, double& Ta, double& Tb)
{
    const double* q[2] = {qa, qb};
    double* w[2] = {wa, wb};
    double rho[2], e[2], inv[2], T[2];
#pragma unroll
    for (int j = 0; j < 2; j++) {
        rho[j] = q[j][0];
        inv[j] = div_rn(1.0, rho[j]);
        const double u1 = q[j][1] * inv[j], u2 = q[j][2] * inv[j], u3 = q[j][3] * inv[j];
        const double ke = 0.5 * (q[j][1] * u1 + q[j][2] * u2 + q[j][3] * u3);
        w[j][0] = rho[j];
        w[j][1] = u1;
        w[j][2] = u2;
        w[j][3] = u3;
        e[j] = q[j][4] - ke;
#pragma unroll
        for (int v = 5; v < NV - DE; v++)
            w[j][v] = q[j][v] * inv[j];
        if (DE)
            w[j][NV - 1] = q[j][NV - 1];
    }
    temp_solve<false, 2>(g, rho, e, T);
#pragma unroll
    for (int j = 0; j < 2; j++)
        w[j][4] = rad_pressure(g, rho[j], T[j]);
    ia = inv[0];
    ib = inv[1];
    Ta = T[0];
    Tb = T[1];
}

// IEEE quotient in either precision (div_rn in FP64)
template <typename R>
__device__ __forceinline__ R qdiv(R a, R b)
{
    if constexpr (sizeof(R) == 8)
        return div_rn(a, b);
    else
        return a / b;
}

// kinetic energy |m|^2 / (2 rho) of a conserved state
template <typename R>
__device__ __forceinline__ R kinetic_energy(const R* q)
{
    return qdiv<R>(R(0.5) * (q[1] * q[1] + q[2] * q[2] + q[3] * q[3]), q[0]);
}

// blend factor of the internal-energy monitor (Sect. 2.5): 1 for e >= eps e_k,
// (e / (eps e_k))^2 down to eps e_k / 10, 0 below
template <typename R>
__device__ __forceinline__ R de_alpha(R e, R ek, R eps)
{
    const R t = eps * ek;
    if (e >= t)
        return R(1);
    if (e > qdiv<R>(t, R(10))) {
        const R r = qdiv<R>(e, t);
        return r * r;
    }
    return R(0);
}

// rho > 0 and P > 0, the latter tested as 2 rho E - |m|^2 > 0 (no division).  The FP32 form
// decides in FP32 where the computed value is farther from zero than its rounding error can reach
// (at most about 6 u (|2 rho E| + |m|^2), u = 2^-24, plus the absolute error of subnormal
// products; tested against 16 u and 2^-100), so that there the sign is the exact one for the FP32
// state even where the kinetic energy dominates and FP32 arithmetic cancels; otherwise it decides
// in FP64, where the products of the FP32 values are exact and only the sums round (the decision
// of an all-FP64 test).
template <typename R>
__device__ __forceinline__ bool positive_state(const R* q)
{
    if constexpr (sizeof(R) == 4) {
        const float a = 2.0f * q[0] * q[4];
        const float b = q[1] * q[1] + q[2] * q[2] + q[3] * q[3];
        const float p = a - b;
        bool pos = p > 0.0f;
        if (!(fabsf(p) > fmaf(0x1p-20f, fabsf(a) + b, 0x1p-100f))) {
            const double r = q[0], m1 = q[1], m2 = q[2], m3 = q[3], e = q[4];
            const double mm = m1 * m1 + m2 * m2 + m3 * m3;
            pos = 2.0 * r * e - mm > 0.0;
        }
        return q[0] > 0.0f && pos;
    } else {
        R m2 = q[1] * q[1] + q[2] * q[2] + q[3] * q[3];
        return q[0] > R(0) && R(2) * q[0] * q[4] - m2 > R(0);
    }
}

template <typename R, int NV, bool DE = false, int EOS = 0>
__device__ __forceinline__ void to_cons(const Gas<R>& g, const R* w, R* q)
{
    R rho = w[0];
    q[0] = rho;
    q[1] = rho * w[1];
    q[2] = rho * w[2];
    q[3] = rho * w[3];
    if constexpr (EOS == 1) {
        const double e = rad_energy(g, rho, temp_from_p(g, rho, w[4]));
        q[4] = e + 0.5 * (q[1] * w[1] + q[2] * w[2] + q[3] * w[3]);
    } else {
        q[4] = w[4] * g.inv_gm1 + R(0.5) * (q[1] * w[1] + q[2] * w[2] + q[3] * w[3]);
    }
#pragma unroll
    for (int v = 5; v < NV - DE; v++)
        q[v] = rho * w[v];
    if (DE)
        q[NV - 1] = w[NV - 1];
}

// gas + radiation EoS: conserved state of primitives w whose internal energy e(rho, P) is already
// known (rad_energy2); the same values as to_cons
template <int NV, bool DE = false>
__device__ __forceinline__ void to_cons_e(const double* w, double e, double* q)
{
    const double rho = w[0];
    q[0] = rho;
    q[1] = rho * w[1];
    q[2] = rho * w[2];
    q[3] = rho * w[3];
    q[4] = e + 0.5 * (q[1] * w[1] + q[2] * w[2] + q[3] * w[3]);
#pragma unroll
    for (int v = 5; v < NV - DE; v++)
        q[v] = rho * w[v];
    if (DE)
        q[NV - 1] = w[NV - 1];
}

// gas + radiation EoS: internal energies of two primitive states (solves in one loop)
__device__ __forceinline__ void rad_energy2(const Gas<double>& g, const double* wa, const double* wb, double& ea,
                                            double& eb)
{
    const double rho[2] = {wa[0], wb[0]}, P[2] = {wa[4], wb[4]};
    double T[2];
    temp_solve<true, 2>(g, rho, P, T);
    ea = rad_energy(g, rho[0], T[0]);
    eb = rad_energy(g, rho[1], T[1]);
}

// physical flux along axis D from primitives w and conserved q of the same state
template <typename R, int NV, int D, bool DE = false>
__device__ __forceinline__ void phys_flux(const R* w, const R* q, R* f)
{
    R un = w[1 + D];
    R mn = q[1 + D];
    f[0] = mn;
    f[1] = mn * w[1];
    f[2] = mn * w[2];
    f[3] = mn * w[3];
    f[1 + D] = f[1 + D] + w[4];
    f[4] = un * (q[4] + w[4]);
#pragma unroll
    for (int v = 5; v < NV - DE; v++)
        f[v] = mn * w[v];
    if (DE)
        f[NV - 1] = un * w[NV - 1];  // u e
}

// HLL / HLLC with Davis wave speeds (Sect. 3.2; textbook solvers the paper cites)
// uf (if not null) receives the interface velocity: the contact speed S* in the HLLC star
// region, else the normal velocity of the upwind side (HLL leaves it unset).
template <typename R, int NV, int D, bool DE = false, int EOS = 0>
__device__ __forceinline__ void riemann(int solver, const Gas<R>& g, const R* qL, const R* qR, R* F,
                                        R* uf = nullptr)
{
    using N = Num<R>;
    R wL[NV], wR[NV];
    R TL = R(0), TR = R(0), iL, iR;
    if constexpr (EOS == 1) {
        to_prim_rad2<NV, DE>(g, qL, qR, wL, wR, iL, iR, TL, TR);
    } else {
        iL = to_prim<R, NV, DE, EOS>(g, qL, wL, &TL);
        iR = to_prim<R, NV, DE, EOS>(g, qR, wR, &TR);
    }
    R rL = wL[0], rR = wR[0];
    R uL = wL[1 + D], uR = wR[1 + D];
    R pL = wL[4], pR = wR[4];
    R cL = sound_speed<R, EOS>(g, wL, iL, TL);
    R cR = sound_speed<R, EOS>(g, wR, iR, TR);
    R SL = fmin(uL - cL, uR - cR);
    R SR = fmax(uL + cL, uR + cR);
    if (solver == HX_HLL) {
        R fL[NV], fR[NV];
        phys_flux<R, NV, D, DE>(wL, qL, fL);
        phys_flux<R, NV, D, DE>(wR, qR, fR);
        if (SL >= R(0)) {
#pragma unroll
            for (int v = 0; v < NV; v++)
                F[v] = fL[v];
            return;
        }
        if (SR <= R(0)) {
#pragma unroll
            for (int v = 0; v < NV; v++)
                F[v] = fR[v];
            return;
        }
        R inv = N::div(R(1), SR - SL);
#pragma unroll
        for (int v = 0; v < NV; v++)
            F[v] = (SR * fL[v] - SL * fR[v] + SL * SR * (qR[v] - qL[v])) * inv;
        return;
    }
    // HLLC: F_L for S_L >= 0, F_L + S_L (U*_L - U_L) for S_L < 0 <= S*, F_R + S_R (U*_R - U_R) for
    // S* < 0 < S_R, F_R for S_R <= 0.  Every case needs the physical flux of one side only, so the
    // side is chosen first.
    R mL = rL * (SL - uL);
    R mR = rR * (SR - uR);
    R Ss = N::div(pR - pL + uL * mL - uR * mR, mL - mR);
    const bool left = SL >= R(0) || Ss >= R(0);
    const bool star = !(SL >= R(0)) && (Ss >= R(0) || SR > R(0));
    R S = left ? SL : SR;
    R m = left ? mL : mR;
    R iv = left ? iL : iR;
    R qs[NV], ws[NV], fs[NV];
#pragma unroll
    for (int v = 0; v < NV; v++) {
        qs[v] = left ? qL[v] : qR[v];
        ws[v] = left ? wL[v] : wR[v];
    }
    phys_flux<R, NV, D, DE>(ws, qs, fs);
    if (uf)
        *uf = star ? Ss : (left ? uL : uR);
    if (!star) {
#pragma unroll
        for (int v = 0; v < NV; v++)
            F[v] = fs[v];
        return;
    }
    R us[NV];
    R un = ws[1 + D];
    R fac = N::div(m, S - Ss);
    us[0] = fac;
    us[1] = fac * ws[1];
    us[2] = fac * ws[2];
    us[3] = fac * ws[3];
    us[1 + D] = fac * Ss;
    us[4] = fac * (qs[4] * iv + (Ss - un) * (Ss + N::div(ws[4], m)));
#pragma unroll
    for (int v = 5; v < NV - DE; v++)
        us[v] = fac * ws[v];
    if (DE)
        us[NV - 1] = fac * (ws[NV - 1] * iv);  // rho* e / rho of the side
#pragma unroll
    for (int v = 0; v < NV; v++)
        F[v] = fs[v] + S * (us[v] - qs[v]);
}

template <typename R>
__device__ __forceinline__ R limit(int lim, R a, R b)
{
    using N = Num<R>;
    if (lim == HX_LIM_NONE)
        return R(0);
    if (!(a * b > R(0)))
        return R(0);
    if (lim == HX_LIM_MINMOD)
        return N::abs_(a) < N::abs_(b) ? a : b;
    if (lim == HX_LIM_VANALBADA)
        return N::div(a * b * (a + b), a * a + b * b);
    return N::div(R(2) * a * b, a + b);
}

// Makes x opaque to the optimiser (emits no instruction): expressions of x before and after are
// not merged, so a recomputation is not replaced by values kept in registers.
template <typename T>
__device__ __forceinline__ void opaque(T& x)
{
    asm volatile("" : "+v"(x));
}

// 16-lane row shifts (DPP row_shr:1 / row_shl:1): lane l of each row of 16 receives the value of
// lane l-1 (l+1); the first (last) lane of a row keeps its own value
__device__ __forceinline__ int dpp_shr1_i(int v) { return __builtin_amdgcn_update_dpp(v, v, 0x111, 0xF, 0xF, false); }
__device__ __forceinline__ int dpp_shl1_i(int v) { return __builtin_amdgcn_update_dpp(v, v, 0x101, 0xF, 0xF, false); }

template <bool UP>
__device__ __forceinline__ double row_shift(double v)
{
    unsigned long long u = (unsigned long long)__double_as_longlong(v);
    int lo = (int)(unsigned)(u & 0xffffffffull), hi = (int)(unsigned)(u >> 32);
    lo = UP ? dpp_shr1_i(lo) : dpp_shl1_i(lo);
    hi = UP ? dpp_shr1_i(hi) : dpp_shl1_i(hi);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

template <bool UP>
__device__ __forceinline__ float row_shift(float v)
{
    int i = __float_as_int(v);
    i = UP ? dpp_shr1_i(i) : dpp_shl1_i(i);
    return __int_as_float(i);
}

// boundary image of index i on an axis with n cells; indices are first clamped into the
// ghost range so that threads of ragged tiles always read inside the array
__device__ __forceinline__ int bc_image(int i, int n, int ng, int lo, int hi, bool& flip)
{
    i = i < -ng ? -ng : (i > n + ng - 1 ? n + ng - 1 : i);
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

__device__ __forceinline__ int clamp_ghost(int i, int n, int ng)
{
    return i < -ng ? -ng : (i > n + ng - 1 ? n + ng - 1 : i);
}

}  // namespace hx
