/*
 * FP64 CPU oracle: one MUSCL-Hancock step of the HERACLES++ scheme, written
 * as plain loops.  TEST INFRASTRUCTURE ONLY (see hydro_oracle.h).
 *
 * The step follows the paper's order (Sect. 3.2):
 *   1. boundary images of the conserved state (periodic / null-gradient /
 *      reflective, Sect. 3.2 last paragraph);
 *   2. primitives (rho, u, P, f) from the ideal-gas EoS (Sect. 2.3, eq. eos_gas) or the gas +
 *      radiation EoS (eqs. eos_gp_rad_ein, eos_gp_rad);
 *   3. limited slopes of the primitives and the reconstructed face values
 *      W_i -/+ (dr_i/2) sigma  (Sect. 3.2, first equation);
 *   4. the Hancock half step U^{n+1/2}_{L,R} = U_{L,R} + dt/(2 dr_i) [F(U_L) - F(U_R)],
 *      summed over all active axes for the unsplit multi-dimensional form;
 *   5. HLL / HLLC fluxes at every face from the half-step states;
 *   6. the Godunov update (eq. godunov) in the finite-volume form
 *      U_new = U + dt/dV (F_L dS_L - F_R dS_R) of Sect. 3.3, plus gravity
 *      (Sect. 2.2) and, in spherical coordinates, the momentum source terms of
 *      Sect. 3.1.2 (eq. source_terms_1 and its theta counterpart), 56Ni decay heating
 *      (Sect. 2.4, eq. heating_ni) and the internal-energy monitor (Sect. 2.5).
 *
 * Readings where the paper is silent are stated at the point of use.
 */
#ifdef _OPENMP
#include <omp.h>
#endif
#include "hydro_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define MAXV 16

/* Marks work that repeats an evaluation made elsewhere in the step; a no-op here.  The
 * op-counting build (opcount.cpp) books the operations inside it apart. */
#ifndef OR_REPEATED_WORK
#define OR_REPEATED_WORK(on)
#endif

typedef struct {
    const or_config *c;
    int nvar;
    int act[3];
    int n[3];
    double gm1;       /* gamma - 1 */
    double inv_gm1;   /* 1 / (gamma - 1) */
    int de;           /* 1: the last field is the monitored internal energy e */
    double gamma;
    int eos;          /* OR_EOS_GAS or OR_EOS_GAS_RAD */
    double R, arad;   /* gas + radiation: specific gas constant k_b/(mu m_u), radiation constant */
    double *gr;       /* radial gravity per interior shell (point / monopole), or NULL */
} Ctx;

/* ------------------------------------------------------------------ geometry */

/* face coordinate i of axis d; active axes carry ng ghost faces on each side */
static double xf(const or_config *c, int d, int i)
{
    if (d < c->ndim)
        return c->faces[d][i + c->ng];
    return c->faces[d][i];
}

static double xcen(const or_config *c, int d, int i) { return 0.5 * (xf(c, d, i) + xf(c, d, i + 1)); }
static double dxc(const or_config *c, int d, int i) { return xf(c, d, i + 1) - xf(c, d, i); }

/* Position of cell i along axis d in the reconstruction with volume centroids (the option
 * `centroid`, reading of the cell centre r_i of Sect. 3.1 on non-uniform spherical cells): the
 * centroid of the cell's volume measure along the axis.  Spherical r, measure r^2 dr:
 * (3/4) (b^4 - a^4) / (b^3 - a^3), written without the cancellation of the differences as
 * (3/4) (b + a) (b^2 + a^2) / (b^2 + b a + a^2); spherical theta, measure sin(theta) dtheta:
 * [sin(t) - t cos(t)]_a^b / (cos a - cos b); Cartesian axes and phi (uniform measure): the face
 * midpoint.  The ghost faces are taken to mirror the interior faces about a non-periodic boundary
 * face and to repeat them across a periodic one (as the grid generators build them). */
static double xrec(const or_config *c, int d, int i)
{
    if (!c->centroid || c->geom != OR_SPH || d == 2)
        return xcen(c, d, i);
    /* a ghost cell is the image of an interior cell (reading 8), so its centroid is the image's,
     * moved like its faces: mirrored about the boundary face, or translated across a periodic axis */
    const int n = c->n[d];
    if (i < 0) {
        if (c->bc[d][0] == OR_BC_PERIODIC)
            return xrec(c, d, i + n) - (xf(c, d, n) - xf(c, d, 0));
        return 2.0 * xf(c, d, 0) - xrec(c, d, -1 - i);
    }
    if (i >= n) {
        if (c->bc[d][1] == OR_BC_PERIODIC)
            return xrec(c, d, i - n) + (xf(c, d, n) - xf(c, d, 0));
        return 2.0 * xf(c, d, n) - xrec(c, d, 2 * n - 1 - i);
    }
    const double a = xf(c, d, i), b = xf(c, d, i + 1);
    if (d == 0)
        return 0.75 * ((b + a) * (b * b + a * a)) / (b * b + b * a + a * a);
    return ((sin(b) - b * cos(b)) - (sin(a) - a * cos(a))) / (cos(a) - cos(b));
}

/* physical width of interior cell (i,j,k) along axis d (Sect. 3.1: dr, r dtheta, r sin(theta) dphi) */
static double width_interior(const or_config *c, int d, int i, int j, int k)
{
    if (c->geom == OR_CART) {
        int id = d == 0 ? i : (d == 1 ? j : k);
        return dxc(c, d, id);
    }
    if (d == 0)
        return dxc(c, 0, i);
    double rc = fabs(xcen(c, 0, i));
    if (d == 1)
        return rc * dxc(c, 1, j);
    return rc * fabs(sin(xcen(c, 1, j))) * dxc(c, 2, k);
}

/* spherical volume and surface elements (Sect. 3.1.1) */
static double sph_vr(const or_config *c, int i)
{
    double rm = xf(c, 0, i), rp = xf(c, 0, i + 1);
    return (rp * rp * rp - rm * rm * rm) / 3.0;
}
static double sph_hr(const or_config *c, int i)
{
    double rm = xf(c, 0, i), rp = xf(c, 0, i + 1);
    return 0.5 * (rp * rp - rm * rm);
}
static double sph_ct(const or_config *c, int j) { return cos(xf(c, 1, j)) - cos(xf(c, 1, j + 1)); }
static double sph_dV(const or_config *c, int i, int j, int k) { return sph_vr(c, i) * sph_ct(c, j) * dxc(c, 2, k); }
/* dS^r on face i (between cells i-1 and i) for column (j,k) */
static double sph_dSr(const or_config *c, int i, int j, int k)
{
    double r = xf(c, 0, i);
    return r * r * sph_ct(c, j) * dxc(c, 2, k);
}
/* dS^theta on face j for cell row (i,k) */
static double sph_dSt(const or_config *c, int i, int j, int k) { return sph_hr(c, i) * sin(xf(c, 1, j)) * dxc(c, 2, k); }
/* dS^phi on face k for (i,j) */
static double sph_dSp(const or_config *c, int i, int j) { return sph_hr(c, i) * dxc(c, 1, j); }

static double cell_volume(const or_config *c, int i, int j, int k)
{
    if (c->geom == OR_SPH)
        return sph_dV(c, i, j, k);
    return dxc(c, 0, i) * dxc(c, 1, j) * dxc(c, 2, k);
}

/* ------------------------------------------------------------------ boundaries */

/* image of index i on an axis of n cells (Sect. 3.2: periodic, null gradient, reflective) */
static int bc_map(int i, int n, int bclo, int bchi, int *flip)
{
    *flip = 0;
    if (i < 0) {
        if (bclo == OR_BC_PERIODIC)
            return i + n;
        if (bclo == OR_BC_TRANSMISSIVE)
            return 0;
        *flip = 1;
        return -1 - i;
    }
    if (i >= n) {
        if (bchi == OR_BC_PERIODIC)
            return i - n;
        if (bchi == OR_BC_TRANSMISSIVE)
            return n - 1;
        *flip = 1;
        return 2 * n - 1 - i;
    }
    return i;
}

/* physical width of any cell along axis d.  A ghost cell takes the widths of its image cell
 * (reading: ghost cells are images of interior cells in state, acceleration and geometry; in
 * spherical coordinates the transverse widths r dtheta and r sin(theta) dphi of a mirrored ghost
 * would otherwise differ from its image's and break the mirror symmetry at reflective walls). */
static double width(const or_config *c, int d, int i, int j, int k)
{
    int fl;
    int ii = c->ndim > 0 ? bc_map(i, c->n[0], c->bc[0][0], c->bc[0][1], &fl) : i;
    int jj = c->ndim > 1 ? bc_map(j, c->n[1], c->bc[1][0], c->bc[1][1], &fl) : j;
    int kk = c->ndim > 2 ? bc_map(k, c->n[2], c->bc[2][0], c->bc[2][1], &fl) : k;
    return width_interior(c, d, ii, jj, kk);
}

/* conserved state of cell (i,j,k), interior or ghost; behind a reflective wall the momentum
 * component normal to that wall changes sign */
static void fetch(const Ctx *x, const double *U, int i, int j, int k, double *q, int flip[3])
{
    const or_config *c = x->c;
    int ii = 0, jj = 0, kk = 0;
    flip[0] = flip[1] = flip[2] = 0;
    if (x->act[0])
        ii = bc_map(i, x->n[0], c->bc[0][0], c->bc[0][1], &flip[0]);
    if (x->act[1])
        jj = bc_map(j, x->n[1], c->bc[1][0], c->bc[1][1], &flip[1]);
    if (x->act[2])
        kk = bc_map(k, x->n[2], c->bc[2][0], c->bc[2][1], &flip[2]);
    long plane = (long)x->n[0] * x->n[1] * x->n[2];
    long off = ((long)kk * x->n[1] + jj) * x->n[0] + ii;
    for (int v = 0; v < x->nvar; v++)
        q[v] = U[v * plane + off];
    for (int d = 0; d < 3; d++)
        if (flip[d])
            q[1 + d] = -q[1 + d];
}

/* gravitational acceleration of cell (i,j,k).  A ghost cell carries the acceleration of its
 * image, with the component normal to a reflective wall negated like the momentum, so that
 * the ghost region is the exact mirror of the interior (reading: the paper does not say how
 * sources act in ghost cells). */
static void gravity_at(const Ctx *x, int i, int j, int k, double g[3])
{
    const or_config *c = x->c;
    g[0] = g[1] = g[2] = 0.0;
    if (c->gravity == OR_GRAV_NONE)
        return;
    int fl[3] = {0, 0, 0};
    int ii = 0;
    if (x->act[0])
        ii = bc_map(i, x->n[0], c->bc[0][0], c->bc[0][1], &fl[0]);
    if (x->act[1])
        (void)bc_map(j, x->n[1], c->bc[1][0], c->bc[1][1], &fl[1]);
    if (x->act[2])
        (void)bc_map(k, x->n[2], c->bc[2][0], c->bc[2][1], &fl[2]);
    if (c->gravity == OR_GRAV_UNIFORM) {
        for (int d = 0; d < 3; d++)
            g[d] = c->g0[d];
    } else {
        g[0] = x->gr[ii];
    }
    for (int d = 0; d < 3; d++)
        if (fl[d])
            g[d] = -g[d];
}

/* ------------------------------------------------------------------ EoS and fluxes */

/* ---- gas + radiation EoS (Sect. 2.3, eqs. eos_gp_rad_ein, eos_gp_rad): e = rho R T/(gamma-1) +
 * a T^4 and P = rho R T + a T^4 / 3.  The temperature follows from e (or, for primitive ->
 * conserved, from P) by Newton's method.  Both residuals are convex and increasing in T, so Newton
 * started from the smaller of the gas-only and the radiation-only temperatures (each an upper
 * bound of the root) decreases monotonically to it.  The iteration runs until a correction is at
 * most EOS_NEWTON_TOL of T, when quadratic convergence ((f''/2f') T <= 3/2 for both residuals)
 * leaves a relative error below 2e-16, and at most ten steps (the paper: about ten) (reading). */
#define EOS_NEWTON_STEPS 10
#define EOS_NEWTON_TOL 1e-8

static double t4(double T) { return (T * T) * (T * T); }

static double temp_from_e(const Ctx *x, double rho, double e)
{
    const double cg = (rho * x->R) / x->gm1;
    const double tg = e / cg, tr = sqrt(sqrt(e / x->arad));
    double T = tg < tr ? tg : tr;
    for (int it = 0; it < EOS_NEWTON_STEPS; it++) {
        const double f = cg * T + x->arad * t4(T) - e;
        const double fp = cg + 4.0 * x->arad * ((T * T) * T);
        const double dT = f / fp;
        T = T - dT;
        if (fabs(dT) <= EOS_NEWTON_TOL * T)
            break;
    }
    return T;
}

static double temp_from_p(const Ctx *x, double rho, double P)
{
    const double cg = rho * x->R;
    const double tg = P / cg, tr = sqrt(sqrt((3.0 * P) / x->arad));
    double T = tg < tr ? tg : tr;
    for (int it = 0; it < EOS_NEWTON_STEPS; it++) {
        const double f = cg * T + (x->arad * t4(T)) / 3.0 - P;
        const double fp = cg + (4.0 * x->arad * ((T * T) * T)) / 3.0;
        const double dT = f / fp;
        T = T - dT;
        if (fabs(dT) <= EOS_NEWTON_TOL * T)
            break;
    }
    return T;
}

/* primitives (rho, u1, u2, u3, P, f...) from conserved (Sect. 2.1; P from eq. eos_gas, or from
 * the temperature of the gas + radiation EoS, returned in *T if T is not NULL); the reciprocal
 * density is returned for the sound speed and the HLLC star energy */
static double prim_inv_t(const Ctx *x, const double *q, double *w, double *T)
{
    double rho = q[0];
    double inv = 1.0 / rho;
    double u1 = q[1] * inv, u2 = q[2] * inv, u3 = q[3] * inv;
    double ke = 0.5 * (q[1] * u1 + q[2] * u2 + q[3] * u3);
    w[0] = rho;
    w[1] = u1;
    w[2] = u2;
    w[3] = u3;
    if (x->eos == OR_EOS_GAS_RAD) {
        const double Tt = temp_from_e(x, rho, q[4] - ke);
        w[4] = (rho * x->R) * Tt + (x->arad * t4(Tt)) / 3.0;
        if (T)
            *T = Tt;
    } else {
        w[4] = x->gm1 * (q[4] - ke);
    }
    for (int v = 5; v < x->nvar - x->de; v++)
        w[v] = q[v] * inv;
    /* the internal energy is reconstructed per unit volume, like the pressure, so that it stays
     * constant across a contact (reading) */
    if (x->de)
        w[x->nvar - 1] = q[x->nvar - 1];
    return inv;
}

static double prim_inv(const Ctx *x, const double *q, double *w) { return prim_inv_t(x, q, w, NULL); }

static void prim(const Ctx *x, const double *q, double *w) { (void)prim_inv(x, q, w); }

/* sound speed of primitives w (reciprocal density inv, temperature T for the gas + radiation
 * EoS): eq. eos_gas, or eq. cs_gp_rad with alpha = P_r / P_g */
static double sound_speed(const Ctx *x, const double *w, double inv, double T)
{
    if (x->eos != OR_EOS_GAS_RAD)
        return sqrt(x->gamma * w[4] * inv);
    const double pg = (w[0] * x->R) * T;
    const double pr = (x->arad * t4(T)) / 3.0;
    const double al = pr / pg;
    const double num = x->gamma / x->gm1 + 20.0 * al + 16.0 * (al * al);
    const double den = 1.0 / x->gm1 + 12.0 * al;
    return sqrt((num / den) * (pg * inv));
}

static void cons(const Ctx *x, const double *w, double *q)
{
    double rho = w[0];
    q[0] = rho;
    q[1] = rho * w[1];
    q[2] = rho * w[2];
    q[3] = rho * w[3];
    if (x->eos == OR_EOS_GAS_RAD) {
        const double T = temp_from_p(x, rho, w[4]);
        const double e = ((rho * x->R) * T) / x->gm1 + x->arad * t4(T);
        q[4] = e + 0.5 * (q[1] * w[1] + q[2] * w[2] + q[3] * w[3]);
    } else {
        q[4] = w[4] * x->inv_gm1 + 0.5 * (q[1] * w[1] + q[2] * w[2] + q[3] * w[3]);
    }
    for (int v = 5; v < x->nvar - x->de; v++)
        q[v] = rho * w[v];
    if (x->de)
        q[x->nvar - 1] = w[x->nvar - 1];
}

/* pressure of density rho and internal energy e per unit volume (the internal-energy monitor's
 * P for its -P div(u) term): (gamma - 1) e, or from the temperature of the gas + radiation EoS */
static double pressure_from_e(const Ctx *x, double rho, double e)
{
    if (x->eos != OR_EOS_GAS_RAD)
        return x->gm1 * e;
    const double T = temp_from_e(x, rho, e);
    return (rho * x->R) * T + (x->arad * t4(T)) / 3.0;
}

static double pressure_of(const Ctx *x, const double *q)
{
    double w[MAXV];
    prim(x, q, w);
    return w[4];
}

/* physical flux along axis d of a state given by primitives w and conserved q */
static void phys_flux(int nvar, int de, int d, const double *w, const double *q, double *f)
{
    double un = w[1 + d];
    double mn = q[1 + d];
    f[0] = mn;
    f[1] = mn * w[1];
    f[2] = mn * w[2];
    f[3] = mn * w[3];
    f[1 + d] = f[1 + d] + w[4];
    f[4] = un * (q[4] + w[4]);
    for (int v = 5; v < nvar - de; v++)
        f[v] = mn * w[v];
    if (de)
        f[nvar - 1] = un * w[nvar - 1];  /* u e */
}

/* HLL and HLLC fluxes with Davis wave-speed estimates (Sect. 3.2; the solvers are those of
 * Toro's textbook, which the paper cites for them). */
/* uf (if not NULL) receives the velocity of the interface: the upwind side's normal velocity
 * outside the star region, the contact speed S* inside it (HLLC; HLL leaves it unset). */
static void riemann(int solver, int d, const Ctx *x, const double *qL, const double *qR, double *F,
                    double *uf)
{
    const int nvar = x->nvar, de = x->de;
    double wL[MAXV], wR[MAXV], fL[MAXV], fR[MAXV];
    double TL = 0.0, TR = 0.0;
    double iL = prim_inv_t(x, qL, wL, &TL);
    double iR = prim_inv_t(x, qR, wR, &TR);
    phys_flux(nvar, de, d, wL, qL, fL);
    phys_flux(nvar, de, d, wR, qR, fR);
    double rL = wL[0], rR = wR[0];
    double uL = wL[1 + d], uR = wR[1 + d];
    double pL = wL[4], pR = wR[4];
    /* sound speeds with the reciprocal densities formed above */
    double cL = sound_speed(x, wL, iL, TL);
    double cR = sound_speed(x, wR, iR, TR);
    double SL = fmin(uL - cL, uR - cR);
    double SR = fmax(uL + cL, uR + cR);
    if (SL >= 0.0) {
        for (int v = 0; v < nvar; v++)
            F[v] = fL[v];
        if (uf)
            *uf = uL;
        return;
    }
    if (solver == OR_HLL) {
        if (SR <= 0.0) {
            for (int v = 0; v < nvar; v++)
                F[v] = fR[v];
            return;
        }
        double inv = 1.0 / (SR - SL);
        for (int v = 0; v < nvar; v++)
            F[v] = (SR * fL[v] - SL * fR[v] + SL * SR * (qR[v] - qL[v])) * inv;
        return;
    }
    /* HLLC: contact speed S*, then the star state of the side the interface lies in */
    double mL = rL * (SL - uL);
    double mR = rR * (SR - uR);
    double Ss = (pR - pL + uL * mL - uR * mR) / (mL - mR);
    const double *q, *w, *f;
    double S, m, iv;
    if (Ss >= 0.0) {
        q = qL; w = wL; f = fL; S = SL; m = mL; iv = iL;
    } else if (SR > 0.0) {
        q = qR; w = wR; f = fR; S = SR; m = mR; iv = iR;
    } else {
        for (int v = 0; v < nvar; v++)
            F[v] = fR[v];
        if (uf)
            *uf = uR;
        return;
    }
    if (uf)
        *uf = Ss;
    double un = w[1 + d];
    double fac = m / (S - Ss);
    double us[MAXV];
    us[0] = fac;
    us[1] = fac * w[1];
    us[2] = fac * w[2];
    us[3] = fac * w[3];
    us[1 + d] = fac * Ss;
    us[4] = fac * (q[4] * iv + (Ss - un) * (Ss + w[4] / m));
    for (int v = 5; v < nvar - de; v++)
        us[v] = fac * w[v];
    if (de)
        us[nvar - 1] = fac * (w[nvar - 1] * iv);  /* rho* e / rho of the side */
    for (int v = 0; v < nvar; v++)
        F[v] = f[v] + S * (us[v] - q[v]);
}

void or_riemann_flux(int solver, int d, int nvar, double gamma, const double *qL, const double *qR,
                     double *flux)
{
    Ctx x;
    memset(&x, 0, sizeof x);
    x.nvar = nvar;
    x.gamma = gamma;
    x.gm1 = gamma - 1.0;
    x.inv_gm1 = 1.0 / x.gm1;
    x.eos = OR_EOS_GAS;
    riemann(solver, d, &x, qL, qR, flux, NULL);
}

/* ------------------------------------------------------------------ limiters */

/* Reconstruction coefficients of cell ic along axis d: the face increments are dl at the upper
 * face and kap dl at the lower one, dl = limiter(cm (w_i - w_{i-1}), cp (w_{i+1} - w_i)).  With
 * centres at the face midpoints both increments are (dx/2) sigma: cm, cp = (dx/2) over the centre
 * distances and kap = 1.  With volume centroids x_c they are (x+ - x_c) sigma and (x_c - x-) sigma,
 * sigma the limited slope over the centroid distances: the limiters are positively homogeneous,
 * so they act on the differences scaled by the upper extrapolation distance, and kap is the ratio
 * of the lower distance to the upper one. */
static void recon_coeffs(const or_config *c, int d, int ic, double *cm, double *cp, double *kap)
{
    if (c->centroid && c->geom == OR_SPH && d < 2) {
        const double xc = xrec(c, d, ic);
        const double hp = xf(c, d, ic + 1) - xc;
        *cm = hp / (xc - xrec(c, d, ic - 1));
        *cp = hp / (xrec(c, d, ic + 1) - xc);
        *kap = (xc - xf(c, d, ic)) / hp;
        return;
    }
    const double half = 0.5 * dxc(c, d, ic);
    *cm = half / (xcen(c, d, ic) - xcen(c, d, ic - 1));
    *cp = half / (xcen(c, d, ic + 1) - xcen(c, d, ic));
    *kap = 1.0;
}

/* Upper face increment from the differences dm = w_i - w_{i-1}, dp = w_{i+1} - w_i (the lower one is
 * kap times it).  About volume centroids an extrapolation distance can exceed half the distance
 * to the neighbouring centroid (next to r = 0 the centroid sits at 3/4 of the first cell), where
 * the textbook limiters would carry a face value beyond the neighbouring cell value; there the
 * increment is also bounded so that both face values stay between the neighbouring cell values:
 * |dl| <= |dp| and kap |dl| <= |dm| (reading).  With face-midpoint centres the bound never binds
 * for these limiters on uniform grids, and it is not applied. */
static double face_increment(const or_config *c, double cm, double cp, double kap, double dm, double dp)
{
    double dl = or_limiter(c->limiter, cm * dm, cp * dp);
    if (c->centroid && c->geom == OR_SPH && dl != 0.0) {
        const double bound = fmin(fabs(dp), fabs(dm) / kap);
        if (fabs(dl) > bound)
            dl = dl > 0.0 ? bound : -bound;
    }
    return dl;
}

/* limited half increment from the two one-sided half increments a, b.  The paper names the
 * limiters (Sect. 3.2) without printing them; these are the textbook forms.  All are
 * positively homogeneous of degree one, so applying them to slopes already scaled by
 * dr_i/2 gives (dr_i/2) sigma directly. */
double or_limiter(int lim, double a, double b)
{
    if (lim == OR_LIM_NONE)
        return 0.0;
    if (!(a * b > 0.0))
        return 0.0;
    if (lim == OR_LIM_MINMOD)
        return fabs(a) < fabs(b) ? a : b;
    if (lim == OR_LIM_VANALBADA)
        return a * b * (a + b) / (a * a + b * b);
    /* van Leer */
    return 2.0 * a * b / (a + b);
}

static double gelu(double z)
{
    return 0.5 * z * (1.0 + tanh(0.7978845608028654 * (z + 0.044715 * z * z * z)));
}

static double gelu_grad(double z)
{
    double k = 0.7978845608028654;
    double t = tanh(k * (z + 0.044715 * z * z * z));
    return 0.5 * (1.0 + t) + 0.5 * z * (1.0 - t * t) * k * (1.0 + 3.0 * 0.044715 * z * z);
}

double or_mlp_phi(const double *w, const double x[4])
{
    const double *W1 = w, *b1 = w + 128, *W2 = w + 160, *b2 = w + 1184, *w3 = w + 1216, *b3 = w + 1248;
    double h1[32], h2[32];
    for (int o = 0; o < 32; o++) {
        double s = b1[o];
        for (int i = 0; i < 4; i++)
            s += W1[o * 4 + i] * x[i];
        h1[o] = gelu(s);
    }
    for (int o = 0; o < 32; o++) {
        double s = b2[o];
        for (int i = 0; i < 32; i++)
            s += W2[o * 32 + i] * h1[i];
        h2[o] = gelu(s);
    }
    double z = b3[0];
    for (int i = 0; i < 32; i++)
        z += w3[i] * h2[i];
    return 2.0 / (1.0 + exp(-z));
}

/* learned limiter: d = the four undivided differences around the cell, cm/cp the geometric
 * factors turning them into half increments.  The network is skipped exactly where the TVD
 * region forces a zero slope, and replaced by van Leer where its output leaves the region
 * 0 <= phi <= min(2, 2r). */
double or_mlp_slope(const double *w, const double d[4], double cm, double cp)
{
    double dm = d[1], dp = d[2];
    if (!(dm * dp > 0.0))
        return 0.0;
    double s = 0.0;
    for (int i = 0; i < 4; i++)
        if (fabs(d[i]) > s)
            s = fabs(d[i]);
    double xin[4];
    for (int i = 0; i < 4; i++)
        xin[i] = d[i] / s;
    double phi = or_mlp_phi(w, xin);
    double a = cm * dm, b = cp * dp;
    double r = b / a;
    double lim = fmin(2.0, 2.0 * r);
    if (phi > lim)
        return 2.0 * a * b / (a + b);
    return phi * a;
}

double or_mlp_loss_grad(const double *w, int B, const double *x, const double *a, const double *t,
                        const double *wt, double *grad)
{
    const double *W1 = w, *b1 = w + 128, *W2 = w + 160, *b2 = w + 1184, *w3 = w + 1216, *b3 = w + 1248;
    double *gW1 = grad, *gb1 = grad + 128, *gW2 = grad + 160, *gb2 = grad + 1184, *gw3 = grad + 1216,
           *gb3 = grad + 1248;
    memset(grad, 0, sizeof(double) * OR_MLP_NPARAM);
    double wsum = 0.0;
    for (int b = 0; b < B; b++)
        wsum += wt[b];
    double loss = 0.0;
    for (int b = 0; b < B; b++) {
        const double *xb = x + 4 * b;
        double s1[32], h1[32], s2[32], h2[32];
        for (int o = 0; o < 32; o++) {
            double s = b1[o];
            for (int i = 0; i < 4; i++)
                s += W1[o * 4 + i] * xb[i];
            s1[o] = s;
            h1[o] = gelu(s);
        }
        for (int o = 0; o < 32; o++) {
            double s = b2[o];
            for (int i = 0; i < 32; i++)
                s += W2[o * 32 + i] * h1[i];
            s2[o] = s;
            h2[o] = gelu(s);
        }
        double z = b3[0];
        for (int i = 0; i < 32; i++)
            z += w3[i] * h2[i];
        double phi = 2.0 / (1.0 + exp(-z));
        double e = phi * a[b] - t[b];
        loss += wt[b] * e * e;
        double dphi = 2.0 * wt[b] * e * a[b] / wsum;
        double dz = dphi * phi * (1.0 - 0.5 * phi);
        gb3[0] += dz;
        double d2[32];
        for (int i = 0; i < 32; i++) {
            gw3[i] += dz * h2[i];
            d2[i] = dz * w3[i] * gelu_grad(s2[i]);
        }
        double dh1[32];
        for (int i = 0; i < 32; i++)
            dh1[i] = 0.0;
        for (int o = 0; o < 32; o++) {
            gb2[o] += d2[o];
            for (int i = 0; i < 32; i++) {
                gW2[o * 32 + i] += d2[o] * h1[i];
                dh1[i] += W2[o * 32 + i] * d2[o];
            }
        }
        for (int o = 0; o < 32; o++) {
            double d1 = dh1[o] * gelu_grad(s1[o]);
            gb1[o] += d1;
            for (int i = 0; i < 4; i++)
                gW1[o * 4 + i] += d1 * xb[i];
        }
    }
    return loss / wsum;
}

/* ------------------------------------------------------------------ setup */

static int ctx_init(Ctx *x, const or_config *c)
{
    memset(x, 0, sizeof *x);
    x->c = c;
    x->nvar = 5 + c->nscalar + (c->dual_energy ? 1 : 0);
    if (c->ndim < 1 || c->ndim > 3 || c->nscalar < 0 || x->nvar > MAXV)
        return OR_EINVAL;
    if (c->dual_energy && (c->riemann != OR_HLLC || !(c->de_eps >= 0.0)))
        return OR_EINVAL;
    if (c->limiter == OR_LIM_MLP && (c->ng < 3 || !c->mlp))
        return OR_EINVAL;
    /* (the learned limiter's TVD test is written for one extrapolation distance per cell) */
    if (c->centroid && c->limiter == OR_LIM_MLP)
        return OR_EINVAL;
    if (c->ng < 2)
        return OR_EINVAL;
    for (int d = 0; d < 3; d++) {
        x->act[d] = d < c->ndim;
        x->n[d] = c->n[d];
        if (x->act[d] && x->n[d] < c->ng)
            return OR_EINVAL;
        if (!x->act[d] && x->n[d] != 1)
            return OR_EINVAL;
    }
    if (c->gravity == OR_GRAV_UNIFORM && c->geom != OR_CART)
        return OR_EINVAL;
    if ((c->gravity == OR_GRAV_POINT || c->gravity == OR_GRAV_POINT_MONOPOLE) && c->geom != OR_SPH)
        return OR_EINVAL;
    x->gm1 = c->gamma - 1.0;
    x->inv_gm1 = 1.0 / x->gm1;
    x->de = c->dual_energy ? 1 : 0;
    x->gamma = c->gamma;
    x->eos = c->eos;
    x->R = c->eos_R;
    x->arad = c->eos_arad;
    if (c->eos != OR_EOS_GAS && c->eos != OR_EOS_GAS_RAD)
        return OR_EINVAL;
    if (c->eos == OR_EOS_GAS_RAD && (!(c->eos_R > 0.0) || !(c->eos_arad >= 0.0)))
        return OR_EINVAL;
    if (c->ni_heating) {
        if (c->ni_scalar < 0 || c->ni_scalar >= c->nscalar || !(c->ni_tau[0] > 0.0) ||
            !(c->ni_tau[1] > c->ni_tau[0]) || !(c->ni_m > 0.0) || !(c->ni_Q[0] >= 0.0) || !(c->ni_Q[1] >= 0.0) ||
            !isfinite(c->time))
            return OR_EINVAL;
    }
    return OR_OK;
}

/* ---- 56Ni decay heating (Sect. 2.4, eq. heating_ni): the energy source rho f_Ni times
 * lambda {[Q_Ni (tau_Co / tau_Ni - 1) - Q_Co] exp(-t / tau_Ni) + Q_Co exp(-t / tau_Co)},
 * lambda = 1 / (56 m_u (tau_Co - tau_Ni)), absorbed locally.  The rate per unit mass of 56Ni: */
double or_ni_rate(const or_config *c, double t)
{
    const double tn = c->ni_tau[0], tc = c->ni_tau[1];
    const double qn = c->ni_Q[0], qc = c->ni_Q[1];
    const double lam = 1.0 / (c->ni_m * (tc - tn));
    return lam * ((qn * (tc / tn - 1.0) - qc) * exp(-t / tn) + qc * exp(-t / tc));
}

/* radial gravity per interior shell; with the monopole term, the enclosed mass is
 * M(r_i) = (4 pi / Omega_w) (sum_{i'<i} m_i' + m_i / 2), m_i the shell mass inside the wedge
 * and Omega_w the wedge's solid angle (reading of eq. internal_gravity for a wedge: the wedge
 * stands for a spherically symmetric star, and half of the cell's own shell is enclosed at
 * its centre). */
static int shell_masses(const Ctx *x, const double *U, double *menc)
{
    const or_config *c = x->c;
    int nr = x->n[0], nt = x->n[1], np = x->n[2];
    double *m = (double *)calloc((size_t)nr, sizeof(double));
    if (!m)
        return OR_ENOMEM;
    double omega_t = 0.0, omega_p = 0.0;
    for (int j = 0; j < nt; j++)
        omega_t += sph_ct(c, j);
    for (int k = 0; k < np; k++)
        omega_p += dxc(c, 2, k);
    double omega = omega_t * omega_p;
    for (int k = 0; k < np; k++)
        for (int j = 0; j < nt; j++)
            for (int i = 0; i < nr; i++)
                m[i] += U[((long)k * nt + j) * nr + i] * sph_dV(c, i, j, k);
    double below = 0.0;
    double scale = 4.0 * M_PI / omega;
    for (int i = 0; i < nr; i++) {
        menc[i] = scale * (below + 0.5 * m[i]);
        below += m[i];
    }
    free(m);
    return OR_OK;
}

int or_enclosed_mass(const or_config *c, const double *U, double *menc)
{
    Ctx x;
    int st = ctx_init(&x, c);
    if (st)
        return st;
    if (c->geom != OR_SPH)
        return OR_EINVAL;
    return shell_masses(&x, U, menc);
}

static int gravity_setup(Ctx *x, const double *U)
{
    const or_config *c = x->c;
    if (c->gravity != OR_GRAV_POINT && c->gravity != OR_GRAV_POINT_MONOPOLE)
        return OR_OK;
    int nr = x->n[0];
    x->gr = (double *)calloc((size_t)nr, sizeof(double));
    double *menc = (double *)calloc((size_t)nr, sizeof(double));
    if (!x->gr || !menc) {
        free(menc);
        return OR_ENOMEM;
    }
    if (c->gravity == OR_GRAV_POINT_MONOPOLE) {
        int st = shell_masses(x, U, menc);
        if (st) {
            free(menc);
            return st;
        }
    }
    for (int i = 0; i < nr; i++) {
        double rc = xcen(c, 0, i);
        x->gr[i] = -(c->G * (c->Mc + menc[i])) / (rc * rc);
    }
    free(menc);
    return OR_OK;
}

/* gravity source S = (0, rho g, rho u.g, 0) (Sect. 2.2 with the acceleration pointing along g:
 * reading of the sign convention of eqs. momentum/energy, where g is also given pointing inward) */
static void grav_source(const Ctx *x, const double *q, const double g[3], double *S)
{
    for (int v = 0; v < x->nvar; v++)
        S[v] = 0.0;
    S[1] = q[0] * g[0];
    S[2] = q[0] * g[1];
    S[3] = q[0] * g[2];
    S[4] = q[1] * g[0] + q[2] * g[1] + q[3] * g[2];
}

/* rho > 0 and P > 0; for rho > 0 the latter is e = E - |m|^2/(2 rho) > 0, tested as
 * 2 rho E - |m|^2 > 0 */
static int positive_state(const double *q)
{
    double m2 = q[1] * q[1] + q[2] * q[2] + q[3] * q[3];
    return q[0] > 0.0 && 2.0 * q[0] * q[4] - m2 > 0.0;
}

static int nonphysical(const Ctx *x, const double *q)
{
    for (int v = 0; v < x->nvar; v++)
        if (!isfinite(q[v]))
            return 1;
    if (!(q[0] > 0.0))
        return 1;
    double p = pressure_of(x, q);
    return !(p > 0.0);
}

/* ------------------------------------------------------------------ the step */

typedef struct {
    int lo[3], ext[3];
} Box;

static long bidx(const Box *b, int i, int j, int k)
{
    return ((long)(k - b->lo[2]) * b->ext[1] + (j - b->lo[1])) * b->ext[0] + (i - b->lo[0]);
}

static int box_grow(Box *b, const int lo[3], const int hi[3], const int act[3], int s)
{
    for (int d = 0; d < 3; d++) {
        int g = act[d] ? s : 0;
        b->lo[d] = lo[d] - g;
        b->ext[d] = hi[d] - lo[d] + 2 * g;
    }
    return 0;
}

static long box_size(const Box *b) { return (long)b->ext[0] * b->ext[1] * b->ext[2]; }

/* e_k = |m|^2 / (2 rho) of a conserved state */
static double kinetic_energy(const double *q)
{
    return 0.5 * (q[1] * q[1] + q[2] * q[2] + q[3] * q[3]) / q[0];
}

double or_eos_state(const or_config *c, double rho, double e, double *P, double *cs)
{
    Ctx x;
    if (ctx_init(&x, c))
        return -1.0;
    double q[MAXV] = {0.0}, w[MAXV];
    q[0] = rho;
    q[4] = e;
    double T = 0.0;
    const double inv = prim_inv_t(&x, q, w, &T);
    if (x.eos != OR_EOS_GAS_RAD)
        T = 0.0;
    if (P)
        *P = w[4];
    if (cs)
        *cs = sound_speed(&x, w, inv, T);
    return T;
}

double or_eos_energy(const or_config *c, double rho, double P)
{
    Ctx x;
    if (ctx_init(&x, c))
        return -1.0;
    double w[MAXV] = {0.0}, q[MAXV];
    w[0] = rho;
    w[4] = P;
    cons(&x, w, q);
    return q[4];
}

double or_de_alpha(double e, double ek, double eps)
{
    /* Sect. 2.5: 1 for e >= eps e_k, (e / (eps e_k))^2 down to eps e_k / 10, 0 below */
    const double t = eps * ek;
    if (e >= t)
        return 1.0;
    if (e > t / 10.0) {
        const double r = e / t;
        return r * r;
    }
    return 0.0;
}

/* One step over the interior box [lo, hi).  fb (optional, the box's cell count) receives 1 for
 * every updated cell whose own half step fell back to first order (step D6 below), else 0. */
static int step_box(const or_config *c, const double *U, double dt, const int lo[3], const int hi[3],
                    double *out, unsigned char *fb)
{
    Ctx x;
    int st = ctx_init(&x, c);
    if (st)
        return st;
    const int nv = x.nvar;
    for (int d = 0; d < 3; d++)
        if (lo[d] < 0 || hi[d] > x.n[d] || lo[d] >= hi[d])
            return OR_EINVAL;
    st = gravity_setup(&x, U);
    if (st)
        return st;
    /* decay heating rates at the start and the middle of the step */
    const double h_n = c->ni_heating ? or_ni_rate(c, c->time) : 0.0;
    const double h_half = c->ni_heating ? or_ni_rate(c, c->time + 0.5 * dt) : 0.0;

    const int s = c->limiter == OR_LIM_MLP ? 3 : 2;
    Box bw, bp, bo;
    box_grow(&bw, lo, hi, x.act, s);   /* primitives */
    box_grow(&bp, lo, hi, x.act, 1);   /* half-step states */
    box_grow(&bo, lo, hi, x.act, 0);   /* updated cells */
    long nw = box_size(&bw), np = box_size(&bp);

    double *Q = (double *)malloc(sizeof(double) * nv * nw);   /* conserved, incl. ghosts */
    double *W = (double *)malloc(sizeof(double) * nv * nw);   /* primitives */
    double *FS = (double *)malloc(sizeof(double) * 6 * nv * np); /* [d][side][v][cell] */
    double *UH = (double *)malloc(sizeof(double) * nv * np);  /* U^n + dU (cell half step) */
    unsigned char *BAD = (unsigned char *)malloc((size_t)np);  /* fallback flag per half-step cell */
    if (!Q || !W || !FS || !UH || !BAD) {
        free(Q); free(W); free(FS); free(UH); free(BAD); free(x.gr);
        return OR_ENOMEM;
    }

    /* 1-2: boundary images and primitives */
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
    for (int k = bw.lo[2]; k < bw.lo[2] + bw.ext[2]; k++)
        for (int j = bw.lo[1]; j < bw.lo[1] + bw.ext[1]; j++)
            for (int i = bw.lo[0]; i < bw.lo[0] + bw.ext[0]; i++) {
                double q[MAXV], w[MAXV];
                int fl[3];
                fetch(&x, U, i, j, k, q, fl);
                prim(&x, q, w);
                long id = bidx(&bw, i, j, k);
                for (int v = 0; v < nv; v++) {
                    Q[v * nw + id] = q[v];
                    W[v * nw + id] = w[v];
                }
            }

    /* 3-4: reconstruction and the Hancock half step for every cell whose face states feed a
     * flux of the box */
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
    for (int k = bp.lo[2]; k < bp.lo[2] + bp.ext[2]; k++)
        for (int j = bp.lo[1]; j < bp.lo[1] + bp.ext[1]; j++)
            for (int i = bp.lo[0]; i < bp.lo[0] + bp.ext[0]; i++) {
                long iw = bidx(&bw, i, j, k);
                long ip = bidx(&bp, i, j, k);
                int cidx[3] = {i, j, k};
                double w[MAXV], q[MAXV];
                for (int v = 0; v < nv; v++) {
                    w[v] = W[v * nw + iw];
                    q[v] = Q[v * nw + iw];
                }
                double um[3][MAXV], up[3][MAXV];
                double du[MAXV];
                for (int v = 0; v < nv; v++)
                    du[v] = 0.0;
                for (int d = 0; d < 3; d++) {
                    if (!x.act[d])
                        continue;
                    int e[3] = {0, 0, 0};
                    e[d] = 1;
                    long im = bidx(&bw, i - e[0], j - e[1], k - e[2]);
                    long ipp = bidx(&bw, i + e[0], j + e[1], k + e[2]);
                    double cm, cp, kap;
                    recon_coeffs(c, d, cidx[d], &cm, &cp, &kap);
                    double wm[MAXV], wp[MAXV];
                    for (int v = 0; v < nv; v++) {
                        double dl;
                        if (c->limiter == OR_LIM_MLP) {
                            long imm = bidx(&bw, i - 2 * e[0], j - 2 * e[1], k - 2 * e[2]);
                            long ip2 = bidx(&bw, i + 2 * e[0], j + 2 * e[1], k + 2 * e[2]);
                            double dd[4] = {W[v * nw + im] - W[v * nw + imm], w[v] - W[v * nw + im],
                                            W[v * nw + ipp] - w[v], W[v * nw + ip2] - W[v * nw + ipp]};
                            dl = or_mlp_slope(c->mlp, dd, cm, cp);
                        } else {
                            dl = face_increment(c, cm, cp, kap, w[v] - W[v * nw + im], W[v * nw + ipp] - w[v]);
                        }
                        wm[v] = w[v] - kap * dl;
                        wp[v] = w[v] + dl;
                    }
                    cons(&x, wm, um[d]);
                    cons(&x, wp, up[d]);
                    double fm[MAXV], fp[MAXV];
                    phys_flux(nv, x.de, d, wm, um[d], fm);
                    phys_flux(nv, x.de, d, wp, up[d], fp);
                    double lam = dt / (2.0 * width(c, d, i, j, k));
                    for (int v = 0; v < nv; v++)
                        du[v] += lam * (fm[v] - fp[v]);
                    /* internal energy: - (dt/2) P div(u) with the reconstructed face velocities
                     * and the pressure of the cell's e ((gamma - 1) e, or through the gas + radiation
                     * EoS; eq. pressure_fix; reading) */
                    if (c->dual_energy)
                        du[nv - 1] += lam * (pressure_from_e(&x, q[0], q[nv - 1]) * (wm[1 + d] - wp[1 + d]));
                }
                if (c->gravity != OR_GRAV_NONE) {
                    double g[3], S[MAXV];
                    gravity_at(&x, i, j, k, g);
                    grav_source(&x, q, g, S);
                    for (int v = 0; v < nv; v++)
                        du[v] += 0.5 * dt * S[v];
                }
                /* decay heating of the state at t^n over the half step; it heats the gas, so the
                 * monitored internal energy takes it too (reading) */
                if (c->ni_heating) {
                    const double sh = h_n * q[5 + c->ni_scalar];
                    du[4] += 0.5 * dt * sh;
                    if (c->dual_energy)
                        du[nv - 1] += 0.5 * dt * sh;
                }
                /* positivity fallback (reading; not in the paper): a cell whose half-step face
                 * states are not physical is advanced at first order (zero slopes, no half step) */
                int bad = 0;
                for (int d = 0; d < 3 && !bad; d++) {
                    if (!x.act[d])
                        continue;
                    double a[MAXV], b[MAXV];
                    for (int v = 0; v < nv; v++) {
                        a[v] = um[d][v] + du[v];
                        b[v] = up[d][v] + du[v];
                    }
                    if (!positive_state(a) || !positive_state(b))
                        bad = 1;
                }
                BAD[ip] = (unsigned char)bad;
                if (bad) {
                    double q0[MAXV];
                    cons(&x, w, q0);
                    for (int d = 0; d < 3; d++)
                        for (int v = 0; v < nv; v++) {
                            FS[((d * 2 + 0) * nv + v) * np + ip] = q0[v];
                            FS[((d * 2 + 1) * nv + v) * np + ip] = q0[v];
                        }
                    for (int v = 0; v < nv; v++)
                        UH[v * np + ip] = q[v];
                } else {
                    for (int d = 0; d < 3; d++) {
                        if (!x.act[d])
                            continue;
                        for (int v = 0; v < nv; v++) {
                            FS[((d * 2 + 0) * nv + v) * np + ip] = um[d][v] + du[v];
                            FS[((d * 2 + 1) * nv + v) * np + ip] = up[d][v] + du[v];
                        }
                    }
                    for (int v = 0; v < nv; v++)
                        UH[v * np + ip] = q[v] + du[v];
                }
            }

    /* 5-6: fluxes at the faces of each updated cell, then the conservative update */
    int nonphys = 0;
    long nbo = box_size(&bo);
#ifdef _OPENMP
#pragma omp parallel for schedule(static) reduction(| : nonphys)
#endif
    for (int k = lo[2]; k < hi[2]; k++)
        for (int j = lo[1]; j < hi[1]; j++)
            for (int i = lo[0]; i < hi[0]; i++) {
                int cidx[3] = {i, j, k};
                long iw = bidx(&bw, i, j, k);
                long ip = bidx(&bp, i, j, k);
                double acc[MAXV], Fm[3][MAXV], Fp[3][MAXV];
                double ufm = 0.0, ufp = 0.0;  /* interface velocities (internal energy) */
                /* P of the cell's half-step internal energy, like the other sources (reading) */
                const double pe =
                    c->dual_energy ? pressure_from_e(&x, UH[0 * np + ip], UH[(nv - 1) * np + ip]) : 0.0;
                for (int v = 0; v < nv; v++)
                    acc[v] = Q[v * nw + iw];
                for (int d = 0; d < 3; d++) {
                    if (!x.act[d])
                        continue;
                    int e[3] = {0, 0, 0};
                    e[d] = 1;
                    long ipm = bidx(&bp, i - e[0], j - e[1], k - e[2]);
                    long ipq = bidx(&bp, i + e[0], j + e[1], k + e[2]);
                    double L[MAXV], R[MAXV];
                    /* left face: right state of the lower neighbour, left state of this cell */
                    for (int v = 0; v < nv; v++) {
                        L[v] = FS[((d * 2 + 1) * nv + v) * np + ipm];
                        R[v] = FS[((d * 2 + 0) * nv + v) * np + ip];
                    }
                    riemann(c->riemann, d, &x, L, R, Fm[d], &ufm);
                    for (int v = 0; v < nv; v++) {
                        L[v] = FS[((d * 2 + 1) * nv + v) * np + ip];
                        R[v] = FS[((d * 2 + 0) * nv + v) * np + ipq];
                    }
                    /* the upper face's flux is the next cell's lower-face flux once more */
                    OR_REPEATED_WORK(1);
                    riemann(c->riemann, d, &x, L, R, Fp[d], &ufp);
                    OR_REPEATED_WORK(0);
                    if (c->geom == OR_CART) {
                        double mu = dt / dxc(c, d, cidx[d]);
                        for (int v = 0; v < nv; v++)
                            acc[v] += mu * (Fm[d][v] - Fp[d][v]);
                        /* internal energy: - dt P div(u) with the interface velocities */
                        if (c->dual_energy)
                            acc[nv - 1] += mu * (pe * (ufm - ufp));
                    } else {
                        double dSm, dSp;
                        if (d == 0) {
                            dSm = sph_dSr(c, i, j, k);
                            dSp = sph_dSr(c, i + 1, j, k);
                        } else if (d == 1) {
                            dSm = sph_dSt(c, i, j, k);
                            dSp = sph_dSt(c, i, j + 1, k);
                        } else {
                            dSm = sph_dSp(c, i, j);
                            dSp = dSm;
                        }
                        double kv = dt / sph_dV(c, i, j, k);
                        for (int v = 0; v < nv; v++)
                            acc[v] += kv * (Fm[d][v] * dSm - Fp[d][v] * dSp);
                        if (c->dual_energy)
                            acc[nv - 1] += kv * (pe * (ufm * dSm - ufp * dSp));
                    }
                }
                /* sources, evaluated with the cell's half-step state */
                double uh[MAXV], S[MAXV];
                for (int v = 0; v < nv; v++) {
                    uh[v] = UH[v * np + ip];
                    S[v] = 0.0;
                }
                int have_src = 0;
                if (c->gravity != OR_GRAV_NONE) {
                    double g[3];
                    gravity_at(&x, i, j, k, g);
                    grav_source(&x, uh, g, S);
                    have_src = 1;
                }
                if (c->geom == OR_SPH) {
                    /* Sect. 3.1.2: the products [rho u_phi u_r], [rho u_phi u_theta], [rho u_theta u_r]
                     * on faces are the Riemann fluxes of the transverse momenta (eq. source_terms_1,
                     * taken for theta as the paper says).  The cot(theta) and 1/r terms that the
                     * paper writes for rho u^2 are taken with the pressure included,
                     * X = rho u^2 + P from the face fluxes, times (dS+ - dS-)/dV, which also supplies
                     * the geometric pressure terms omitted in the printed equations (reading). */
                    double dV = sph_dV(c, i, j, k);
                    double rm = xf(c, 0, i), rp = xf(c, 0, i + 1);
                    double dSrm = sph_dSr(c, i, j, k), dSrp = sph_dSr(c, i + 1, j, k);
                    double cr = (rp - rm) / ((rp + rm) * dV);
                    double grg = (dSrp - dSrm) / dV;
                    double pu = pressure_of(&x, uh);
                    double Xt, Xp, Tt = 0.0, gtg = 0.0;
                    if (x.act[1]) {
                        double sm = sin(xf(c, 1, j)), sp = sin(xf(c, 1, j + 1));
                        double dStm = sph_dSt(c, i, j, k), dStp = sph_dSt(c, i, j + 1, k);
                        double ct = (sp - sm) / ((sp + sm) * dV);
                        gtg = (dStp - dStm) / dV;
                        Xt = 0.5 * (Fm[1][2] + Fp[1][2]);
                        Tt = -ct * (Fp[1][3] * dStp + Fm[1][3] * dStm);
                    } else {
                        Xt = uh[2] * (uh[2] / uh[0]) + pu;
                    }
                    if (x.act[2])
                        Xp = 0.5 * (Fm[2][3] + Fp[2][3]);
                    else
                        Xp = uh[3] * (uh[3] / uh[0]) + pu;
                    double Trt = -cr * (Fp[0][2] * dSrp + Fm[0][2] * dSrm);
                    double Trp = -cr * (Fp[0][3] * dSrp + Fm[0][3] * dSrm);
                    S[1] = S[1] + 0.5 * (Xt + Xp) * grg;
                    S[2] = S[2] + (Trt + Xp * gtg);
                    S[3] = S[3] + (Trp + Tt);
                    have_src = 1;
                }
                /* decay heating of the half-step state at t^n + dt/2 (reading: the midpoint in time,
                 * like the other sources) */
                if (c->ni_heating) {
                    const double sh = h_half * uh[5 + c->ni_scalar];
                    S[4] = S[4] + sh;
                    if (c->dual_energy)
                        S[nv - 1] = S[nv - 1] + sh;
                    have_src = 1;
                }
                if (have_src)
                    for (int v = 0; v < nv; v++)
                        acc[v] += dt * S[v];
                /* internal energy (Sect. 2.5): e_new = e + alpha d1e + (1 - alpha) d2e, d1e from the
                 * total energy (E - |m|^2 / (2 rho) of the updated cell), d2e from eq. pressure_fix
                 * (acc above); alpha from e and e_k of the cell at time n (reading) */
                if (c->dual_energy) {
                    const double en = Q[(nv - 1) * nw + iw];
                    double qn[5];
                    for (int v = 0; v < 5; v++)
                        qn[v] = Q[v * nw + iw];
                    const double alpha = or_de_alpha(en, kinetic_energy(qn), c->de_eps);
                    const double d1 = (acc[4] - kinetic_energy(acc)) - en;
                    const double d2 = acc[nv - 1] - en;
                    acc[nv - 1] = en + alpha * d1 + (1.0 - alpha) * d2;
                }
                if (nonphysical(&x, acc))
                    nonphys = 1;
                long io = bidx(&bo, i, j, k);
                for (int v = 0; v < nv; v++)
                    out[v * nbo + io] = acc[v];
                if (fb)
                    fb[io] = BAD[ip];
            }

    free(Q);
    free(W);
    free(FS);
    free(UH);
    free(BAD);
    free(x.gr);
    return nonphys ? OR_ENONPHYS : OR_OK;
}

int or_step_box(const or_config *c, const double *U, double dt, const int lo[3], const int hi[3],
                double *out)
{
    return step_box(c, U, dt, lo, hi, out, NULL);
}

int or_step_box_fb(const or_config *c, const double *U, double dt, const int lo[3], const int hi[3],
                   double *out, unsigned char *fb)
{
    return step_box(c, U, dt, lo, hi, out, fb);
}

int or_face_states(const or_config *c, const double *U, int i, int j, int k, int d, double *wm, double *wp)
{
    Ctx x;
    int st = ctx_init(&x, c);
    if (st)
        return st;
    if (d < 0 || d >= 3 || !x.act[d] || c->limiter == OR_LIM_MLP)
        return OR_EINVAL;
    int e[3] = {0, 0, 0};
    e[d] = 1;
    int cidx[3] = {i, j, k};
    double q[3][MAXV], w[3][MAXV];
    for (int s = 0; s < 3; s++) {
        int fl[3];
        fetch(&x, U, i + (s - 1) * e[0], j + (s - 1) * e[1], k + (s - 1) * e[2], q[s], fl);
        prim(&x, q[s], w[s]);
    }
    double cm, cp, kap;
    recon_coeffs(c, d, cidx[d], &cm, &cp, &kap);
    for (int v = 0; v < x.nvar; v++) {
        const double dl = face_increment(c, cm, cp, kap, w[1][v] - w[0][v], w[2][v] - w[1][v]);
        wm[v] = w[1][v] - kap * dl;
        wp[v] = w[1][v] + dl;
    }
    return OR_OK;
}

int or_step(const or_config *c, const double *U, double dt, double *Unew)
{
    int lo[3] = {0, 0, 0};
    int hi[3] = {c->n[0], c->n[1], c->n[2]};
    return or_step_box(c, U, dt, lo, hi, Unew);
}

/* The CFL step of the cells of the box [lo, hi) (the whole grid in or_compute_dt) */
static int compute_dt_box(const or_config *c, const double *U, const int lo[3], const int hi[3], double *dt)
{
    Ctx x;
    int st = ctx_init(&x, c);
    if (st)
        return st;
    for (int d = 0; d < 3; d++)
        if (lo[d] < 0 || hi[d] > x.n[d] || lo[d] >= hi[d]) {
            free(x.gr);
            return OR_EINVAL;
        }
    double smax = 0.0;
    int bad = 0;
    /* (a maximum does not depend on the order of its terms: any thread count gives the same dt) */
#ifdef _OPENMP
#pragma omp parallel for schedule(static) reduction(max : smax) reduction(| : bad)
#endif
    for (int k = lo[2]; k < hi[2]; k++)
        for (int j = lo[1]; j < hi[1]; j++)
            for (int i = lo[0]; i < hi[0]; i++) {
                double q[MAXV], w[MAXV];
                int fl[3];
                fetch(&x, U, i, j, k, q, fl);
                if (nonphysical(&x, q)) {
                    bad = 1;
                    continue;
                }
                double T = 0.0;
                double inv = prim_inv_t(&x, q, w, &T);
                double cs = sound_speed(&x, w, inv, T);
                double s = 0.0;
                for (int d = 0; d < 3; d++)
                    if (x.act[d])
                        s += (fabs(w[1 + d]) + cs) / width(c, d, i, j, k);
                if (s > smax)
                    smax = s;
            }
    free(x.gr);
    *dt = c->cfl / smax;
    return bad ? OR_ENONPHYS : OR_OK;
}

int or_compute_dt(const or_config *c, const double *U, double *dt)
{
    const int lo[3] = {0, 0, 0};
    const int hi[3] = {c->n[0], c->n[1], c->n[2]};
    return compute_dt_box(c, U, lo, hi, dt);
}

int or_compute_dt_box(const or_config *c, const double *U, const int lo[3], const int hi[3], double *dt)
{
    return compute_dt_box(c, U, lo, hi, dt);
}

/* ---- grid shift (Sect. 3.1.1, moving grid): every face of axis 0 moves by delta and the state
 * is carried over conservatively.  Reading: the paper only says that the grid can be shifted
 * along an axis to follow the ejecta.  Each old cell holds the linear profile U_m + s_m (x - c_m)
 * of its conserved variables, c_m its volume centroid (so the profile integrates to the cell's
 * content), s_m the minmod of the differences to its neighbours over the centroid distances; a new
 * cell takes the integral of the profiles over its overlap with the old cells (|delta| at most
 * the narrowest cell, so at most two), with the volume measure dx (Cartesian) or r^2 dr
 * (spherical: the angular factor is common to the row), divided by its new volume.  Material
 * beyond the old grid comes from the boundary images; what leaves the grid is dropped.  A cell
 * whose result has rho <= 0, P <= 0 (or e <= 0 with the monitor) takes the piecewise-constant
 * remap instead, a convex combination of the old cells, which keeps them positive. */
static double shift_m0(int sph, double a, double b)
{
    return sph ? (b * b * b - a * a * a) / 3.0 : b - a;
}

static double shift_m1(int sph, double a, double b)
{
    return sph ? (b * b * b * b - a * a * a * a) / 4.0 : 0.5 * (b * b - a * a);
}

static double minmod(double a, double b)
{
    if (a * b <= 0.0)
        return 0.0;
    return fabs(a) < fabs(b) ? a : b;
}

int or_shift_grid(const or_config *c, const double *U, double delta, double *Unew)
{
    Ctx x;
    int st = ctx_init(&x, c);
    if (st)
        return st;
    const int n = x.n[0], nv = x.nvar, sph = c->geom == OR_SPH;
    for (int i = -2; i < n + 2; i++)
        if (!(fabs(delta) <= dxc(c, 0, i)))
            return OR_EINVAL;
    if (sph && !(xf(c, 0, 0) + delta >= 0.0))
        return OR_EINVAL;
    const long plane = (long)x.n[0] * x.n[1] * x.n[2];
    for (int k = 0; k < x.n[2]; k++)
        for (int j = 0; j < x.n[1]; j++)
            for (int i = 0; i < n; i++) {
                const double a = xf(c, 0, i) + delta, b = xf(c, 0, i + 1) + delta;
                const double vnew = shift_m0(sph, a, b);
                /* the old cells under the new one */
                const int m0 = delta > 0.0 ? i : i - 1;
                double out[2][MAXV];  /* [0]: linear profiles, [1]: constant profiles */
                for (int v = 0; v < nv; v++)
                    out[0][v] = out[1][v] = 0.0;
                for (int m = m0; m <= m0 + 1; m++) {
                    const double lo = fmax(a, xf(c, 0, m)), hi = fmin(b, xf(c, 0, m + 1));
                    if (!(hi > lo))
                        continue;
                    double q[3][MAXV], cm[3];
                    for (int s = 0; s < 3; s++) {
                        int fl[3];
                        fetch(&x, U, m - 1 + s, j, k, q[s], fl);
                        const double fa = xf(c, 0, m - 1 + s), fb = xf(c, 0, m + s);
                        cm[s] = shift_m1(sph, fa, fb) / shift_m0(sph, fa, fb);
                    }
                    const double w0 = shift_m0(sph, lo, hi), w1 = shift_m1(sph, lo, hi);
                    for (int v = 0; v < nv; v++) {
                        const double sl = minmod((q[1][v] - q[0][v]) / (cm[1] - cm[0]),
                                                 (q[2][v] - q[1][v]) / (cm[2] - cm[1]));
                        out[0][v] += q[1][v] * w0 + sl * (w1 - cm[1] * w0);
                        out[1][v] += q[1][v] * w0;
                    }
                }
                const double *r = out[0];
                const double m2 = r[1] * r[1] + r[2] * r[2] + r[3] * r[3];
                const int ok = r[0] > 0.0 && 2.0 * r[0] * r[4] - m2 > 0.0 && (!x.de || r[nv - 1] > 0.0);
                const long off = ((long)k * x.n[1] + j) * x.n[0] + i;
                for (int v = 0; v < nv; v++)
                    Unew[v * plane + off] = out[ok ? 0 : 1][v] / vnew;
            }
    return OR_OK;
}

/* threads the step's loops run on: OpenMP's team size in the OpenMP build, 1 in the serial one */
int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void or_totals(const or_config *c, const double *U, double *tot)
{
    /* every field, the monitored internal energy included */
    int nv = 5 + c->nscalar + (c->dual_energy ? 1 : 0);
    long plane = (long)c->n[0] * c->n[1] * c->n[2];
    for (int v = 0; v < nv; v++) {
        double s = 0.0;
        for (int k = 0; k < c->n[2]; k++)
            for (int j = 0; j < c->n[1]; j++)
                for (int i = 0; i < c->n[0]; i++)
                    s += U[v * plane + ((long)k * c->n[1] + j) * c->n[0] + i] * cell_volume(c, i, j, k);
        tot[v] = s;
    }
}

/* ------------------------------------------------------------------ learned-limiter samples */

static void restrict_prim(const double *U, long plane, long row_off, int ratio, int i, double gm1, double *w)
{
    double q[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int f = 0; f < ratio; f++)
        for (int v = 0; v < 5; v++)
            q[v] += U[v * plane + row_off + (long)i * ratio + f];
    for (int v = 0; v < 5; v++)
        q[v] = q[v] / ratio;
    double inv = 1.0 / q[0];
    w[0] = q[0];
    w[1] = q[1] * inv;
    w[2] = q[2] * inv;
    w[3] = q[3] * inv;
    w[4] = gm1 * (q[4] - 0.5 * (q[1] * w[1] + q[2] * w[2] + q[3] * w[3]));
}

void or_mlp_features(const double *U, int nrows, int nf, int ratio, double gamma, double *x, double *a,
                     double *t, double *wt)
{
    int nc = nf / ratio;
    long plane = (long)nrows * nf;
    double gm1 = gamma - 1.0;
    for (int row = 0; row < nrows; row++)
        for (int i = 0; i < nc; i++) {
            long row_off = (long)row * nf;
            double W[5][5] = {{0.0}}; /* initialised: gcc 11 -O2 mis-handles it conditionally set */
            int inside = i >= 2 && i <= nc - 3;
            if (inside)
                for (int s = 0; s < 5; s++)
                    restrict_prim(U, plane, row_off, ratio, i - 2 + s, gm1, W[s]);
            for (int v = 0; v < 5; v++) {
                long e = ((long)row * nc + i) * 5 + v;
                for (int k = 0; k < 4; k++)
                    x[4 * e + k] = 0.0;
                a[e] = t[e] = wt[e] = 0.0;
                if (!inside)
                    continue;
                double d[4] = {W[1][v] - W[0][v], W[2][v] - W[1][v], W[3][v] - W[2][v], W[4][v] - W[3][v]};
                double s = 0.0;
                for (int k = 0; k < 4; k++)
                    if (fabs(d[k]) > s)
                        s = fabs(d[k]);
                if (!(d[1] * d[2] > 0.0 && s > 0.0))
                    continue;
                /* least-squares slope of the fine primitive values at fine-cell offsets f - (ratio-1)/2 */
                double num = 0.0, den = 0.0, mid = 0.5 * (ratio - 1);
                for (int f = 0; f < ratio; f++) {
                    double q[5], w[5];
                    for (int u = 0; u < 5; u++)
                        q[u] = U[u * plane + row_off + (long)i * ratio + f];
                    double inv = 1.0 / q[0];
                    w[0] = q[0];
                    w[1] = q[1] * inv;
                    w[2] = q[2] * inv;
                    w[3] = q[3] * inv;
                    w[4] = gm1 * (q[4] - 0.5 * (q[1] * w[1] + q[2] * w[2] + q[3] * w[3]));
                    num += (f - mid) * w[v];
                    den += (f - mid) * (f - mid);
                }
                double slope = ratio * num / den;
                for (int k = 0; k < 4; k++)
                    x[4 * e + k] = d[k] / s;
                a[e] = d[1] / s;
                t[e] = slope / s;
                wt[e] = 1.0;
            }
        }
}
