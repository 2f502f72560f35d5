/*
 * FP64 CPU oracle for one MUSCL-Hancock step of the HERACLES++ Godunov scheme.
 *
 * TEST INFRASTRUCTURE ONLY.  This is the plain, slow, single-threaded
 * reference that the HIP library is checked against.  Built with OpenMP (liboracle_omp.so), the
 * step's cell loops run over z planes in parallel; every cell is computed by the same expressions
 * and the time step is a maximum, so the results are bit for bit those of the serial build.  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg may load it; the
 * product path never does.  It shares no code, header or table with the HIP
 * library.
 *
 * Units of the paper followed here:
 *   Sect. 2.1 (eqs. continuity, momentum, energy with its heating term, passive scalar),
 *   Sect. 2.2 (uniform / point / enclosed-mass gravity), Sect. 2.3 (ideal-gas and gas + radiation
 *   EoS), Sect. 2.4 (56Ni decay heating, eq. heating_ni), Sect. 2.5 (internal-energy monitor),
 *   Sect. 3.1.1 (mesh, dS, dV), Sect. 3.1.2 (spherical momentum sources,
 *   eq. source_terms_1 and the theta counterpart), Sect. 3.2 (slope-limited
 *   reconstruction, Hancock half step, Godunov update eq. godunov, HLL/HLLC,
 *   boundary conditions).
 *
 * Pins (tests/test_oracle_*.py): limiters against closed forms and the TVD region; HLL/HLLC
 * against consistency, exact contact resolution, mirror symmetry and the exact Godunov flux for
 * weak waves; the whole step against the exact Sod solution (convergence), first-order Godunov by
 * brute force, conservation, free stream, mirror/permutation symmetry, 1D data in 3D, free fall
 * under uniform gravity, a static spherical wedge, discrete angular momentum, the closed-form
 * enclosed mass and the Sedov-Taylor shock radius; the MLP against torch and finite differences;
 * the internal-energy monitor's blend branches and second-order agreement with the total energy;
 * the gas + radiation EoS against round trips, its limits and the isentropic sound speed; the
 * 56Ni heating rate against the decay chain's populations, its total release and second-order
 * convergence of a heated flow.
 */
#ifndef HYDRO_ORACLE_H
#define HYDRO_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

enum { OR_CART = 0, OR_SPH = 1 };
enum { OR_HLL = 0, OR_HLLC = 1 };
enum { OR_LIM_NONE = 0, OR_LIM_MINMOD = 1, OR_LIM_VANLEER = 2, OR_LIM_VANALBADA = 3, OR_LIM_MLP = 4 };
enum { OR_BC_PERIODIC = 0, OR_BC_TRANSMISSIVE = 1, OR_BC_REFLECTIVE = 2 };
enum { OR_GRAV_NONE = 0, OR_GRAV_UNIFORM = 1, OR_GRAV_POINT = 2, OR_GRAV_POINT_MONOPOLE = 3 };
enum { OR_EOS_GAS = 0, OR_EOS_GAS_RAD = 1 };
enum { OR_OK = 0, OR_EINVAL = -1, OR_ENONPHYS = -3, OR_ENOMEM = -5 };

#define OR_MLP_NPARAM 1249   /* 4*32+32 + 32*32+32 + 32+1 */

typedef struct {
    int ndim;                 /* 1..3 active axes (x1, x2, x3 in that order) */
    int geom;                 /* OR_CART or OR_SPH */
    int n[3];                 /* interior cells per axis (1 for inactive axes) */
    int ng;                   /* ghost layers (2; 3 for the MLP limiter) */
    const double *faces[3];   /* active: n+1+2ng faces incl. ghost faces; inactive: 2 faces */
    int nscalar;
    double gamma;
    double cfl;
    int riemann;
    int limiter;
    int bc[3][2];
    int gravity;
    double g0[3];
    double G, Mc;
    const double *mlp;        /* OR_MLP_NPARAM weights, W1[32][4] b1 W2[32][32] b2 w3[32] b3 */
    int dual_energy;          /* 1: the last field is the monitored internal energy e (Sect. 2.5,
                                 eq. pressure_fix); needs HLLC */
    double de_eps;            /* the criterion epsilon of the blend factor alpha (paper: 1e-6) */
    int eos;                  /* OR_EOS_GAS (eq. eos_gas) or OR_EOS_GAS_RAD (eqs. eos_gp_rad_ein,
                                 eos_gp_rad, cs_gp_rad) */
    double eos_R;             /* gas + radiation: specific gas constant k_b / (mu m_u) */
    double eos_arad;          /* gas + radiation: radiation constant a_r */
    int ni_heating;           /* 1: 56Ni -> 56Co -> 56Fe decay heating (Sect. 2.4, eq. heating_ni)
                                 added to E (and to e with dual_energy) */
    int ni_scalar;            /* the passive scalar that carries rho f_Ni (0 .. nscalar-1) */
    double ni_Q[2];           /* energy released per decay of 56Ni and of 56Co */
    double ni_tau[2];         /* lifetimes tau_Ni < tau_Co */
    double ni_m;              /* mass of one 56Ni nucleus (56 m_u) */
    double time;              /* time t^n at the start of the step (the decay clock) */
    int centroid;             /* 1: reconstruction about the volume centroids of spherical cells
                                 (r and theta; Cartesian axes and phi keep the face midpoints);
                                 0: every cell centre at its face midpoint.  Not with the MLP */
} or_config;

/* Full step of interior U (layout [nvar][n3][n2][n1]) with time step dt into Unew.
 * Returns OR_OK, or OR_ENONPHYS if any updated cell has rho<=0, p<=0 or a non-finite value
 * (Unew is written in every case), or OR_EINVAL. */
int or_step(const or_config *c, const double *U, double dt, double *Unew);

/* Same step, evaluated only for the interior box [lo, hi) (per axis); out has the box's
 * shape [nvar][hi2-lo2][hi1-lo1][hi0-lo0].  Used for sampled checks of large grids. */
int or_step_box(const or_config *c, const double *U, double dt, const int lo[3], const int hi[3],
                double *out);

/* or_step_box that also reports, per updated cell (fb, the box's cell count, layout [k][j][i]),
 * 1 where the cell's own half-step face states were not all physical and the cell was advanced at
 * first order (the positivity fallback: zero slopes and no half step), else 0. */
int or_step_box_fb(const or_config *c, const double *U, double dt, const int lo[3], const int hi[3],
                   double *out, unsigned char *fb);

/* CFL time step: dt = cfl / max over interior cells of sum_d (|u_d| + c_s)/dx_d. */
/* The limited face states (primitives) of cell (i, j, k) along axis d before the half step, as the
 * step forms them: wm at the lower face, wp at the upper (nvar values each; not for the MLP). */
int or_face_states(const or_config *c, const double *U, int i, int j, int k, int d, double *wm, double *wp);
int or_compute_dt(const or_config *c, const double *U, double *dt);
int or_num_threads(void);
/* the same over the cells of the box [lo, hi) only (the grid's step where every cell outside the
 * box has the state of a cell inside it) */
int or_compute_dt_box(const or_config *c, const double *U, const int lo[3], const int hi[3], double *dt);

/* Grid shift along axis 0 (Sect. 3.1.1, moving grid): the state U on the faces of c, carried
 * conservatively onto the faces moved by delta (|delta| <= the narrowest cell incl. the two ghost
 * layers; spherical: the inner radius stays >= 0), written to Unew.  OR_EINVAL otherwise. */
int or_shift_grid(const or_config *c, const double *U, double delta, double *Unew);

/* Conserved totals sum_cells U_v dV, one per variable (all nvar, the monitored e included). */
void or_totals(const or_config *c, const double *U, double *tot);

/* Enclosed mass M_enc(r_i) per radial shell (spherical wedge, Sect. 2.2 eq. internal_gravity). */
int or_enclosed_mass(const or_config *c, const double *U, double *menc);

/* EoS of configuration c at rest: the temperature (0 for the ideal gas) of internal energy e per
 * unit volume at density rho, with its pressure *P and sound speed *cs (Sect. 2.3). */
double or_eos_state(const or_config *c, double rho, double e, double *P, double *cs);

/* Internal energy per unit volume of density rho and pressure P (Sect. 2.3). */
double or_eos_energy(const or_config *c, double rho, double P);

/* 56Ni decay heating rate per unit mass of 56Ni at time t (eq. heating_ni without rho f_Ni). */
double or_ni_rate(const or_config *c, double t);

/* Blend factor alpha of the internal-energy monitor (Sect. 2.5) for internal energy e and kinetic
 * energy e_k (per unit volume) and the criterion eps. */
double or_de_alpha(double e, double ek, double eps);

/* Single-interface Riemann flux in direction d for conserved states qL, qR (nvar each). */
void or_riemann_flux(int solver, int d, int nvar, double gamma, const double *qL, const double *qR,
                     double *flux);

/* Half increment of a limited slope, limiter(a, b) (Sect. 3.2). */
double or_limiter(int lim, double a, double b);

/* MLP limiter network on one normalised stencil x[4]: returns phi in (0, 2). */
double or_mlp_phi(const double *w, const double x[4]);

/* MLP limited half increment for the undivided differences d[4] and geometric factors. */
double or_mlp_slope(const double *w, const double d[4], double cm, double cp);

/* Batched MLP forward + loss + gradient in FP64 (training, Sect. "learned limiter").
 * x: [B][4] normalised inputs, a: [B] base (phi multiplies a), t: [B] target, wt: [B] weights.
 * Loss L = sum_b wt_b (phi_b a_b - t_b)^2 / sum_b wt_b. grad: OR_MLP_NPARAM. Returns L. */
double or_mlp_loss_grad(const double *w, int B, const double *x, const double *a, const double *t,
                        const double *wt, double *grad);

/* Training samples of the learned limiter from a batch of 1D fine solutions U [5][nrows][nf]:
 * for every row, coarse cell i (averages of `ratio` fine cells) and primitive v: x[4] = the four
 * undivided coarse differences around i over their largest magnitude s, a = left difference / s,
 * t = least-squares slope of the fine primitive inside i, times the coarse width, / s, wt = 1 where
 * the network is used (differences on both sides of the same sign, not within 2 cells of a row end),
 * else all zero.  Outputs have nrows*(nf/ratio)*5 entries (x four times that). */
void or_mlp_features(const double *U, int nrows, int nf, int ratio, double gamma, double *x, double *a,
                     double *t, double *wt);

#ifdef __cplusplus
}
#endif
#endif
