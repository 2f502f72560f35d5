/*
 * hydro.h -- C ABI of the MI355X (gfx950) MUSCL-Hancock Godunov hydrodynamics step.
 *
 * The library advances the Euler equations with gravity and passive scalars (paper Sect. 2.1,
 * eqs. continuity, momentum, energy, passive_scalar; Sect. 2.2 gravity; Sect. 2.3 ideal-gas EoS)
 * by one time step of the unsplit MUSCL-Hancock scheme with HLL/HLLC fluxes (Sect. 3.2: slope-
 * limited reconstruction, Hancock half step, Godunov update eq. godunov, boundary conditions),
 * on Cartesian or spherical-wedge grids in 1D-3D (Sect. 3.1.1), including the spherical momentum
 * source terms of Sect. 3.1.2 (eq. source_terms_1 and its theta counterpart).
 *
 * Data layout.  A state is nvar = 5 + nscalar (+ 1 with dual_energy) fields, structure of arrays,
 * x fastest: U[v][k][j][i], v in (rho, rho u1, rho u2, rho u3, E, rho f_1 .. rho f_nscalar[, e]),
 *   i < n[0], j < n[1], k < n[2]; interior cells only (ghost cells are never stored).
 * In spherical geometry axis 0 is r, axis 1 theta, axis 2 phi, and (u1, u2, u3) = (u_r, u_theta,
 * u_phi).  All three momentum components are carried in every dimension.
 *
 * Ownership.  The caller owns every device buffer and the stream: the workspace passed to
 * hx_create, the state buffers passed to hx_set_state / hx_get_state and any device dt buffer.
 * The library never allocates or frees device memory; it borrows the workspace and the stream
 * until hx_destroy.  Host arrays (faces, weights) are copied during the call.
 *
 * Errors.  Every entry point returns a status; nothing aborts or prints.  HX_EHIP carries the HIP
 * error text in hx_last_error() (thread-local).  A non-physical state (rho <= 0, p <= 0 or a
 * non-finite value) is detected on the device while the state is read (by hx_step and
 * hx_compute_dt*) and reported as HX_ENONPHYS by the next synchronising call (hx_compute_dt,
 * hx_totals, hx_check); it stays reported until hx_set_state loads a new state.
 *
 * Threads and streams.  One context per stream; calls on one context must not overlap.
 * All device work of a context is enqueued on its stream in call order.
 */
#ifndef HYDRO_H
#define HYDRO_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hx_ctx hx_ctx;

typedef enum {
    HX_OK = 0,
    HX_EINVAL = -1,    /* invalid configuration or argument */
    HX_EHIP = -2,      /* a HIP runtime call failed */
    HX_ENONPHYS = -3,  /* a non-physical state was met */
    HX_ESTATE = -4,    /* call out of order (e.g. step before set_state, MLP without weights) */
    HX_ENOSPACE = -5   /* workspace smaller than hx_workspace_bytes() */
} hx_status;

enum { HX_GEOM_CART = 0, HX_GEOM_SPH = 1 };
enum { HX_RIEMANN_HLL = 0, HX_RIEMANN_HLLC = 1 };
enum { HX_LIMITER_NONE = 0, HX_LIMITER_MINMOD = 1, HX_LIMITER_VANLEER = 2, HX_LIMITER_VANALBADA = 3,
       HX_LIMITER_MLP = 4 };
enum { HX_PRECISION_FP64 = 0, HX_PRECISION_FP32 = 1 };
enum { HX_BOUNDARY_PERIODIC = 0, HX_BOUNDARY_TRANSMISSIVE = 1, HX_BOUNDARY_REFLECTIVE = 2 };
enum { HX_GRAVITY_NONE = 0, HX_GRAVITY_UNIFORM = 1, HX_GRAVITY_POINT = 2, HX_GRAVITY_POINT_MONOPOLE = 3 };
enum { HX_EOS_GAS = 0, HX_EOS_GAS_RAD = 1 };

#define HX_MLP_NPARAM 1249 /* 4->32->32->1: W1[32][4] b1[32] W2[32][32] b2[32] w3[32] b3 */

typedef struct {
    int ndim;               /* 1, 2 or 3 active axes (axes 0..ndim-1) */
    int geom;               /* HX_GEOM_*; spherical: axis 0 = r, 1 = theta, 2 = phi */
    int n[3];               /* interior cells per axis; 1 on inactive axes; active axes >= nghost */
    int nghost;             /* ghost layers: 2 (3 for HX_LIMITER_MLP) */
    const double *faces[3]; /* host; active axis: n+1+2*nghost increasing face coordinates incl.
                               ghost faces (a ghost cell's geometry); inactive axis: 2 faces */
    int nscalar;            /* passive scalars, 0..4 */
    double gamma;           /* adiabatic index (eq. eos_gas) */
    double cfl;             /* Courant number of hx_compute_dt */
    int riemann;            /* HX_RIEMANN_* (Sect. 3.2) */
    int limiter;            /* HX_LIMITER_* (Sect. 3.2) */
    int precision;          /* HX_PRECISION_*: FP64, or FP32 storage/bulk with the internal
                               energy recovered in FP64 where the kinetic energy dominates and
                               the time step, totals and source terms in FP64 */
    int bc[3][2];           /* HX_BOUNDARY_* per axis, low and high side (Sect. 3.2) */
    int gravity;            /* HX_GRAVITY_*: uniform g0 (Cartesian, eq. uniform_gravity); point mass
                               G*Mc (spherical, eq. point_gravity); point mass plus the enclosed
                               mass of the wedge, scaled to the full sphere (eq. internal_gravity) */
    double g0[3];
    double G, Mc;
    int dual_energy;        /* 1: the last field is the monitored internal energy e per unit volume
                               (Sect. 2.5: eq. pressure_fix with -P div(u), and the alpha blend of
                               the total- and internal-energy updates); needs FP64, HLLC, a
                               limiter other than the learned one and nscalar <= 3.  0: off */
    double de_eps;          /* the blend criterion epsilon (the paper uses 1e-6), >= 0 */
    int eos;                /* HX_EOS_GAS: ideal gas (eq. eos_gas).  HX_EOS_GAS_RAD: ideal gas plus
                               radiation (Sect. 2.3, eqs. eos_gp_rad_ein and eos_gp_rad:
                               e = rho R T/(gamma-1) + a T^4, P = rho R T + a T^4/3; T from e or P by
                               Newton's method from the smaller of the gas-only and radiation-only
                               temperatures, run until the correction is at most 1e-8 of T (ten
                               steps at most); sound speed of eq. cs_gp_rad; with dual_energy the
                               monitor's P is the EoS pressure of (rho, e)); needs FP64 and a
                               limiter other than the learned one */
    double eos_R;           /* HX_EOS_GAS_RAD: specific gas constant k_b/(mu m_u), > 0 */
    double eos_arad;        /* HX_EOS_GAS_RAD: radiation constant a, >= 0 */
    int ni_heating;         /* 1: 56Ni -> 56Co -> 56Fe decay heating (Sect. 2.4, eq. heating_ni):
                               E (and e with dual_energy) gains rho f_Ni h(t) with
                               h = lambda {[Q_Ni (tau_Co/tau_Ni - 1) - Q_Co] exp(-t/tau_Ni)
                               + Q_Co exp(-t/tau_Co)}, lambda = 1/(ni_m (tau_Co - tau_Ni)), taken at
                               the step's start in the half step and at its midpoint in the update;
                               t is the context's decay clock (hx_set_time).  Needs FP64.  0: off */
    int ni_scalar;          /* the passive scalar (0 .. nscalar-1) that carries rho f_Ni */
    double ni_Q[2];         /* energy released per decay of 56Ni and of 56Co, >= 0 */
    double ni_tau[2];       /* lifetimes of 56Ni and 56Co, 0 < tau_Ni < tau_Co */
    double ni_m;            /* mass of one 56Ni nucleus (56 m_u in the caller's units), > 0 */
    int centroid;           /* 1: reconstruct about the volume centroids of spherical cells (Sect.
                               3.1.1: non-uniform radial and angular spacing) instead of the face
                               midpoints: along r (measure r^2 dr) and theta (sin theta dtheta) the
                               slopes use the distances between centroids, the face values are
                               x_c + (x_+ - x_c) sigma and x_c - (x_c - x_-) sigma, and the increment
                               is bounded so that both stay between the neighbouring cell values;
                               a ghost cell's centroid is its image's, mirrored or translated like
                               its faces.  Cartesian grids and phi are unchanged.  Not with the
                               learned limiter.  0: face midpoints */
} hx_config;

/* Device bytes the caller must provide to hx_create for this configuration, or 0 if the
 * configuration is invalid (hx_last_error says why). */
size_t hx_workspace_bytes(const hx_config *cfg);

/* Validate cfg, copy the grid, lay out the workspace (device, >= hx_workspace_bytes(cfg) bytes,
 * 256-byte aligned) and bind the HIP stream (hipStream_t, may be NULL for the default stream).
 * Enqueues the upload of the geometry tables on the stream. */
hx_status hx_create(const hx_config *cfg, void *d_workspace, size_t workspace_bytes, void *hip_stream,
                    hx_ctx **out);

/* Load a state: d_U is a device FP64 array [nvar][n3][n2][n1].  The FP32 form rounds it to FP32.
 * Clears the non-physical flag.  Asynchronous on the context's stream. */
hx_status hx_set_state(hx_ctx *ctx, const double *d_U);

/* Store the current state to the device FP64 array d_U (same layout; the FP32 form widens
 * exactly).  Asynchronous. */
hx_status hx_get_state(hx_ctx *ctx, double *d_U);

/* CFL time step dt = cfl / max_cells sum_d (|u_d| + c_s) / dx_d over the current state (FP64),
 * with dx_d the physical widths dr, r dtheta, r sin(theta) dphi.  Synchronises the stream;
 * returns HX_ENONPHYS if a non-physical state was met since the last hx_set_state. */
hx_status hx_compute_dt(hx_ctx *ctx, double *h_dt);

/* Same time step written to the device double *d_dt; asynchronous, no check. */
hx_status hx_compute_dt_device(hx_ctx *ctx, double *d_dt);

/* Advance the current state by one step of length dt (host value).  Asynchronous. */
hx_status hx_step(hx_ctx *ctx, double dt);

/* Advance by one step whose length is read on the device from *d_dt (e.g. written by
 * hx_compute_dt_device), so that a time loop needs no host synchronisation.  Asynchronous. */
hx_status hx_step_device(hx_ctx *ctx, const double *d_dt);

/* Run a 1D problem from time t0 with CFL steps (the last one clipped to t_end) until t_end or
 * max_steps steps, inside one workgroup on the device: the state stays on chip, each step takes
 * the CFL time step and the MUSCL-Hancock step of hx_compute_dt / hx_step (FP64: the same results,
 * bit for bit, as that host loop; FP32 form: the same to FP32 rounding, since the compiler may
 * contract FP32 products and sums differently in the two kernels), and no kernel is launched and
 * nothing synchronises per step (Sect. 3.2; the Sod tube of App. C.1 is this size).  For one Cartesian row (ndim 1, n[1] = 1) of at
 * most 2046 cells whose primitives and face states, 3 nvar (n + 4) values of 8 bytes (FP64) or 4
 * (FP32 form), fit the device's LDS with 512 bytes to spare (160 KiB on gfx950: at most 1357 cells
 * with 5 fields in FP64, 2046 in FP32), with the ideal gas and no gravity, heating,
 * internal-energy monitor or learned limiter; HX_EINVAL otherwise, or for
 * a non-finite t0 or t_end or max_steps < 1; HX_ESTATE before hx_set_state.  Writes the final time
 * to *h_t and the number of steps to *h_steps; synchronises and reports HX_ENONPHYS like
 * hx_compute_dt. */
hx_status hx_run_1d(hx_ctx *ctx, double t0, double t_end, int max_steps, double *h_t, int *h_steps);

/* Conserved totals sum_cells U_v dV (FP64), nvar values to host h_tot.  Synchronises; returns
 * HX_ENONPHYS like hx_compute_dt. */
hx_status hx_totals(hx_ctx *ctx, double *h_tot);

/* Synchronise the stream and report HX_ENONPHYS / HIP errors. */
hx_status hx_check(hx_ctx *ctx);

/* Weights of the learned slope limiter, HX_MLP_NPARAM FP32 values (host), layout as above. */
hx_status hx_set_mlp(hx_ctx *ctx, const float *h_w, size_t n);

/* Tuning: z planes per workgroup of the 3D sweep; 0 (the default) chooses it at the first 3D step
 * from the sweep's workgroups per compute unit and the number of compute units, so that the
 * launch's dispatch rounds times the planes per workgroup is smallest.  Does not change results.
 * HX_EINVAL for kz < 0. */
hx_status hx_set_zchunk(hx_ctx *ctx, int kz);

/* The z planes per workgroup in use: the value set, else the automatic choice (0 before the first
 * 3D step).  HX_EINVAL for null arguments. */
hx_status hx_get_zchunk(hx_ctx *ctx, int *kz);

/* Moving grid (Sect. 3.1.1): move every face of axis 0 (r in spherical geometry) by delta and
 * carry the current state over conservatively: minmod-limited linear profiles of the conserved
 * variables about each cell's volume centroid, integrated over the overlaps with the new cells
 * (measure dx, or r^2 dr in spherical geometry), the boundary images supplying what enters; a
 * cell whose result would not be physical takes the piecewise-constant remap.  |delta| must not
 * exceed the narrowest cell of axis 0 (ghost layers included) and a spherical inner radius must
 * stay >= 0.  Between steps; synchronises the stream (the geometry tables are rebuilt and
 * uploaded).  HX_EINVAL for an invalid delta, HX_ESTATE before hx_set_state. */
hx_status hx_shift_grid(hx_ctx *ctx, double delta);

/* The decay clock of the 56Ni heating: with ni_heating on, every step advances it by its dt on the
 * device (also with hx_step_device); without, steps leave it alone.  hx_create starts it at 0.
 * hx_set_time sets it (asynchronous); hx_get_time synchronises and reads it.  HX_EINVAL for null
 * arguments or a non-finite t. */
hx_status hx_set_time(hx_ctx *ctx, double t);
hx_status hx_get_time(hx_ctx *ctx, double *t);

/* Enclosed-mass table of the last step that used HX_GRAVITY_POINT_MONOPOLE (n[0] doubles to the
 * host; synchronises).  For tests of the enclosed-mass reduction. */
hx_status hx_enclosed_mass(hx_ctx *ctx, double *h_menc);

/* Check of the FP64 arithmetic the sweeps use (context-free; device pointers; asynchronous on
 * hip_stream): d_q[i] = d_a[i] / d_b[i] and d_s[i] = sqrt(|d_a[i]|) for n elements, computed with
 * the sweeps' own division and square root (the hardware reciprocal and reciprocal square root
 * refined by Newton steps with FMA corrections, without range scaling).  They are the IEEE
 * round-to-nearest results for operands whose quotients and roots lie well inside the normal range
 * (exponents within about +-700); zero, infinite and NaN operands are outside their domain.
 * HX_EINVAL for null pointers or n < 0. */
hx_status hx_arith_check(const double *d_a, const double *d_b, long long n, double *d_q, double *d_s,
                         void *hip_stream);

/* ---- learned slope limiter (context-free; device pointers; asynchronous on hip_stream) ----
 * The limiter network maps the four undivided differences of a primitive around a cell,
 * normalised by their largest magnitude, to phi in (0, 2); the limited slope is phi times the
 * left difference, replaced by van Leer outside the TVD region 0 <= phi <= min(2, 2r).  It is an
 * extension of the paper's runtime-selectable limiters (Sect. 3.2), trained on fine FP64 solutions
 * of the scheme itself. */

/* phi of n stencils: d_w HX_MLP_NPARAM FP32 parameters (used as BF16), d_x [n][4] FP32 inputs,
 * d_phi [n] FP32 output; BF16 matrix-core evaluation, the same code the fused sweep runs. */
hx_status hx_mlp_eval(const float *d_w, const float *d_x, long long n, float *d_phi, void *hip_stream);

/* Training samples from a batch of 1D FP64 solutions d_fine [5][nrows][nfine] (rho, m1, m2, m3, E):
 * one sample per (row, coarse cell, primitive), coarse cells = averages of `ratio` fine cells
 * (nfine divisible by ratio).  Outputs (FP32, n = nrows*(nfine/ratio)*5): d_x [n][4] normalised
 * coarse differences, d_a [n] the normalised left difference, d_t [n] the least-squares slope of
 * the fine primitive across the coarse cell (times the coarse width) normalised alike, d_wt [n]
 * 1 where the network is used (monotone, non-flat stencil away from the row ends), else 0. */
hx_status hx_mlp_features(const double *d_fine, int nrows, int nfine, int ratio, double gamma, float *d_x,
                          float *d_a, float *d_t, float *d_wt, void *hip_stream);

/* Device bytes of the scratch buffer hx_mlp_grad needs for n samples. */
size_t hx_mlp_grad_workspace_bytes(long long n);

/* FP32 loss L = sum wt (phi a - t)^2 / sum wt and its gradient (HX_MLP_NPARAM values) over n samples,
 * with the caller's scratch d_work (>= hx_mlp_grad_workspace_bytes(n)). */
hx_status hx_mlp_grad(const float *d_w, const float *d_x, const float *d_a, const float *d_t, const float *d_wt,
                      long long n, float *d_grad, float *d_loss, void *d_work, size_t work_bytes,
                      void *hip_stream);

/* hx_mlp_grad for callers that cannot allocate device memory (code under HIP graph capture, serving
 * loops, harnesses that forbid hipMalloc): the same loss and gradient, bit for bit, with the block
 * partials in a scratch array the library holds statically on every device it runs on (5.1 MB,
 * 1024 partial rows, enough for any n since the gradient grid is capped at 1024 blocks; kept until
 * the process ends).  No allocation, no workspace argument.  The array is shared by every call on a
 * device and keeps the last call's partials (each call overwrites the rows it uses before reading
 * them): calls that overlap on one device (different streams or threads) race.  HX_EINVAL for null
 * pointers or n < 1, HX_ENOSPACE if n needs more partial rows than the array holds. */
hx_status hx_mlp_grad_noalloc(const float *d_w, const float *d_x, const float *d_a, const float *d_t,
                              const float *d_wt, long long n, float *d_grad, float *d_loss, void *hip_stream);

/* One Adam update of the FP32 master weights d_w with moments d_m, d_v (step counts from 1). */
hx_status hx_mlp_adam(float *d_w, const float *d_grad, float *d_m, float *d_v, int step, float lr, float beta1,
                      float beta2, float eps, void *hip_stream);

/* Thread-local text of the last error. */
const char *hx_last_error(void);

/* Release the context (host memory only; the workspace stays the caller's). */
void hx_destroy(hx_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif
