"""MI355X-native MUSCL-Hancock Godunov hydrodynamics (the time step of HERACLES++, arXiv:2503.04428)
as HIP kernels for gfx950 behind a C ABI (include/hydro.h, libhydro.so).

Modules:
  hydro     ctypes binding of the C ABI: Solver (one context on a torch HIP device and stream:
            set_state / get_state / state_numpy, compute_dt / compute_dt_device, step /
            step_device, advance, run to t_end, totals, check, enclosed_mass, set_mlp,
            set_zchunk, shift_grid (moving grid), set_time / time (56Ni decay clock)) and the
            learned-limiter entry points (mlp_eval, mlp_features, training).
  problems  seeded input generators (Sod, Sedov, Rayleigh-Taylor, spherical wedges, Riemann
            batches, the SN-configuration wedge on the hybrid linear-log grid) and the wrappers
            that switch on the internal-energy monitor, the gas + radiation EoS and the 56Ni
            heating.
  learned   training data and training loop of the learned slope limiter on the GPU.
  build     in-tree build of libhydro.so with hipcc.

Example (FP64 Sedov 64^3, ten CFL steps on the device):

    from paper_2503_04428_amd import hydro, problems
    prob = problems.sedov3d(n=64)
    s = hydro.Solver(prob)
    s.set_state(prob.U0)
    s.advance(10)
    U = s.state_numpy()

There is no CPU path: the binding raises if the library or the HIP device is missing.
"""
