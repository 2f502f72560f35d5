"""Writes the exact-solution references that bench.py reads to state its L1 errors against exact
solutions (the benchmark may not call the oracle outside its CPU-baseline leg):

  sod1024_exact_t0.2.txt    cell averages of the exact Sod solution (paper App. C.1: left
                            (rho, u, P) = (1, 0, 1), right (0.125, 0, 0.1), interface at 0.5,
                            gamma 1.4) at t = 0.2 over the 1024 uniform cells of [0, 1]
                            (exact Riemann solver, 64 sub-samples per cell)
  sedov_xi0_gamma1.4.txt    the Sedov-Taylor constant xi0(1.4) of eq. analytical_sedov
                            (Sect. 4.3), from the similarity solution's energy integral
  sedov_profile_gamma1.4.txt  the self-similar density, velocity and pressure profiles
                            G, U, P (rho / rho0, u / Rdot, P / (rho0 Rdot^2)) against
                            lam = r / R(t) on 2001 points of [1e-6, 1]

Only oracle/exact.py is called.  Run from the repository root:
    python tests/golden/make_exact_references.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import exact  # noqa: E402


def main():
    n = 1024
    faces = np.linspace(0.0, 1.0, n + 1)
    r, u, p = exact.cell_average(1.0, 0.0, 1.0, 0.125, 0.0, 0.1, faces, 0.5, 0.2, g=1.4, sub=64)
    with open(os.path.join(HERE, "sod1024_exact_t0.2.txt"), "w") as f:
        f.write("# exact Sod solution (paper App. C.1), cell averages over 1024 uniform cells of [0,1] at t = 0.2,\n"
                "# gamma 1.4; written by tests/golden/make_exact_references.py (oracle/exact.py)\n"
                "# rho u P\n")
        for a, b, c in zip(r, u, p):
            f.write(f"{float(a)!r} {float(b)!r} {float(c)!r}\n")
    xi0 = exact.sedov_xi0(1.4)
    with open(os.path.join(HERE, "sedov_xi0_gamma1.4.txt"), "w") as f:
        f.write("# Sedov-Taylor constant xi0 for gamma = 1.4 in d_sh = xi0 (E t^2 / rho0)^(1/5) (Sect. 4.3),\n"
                "# from the similarity solution's energy integral; written by tests/golden/make_exact_references.py\n")
        f.write(f"{float(xi0)!r}\n")
    sol = exact.sedov_profiles(1.4)
    lam = np.linspace(1e-6, 1.0, 2001)
    G, U, P = sol.sol(lam)
    with open(os.path.join(HERE, "sedov_profile_gamma1.4.txt"), "w") as f:
        f.write("# Sedov-Taylor self-similar profiles for gamma = 1.4 (Sect. 4.3): lam = r / R, G = rho / rho0,\n"
                "# U = u / Rdot, P = p / (rho0 Rdot^2), Rdot = (2/5) R / t; written by\n"
                "# tests/golden/make_exact_references.py (oracle/exact.py)\n# lam G U P\n")
        for a, b, c, d in zip(lam, G, U, P):
            f.write(f"{float(a)!r} {float(b)!r} {float(c)!r} {float(d)!r}\n")


if __name__ == "__main__":
    main()
