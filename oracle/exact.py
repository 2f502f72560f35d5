"""Exact solutions used to pin the oracle.  TEST INFRASTRUCTURE ONLY.

* Exact Riemann solver for the ideal-gas Euler equations (the Sod tube of the
  paper's App. C.1 "is known analytically"): the star pressure solves
  f_L(p) + f_R(p) + (u_R - u_L) = 0 with the shock (Rankine-Hugoniot) and
  rarefaction (isentropic) branches of each f_K; it is found by a safeguarded
  Newton iteration and the self-similar solution is sampled at x/t.
* Sedov-Taylor point blast: shock radius d_sh = xi0 (E t^2 / rho0)^(1/5)
  (paper Sect. 4.3, eq. analytical_sedov).  xi0(gamma) follows from the energy
  integral of the self-similar profiles, obtained by integrating the
  similarity ODEs of the spherically symmetric Euler equations inward from
  the strong-shock jump conditions.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.integrate import solve_ivp


# ---------------------------------------------------------------------------
# exact Riemann solver
# ---------------------------------------------------------------------------

def _fk(p, rho, pk, ck, g):
    """Velocity change across the K wave as a function of the star pressure, and its derivative."""
    if p > pk:  # shock
        A = 2.0 / ((g + 1.0) * rho)
        B = (g - 1.0) / (g + 1.0) * pk
        s = math.sqrt(A / (p + B))
        return (p - pk) * s, s * (1.0 - 0.5 * (p - pk) / (p + B))
    # rarefaction
    r = (p / pk) ** ((g - 1.0) / (2.0 * g))
    return 2.0 * ck / (g - 1.0) * (r - 1.0), 1.0 / (rho * ck) * (p / pk) ** (-(g + 1.0) / (2.0 * g))


def star_state(rL, uL, pL, rR, uR, pR, g=1.4, tol=1e-14):
    """Star pressure and velocity of the exact Riemann problem (Newton with bisection fallback)."""
    cL = math.sqrt(g * pL / rL)
    cR = math.sqrt(g * pR / rR)
    if 2.0 * (cL + cR) / (g - 1.0) <= uR - uL:
        raise ValueError("vacuum generated")

    def F(p):
        a, da = _fk(p, rL, pL, cL, g)
        b, db = _fk(p, rR, pR, cR, g)
        return a + b + (uR - uL), da + db

    lo, hi = 1e-300, max(pL, pR)
    while F(hi)[0] < 0:
        hi *= 2.0
    p = 0.5 * (pL + pR)
    for _ in range(200):
        f, df = F(p)
        pn = p - f / df
        if not (lo < pn < hi):
            pn = 0.5 * (lo + hi)
        if F(pn)[0] > 0:
            hi = pn
        else:
            lo = pn
        if abs(pn - p) <= tol * 0.5 * (pn + p):
            p = pn
            break
        p = pn
    u = 0.5 * (uL + uR) + 0.5 * (_fk(p, rR, pR, cR, g)[0] - _fk(p, rL, pL, cL, g)[0])
    return p, u


def star_densities(rL, pL, rR, pR, ps, g=1.4):
    def rho_star(rk, pk):
        if ps > pk:
            q = ps / pk
            gr = (g - 1.0) / (g + 1.0)
            return rk * (q + gr) / (gr * q + 1.0)
        return rk * (ps / pk) ** (1.0 / g)
    return rho_star(rL, pL), rho_star(rR, pR)


def sample(rL, uL, pL, rR, uR, pR, xi, g=1.4):
    """Exact solution (rho, u, p) at similarity coordinates xi = (x - x0)/t (array)."""
    ps, us = star_state(rL, uL, pL, rR, uR, pR, g)
    rsL, rsR = star_densities(rL, pL, rR, pR, ps, g)
    cL = math.sqrt(g * pL / rL)
    cR = math.sqrt(g * pR / rR)
    xi = np.asarray(xi, dtype=np.float64)
    rho = np.empty_like(xi)
    u = np.empty_like(xi)
    p = np.empty_like(xi)
    gm = (g - 1.0) / (g + 1.0)
    for n, s in enumerate(xi.ravel()):
        if s <= us:  # left of contact
            if ps > pL:
                SL = uL - cL * math.sqrt((g + 1) / (2 * g) * ps / pL + (g - 1) / (2 * g))
                st = (rL, uL, pL) if s <= SL else (rsL, us, ps)
            else:
                csL = cL * (ps / pL) ** ((g - 1) / (2 * g))
                SH, ST = uL - cL, us - csL
                if s <= SH:
                    st = (rL, uL, pL)
                elif s >= ST:
                    st = (rsL, us, ps)
                else:
                    f = 2.0 / (g + 1) + gm / cL * (uL - s)
                    st = (rL * f ** (2.0 / (g - 1)), 2.0 / (g + 1) * (cL + (g - 1) / 2 * uL + s),
                          pL * f ** (2 * g / (g - 1)))
        else:
            if ps > pR:
                SR = uR + cR * math.sqrt((g + 1) / (2 * g) * ps / pR + (g - 1) / (2 * g))
                st = (rR, uR, pR) if s >= SR else (rsR, us, ps)
            else:
                csR = cR * (ps / pR) ** ((g - 1) / (2 * g))
                SH, ST = uR + cR, us + csR
                if s >= SH:
                    st = (rR, uR, pR)
                elif s <= ST:
                    st = (rsR, us, ps)
                else:
                    f = 2.0 / (g + 1) - gm / cR * (uR - s)
                    st = (rR * f ** (2.0 / (g - 1)), 2.0 / (g + 1) * (-cR + (g - 1) / 2 * uR + s),
                          pR * f ** (2 * g / (g - 1)))
        rho.flat[n], u.flat[n], p.flat[n] = st
    return rho, u, p


def cell_average(rL, uL, pL, rR, uR, pR, faces, x0, t, g=1.4, sub=64):
    """Cell averages of the exact (rho, u, p) over cells with the given faces (midpoint sub-sampling)."""
    faces = np.asarray(faces)
    n = len(faces) - 1
    frac = (np.arange(sub) + 0.5) / sub
    xs = faces[:-1, None] + (faces[1:] - faces[:-1])[:, None] * frac[None, :]
    r, u, p = sample(rL, uL, pL, rR, uR, pR, (xs - x0) / t, g)
    return r.mean(axis=1), u.mean(axis=1), p.mean(axis=1)


# ---------------------------------------------------------------------------
# Sedov-Taylor
# ---------------------------------------------------------------------------

def sedov_profiles(gamma: float, lam_min: float = 1e-6):
    """Self-similar profiles G (density / rho0), U (velocity / shock speed) and P
    (pressure / (rho0 Rdot^2)) of the spherical point blast versus lam = r / R(t), with
    R = xi0 (E t^2/rho0)^(1/5).  Substituting into the 1D spherical Euler equations gives
        (U - lam) G' + G U' = -2 G U / lam
        (U - lam) U' + P'/G = 3 U / 2
        (U - lam) (P'/P - gamma G'/G) = 3
    with the strong-shock values at lam = 1: G = (g+1)/(g-1), U = P = 2/(g+1)."""
    g = gamma

    def rhs(lam, y):
        G, U, P = y
        a = U - lam
        A = np.array([[a, G, 0.0], [0.0, a, 1.0 / G], [-g * a / G, 0.0, a / P]])
        b = np.array([-2.0 * G * U / lam, 1.5 * U, 3.0])
        return np.linalg.solve(A, b)

    y0 = [(g + 1.0) / (g - 1.0), 2.0 / (g + 1.0), 2.0 / (g + 1.0)]
    sol = solve_ivp(rhs, (1.0, lam_min), y0, method="LSODA", rtol=1e-11, atol=1e-14, dense_output=True)
    return sol


def sedov_xi0(gamma: float) -> float:
    """xi0 from the energy integral E = 4 pi rho0 Rdot^2 R^3 I, I = int_0^1 (G U^2/2 + P/(g-1)) lam^2 dlam,
    with Rdot = (2/5) R / t, giving xi0^5 = 25 / (16 pi I)."""
    sol = sedov_profiles(gamma)
    lam = np.concatenate([np.linspace(sol.t[-1], 1.0, 20001)])
    G, U, P = sol.sol(lam)
    f = (0.5 * G * U * U + P / (gamma - 1.0)) * lam * lam
    I = np.trapz(f, lam) if hasattr(np, "trapz") else np.trapezoid(f, lam)
    return (25.0 / (16.0 * math.pi * I)) ** 0.2


def sedov_radius(E: float, rho0: float, t: float, gamma: float) -> float:
    return sedov_xi0(gamma) * (E * t * t / rho0) ** 0.2
