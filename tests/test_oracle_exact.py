"""Pins of the exact solutions themselves (exact Riemann solver, Sedov-Taylor constant)
against published values and the jump relations they must satisfy."""
import math
import os

import numpy as np
import pytest

from oracle import exact

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    out = {}
    for line in open(os.path.join(GOLD, name)):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        k, *v = line.split()
        out[k] = [float(x) for x in v]
    return out


def test_sod_star_state_textbook_values():
    g = _golden("sod_star_state.txt")
    ps, us = exact.star_state(1.0, 0.0, 1.0, 0.125, 0.0, 0.1, 1.4)
    rl, rr = exact.star_densities(1.0, 1.0, 0.125, 0.1, ps, 1.4)
    assert abs(ps - g["p_star"][0]) < 1e-5
    assert abs(us - g["u_star"][0]) < 1e-5
    assert abs(rl - g["rho_star_left"][0]) < 1e-5
    assert abs(rr - g["rho_star_right"][0]) < 1e-5


def test_sod_star_state_satisfies_jump_relations():
    """Right shock: Rankine-Hugoniot mass and momentum fluxes match in the shock frame.
    Left rarefaction: isentropic (p/rho^g const) and the Riemann invariant u + 2c/(g-1) const."""
    g = 1.4
    ps, us = exact.star_state(1.0, 0.0, 1.0, 0.125, 0.0, 0.1, g)
    rl, rr = exact.star_densities(1.0, 1.0, 0.125, 0.1, ps, g)
    # shock speed from mass conservation, then momentum conservation must hold
    S = (rr * us - 0.125 * 0.0) / (rr - 0.125)
    mom_pre = 0.125 * (0.0 - S) ** 2 + 0.1
    mom_post = rr * (us - S) ** 2 + ps
    assert abs(mom_pre - mom_post) < 1e-10
    # energy flux across the shock
    def eflux(r, u, p):
        v = u - S
        return v * (p / (g - 1) + 0.5 * r * v * v + p)
    assert abs(eflux(0.125, 0.0, 0.1) - eflux(rr, us, ps)) < 1e-10
    # rarefaction: isentrope and Riemann invariant
    assert abs(ps / rl ** g - 1.0) < 1e-12
    cl = math.sqrt(g * ps / rl)
    assert abs((us + 2 * cl / (g - 1)) - (0.0 + 2 * math.sqrt(g) / (g - 1))) < 1e-12


def test_sod_wave_positions():
    """Sampled solution at t = 0.2: rarefaction head/tail, contact and shock positions."""
    g = 1.4
    ps, us = exact.star_state(1.0, 0.0, 1.0, 0.125, 0.0, 0.1, g)
    rl, rr = exact.star_densities(1.0, 1.0, 0.125, 0.1, ps, g)
    S = rr * us / (rr - 0.125)
    head = 0.5 - 0.2 * math.sqrt(g)
    tail = 0.5 + 0.2 * (us - math.sqrt(g * ps / rl))
    x = np.array([head - 1e-6, head + 1e-6, tail + 1e-6, 0.5 + 0.2 * us - 1e-6, 0.5 + 0.2 * us + 1e-6,
                  0.5 + 0.2 * S - 1e-6, 0.5 + 0.2 * S + 1e-6])
    r, u, p = exact.sample(1.0, 0.0, 1.0, 0.125, 0.0, 0.1, (x - 0.5) / 0.2, g)
    assert abs(r[0] - 1.0) < 1e-12 and r[1] < 1.0
    assert abs(r[2] - rl) < 1e-4
    assert abs(r[3] - rl) < 1e-12 and abs(r[4] - rr) < 1e-12
    assert abs(r[5] - rr) < 1e-12 and abs(r[6] - 0.125) < 1e-12
    # wave positions printed in many references for the Sod problem at t = 0.2
    assert abs(head - 0.26334) < 1e-4
    assert abs(tail - 0.48594) < 2e-4
    assert abs(0.5 + 0.2 * us - 0.68549) < 1e-4
    assert abs(0.5 + 0.2 * S - 0.85044) < 1e-4


def test_sedov_xi0_values():
    g = _golden("sedov_xi0.txt")
    v, tol = g["gamma_5_3"]
    assert abs(exact.sedov_xi0(5.0 / 3.0) - v) < tol
    v, tol = g["gamma_1_4"]
    assert abs(exact.sedov_xi0(1.4) - v) < tol


def test_sedov_profile_center_behaviour():
    """Near the centre the pressure is uniform, and continuity plus constant entropy along
    particle paths force the homologous asymptote U(lam) = lam / gamma (velocity in units of the
    shock speed), with the density vanishing."""
    for g in (1.4, 5.0 / 3.0):
        sol = exact.sedov_profiles(g, lam_min=1e-4)
        G, U, P = sol.sol(np.array([1e-2, 0.05]))
        assert np.all(np.abs(U / np.array([1e-2, 0.05]) - 1.0 / g) < 1e-4)
        assert G[0] < 1e-8
        assert abs(P[0] - P[1]) < 1e-8 * P[0]


def test_stored_exact_references_are_current():
    """The exact references the benchmark reads (tests/golden, written by make_exact_references.py)
    equal what the exact solvers give now, and the Sod file holds the textbook star state."""
    import os

    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    sod = np.loadtxt(os.path.join(here, "sod1024_exact_t0.2.txt"))
    faces = np.linspace(0.0, 1.0, 1025)
    r, u, p = exact.cell_average(1.0, 0.0, 1.0, 0.125, 0.0, 0.1, faces, 0.5, 0.2, g=1.4, sub=64)
    assert np.array_equal(sod, np.stack([r, u, p], axis=1))
    # cell 600 (x = 0.586) sits between the rarefaction tail and the contact: the left star state
    assert sod[600, 0] == pytest.approx(0.42632, abs=1e-5)
    assert sod[600, 1] == pytest.approx(0.92745, abs=1e-5)
    assert sod[600, 2] == pytest.approx(0.30313, abs=1e-5)
    xi0 = float(np.loadtxt(os.path.join(here, "sedov_xi0_gamma1.4.txt")))
    assert xi0 == exact.sedov_xi0(1.4)
    assert xi0 == pytest.approx(1.033, abs=0.002)
    prof = np.loadtxt(os.path.join(here, "sedov_profile_gamma1.4.txt"))
    sol = exact.sedov_profiles(1.4)
    assert np.array_equal(prof[:, 1:], np.stack(sol.sol(prof[:, 0]), axis=1))
    # strong-shock jump at lam = 1: G = (g+1)/(g-1), U = P = 2/(g+1)
    assert prof[-1, 1:] == pytest.approx([6.0, 1.0 / 1.2, 1.0 / 1.2], rel=1e-12)
