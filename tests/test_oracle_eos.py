"""Pins of the oracle's gas + radiation EoS (Sect. 2.3, eqs. eos_gp_rad_ein, eos_gp_rad,
cs_gp_rad): temperature and energy round trips across gas- and radiation-dominated states, the
printed sound speed against the isentropic derivative (dP/drho)_s computed independently, the
ideal-gas limit, conservation, and the compression ratio 7 of a strong radiation-dominated shock."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2503_04428_amd import problems as P

R, A, G = 1.0, 30.0, 5.0 / 3.0


def _oracle(arad=A, gamma=G):
    pr = P.sod(40).with_(gamma=gamma, eos="gas_rad", eos_R=R, eos_arad=arad)
    return O.Oracle(pr)


def _e_of(rho, T, arad=A, gamma=G):
    return rho * R * T / (gamma - 1) + arad * T ** 4


def _p_of(rho, T, arad=A):
    return rho * R * T + arad * T ** 4 / 3


@pytest.mark.parametrize("rho", [1e-3, 1.0, 1e3])
@pytest.mark.parametrize("T", [1e-2, 0.3, 1.0, 3.0, 1e2])
def test_temperature_round_trip(rho, T):
    o = _oracle()
    e = _e_of(rho, T)
    Tn, Pn, cs = o.eos_state(rho, e)
    assert Tn == pytest.approx(T, rel=2e-14)
    assert Pn == pytest.approx(_p_of(rho, T), rel=2e-14)
    assert o.eos_energy(rho, _p_of(rho, T)) == pytest.approx(e, rel=2e-14)
    assert cs > 0


@pytest.mark.parametrize("rho,T", [(1.0, 0.05), (1.0, 1.0), (0.01, 2.0), (50.0, 0.5)])
def test_sound_speed_is_the_isentropic_derivative(rho, T):
    """(dP/drho)_s from the first law along an isentrope, de/drho = (e + P)/rho (e per unit
    volume), integrated with RK4 through the oracle's own P(rho, e), then differenced."""
    o = _oracle()

    def P_of(r, e):
        return o.eos_state(r, e)[1]

    def rhs(r, e):
        return (e + P_of(r, e)) / r

    def walk(h, nsub=40):
        r, e = rho, _e_of(rho, T)
        dr = h / nsub
        for _ in range(nsub):
            k1 = rhs(r, e)
            k2 = rhs(r + dr / 2, e + dr / 2 * k1)
            k3 = rhs(r + dr / 2, e + dr / 2 * k2)
            k4 = rhs(r + dr, e + dr * k3)
            e += dr / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
            r += dr
        return r, e

    h = 1e-3 * rho
    rp, ep = walk(h)
    rm, em = walk(-h)
    dPdrho = (P_of(rp, ep) - P_of(rm, em)) / (rp - rm)
    cs = o.eos_state(rho, _e_of(rho, T))[2]
    assert cs * cs == pytest.approx(dPdrho, rel=1e-6)


def test_limits():
    """No radiation: the ideal-gas pressure and sound speed; radiation-dominated: Gamma_1 -> 4/3."""
    o = _oracle(arad=0.0)
    T, Pn, cs = o.eos_state(2.0, 3.0)
    assert Pn == pytest.approx((G - 1) * 3.0, rel=1e-15)
    assert cs == pytest.approx(np.sqrt(G * Pn / 2.0), rel=1e-15)
    o = _oracle(arad=1e8)
    T, Pn, cs = o.eos_state(1.0, _e_of(1.0, 1.0, arad=1e8))
    assert cs * cs / (Pn / 1.0) == pytest.approx(4.0 / 3.0, rel=1e-6)


def test_ideal_gas_limit_of_the_step():
    """With a negligible radiation constant the gas + radiation step equals the ideal-gas step to
    rounding (the temperature path rounds differently)."""
    base = P.random_periodic(n=(12, 10, 8), ndim=3, nscalar=1, seed=31)
    rad = P.with_gas_rad(base, R=1.0, arad=1e-300)
    oa, ob = O.Oracle(base), O.Oracle(rad)
    dt, _ = oa.compute_dt(base.U0)
    dtb, _ = ob.compute_dt(rad.U0)
    assert dtb == pytest.approx(dt, rel=1e-13)
    Ua, _ = oa.step(base.U0, dt)
    Ub, st = ob.step(rad.U0, dt)
    assert st == 0
    assert np.max(np.abs(Ub - Ua) / (np.abs(Ua) + 1e-12)) < 1e-11


def test_conservation_radiation_dominated():
    pr = P.with_gas_rad(P.random_periodic(n=(14, 12, 10), ndim=3, nscalar=1, seed=32))
    o = O.Oracle(pr)
    U = pr.U0.copy()
    t0 = o.totals(U)
    for _ in range(5):
        dt, _ = o.compute_dt(U)
        U, st = o.step(U, dt)
        assert st == 0
    t1 = o.totals(U)
    assert np.max(np.abs(t1 - t0) / np.maximum(np.abs(t0), 1.0)) < 1e-13


def test_strong_radiation_shock_compresses_seven_times():
    """Radiation-dominated gas hitting a wall at Mach ~26: the shocked plateau's density is the
    strong-shock ratio (Gamma + 1)/(Gamma - 1) = 7 of index 4/3 (a gamma = 5/3 ideal gas gives 4)."""
    pr = P.rad_wall1d(n=400, u0=-100.0)
    o = O.Oracle(pr)
    U = pr.U0.copy()
    t = 0.0
    while t < 0.01:
        dt, _ = o.compute_dt(U)
        U, st = o.step(U, dt)
        assert st == 0
        t += dt
    rho = U[0, 0, 0]
    plateau = rho[rho > 3.0]
    assert len(plateau) > 40
    med = np.median(plateau[5:-5])
    assert med == pytest.approx(7.0, rel=0.03), med


@pytest.mark.parametrize("rho", [1e-8, 1e-4, 1e4, 1e8])
@pytest.mark.parametrize("T", [1e-5, 1e-3, 0.3, 2.5, 1e3, 1e5])
def test_converged_temperature_over_wide_ranges(rho, T):
    """Newton stops once a correction is at most 1e-8 of T (ten steps at most): across sixteen
    decades of density and ten of temperature, from deeply gas- to deeply radiation-dominated and
    through the crossover where the start is farthest from the root, the stopped iterate is the
    root to rounding, from e and from P."""
    o = _oracle()
    e = _e_of(rho, T)
    Tn, Pn, _ = o.eos_state(rho, e)
    assert Tn == pytest.approx(T, rel=4e-15)
    assert Pn == pytest.approx(_p_of(rho, T), rel=4e-15)
    assert o.eos_energy(rho, _p_of(rho, T)) == pytest.approx(e, rel=4e-15)


def test_crossover_start_needs_several_steps():
    """At P_r = P_g the start min(T_gas, T_rad) is 2^(1/4) T above the root (from P); the stopped
    iterate must still be the root, so the convergence test cannot stop after the first step."""
    o = _oracle()
    rho = 1.0
    T = (3.0 * rho * R / A) ** (1.0 / 3.0)  # rho R T = a T^4 / 3
    P = _p_of(rho, T)
    assert rho * R * T == pytest.approx(A * T ** 4 / 3, rel=1e-14)
    assert o.eos_energy(rho, P) == pytest.approx(_e_of(rho, T), rel=4e-15)
    Tn, Pn, _ = o.eos_state(rho, _e_of(rho, T))
    assert Tn == pytest.approx(T, rel=4e-15)
