"""Pins of the oracle's internal-energy monitor (Sect. 2.5, eq. pressure_fix and the blend factor
alpha): the blend factor's branches, the two limits of the blend, a passive-scalar identity, and
second-order agreement of the internal-energy equation with the total-energy equation in a smooth
flow (which a dropped or sign-flipped P div(u) term would break)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2503_04428_amd import problems as P


def _run(pr, nsteps):
    o = O.Oracle(pr)
    U = pr.U0.copy()
    for _ in range(nsteps):
        dt, st = o.compute_dt(U)
        assert st == 0
        U, st = o.step(U, dt)
        assert st == 0
    return U


def _eint(U):
    return U[4] - 0.5 * (U[1] ** 2 + U[2] ** 2 + U[3] ** 2) / U[0]


def test_alpha_branches():
    eps, ek = 1e-6, 3.0e6  # eps e_k = 3
    assert O.de_alpha(3.0, ek, eps) == 1.0          # e = eps e_k: first branch
    assert O.de_alpha(7.0, ek, eps) == 1.0
    assert O.de_alpha(1.5, ek, eps) == pytest.approx(0.25, rel=1e-15)
    assert O.de_alpha(0.6, ek, eps) == pytest.approx(0.04, rel=1e-15)
    assert O.de_alpha(0.3, ek, eps) == 0.0          # e = eps e_k / 10: last branch
    assert O.de_alpha(0.1, ek, eps) == 0.0
    assert O.de_alpha(1.0, 0.0, eps) == 1.0         # at rest: total-energy path


def test_alpha_one_is_the_total_energy_path():
    """eps = 0: alpha = 1 everywhere and the monitored e equals E - |m|^2/(2 rho) of the new state;
    the other fields are those of the run without the monitor (bit for bit)."""
    base = P.random_periodic(n=(10, 9, 8), ndim=3, nscalar=1, seed=21, ng=2)
    pr = P.with_internal_energy(base, eps=0.0)
    Ua = _run(base, 3)
    Ub = _run(pr, 3)
    assert np.array_equal(Ub[:-1], Ua)
    e = _eint(Ub)
    assert np.max(np.abs(Ub[-1] - e) / np.abs(e)) < 1e-13


def test_moving_contact_keeps_internal_energy():
    """Uniform velocity and pressure with a density jump (a moving contact): div(u) vanishes, and
    e, reconstructed per unit volume like the pressure, stays at P/(gamma - 1) to rounding with
    alpha = 0 (huge eps); a passive scalar carrying e/rho does not (its product with rho is not
    kept across the jump), which is why e is not reconstructed that way."""
    n = 64
    f = np.linspace(0.0, 1.0, n + 1)
    x = 0.5 * (f[:-1] + f[1:])
    rho = np.where((x > 0.3) & (x < 0.6), 2.0, 1.0)
    u, p, g = 0.7, 1.0, 1.4
    U = np.zeros((6, 1, 1, n))
    U[0, 0, 0] = rho
    U[1, 0, 0] = rho * u
    U[4, 0, 0] = p / (g - 1) + 0.5 * rho * u * u
    e = p / (g - 1) * np.ones(n)
    U[5, 0, 0] = e  # conserved passive scalar rho f with f = e / rho
    base = P.Problem(name="contact", ndim=1, geom="cart", n=(n, 1, 1), ng=2,
                     faces=[P.ghost_faces(f, 2, "periodic", "periodic"), np.array([0.0, 1.0]),
                            np.array([0.0, 1.0])],
                     nscalar=1, gamma=g, cfl=0.5, riemann="hllc", limiter="vanleer",
                     bc=[["periodic"] * 2] * 3, U0=U)
    pr = base.with_(U0=np.concatenate([U, e[None, None, None, :]], axis=0), dual_energy=True, de_eps=1e30)
    Ua = _run(base, 20)
    Ub = _run(pr, 20)
    assert np.array_equal(Ub[:6], Ua)  # the monitor does not touch the other fields
    assert np.max(np.abs(Ub[-1] - e)) < 1e-12 * e[0]
    assert np.max(np.abs(Ua[5] - e)) > 1e-3 * e[0]


def test_internal_energy_equation_converges_to_total_energy():
    """Smooth acoustic wave, alpha = 0 (huge eps): the monitored e and E - |m|^2/(2 rho) are two
    second-order discretisations of the same internal energy, so their difference falls by about
    4x per doubling of the resolution."""
    errs = []
    for n in (64, 128, 256):
        pr = P.with_internal_energy(P.acoustic_wave1d(n=n, amp=1e-2), eps=1e30)
        o = O.Oracle(pr)
        U = pr.U0.copy()
        t, t_end = 0.0, 0.25
        while t < t_end * (1 - 1e-12):
            dt, _ = o.compute_dt(U)
            dt = min(dt, t_end - t)
            U, st = o.step(U, dt)
            assert st == 0
            t += dt
        errs.append(np.mean(np.abs(U[-1] - _eint(U))))
    rates = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(rates) > 1.7, (errs, rates)


def test_boosted_blast_branches():
    """Sedov blast in gas moving at Mach ~300 with eps = 1e-3: the ambient gas (e/e_k = 3.8e-5)
    takes the internal-energy path (alpha = 0) and keeps its e to rounding where the blast has not
    arrived; the blast core (alpha = 1) takes the total-energy path."""
    pr = P.boosted_sedov3d(n=16, eps=1e-3)
    o = O.Oracle(pr)
    U0 = pr.U0
    dt, _ = o.compute_dt(U0)
    U, st = o.step(U0, dt)
    assert st == 0 and np.all(U[-1] > 0)
    ek0 = 0.5 * (U0[1] ** 2 + U0[2] ** 2 + U0[3] ** 2) / U0[0]
    alpha = np.vectorize(lambda e, k: O.de_alpha(e, k, 1e-3))(U0[-1], ek0)
    untouched = (np.abs(U[0] - U0[0]) == 0) & (alpha == 0.0)
    assert untouched.sum() > 100
    assert np.max(np.abs(U[-1][untouched] - U0[-1][untouched]) / U0[-1][untouched]) < 1e-12
    core = alpha == 1.0
    assert core.sum() >= 8
    e = _eint(U)
    assert np.max(np.abs(U[-1][core] - e[core]) / np.abs(e[core])) < 1e-12


def test_monitor_with_gas_radiation_eos_converges_to_total_energy():
    """With the gas + radiation EoS the monitor's P comes from the EoS at (rho, e): in a smooth
    flow (alpha = 0) e and E - |m|^2/(2 rho) again differ at second order; taking (gamma - 1) e
    there instead leaves an O(1) gap (checked against the same run: its error does not fall)."""
    errs = []
    for n in (64, 128, 256):
        pr = P.with_internal_energy(P.with_gas_rad(P.acoustic_wave1d(n=n, amp=1e-2), arad=3.0), eps=1e30)
        o = O.Oracle(pr)
        U = pr.U0.copy()
        t, t_end = 0.0, 0.25
        while t < t_end * (1 - 1e-12):
            dt, _ = o.compute_dt(U)
            dt = min(dt, t_end - t)
            U, st = o.step(U, dt)
            assert st == 0
            t += dt
        errs.append(np.mean(np.abs(U[-1] - _eint(U))))
    rates = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(rates) > 1.7, (errs, rates)


def test_totals_cover_the_monitored_internal_energy():
    # sum_cells U_v dV for every field, the monitored e (the last one) included; on a uniform
    # Cartesian grid dV is the same for every cell, so the totals are plain sums times dV
    prob = P.with_internal_energy(P.random_periodic(n=(8, 6, 4), ndim=3, nscalar=1))
    tot = O.Oracle(prob).totals(prob.U0)
    dV = (1.0 / 8) * (1.0 / 6) * (1.0 / 4)
    ref = prob.U0.reshape(prob.nvar, -1).sum(axis=1) * dV
    assert tot.shape == (prob.nvar,)
    assert np.allclose(tot, ref, rtol=1e-13, atol=0)
    assert tot[-1] > 0
