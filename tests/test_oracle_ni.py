"""Pins of the oracle's 56Ni decay heating (Sect. 2.4, eq. heating_ni): the rate against the
decay chain's populations integrated as an ODE (Bateman), its value at t = 0 and its time integral
(every 56Ni nucleus releases Q_Ni + Q_Co in the end), and the step: a uniform medium at rest gains
exactly dt h(t + dt/2) rho f_Ni per step, second order in time against the integral; the monitored
internal energy and the gas + radiation EoS take the same heat."""
import numpy as np
import pytest
from scipy.integrate import quad, solve_ivp

from oracle import oracle as O
from paper_2503_04428_amd import problems as P


def _uniform(n=6, nscalar=2, fni=0.6, rho=1.3, p=0.9, gamma=5.0 / 3.0, ndim=3):
    base = P.random_periodic(n=(n,) * ndim, ndim=ndim, nscalar=nscalar, seed=1)
    U = np.zeros_like(base.U0)
    U[0] = rho
    U[4] = p / (gamma - 1.0)
    U[5] = rho * fni
    if nscalar > 1:
        U[6] = rho * 0.25
    return base.with_(U0=U, gamma=gamma)


def test_rate_matches_the_decay_chain_populations():
    """Power of the chain from the populations N_Ni, N_Co of dN_Ni/dt = -N_Ni/tau_Ni,
    dN_Co/dt = N_Ni/tau_Ni - N_Co/tau_Co (integrated numerically, per unit initial mass of 56Ni):
    Q_Ni N_Ni/tau_Ni + Q_Co N_Co/tau_Co."""
    pr = P.with_ni_heating(_uniform(), **{"Q": P.NI_CGS["ni_Q"], "tau": P.NI_CGS["ni_tau"], "m": P.NI_CGS["ni_m"]})
    o = O.Oracle(pr)
    (qn, qc), (tn, tc), m = pr.ni_Q, pr.ni_tau, pr.ni_m
    ts = np.array([0.0, 1e4, 3e5, 8.8 * 86400, 30 * 86400, 200 * 86400, 1000 * 86400])
    sol = solve_ivp(lambda t, y: [-y[0] / tn, y[0] / tn - y[1] / tc], (0, ts[-1]), [1.0 / m, 0.0],
                    t_eval=ts, rtol=1e-12, atol=1e-30, method="DOP853")
    for t, nni, nco in zip(ts, sol.y[0], sol.y[1]):
        ref = qn * nni / tn + qc * nco / tc
        assert o.ni_rate(t) == pytest.approx(ref, rel=1e-9)
    # at t = 0 only 56Ni decays
    assert o.ni_rate(0.0) == pytest.approx(qn / (m * tn), rel=1e-14)


def test_total_release_is_both_decay_energies():
    pr = P.with_ni_heating(_uniform(), Q=(1.0, 2.0), tau=(0.05, 0.6), m=2.0)
    o = O.Oracle(pr)
    tot, err = quad(o.ni_rate, 0.0, np.inf, epsabs=0, epsrel=1e-13, limit=200)
    assert tot == pytest.approx((1.0 + 2.0) / 2.0, rel=1e-10)


def _heat_run(pr, t0, t1, nsteps):
    o = O.Oracle(pr)
    U = pr.U0.copy()
    dt = (t1 - t0) / nsteps
    t = t0
    for _ in range(nsteps):
        Un, st = o.step(U, dt, t)
        assert st == 0
        U = Un
        t += dt
    return o, U


def test_uniform_medium_gains_the_midpoint_heat_each_step():
    pr = P.with_ni_heating(_uniform(), Q=(1.0, 2.0), tau=(0.05, 0.6))
    o = O.Oracle(pr)
    U0 = pr.U0
    t, dt = 0.03, 0.004
    U1, st = o.step(U0, dt, t)
    assert st == 0
    gain = dt * o.ni_rate(t + 0.5 * dt) * U0[5]
    assert np.allclose(U1[4] - U0[4], gain, rtol=1e-12, atol=0)
    for v in (0, 1, 2, 3, 5, 6):
        assert np.array_equal(U1[v], U0[v])
    # without heating nothing changes
    Ub, _ = O.Oracle(pr.with_(ni_heating=False)).step(U0, dt, t)
    assert np.array_equal(Ub, U0)


def test_heat_over_many_steps_is_second_order_in_time():
    pr = P.with_ni_heating(_uniform(n=4), Q=(1.0, 2.0), tau=(0.05, 0.6))
    o = O.Oracle(pr)
    t0, t1 = 0.0, 0.2
    exact = quad(o.ni_rate, t0, t1, epsabs=0, epsrel=1e-13)[0] * pr.U0[5, 0, 0, 0]
    errs = []
    for nsteps in (10, 20, 40):
        _, U = _heat_run(pr, t0, t1, nsteps)
        errs.append(abs((U[4, 0, 0, 0] - pr.U0[4, 0, 0, 0]) - exact))
    rates = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(rates) > 1.9, (errs, rates)


def test_heat_goes_to_the_monitored_internal_energy():
    """With the internal-energy monitor at alpha = 0 (huge eps) the heat reaches e by its own
    equation: e and E - |m|^2/(2 rho) gain the same."""
    pr = P.with_ni_heating(P.with_internal_energy(_uniform(), eps=1e30), Q=(1.0, 2.0), tau=(0.05, 0.6))
    o, U = _heat_run(pr, 0.01, 0.05, 8)
    assert np.allclose(U[-1] - pr.U0[-1], U[4] - pr.U0[4], rtol=1e-12, atol=0)
    assert np.all(U[-1] > pr.U0[-1] * 1.01)


def test_heat_with_gas_radiation_eos():
    """Gas + radiation EoS: the heat raises E by the same amount (the EoS only sets P from it), and
    the pressure follows the EoS at the new energy."""
    base = P.with_gas_rad(_uniform(), arad=3.0)
    pr = P.with_ni_heating(base, Q=(1.0, 2.0), tau=(0.05, 0.6))
    o = O.Oracle(pr)
    t, dt = 0.0, 0.01
    U1, st = o.step(pr.U0, dt, t)
    assert st == 0
    gain = dt * o.ni_rate(t + 0.5 * dt) * pr.U0[5]
    assert np.allclose(U1[4] - pr.U0[4], gain, rtol=1e-12, atol=0)
    T0, P0, _ = o.eos_state(pr.U0[0, 0, 0, 0], pr.U0[4, 0, 0, 0])
    T1, P1, _ = o.eos_state(U1[0, 0, 0, 0], U1[4, 0, 0, 0])
    assert T1 > T0 and P1 > P0


def test_invalid_heating_configurations():
    pr = P.with_ni_heating(_uniform(), Q=(1.0, 2.0), tau=(0.05, 0.6))
    for bad in (dict(ni_scalar=2), dict(ni_scalar=-1), dict(ni_tau=(0.6, 0.05)), dict(ni_m=0.0),
                dict(ni_Q=(-1.0, 2.0))):
        with pytest.raises(ValueError):
            O.Oracle(pr.with_(**bad)).step(pr.U0, 0.001)


def _heated_wave(n):
    """Smooth acoustic wave carrying a non-uniform 56Ni fraction, strongly heated."""
    pr = P.acoustic_wave1d(n=n, amp=1e-2)
    f = np.linspace(0.0, 1.0, n + 1)
    x = 0.5 * (f[:-1] + f[1:])
    fni = 0.5 + 0.4 * np.sin(2.0 * np.pi * x + 0.3)
    U = np.concatenate([pr.U0, (pr.U0[0] * fni)[None]], axis=0)
    return P.with_ni_heating(pr.with_(U0=U, nscalar=1), Q=(1.0, 2.0), tau=(0.05, 0.6))


def test_heated_flow_converges_at_second_order():
    """The heat enters the Hancock half step too: without it the half-step pressures lag by
    (dt/2) h rho f_Ni (gamma - 1) and the energy converges at first order only (checked by planting
    that omission); with it, second order against a 4x finer run."""
    def run(n, t_end=0.1):
        pr = _heated_wave(n)
        o = O.Oracle(pr)
        U, t = pr.U0.copy(), 0.0
        while t < t_end * (1 - 1e-12):
            dt = min(o.compute_dt(U)[0], t_end - t)
            U, st = o.step(U, dt, t)
            assert st == 0
            t += dt
        return U
    ref = run(1024)
    errs = []
    for n in (64, 128, 256):
        R = ref.reshape(ref.shape[0], 1, 1, n, 1024 // n).mean(axis=-1)
        errs.append(np.abs(run(n)[4] - R[4]).mean())
    rates = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(rates) > 1.8, (errs, rates)
