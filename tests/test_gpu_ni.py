"""GPU parity of the 56Ni decay heating (Sect. 2.4, eq. heating_ni) against the FP64 oracle on the
same seeded inputs: the ideal-gas sweeps (fixed HLLC + van Leer and run-time choices), the gas +
radiation EoS, the internal-energy monitor, 1D-3D, Cartesian and spherical, with the decay clock
advanced on the device by host and device time steps.  Both sides evaluate the decay exponentials
with their own exp, so the bar is the FP64 tolerance (per cell |dU| <= 1e-12 |U_oracle| +
1e-14 s_field, s_field = max|U_oracle,field|), not bit equality."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2503_04428_amd import problems as P

from parity import announce, assert_parity, max_rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2503_04428_amd import hydro
    hydro.load_library()
    return hydro


def _heated_wave(n=200, riemann="hll", limiter="minmod"):
    pr = P.acoustic_wave1d(n=n, amp=1e-2, limiter=limiter)
    f = np.linspace(0.0, 1.0, n + 1)
    x = 0.5 * (f[:-1] + f[1:])
    fni = 0.5 + 0.4 * np.sin(2.0 * np.pi * x + 0.3)
    U = np.concatenate([pr.U0, (pr.U0[0] * fni)[None]], axis=0)
    return P.with_ni_heating(pr.with_(U0=U, nscalar=1, riemann=riemann), Q=(1.0, 2.0), tau=(0.05, 0.6))


CASES = {
    "wave1d_hll_minmod": (lambda: _heated_wave(), 0.02, 60, None),
    "blob3d_hllc_vl_kz5": (lambda: P.ni_blob3d(), 0.0, 25, 5),
    "blob3d_scalar1_vanalbada": (lambda: P.ni_blob3d().with_(ni_scalar=1, limiter="vanalbada"), 0.1, 20, None),
    "blob3d_gas_rad": (lambda: P.ni_blob3d(eos="gas_rad"), 0.0, 20, 6),
    "blob3d_dual_energy": (lambda: P.with_internal_energy(P.ni_blob3d(), eps=2.0), 0.0, 20, 7),
    "wave1d_dual_energy": (lambda: P.with_internal_energy(_heated_wave(riemann="hllc"), eps=1e30), 0.0, 60, None),
    "wedge3d_point": (lambda: P.with_ni_heating(P.random_wedge(
        nr=16, nth=9, nph=12, nscalar=2, gravity="point",
        bc=[["reflective", "transmissive"], ["reflective"] * 2, ["periodic"] * 2])), 0.01, 20, None),
    "wedge2d_late_clock": (lambda: P.with_ni_heating(P.random_wedge(
        nr=20, nth=18, ndim=2, nscalar=1), Q=(2.0, 5.0), tau=(0.3, 1.1), m=0.5), 1e-3, 30, None),
    # the paper's SN configuration: gas + radiation EoS, monitor, heating, point mass, minmod, HLLC,
    # hybrid linear-log radial grid
    "sn_wedge3d_kz6": (lambda: P.sn_wedge3d(n_lin=24, n_log=24, nth=12, nph=12), 0.0, 20, 6),
    "sn_wedge2d": (lambda: P.sn_wedge3d(n_lin=40, n_log=40, nth=24, ndim=2), 0.2, 30, None),
    "sn_wedge1d": (lambda: P.sn_wedge3d(n_lin=100, n_log=100, ndim=1), 0.0, 60, None),
}


@pytest.mark.parametrize("name", list(CASES))
def test_ni_heating_parity(H, name):
    make, t0, nsteps, kz = CASES[name]
    pr = make()
    assert pr.ni_heating
    announce(f"56Ni heating parity {name} ({nsteps} steps from t = {t0}, kz {kz})")
    o = O.Oracle(pr)
    s = H.Solver(pr, zchunk=kz)
    U = pr.U0.copy()
    s.set_state(U)
    s.set_time(t0)
    t = t0
    for _ in range(nsteps):
        dt, st = o.compute_dt(U)
        assert st == 0
        U, st = o.step(U, dt, t)
        assert st == 0
        t += dt
        s.step(dt)
    assert s.time() == t  # the same FP64 sums on both sides
    G = s.state_numpy()
    s.check()
    s.close()
    print(f"{name}: max relative difference {max_rel(G, U):.3e}")
    assert_parity(G, U, what=name)


def test_heating_changes_the_flow():
    """The cases above are heated noticeably (CPU-side check through the oracle: the same run
    without heating differs well above the parity bar)."""
    pr = P.ni_blob3d()
    o, oc = O.Oracle(pr), O.Oracle(pr.with_(ni_heating=False))
    U = pr.U0
    dt, _ = o.compute_dt(U)
    a, _ = o.step(U, dt, 0.0)
    b, _ = oc.step(U, dt, 0.0)
    assert np.max(np.abs(a[4] - b[4]) / np.abs(b[4])) > 1e-3


def test_device_dt_loop_advances_the_clock(H):
    """hx_step_device reads dt on the device; the decay clock follows the same steps."""
    pr = P.ni_blob3d(n=(20, 18, 14))
    announce("56Ni heating: device-dt loop vs host-dt loop")
    a, b = H.Solver(pr), H.Solver(pr)
    for s in (a, b):
        s.set_state(pr.U0)
        s.set_time(0.02)
    for _ in range(12):
        a.step(a.compute_dt())
        b.compute_dt_device()
        b.step_device()
    assert a.time() == b.time() and a.time() > 0.02
    Ga, Gb = a.state_numpy(), b.state_numpy()
    a.close()
    b.close()
    assert np.array_equal(Ga, Gb)


def test_clock_survives_a_new_state(H):
    pr = P.ni_blob3d(n=(12, 10, 8))
    s = H.Solver(pr)
    s.set_state(pr.U0)
    s.set_time(1.25)
    dt = s.compute_dt()
    s.step(dt)
    s.set_state(pr.U0)
    assert s.time() == 1.25 + dt
    s.close()


def test_heating_rejected_configurations(H):
    pr = P.ni_blob3d(n=(9, 8, 7))
    for bad in (dict(precision="fp32"), dict(ni_scalar=2), dict(ni_tau=(0.6, 0.05)), dict(ni_m=-1.0)):
        with pytest.raises(Exception):
            H.Solver(pr.with_(**bad))
