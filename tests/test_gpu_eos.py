"""GPU parity of the gas + radiation EoS (Sect. 2.3; variant 4 of the fused sweep, FP64) against the
FP64 oracle on the same seeded inputs: 1D-3D, Cartesian and spherical, both Riemann solvers, every
limiter but the learned one, every boundary kind, gravity, ragged z chunks, radiation- and
gas-dominated states in one grid.  FP64 bar: per cell |dU| <= 1e-12 |U_oracle| + 1e-14 s_field,
s_field = max|U_oracle,field|; the time step to 1e-14.  The kernel's temperature solve takes the
oracle's Newton sequence operation for operation (IEEE division and square roots, each cell
stopping on its own correction), so its results do not depend on the tile or z-chunk layout."""
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


def _boost(pr, v, seed):
    """Add a velocity v * w^3, w uniform in [0, 1] per cell, with its kinetic energy (so that the
    monitor's alpha takes all of its branches)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    U = pr.U0.copy()
    w = rng.uniform(0.0, 1.0, size=U.shape[1:]) ** 3
    for d in range(3):
        vd = v[d] * w
        U[4] += U[1 + d] * vd + 0.5 * U[0] * vd * vd
        U[1 + d] += U[0] * vd
    return pr.with_(U0=U)


def _pr_over_pg(pr):
    """P_r / P_g per cell of a gas + radiation problem's initial state (oracle EoS)."""
    o = O.Oracle(pr)
    U = pr.U0
    ke = 0.5 * (U[1] ** 2 + U[2] ** 2 + U[3] ** 2) / U[0]
    out = np.empty(U[0].size)
    for c, (rho, e) in enumerate(zip(U[0].ravel(), (U[4] - ke).ravel())):
        T, P_, _ = o.eos_state(rho, e)
        pg = rho * pr.eos_R * T
        out[c] = (P_ - pg) / pg
    return out


def _wide_range1d(n=400):
    """A 1D periodic state in pressure balance (P = 1, small velocity) whose density spans eight
    decades (1e-4 .. 1e4, smoothly): the temperature solves run from deeply gas-dominated cells
    through the crossover to radiation-dominated ones, where the Newton start is farthest from the
    root."""
    pr = P.random_periodic(n=(n,), ndim=1, nscalar=1, seed=57)
    x = (np.arange(n) + 0.5) / n
    rho = 10.0 ** (4.0 * np.sin(2.0 * np.pi * x))
    u = 0.01 * np.sin(4.0 * np.pi * x)
    U = np.zeros_like(pr.U0)
    U[0, 0, 0] = rho
    U[1, 0, 0] = rho * u
    U[4, 0, 0] = 1.0 / (pr.gamma - 1.0) + 0.5 * rho * u * u
    U[5, 0, 0] = rho * (0.5 + 0.5 * np.cos(2.0 * np.pi * x))
    return P.with_gas_rad(pr.with_(U0=U), arad=30.0)


CASES = {
    "wide_range1d": (lambda: _wide_range1d(), 40, None),
    "rad_wall1d_strong": (lambda: P.rad_wall1d(n=200, u0=-100.0), 60, None),
    "sod1d_hll_minmod": (lambda: P.with_gas_rad(P.sod(n=300, limiter="minmod", riemann="hll"), arad=3.0), 60, None),
    "sod1d_arad0": (lambda: P.with_gas_rad(P.sod(n=150), arad=0.0), 40, None),
    "rand1d_s2_vanalbada": (lambda: P.with_gas_rad(P.random_periodic(
        n=(131,), ndim=1, nscalar=2, seed=51, limiter="vanalbada")), 40, None),
    "rand2d_mixed_s1_none_hll": (lambda: P.with_gas_rad(P.random_periodic(
        n=(37, 29), ndim=2, nscalar=1, seed=52, limiter="none", riemann="hll",
        bc=[["transmissive", "reflective"], ["reflective", "transmissive"], ["periodic"] * 2]), arad=0.3), 40, None),
    "rt2d_gravity": (lambda: P.with_gas_rad(P.rt2d(24, 48), arad=1.0), 40, None),
    "rand3d_periodic_s0_kz5": (lambda: P.with_gas_rad(P.random_periodic(
        n=(31, 23, 19), ndim=3, nscalar=0, seed=53)), 25, 5),
    "rand3d_mixed_s4_minmod_kz7": (lambda: P.with_gas_rad(P.random_periodic(
        n=(17, 20, 13), ndim=3, nscalar=4, seed=54, limiter="minmod",
        bc=[["transmissive"] * 2, ["reflective"] * 2, ["periodic"] * 2]), arad=3.0), 25, 7),
    "sedov3d_24": (lambda: P.with_gas_rad(P.sedov3d(n=24)), 30, None),
    "wedge3d_point_s1": (lambda: P.with_gas_rad(P.random_wedge(
        nr=16, nth=9, nph=20, nscalar=1, gravity="point",
        bc=[["reflective", "transmissive"], ["reflective"] * 2, ["periodic"] * 2])), 25, 6),
    "wedge3d_monopole_hll": (lambda: P.with_gas_rad(P.random_wedge(
        nr=14, nth=10, nph=8, nscalar=1, gravity="point_monopole", riemann="hll",
        bc=[["reflective", "transmissive"], ["reflective"] * 2, ["periodic"] * 2]), arad=3.0), 20, None),
    "wedge2d_point": (lambda: P.with_gas_rad(P.random_wedge(
        nr=20, nth=18, ndim=2, nscalar=1, gravity="point",
        bc=[["reflective", "transmissive"], ["reflective"] * 2, ["periodic"] * 2])), 30, None),
    "sedov_sph1d": (lambda: P.with_gas_rad(P.sedov_sph1d(n=200)), 40, None),
    # with the internal-energy monitor (variant 5: the monitor's P through the EoS)
    "monitor_wave1d_alpha0": (lambda: P.with_internal_energy(
        P.with_gas_rad(P.acoustic_wave1d(n=200, amp=1e-2), arad=3.0), eps=1e30), 60, None),
    "monitor_rand3d_s1_kz5": (lambda: P.with_internal_energy(P.with_gas_rad(_boost(P.random_periodic(
        n=(31, 23, 19), ndim=3, nscalar=1, seed=56), (6.0, 3.0, -4.0), 56)), eps=2.0), 25, 5),
    "monitor_boosted_sedov24": (lambda: P.with_internal_energy(P.with_gas_rad(
        P.boosted_sedov3d(n=24).with_(dual_energy=False, U0=P.boosted_sedov3d(n=24).U0[:-1])), eps=1e-3), 25, None),
    "monitor_wedge3d_point_minmod": (lambda: P.with_internal_energy(P.with_gas_rad(_boost(P.random_wedge(
        nr=16, nth=9, nph=12, nscalar=2, gravity="point", limiter="minmod",
        bc=[["reflective", "transmissive"], ["reflective"] * 2, ["periodic"] * 2]), (0.0, 0.0, 6.0), 57)),
        eps=2.0), 20, 5),
}


@pytest.mark.parametrize("name", list(CASES))
def test_gas_rad_parity(H, name):
    make, nsteps, kz = CASES[name]
    pr = make()
    assert pr.eos == "gas_rad" and pr.nvar == pr.U0.shape[0]
    announce(f"gas+rad EoS parity {name} ({nsteps} steps, kz {kz})")
    o = O.Oracle(pr)
    s = H.Solver(pr, zchunk=kz)
    U = pr.U0.copy()
    s.set_state(U)
    for n in range(nsteps):
        dt, st = o.compute_dt(U)
        assert st == 0
        if n in (0, nsteps - 1):
            assert s.compute_dt() == pytest.approx(dt, rel=1e-14, abs=0)
        U, st = o.step(U, dt)
        assert st == 0
        s.step(dt)
    G = s.state_numpy()
    s.check()
    s.close()
    print(f"{name}: max relative difference {max_rel(G, U):.3e}")
    assert_parity(G, U, what=name)


def test_gas_rad_independent_of_layout(H):
    """The same steps with three z-chunk sizes give bit-identical states: a cell's temperature
    iterations do not depend on which cells share its wave."""
    pr = CASES["rand3d_periodic_s0_kz5"][0]()
    announce("gas+rad layout independence (kz 3, 5, 19)")
    o = O.Oracle(pr)
    dts = []
    U = pr.U0.copy()
    for _ in range(6):
        dt, st = o.compute_dt(U)
        assert st == 0
        dts.append(dt)
        U, st = o.step(U, dt)
        assert st == 0
    out = []
    for kz in (3, 5, 19):
        s = H.Solver(pr, zchunk=kz)
        s.set_state(pr.U0)
        for dt in dts:
            s.step(dt)
        out.append(s.state_numpy())
        s.check()
        s.close()
    assert np.array_equal(out[0], out[1]) and np.array_equal(out[0], out[2])
    assert_parity(out[0], U, what="gas+rad layout case")


def test_cases_span_both_regimes():
    """The cases cover radiation-dominated (P_r/P_g > 1) and gas-dominated cells, in one grid and
    apart (CPU check of their inputs)."""
    a = _pr_over_pg(CASES["rand3d_periodic_s0_kz5"][0]())
    assert a.min() < 0.7 and a.max() > 1.5
    b = _pr_over_pg(CASES["rand3d_mixed_s4_minmod_kz7"][0]())
    assert b.max() < 1.0  # arad = 3: gas-dominated throughout
    c = _pr_over_pg(CASES["sedov3d_24"][0]())
    assert c.min() < 1e-10 and c.max() > 10.0  # cold ambient gas, radiation-dominated blast
    assert np.all(_pr_over_pg(CASES["rad_wall1d_strong"][0]()) == pytest.approx(10.0, rel=1e-12))
    w = _pr_over_pg(CASES["wide_range1d"][0]())
    assert w.min() < 1e-6 and w.max() > 1e3 and np.any((w > 0.3) & (w < 3.0))


def test_gas_rad_full_size_sedov_sampled(H):
    """Sedov 256^3 with the gas + radiation EoS (the benchmark's workload and launch configuration):
    the first step on sampled boxes (the blast centre, random interior boxes, tile and chunk seams,
    the domain corners)."""
    prob = P.with_gas_rad(P.sedov3d(n=256))
    announce("gas+rad full-size sedov 256^3 first step")
    o = O.Oracle(prob)
    U0 = prob.U0
    dt, st = o.compute_dt(U0)
    assert st == 0
    s = H.Solver(prob)
    s.set_state(U0)
    assert s.compute_dt() == pytest.approx(dt, rel=1e-14, abs=0)
    s.step(dt)
    Ug = s.state_numpy()
    s.close()
    rng = np.random.default_rng(1)
    boxes = [((124, 124, 124), (132, 132, 132)), ((0, 0, 0), (3, 3, 3)), ((253, 253, 253), (256, 256, 256)),
             ((12, 12, 30), (17, 17, 34)), ((138, 26, 62), (142, 30, 66))]
    for _ in range(5):
        lo = rng.integers(0, 252, size=3)
        boxes.append((tuple(int(v) for v in lo), tuple(int(v) + 4 for v in lo)))
    for lo, hi in boxes:
        ob, st = o.step_box(U0, dt, lo, hi)
        gb = Ug[:, lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]]
        assert_parity(gb, ob, what=f"gas+rad sedov256 box {lo}-{hi}")


def test_gas_rad_nonphysical_state_reported(H):
    """A cell with E below its kinetic energy has no temperature: reported like any other
    non-physical state, by the time step and by the sweep."""
    prob = P.with_gas_rad(P.random_periodic(n=(20, 18, 9), ndim=3, nscalar=1, seed=55))
    announce("gas+rad non-physical state report")
    U = prob.U0.copy()
    ke = 0.5 * (U[1, 3, 4, 5] ** 2 + U[2, 3, 4, 5] ** 2 + U[3, 3, 4, 5] ** 2) / U[0, 3, 4, 5]
    U[4, 3, 4, 5] = 0.5 * ke
    s = H.Solver(prob)
    s.set_state(U)
    with pytest.raises(H.NonPhysicalState):
        s.compute_dt()
    s.set_state(prob.U0)
    assert s.compute_dt() > 0
    s.set_state(U)
    s.step(1e-4)
    with pytest.raises(H.NonPhysicalState):
        s.check()
    s.close()
