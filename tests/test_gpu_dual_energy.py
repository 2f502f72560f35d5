"""GPU parity of the internal-energy monitor (Sect. 2.5; variant 3 of the fused sweep, FP64)
against the FP64 oracle on the same seeded inputs: every geometry and dimension, boundary kinds,
gravity, ragged z chunks, and blend factors alpha in all three branches.  FP64 bar as for the
other sweeps: per cell |dU| <= 1e-12 |U_oracle| + 1e-14 max|U_oracle,field|."""
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
    """Add a velocity v * w(x)^3 with w uniform in [0, 1] per cell (and the matching kinetic
    energy), so that e / e_k spans orders of magnitude and alpha takes all of its branches."""
    rng = np.random.Generator(np.random.PCG64(seed))
    U = pr.U0.copy()
    w = rng.uniform(0.0, 1.0, size=U.shape[1:]) ** 3
    for d in range(3):
        vd = v[d] * w
        U[4] += U[1 + d] * vd + 0.5 * U[0] * vd * vd
        U[1 + d] += U[0] * vd
    return pr.with_(U0=U)


def _alpha_mix(pr, eps):
    U = pr.U0
    ek = 0.5 * (U[1] ** 2 + U[2] ** 2 + U[3] ** 2) / U[0]
    a = np.vectorize(lambda e, k: O.de_alpha(e, k, eps))(U[-1], ek)
    return (a == 1.0).mean(), ((a > 0) & (a < 1)).mean(), (a == 0.0).mean()


CASES = {
    "acoustic1d_alpha0": (lambda: P.with_internal_energy(P.acoustic_wave1d(n=200), eps=1e30), 60, None),
    "rand1d_s1_boost": (lambda: P.with_internal_energy(
        _boost(P.random_periodic(n=(131,), ndim=1, nscalar=1, seed=41), (8.0, 0, 0), 41), eps=2.0), 40, None),
    "rand2d_mixed_s2_minmod": (lambda: P.with_internal_energy(_boost(P.random_periodic(
        n=(37, 29), ndim=2, nscalar=2, seed=42, limiter="minmod",
        bc=[["transmissive", "reflective"], ["reflective", "transmissive"], ["periodic"] * 2]),
        (6.0, -5.0, 2.0), 42), eps=2.0), 40, None),
    "rt2d_gravity": (lambda: P.with_internal_energy(P.rt2d(24, 48), eps=1e-6), 40, None),
    "rand3d_periodic_s1_kz5": (lambda: P.with_internal_energy(_boost(P.random_periodic(
        n=(31, 23, 19), ndim=3, nscalar=1, seed=43), (6.0, 3.0, -4.0), 43), eps=2.0), 25, 5),
    "rand3d_mixed_s3_vanalbada_kz7": (lambda: P.with_internal_energy(_boost(P.random_periodic(
        n=(17, 20, 13), ndim=3, nscalar=3, seed=44, limiter="vanalbada",
        bc=[["transmissive"] * 2, ["reflective"] * 2, ["periodic"] * 2]), (0.0, 0.0, 8.0), 44), eps=2.0), 25, 7),
    "boosted_sedov24": (lambda: P.boosted_sedov3d(n=24, eps=1e-3), 30, None),
    "wedge3d_point_s1": (lambda: P.with_internal_energy(_boost(P.random_wedge(
        nr=16, nth=9, nph=20, nscalar=1, gravity="point",
        bc=[["reflective", "transmissive"], ["reflective"] * 2, ["periodic"] * 2]), (0.0, 0.0, 6.0), 47), eps=2.0), 25, 6),
    "wedge2d_point": (lambda: P.with_internal_energy(_boost(P.random_wedge(
        nr=20, nth=18, ndim=2, nscalar=1, gravity="point",
        bc=[["reflective", "transmissive"], ["reflective"] * 2, ["periodic"] * 2]), (0.0, 0.0, 6.0), 48), eps=2.0), 30, None),
}


@pytest.mark.parametrize("name", list(CASES))
def test_dual_energy_parity(H, name):
    make, nsteps, kz = CASES[name]
    pr = make()
    assert pr.dual_energy and pr.nvar == pr.U0.shape[0]
    announce(f"dual energy parity {name} ({nsteps} steps, kz {kz})")
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
    print(f"{name}: alpha branches (1, mixed, 0) = {_alpha_mix(pr.with_(U0=U), pr.de_eps)}, "
          f"max relative difference {max_rel(G, U):.3e}")
    assert_parity(G, U, what=name)


def test_blend_regimes_are_exercised():
    """The boosted cases above reach all three branches of alpha (CPU check of their inputs)."""
    a1, am, a0 = _alpha_mix(CASES["rand3d_periodic_s1_kz5"][0](), 2.0)
    assert a1 > 0.05 and am > 0.05 and a0 > 0.05, (a1, am, a0)


def test_dual_energy_leaves_hydro_fields_unchanged(H):
    """The monitored field does not feed back: the other fields equal those of the same sweep
    without the monitor (different kernel variant), to the FP64 parity bar."""
    base = _boost(P.random_periodic(n=(23, 19, 17), ndim=3, nscalar=1, seed=45), (1.5, 0.0, 0.0), 45)
    pr = P.with_internal_energy(base, eps=1e-2)
    announce("dual energy: hydro fields vs the plain sweep")
    a, b = H.Solver(base), H.Solver(pr)
    a.set_state(base.U0)
    b.set_state(pr.U0)
    for _ in range(10):
        dt = a.compute_dt()
        a.step(dt)
        b.step(dt)
    Ga, Gb = a.state_numpy(), b.state_numpy()
    a.close()
    b.close()
    assert_parity(Gb[:-1], Ga, what="hydro fields with and without the monitor")


def test_dual_energy_rejected_configurations(H):
    base = P.with_internal_energy(P.random_periodic(n=(9, 8, 7), ndim=3, nscalar=1, seed=46))
    for bad in (dict(precision="fp32"), dict(riemann="hll")):
        with pytest.raises(Exception):
            H.Solver(base.with_(**bad))
