"""GPU parity of the grid shift (moving grid, Sect. 3.1.1) against the FP64 oracle on the same
seeded inputs: Cartesian and spherical, 1D-3D, both signs of the shift, every boundary kind, the
monitored internal energy, a blast (fallback path), the FP32 form, and shifts interleaved with
steps (the geometry tables follow the faces).  FP64 bar as for the sweeps; the FP32 form to its
storage precision."""
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


def _minw(pr):
    return float(np.diff(pr.faces[0]).min())


CASES = {
    "rand1d_transmissive_pos": (lambda: P.random_periodic(
        n=(131,), ndim=1, nscalar=2, seed=91, bc=[["transmissive"] * 2, ["periodic"] * 2, ["periodic"] * 2]), 0.6),
    "rand1d_reflective_neg": (lambda: P.random_periodic(
        n=(77,), ndim=1, nscalar=1, seed=92, bc=[["reflective", "transmissive"], ["periodic"] * 2, ["periodic"] * 2]),
        -0.8),
    "rand3d_periodic": (lambda: P.random_periodic(n=(29, 17, 11), ndim=3, nscalar=2, seed=93), 0.37),
    "rand2d_mixed_full_cell": (lambda: P.random_periodic(
        n=(33, 21), ndim=2, nscalar=0, seed=94,
        bc=[["transmissive", "reflective"], ["reflective", "transmissive"], ["periodic"] * 2]), -1.0),
    "wedge3d_out": (lambda: P.random_wedge(nr=24, nth=9, nph=10, nscalar=2,
                                           bc=[["reflective", "transmissive"], ["reflective"] * 2, ["periodic"] * 2]), 0.9),
    "wedge2d_in": (lambda: P.random_wedge(nr=30, nth=12, ndim=2, nscalar=1), -0.7),
    "sedov3d_blast": (lambda: P.sedov3d(n=24), 0.95),
    "monitor_boosted": (lambda: P.boosted_sedov3d(n=16, eps=1e-3), -0.5),
    "sn_wedge3d": (lambda: P.sn_wedge3d(n_lin=20, n_log=20, nth=8, nph=8), 0.8),
}


@pytest.mark.parametrize("name", list(CASES))
def test_shift_parity(H, name):
    make, frac = CASES[name]
    pr = make()
    d = frac * _minw(pr)
    announce(f"grid shift parity {name} (delta {d:.4g})")
    o = O.Oracle(pr)
    Uo = o.shift_grid(pr.U0, d)
    s = H.Solver(pr)
    s.set_state(pr.U0)
    s.shift_grid(d)
    G = s.state_numpy()
    s.check()
    s.close()
    print(f"{name}: max relative difference {max_rel(G, Uo):.3e}")
    assert_parity(G, Uo, what=name)


def test_shift_fp32_form(H):
    pr = P.random_wedge(nr=24, nth=9, nph=10, nscalar=2)
    d = 0.6 * _minw(pr)
    announce("grid shift FP32 form")
    Uo = O.Oracle(pr).shift_grid(pr.U0, d)
    s = H.Solver(pr, precision="fp32")
    s.set_state(pr.U0)
    s.shift_grid(d)
    G = s.state_numpy()
    s.close()
    U32 = pr.U0.astype(np.float32).astype(np.float64)
    ref32 = O.Oracle(pr).shift_grid(U32, d)
    assert_parity(G, ref32, rel=2e-6, absf=1e-6, what="fp32 shift")
    # and against the FP64 shift of the unrounded state, to FP32 storage precision
    assert_parity(G, Uo, rel=1e-6, absf=1e-6, what="fp32 shift vs fp64", flow_scale=True)


@pytest.mark.parametrize("name", ["sn_wedge3d", "wedge2d"])
def test_steps_and_shifts(H, name):
    """Steps between shifts: the step after a shift uses the moved geometry (its time step and
    update) on both sides."""
    if name == "sn_wedge3d":
        pr = P.sn_wedge3d(n_lin=16, n_log=16, nth=8, nph=8)
    else:
        pr = P.random_wedge(nr=24, nth=14, ndim=2, nscalar=1, gravity="point",
                            bc=[["reflective", "transmissive"], ["reflective"] * 2, ["periodic"] * 2])
    announce(f"steps and grid shifts {name}")
    o = O.Oracle(pr)
    s = H.Solver(pr)
    U = pr.U0.copy()
    s.set_state(U)
    t = 0.0
    for cycle in range(3):
        for _ in range(5):
            dt, st = o.compute_dt(U)
            assert st == 0
            assert s.compute_dt() == pytest.approx(dt, rel=1e-13, abs=0)
            U, st = o.step(U, dt, t)
            assert st == 0
            s.step(dt)
            t += dt
        d = (0.5 if cycle != 1 else -0.3) * float(np.diff(o._faces[0]).min())
        U = o.shift_grid(U, d)
        s.shift_grid(d)
    G = s.state_numpy()
    s.check()
    s.close()
    print(f"{name}: max relative difference {max_rel(G, U):.3e}")
    assert_parity(G, U, what=f"steps and shifts {name}")


def test_shift_rejected(H):
    pr = P.random_periodic(n=(10, 4, 4), ndim=3, nscalar=1, seed=95)
    s = H.Solver(pr)
    with pytest.raises(H.HydroError):
        s.shift_grid(0.01)  # before a state
    s.set_state(pr.U0)
    for bad in (0.11, -0.2, float("nan")):
        with pytest.raises(H.HydroError):
            s.shift_grid(bad)
    s.close()
    w = P.static_wedge()
    s = H.Solver(w)
    s.set_state(w.U0)
    with pytest.raises(H.HydroError):
        s.shift_grid(-1.5)
    s.close()
