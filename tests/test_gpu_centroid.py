"""GPU parity of the reconstruction about volume centroids (option `centroid`, a reading of the cell
position r_i of Sect. 3.1.1 on the non-uniform spherical cells of the paper's SN grids: slopes over
centroid distances, face values x_c + (x_+ - x_c) sigma and x_c - (x_c - x_-) sigma, the increment
bounded between the neighbouring values) against the oracle, through the C ABI: spherical wedges in
1D-3D on logarithmic and hybrid linear-log radial grids, every limiter and both solvers, gravity
(point, point + enclosed mass), the SN configuration (gas + radiation EoS, internal-energy
monitor, 56Ni heating), the FP32 form at its bar, and a Cartesian grid, where the option changes
nothing.  FP64 at the per-cell bar."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2503_04428_amd import problems as P

from parity import announce, assert_parity, max_rel

pytestmark = pytest.mark.gpu

FP32_REL, FP32_ABS = 2e-5, 2e-6


@pytest.fixture(scope="module")
def H():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2503_04428_amd import hydro
    hydro.load_library()
    return hydro


def _run(H, prob, nsteps, zchunk=None, t0=None, precision=None):
    o = O.Oracle(prob)
    s = H.Solver(prob, zchunk=zchunk, precision=precision)
    U = prob.U0.copy()
    if precision == "fp32":
        U = U.astype(np.float32).astype(np.float64)
    s.set_state(U)
    t = 0.0 if t0 is None else t0
    if t0 is not None:
        s.set_time(t0)
    for _ in range(nsteps):
        dt, st = o.compute_dt(U)
        assert st == 0
        U, st = o.step(U, dt, t)
        assert st == 0
        t += dt
        s.step(dt)
    G = s.state_numpy()
    s.check()
    s.close()
    return G, U


CASES = {
    # name: (problem, steps, z chunk)
    "wedge3d_vl_hllc_monopole_s4": (lambda: P.random_wedge(
        nr=17, nth=15, nph=13, nscalar=4, gravity="point_monopole",
        bc=[["reflective", "transmissive"], ["reflective"] * 2, ["periodic"] * 2]), 30, 4),
    "wedge3d_minmod_hll_point": (lambda: P.random_wedge(
        nr=16, nth=9, nph=20, nscalar=1, gravity="point", limiter="minmod", riemann="hll",
        bc=[["reflective"] * 2, ["reflective"] * 2, ["reflective"] * 2]), 30, 7),
    "wedge3d_vanalbada_periodic_theta": (lambda: P.random_wedge(
        nr=15, nth=14, nph=9, nscalar=0, limiter="vanalbada", th=(0.3, 1.2),
        bc=[["transmissive"] * 2, ["periodic"] * 2, ["periodic"] * 2]), 30, 5),
    "wedge2d_point_near_axis": (lambda: P.random_wedge(nr=20, nth=18, ndim=2, nscalar=1, gravity="point",
                                                       th=(0.05, 1.5),
                                                       bc=[["reflective", "transmissive"], ["reflective"] * 2,
                                                           ["periodic"] * 2]), 30, None),
    "wedge1d_point": (lambda: P.random_wedge(nr=60, ndim=1, nscalar=1, gravity="point",
                                             bc=[["reflective", "transmissive"], ["reflective"] * 2,
                                                 ["periodic"] * 2]), 60, None),
    "sn_wedge3d": (lambda: P.sn_wedge3d(n_lin=24, n_log=24, nth=12, nph=12), 20, 6),
    "sn_wedge1d": (lambda: P.sn_wedge3d(n_lin=100, n_log=100, ndim=1), 60, None),
}


@pytest.mark.parametrize("name", list(CASES))
def test_centroid_parity(H, name):
    make, nsteps, kz = CASES[name]
    prob = make().with_(centroid=True)
    announce(f"centroid parity {name} n={prob.n} nvar={prob.nvar} steps={nsteps} kz={kz}")
    t0 = 0.0 if getattr(prob, "ni_heating", False) else None
    G, U = _run(H, prob, nsteps, zchunk=kz, t0=t0)
    assert_parity(G, U, what=name)
    # the option is not a no-op on these grids: the face-midpoint run differs
    G0, _ = _run(H, prob.with_(centroid=False), min(nsteps, 5), zchunk=kz, t0=t0)
    G1, _ = _run(H, prob, min(nsteps, 5), zchunk=kz, t0=t0)
    assert not np.array_equal(G0, G1)
    print(f"{name}: max relative difference {max_rel(G, U):.3e}")


def test_centroid_fp32_form(H):
    prob = P.random_wedge(nr=17, nth=15, nph=13, nscalar=2, gravity="point_monopole", precision="fp32",
                          bc=[["reflective", "transmissive"], ["reflective"] * 2, ["periodic"] * 2]).with_(
        centroid=True)
    announce("centroid parity FP32 form wedge 17x15x13")
    G, U = _run(H, prob, 3, zchunk=4, precision="fp32")
    assert_parity(G, U, rel=FP32_REL, absf=FP32_ABS, what="centroid fp32", flow_scale=True)


def test_centroid_is_inert_on_cartesian_grids(H):
    prob = P.random_periodic(n=(19, 17, 13), ndim=3, nscalar=2, seed=31, limiter="minmod")
    announce("centroid on a Cartesian grid")
    a, _ = _run(H, prob, 5, zchunk=4)
    b, _ = _run(H, prob.with_(centroid=True), 5, zchunk=4)
    assert np.array_equal(a, b)
