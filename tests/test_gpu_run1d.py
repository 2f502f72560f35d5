"""GPU tests of the persistent one-workgroup 1D run (hx_run_1d, through the C ABI): the whole time
loop to t_end inside one workgroup equals the host-driven loop of hx_compute_dt / hx_step bit for
bit (the same operations in the same order) and the FP64 oracle at the per-cell bar, with the same
step count and final time, for the Sod tube of App. C.1 (1024 cells; the FP32 form to FP32
rounding of its own host loop), every limiter
and both solvers, periodic and reflective ends, passive scalars, the largest rows the LDS holds
(1357 cells of 5 fields in FP64, 2046 in FP32) and a run cut by max_steps; unsupported
configurations are refused."""
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


def _host_loop(H, prob, t_end, precision=None, max_steps=None):
    s = H.Solver(prob, precision=precision)
    s.set_state(prob.U0)
    t, n = s.run(t_end=t_end, nsteps=max_steps)
    G = s.state_numpy()
    s.close()
    return G, t, n


def _device_loop(H, prob, t_end, precision=None, max_steps=1 << 30):
    s = H.Solver(prob, precision=precision)
    s.set_state(prob.U0)
    t, n = s.run_1d(t_end, max_steps=max_steps)
    G = s.state_numpy()
    s.check()
    s.close()
    return G, t, n


CASES = {
    "sod1024_vl_hllc": (lambda: P.sod(1024), 0.2),
    "sod1000_minmod_hll": (lambda: P.sod(1000, limiter="minmod", riemann="hll"), 0.15),
    "sod777_vanalbada_hllc": (lambda: P.sod(777, limiter="vanalbada"), 0.1),
    "sod300_first_order": (lambda: P.sod(300, limiter="none"), 0.2),
    "rand1d_periodic_s2": (lambda: P.random_periodic(n=(131,), ndim=1, nscalar=2, seed=21), 0.05),
    "rand1d_reflective_s1": (lambda: P.random_periodic(n=(200,), ndim=1, nscalar=1, seed=22,
                                                       bc=[["reflective"] * 2, ["periodic"] * 2,
                                                           ["periodic"] * 2]), 0.05),
    "sod1357_largest_fp64": (lambda: P.sod(1357), 0.05),
}


@pytest.mark.parametrize("name", list(CASES))
def test_device_loop_equals_host_loop_and_oracle(H, name):
    make, t_end = CASES[name]
    prob = make()
    announce(f"run_1d {name} n={prob.n[0]} t_end={t_end}")
    Gd, td, nd = _device_loop(H, prob, t_end)
    Gh, th, nh = _host_loop(H, prob, t_end)
    assert (nd, td) == (nh, th)
    assert np.array_equal(Gd, Gh)
    Uo, to, no, _ = O.Oracle(prob).run(prob.U0.copy(), t_end=t_end)
    assert no == nd and to == td
    assert_parity(Gd, Uo, what=name)
    print(f"{name}: {nd} steps to t = {td}, max relative difference to the oracle {max_rel(Gd, Uo):.3e}")


@pytest.mark.parametrize("n,t_end", [(1024, 0.2), (2046, 0.05)])
def test_fp32_form_device_loop_matches_host_loop(H, n, t_end):
    # FP32 products and sums may be contracted into FMAs, and the compiler decides that per kernel,
    # so the FP32 form of the device loop agrees with its host loop to FP32 rounding (not bitwise):
    # every field within 1e-5 of its largest value after hundreds of steps, the same time reached
    prob = P.sod(n)
    announce(f"run_1d sod{n} fp32")
    Gd, td, nd = _device_loop(H, prob, t_end, precision="fp32")
    Gh, th, nh = _host_loop(H, prob, t_end, precision="fp32")
    scale = np.abs(Gh).reshape(Gh.shape[0], -1).max(axis=1)
    rel = (np.abs(Gd - Gh).reshape(Gh.shape[0], -1).max(axis=1) / np.maximum(scale, 1e-30))
    print(f"fp32 sod{n}: {nd} / {nh} steps, largest difference per field / field scale {rel.max():.3e}")
    assert abs(nd - nh) <= 1 and abs(td - th) <= 1e-12 * t_end
    assert td == pytest.approx(t_end, rel=1e-13)
    assert np.all(rel <= 1e-5)


def test_max_steps_cuts_the_run(H):
    prob = P.sod(1024)
    announce("run_1d max_steps")
    Gd, td, nd = _device_loop(H, prob, 0.2, max_steps=37)
    Gh, th, nh = _host_loop(H, prob, 0.2, max_steps=37)
    assert nd == nh == 37 and td == th < 0.2
    assert np.array_equal(Gd, Gh)


def test_unsupported_configurations_are_refused(H):
    announce("run_1d refusals")
    # a 2D problem, a row longer than one workgroup holds, an FP64 row whose face states exceed
    # the LDS (checked on the host before any launch), gravity
    for prob in (P.random_periodic(n=(12, 10), ndim=2, nscalar=0, seed=1), P.sod(2047), P.sod(1358),
                 P.rt2d(8, 16)):
        s = H.Solver(prob)
        s.set_state(prob.U0)
        with pytest.raises(H.HydroError):
            s.run_1d(0.1)
        s.close()
