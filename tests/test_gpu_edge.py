"""GPU edge cases through the C ABI: the smallest grids the method allows (as many cells per axis
as ghost layers, so that every ghost image of a periodic or reflective end is an interior cell of
the far side), and a uniform moving state, which every form must leave exactly as it is (all
faces see the same two states, so every flux difference is zero) with the oracle's time step."""
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


def _pair(H, prob, nsteps, zchunk=None):
    o = O.Oracle(prob)
    s = H.Solver(prob, zchunk=zchunk)
    U = prob.U0.copy()
    s.set_state(U)
    for _ in range(nsteps):
        dt, st = o.compute_dt(U)
        assert st == 0
        assert s.compute_dt() == pytest.approx(dt, rel=1e-14, abs=0)
        U, st = o.step(U, dt)
        assert st == 0
        s.step(dt)
    Ug = s.state_numpy()
    s.check()
    s.close()
    return Ug, U


REFL = ["reflective"] * 2
TRAN = ["transmissive"] * 2
PER = ["periodic"] * 2
SMALL = {
    "1d_n2_periodic": dict(n=(2,), ndim=1, nscalar=1, seed=31),
    "1d_n2_reflective": dict(n=(2,), ndim=1, nscalar=0, seed=32, bc=[REFL, PER, PER]),
    "1d_n3_transmissive_hll": dict(n=(3,), ndim=1, nscalar=1, seed=33, bc=[TRAN, PER, PER], riemann="hll"),
    "2d_2x2_periodic": dict(n=(2, 2), ndim=2, nscalar=2, seed=34),
    "2d_3x2_reflective_transmissive": dict(n=(3, 2), ndim=2, nscalar=1, seed=35, bc=[REFL, TRAN, PER],
                                           limiter="minmod"),
    "3d_2x2x2_periodic": dict(n=(2, 2, 2), ndim=3, nscalar=2, seed=36),
    "3d_3x2x2_mixed": dict(n=(3, 2, 2), ndim=3, nscalar=1, seed=37, bc=[REFL, PER, TRAN]),
    "3d_2x3x5_reflective_vanalbada": dict(n=(2, 3, 5), ndim=3, nscalar=0, seed=38, bc=[REFL, REFL, REFL],
                                          limiter="vanalbada"),
}


@pytest.mark.parametrize("name", list(SMALL))
def test_smallest_grids_match_oracle(H, name):
    prob = P.random_periodic(**SMALL[name])
    announce(f"smallest grid {name} n={prob.n}")
    Ug, Uo = _pair(H, prob, 15, zchunk=1 if prob.ndim == 3 else None)
    assert_parity(Ug, Uo, what=name)
    print(f"{name}: max relative difference {max_rel(Ug, Uo):.3e}")


@pytest.mark.parametrize("name", list(SMALL))
def test_smallest_grids_fp32_form(H, name):
    """The FP32 form on the same smallest grids, with the oracle's time steps, at the FP32-form bar
    of the parity tests (2e-5 of the value plus 2e-6 of the field's scale, momenta on the flow's
    momentum scale)."""
    prob = P.random_periodic(**SMALL[name])
    announce(f"smallest grid {name} n={prob.n}, fp32 form")
    o = O.Oracle(prob)
    s = H.Solver(prob, precision="fp32", zchunk=1 if prob.ndim == 3 else None)
    U = prob.U0.copy()
    s.set_state(U)
    for _ in range(15):
        dt, st = o.compute_dt(U)
        assert st == 0
        U, st = o.step(U, dt)
        assert st == 0
        s.step(dt)
    Ug = s.state_numpy()
    s.check()
    s.close()
    assert_parity(Ug, U, rel=2e-5, absf=2e-6, what=f"{name} fp32", flow_scale=True)


def _uniform(n, ndim, nscalar, precision, limiter="vanleer", ng=2):
    pr = P.random_periodic(n=n, ndim=ndim, nscalar=nscalar, seed=1, amp=0.0, ng=ng, precision=precision,
                           limiter=limiter)
    shape = pr.U0.shape[1:]
    u = (0.3, -0.2, 0.1)
    U = P._pack(np.full(shape, 1.25), np.full(shape, u[0]), np.full(shape, u[1] if ndim >= 2 else 0.0),
                np.full(shape, u[2] if ndim == 3 else 0.0), np.full(shape, 0.8),
                [np.full(shape, 0.25 + 0.5 * k) for k in range(nscalar)], 1.4)
    return pr.with_(U0=U)


@pytest.mark.parametrize("form", ["fp64", "fp32", "learned"])
def test_uniform_moving_state_is_kept_exactly(H, form):
    from paper_2503_04428_amd import learned
    if form == "learned":
        try:
            w = learned.load_weights()
        except OSError:
            pytest.skip("no trained weights")
        prob = _uniform((20, 18, 17), 3, 0, "fp32", limiter="mlp", ng=3)
    else:
        prob = _uniform((20, 18, 17), 3, 2, form)
    announce(f"uniform moving state, {form}")
    s = H.Solver(prob, precision="fp32" if form != "fp64" else "fp64", zchunk=5)
    if form == "learned":
        s.set_mlp(w)
    s.set_state(prob.U0)
    dt0 = None
    for _ in range(10):
        dt = s.compute_dt()
        dt0 = dt if dt0 is None else dt0
        assert dt == dt0
        s.step(dt)
    G = s.state_numpy()
    s.check()
    s.close()
    # FP32 form: the state round-trips through FP32 once, and stays there exactly
    ref = prob.U0 if form == "fp64" else prob.U0.astype(np.float32).astype(np.float64)
    assert np.array_equal(G, ref)
    # the time step of a uniform state: cfl / sum_d (|u_d| + c_s) / dx_d, as the oracle computes it
    dto, st = O.Oracle(prob.with_(limiter="vanleer")).compute_dt(prob.U0.copy())
    assert st == 0
    if form == "fp64":
        assert dt0 == pytest.approx(dto, rel=1e-15)
    else:
        assert dt0 == pytest.approx(dto, rel=1e-6)
