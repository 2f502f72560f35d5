"""GPU parity where the positivity fallback fires (a reading: a cell whose Hancock half-step face
states leave rho > 0, P > 0 is advanced at first order; the paper's Sect. 3.2 scheme says nothing of
such states).  Cold expanding flows (problems.expansion) reach it in a few per cent of the cells;
each case asserts through the oracle's fallback mask that the branch fired, then compares the HIP
path with the oracle after several steps in the instantiations the workloads run:

  * FP64 HLLC + van Leer with 7 fields (the benchmark's one-wave-per-SIMD sweep, whose face states
    are formed again after the fallback) and with 5 fields (the two-wave sweep, which keeps the
    positivity check's face states), and the run-time limiter/solver variant;
  * the FP32 form with 7 and 5 fields (the same two face-state paths).

FP64 at the per-cell bar (the fallback decisions are then the oracle's, bit for bit).  FP32 at the
FP32-form bar of the full-size tests, on a flow whose fallback mask does not change under 1e-4
relative perturbations of its primitives (checked here with the oracle), so that FP32 rounding
cannot flip a decision."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2503_04428_amd import problems as P

from parity import announce, assert_parity

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


def _perturbed(U, eps, rng, gamma):
    """the same flow with its primitives scaled by 1 + eps U(-1, 1) (seeded)"""
    rho = U[0]
    u = U[1:4] / rho
    p = (gamma - 1.0) * (U[4] - 0.5 * (U[1] ** 2 + U[2] ** 2 + U[3] ** 2) / rho)
    f = U[5:] / rho
    r2 = rho * (1 + eps * rng.uniform(-1, 1, size=rho.shape))
    u2 = u * (1 + eps * rng.uniform(-1, 1, size=u.shape))
    p2 = p * (1 + eps * rng.uniform(-1, 1, size=rho.shape))
    V = np.empty_like(U)
    V[0] = r2
    V[1:4] = r2 * u2
    V[4] = p2 / (gamma - 1.0) + 0.5 * r2 * (u2 ** 2).sum(axis=0)
    V[5:] = r2 * f
    return V


def _oracle_run(prob, U, nsteps):
    o = O.Oracle(prob)
    masks, dts = [], []
    for _ in range(nsteps):
        dt, st = o.compute_dt(U)
        assert st == 0
        U, fb, st = o.step_fallback(U, dt)
        assert st == 0
        masks.append(fb)
        dts.append(dt)
    return U, masks, dts


CASES = {
    # name: (problem, precision, steps, z chunk)
    "fp64_vl_hllc_7f": (lambda: P.expansion(n=(20, 18, 17), ndim=3, nscalar=2), "fp64", 4, 6),
    "fp64_vl_hllc_5f": (lambda: P.expansion(n=(19, 20, 15), ndim=3, nscalar=0), "fp64", 4, 4),
    "fp64_minmod_hll_6f": (lambda: P.expansion(n=(17, 16, 18), ndim=3, nscalar=1, riemann="hll",
                                               limiter="minmod"), "fp64", 4, 5),
    "fp64_vanalbada_hllc_7f_2d": (lambda: P.expansion(n=(33, 30), ndim=2, nscalar=2, limiter="vanalbada"),
                                  "fp64", 4, None),
    "fp32_vl_hllc_7f": (lambda: P.expansion(n=(20, 18, 17), ndim=3, nscalar=2, V=4.0, p0=1e-2,
                                            precision="fp32"), "fp32", 3, 6),
    "fp32_vl_hllc_5f": (lambda: P.expansion(n=(19, 20, 15), ndim=3, nscalar=0, V=4.0, p0=1e-2,
                                            precision="fp32"), "fp32", 3, 4),
}


@pytest.mark.parametrize("name", list(CASES))
def test_fallback_parity(H, name):
    make, precision, nsteps, kz = CASES[name]
    prob = make()
    announce(f"fallback parity {name} n={prob.n} nvar={prob.nvar} {precision} steps={nsteps} kz={kz}")
    U0 = prob.U0
    if precision == "fp32":
        U0 = U0.astype(np.float32).astype(np.float64)  # the FP32 form's own initial state
    Uo, masks, dts = _oracle_run(prob, U0.copy(), nsteps)
    fired = [int(m.sum()) for m in masks]
    assert fired[0] > 0 and min(fired) > 0, f"the fallback must fire in every step: {fired}"
    assert all(int((~m).sum()) > 0 for m in masks), "a mix of fallback and limited cells"
    if precision == "fp32":
        rng = np.random.default_rng(5)
        for _ in range(2):
            _, pm, _ = _oracle_run(prob, _perturbed(U0, 1e-4, rng, prob.gamma), nsteps)
            assert all(np.array_equal(a, b) for a, b in zip(masks, pm)), "a fallback decision is marginal"
    s = H.Solver(prob, precision=precision, zchunk=kz)
    s.set_state(U0)
    for dt in dts:
        s.step(dt)
    Ug = s.state_numpy()
    s.check()
    s.close()
    if precision == "fp64":
        assert_parity(Ug, Uo, what=name)
    else:
        assert_parity(Ug, Uo, rel=FP32_REL, absf=FP32_ABS, what=name, flow_scale=True)
    print(f"{name}: fallback cells per step {fired} of {masks[0].size}")
