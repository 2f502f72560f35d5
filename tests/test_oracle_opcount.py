"""The op-counting build of the oracle (the same C source with a counting FP64 type): it must give
the plain oracle's results bit for bit, and its counts must behave like counts of the algorithm."""
import numpy as np

from oracle import oracle as O
from paper_2503_04428_amd import problems as P


def test_opcount_build_is_the_oracle():
    for pr in (P.sedov3d(n=12), P.random_periodic(n=(9, 8, 7), ndim=3, nscalar=1, seed=3, ng=2),
               P.static_wedge()):
        o = O.Oracle(pr)
        dt, _ = o.compute_dt(pr.U0)
        ref, _ = o.step(pr.U0, dt)
        r = O.opcount_step(pr, pr.U0, dt)
        assert np.array_equal(ref, r["state"]), pr.name
        assert r["flops"] > 0


def test_opcount_scales_with_cells():
    """The count of a uniform periodic row is affine in its length (a fixed part for the boundary
    images and the predicted ghost neighbours, the same work for every further cell), and a
    first-order step costs less than a limited one."""
    def per_cell(n, limiter="vanleer"):
        pr = P.random_periodic(n=(n, 1, 1), ndim=1, nscalar=0, seed=1, ng=2, limiter=limiter)
        U = pr.U0.copy()
        U[:] = U[:, :1, :1, :1]  # uniform state
        o = O.Oracle(pr)
        dt, _ = o.compute_dt(U)
        return O.opcount_step(pr, U, dt)

    a, b, c = per_cell(40), per_cell(80), per_cell(120)
    for k in ("add", "mul", "div", "sqrt"):
        assert c[k] - b[k] == b[k] - a[k], k
    lim, first = per_cell(40), per_cell(40, limiter="none")
    assert first["flops"] < lim["flops"]
    # one sound speed per half-step face state: 2 per cell in 1D (HLLC wave speeds of each face)
    assert b["sqrt"] - a["sqrt"] == 2 * 40
