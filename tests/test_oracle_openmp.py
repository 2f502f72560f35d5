"""The OpenMP build of the oracle (liboracle_omp.so: the same C source with its cell loops shared
over z planes) gives bit for bit the serial oracle's steps, time steps and fallback masks: every
cell is computed by the same expressions, and the time step is a maximum."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2503_04428_amd import problems as P


def _cases():
    return [
        ("sod", P.sod(n=256), 3),
        ("sedov32", P.sedov3d(n=32), 3),
        ("wedge", P.random_wedge(nr=16, nth=10, nph=8, gravity="point_monopole"), 2),
        ("expansion", P.expansion(n=(14, 12, 10), ndim=3, nscalar=2), 1),
    ]


@pytest.mark.parametrize("name,prob,steps", _cases(), ids=[c[0] for c in _cases()])
def test_openmp_oracle_is_bitwise_serial(name, prob, steps):
    so = O.Oracle(prob)
    po = O.Oracle(prob, library=O.OMP_LIB_PATH)
    U = prob.U0.copy()
    for _ in range(steps):
        dt, st = so.compute_dt(U)
        dtp, stp = po.compute_dt(U)
        assert dt == dtp and st == stp
        Us, fbs, st = so.step_fallback(U, dt)
        Up, fbp, stp = po.step_fallback(U, dt)
        assert st == stp
        assert np.array_equal(Us, Up) and np.array_equal(fbs, fbp)
        U = Us
