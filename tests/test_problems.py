"""Input generators (host, CPU): the hybrid linear-log radial grid of the paper's SN runs and the
SN-like wedge built on it."""
import numpy as np
import pytest

from paper_2503_04428_amd import problems as P


def test_hybrid_linlog_faces():
    f = P.hybrid_linlog_faces(0.1, 1.0, 10.0, 64, 96)
    d = np.diff(f)
    assert len(f) == 64 + 96 + 1 and f[0] == 0.1 and f[-1] == 10.0
    assert f[64] == pytest.approx(1.0, rel=1e-15)
    assert np.all(d > 0)
    assert np.allclose(d[:64], 0.9 / 64, rtol=1e-12)
    assert d[64] == pytest.approx(d[63], rel=1e-9)          # continuous spacing at the break
    q = d[65:] / d[64:-1]
    assert np.allclose(q[:-1], q[0], rtol=1e-9) and q[0] > 1  # constant growth beyond it
    with pytest.raises(ValueError):
        P.hybrid_linlog_faces(0.1, 1.0, 1.5, 64, 96)          # cannot widen


@pytest.mark.parametrize("ndim", [1, 2, 3])
def test_sn_wedge_inputs(ndim):
    pr = P.sn_wedge3d(n_lin=16, n_log=16, nth=8, nph=8, ndim=ndim)
    assert pr.eos == "gas_rad" and pr.ni_heating and pr.dual_energy and pr.gravity == "point"
    assert pr.U0.shape == (8,) + tuple(reversed(pr.n))
    U = pr.U0
    e = U[4] - 0.5 * (U[1] ** 2 + U[2] ** 2 + U[3] ** 2) / U[0]
    assert np.all(U[0] > 0) and np.all(e > 0)
    assert np.allclose(U[-1], e, rtol=1e-14)
    assert U[5].max() > 0 and U[6].max() > 0
