"""Pins of the oracle's grid shift (Sect. 3.1.1, moving grid: the faces of axis 0 move and the
state is carried over conservatively): identity at zero shift, exactness for linear profiles
(Cartesian and spherical, uniform and stretched grids) against the closed-form cell averages,
conservation on a periodic grid, a shift by one uniform cell is an index shift, second-order
accuracy for a smooth profile, the slabs that leave and enter at transmissive boundaries, uniform
states stay uniform, positivity across a blast, and the limit on the shift."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2503_04428_amd import problems as P


def _cart1d(f, U, bc=("transmissive", "transmissive"), nscalar=0):
    n = len(f) - 1
    return P.Problem(name="shift", ndim=1, geom="cart", n=(n, 1, 1), ng=2,
                     faces=[P.ghost_faces(f, 2, bc[0], bc[1]), np.array([0.0, 1.0]), np.array([0.0, 1.0])],
                     nscalar=nscalar, gamma=1.4, cfl=0.5, riemann="hllc", limiter="vanleer",
                     bc=[list(bc), ["periodic"] * 2, ["periodic"] * 2], U0=U)


def _sph1d(f, U):
    n = len(f) - 1
    bc = ("reflective", "transmissive")
    return P.Problem(name="shift", ndim=1, geom="sph", n=(n, 1, 1), ng=2,
                     faces=[P.ghost_faces(f, 2, bc[0], bc[1]), np.array([0.0, math.pi]), np.array([0.0, 2 * math.pi])],
                     nscalar=0, gamma=1.4, cfl=0.5, riemann="hllc", limiter="vanleer",
                     bc=[list(bc), ["periodic"] * 2, ["periodic"] * 2], U0=U)


def _linear_state(xc, coef):
    """Every field linear in x: U_v = a_v + b_v x, positive and with P > 0."""
    U = np.zeros((5, 1, 1, len(xc)))
    for v, (a, b) in enumerate(coef):
        U[v, 0, 0] = a + b * xc
    return U


COEF = [(2.0, 0.3), (0.1, -0.05), (0.2, 0.02), (-0.1, 0.04), (20.0, 1.5)]


def test_zero_shift_is_the_identity():
    pr = P.random_periodic(n=(13, 7, 5), ndim=3, nscalar=2, seed=81)
    o = O.Oracle(pr)
    U = o.shift_grid(pr.U0, 0.0)
    assert np.allclose(U, pr.U0, rtol=1e-14, atol=1e-16)


@pytest.mark.parametrize("grid", ["uniform", "stretched"])
@pytest.mark.parametrize("delta_frac", [0.37, -0.61, 1.0])
def test_linear_profiles_are_exact_cartesian(grid, delta_frac):
    n = 24
    if grid == "uniform":
        f = np.linspace(0.0, 1.0, n + 1)
    else:
        f = np.cumsum(np.concatenate([[0.0], 0.02 * 1.07 ** np.arange(n)]))
    xc = 0.5 * (f[:-1] + f[1:])  # the cell average of a linear function is its value at the midpoint
    pr = _cart1d(f, _linear_state(xc, COEF))
    d = delta_frac * np.diff(f).min()
    U = O.Oracle(pr).shift_grid(pr.U0, d)
    xn = xc + d
    ref = _linear_state(xn, COEF)
    # away from the boundaries (their images are not linear continuations)
    assert np.allclose(U[..., 2:-2], ref[..., 2:-2], rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("delta_frac", [0.45, -0.8])
def test_linear_profiles_are_exact_spherical(delta_frac):
    """Spherical shells on a log grid: the average of a + b r over a shell is a + b times the
    shell's volume centroid (3/4)(r+^4 - r-^4)/(r+^3 - r-^3)."""
    n = 30
    f = 0.5 * 20.0 ** (np.arange(n + 1) / n)

    def cen(a, b):
        return 0.75 * (b ** 4 - a ** 4) / (b ** 3 - a ** 3)

    pr = _sph1d(f, _linear_state(cen(f[:-1], f[1:]), COEF))
    d = delta_frac * np.diff(f).min()
    U = O.Oracle(pr).shift_grid(pr.U0, d)
    ref = _linear_state(cen(f[:-1] + d, f[1:] + d), COEF)
    assert np.allclose(U[..., 2:-2], ref[..., 2:-2], rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("delta", [0.013, -0.029])
def test_periodic_shift_conserves(delta):
    pr = P.random_periodic(n=(24, 9, 7), ndim=3, nscalar=2, seed=82)
    o = O.Oracle(pr)
    t0 = o.totals(pr.U0)
    U = o.shift_grid(pr.U0, delta)
    t1 = o.totals(U)
    assert np.allclose(t1, t0, rtol=1e-13, atol=1e-14 * np.abs(t0).max())


def test_shift_by_one_uniform_cell_is_an_index_shift():
    pr = P.random_periodic(n=(16, 5, 4), ndim=3, nscalar=1, seed=83)
    dx = 1.0 / 16
    o = O.Oracle(pr)
    U = o.shift_grid(pr.U0, dx)
    assert np.allclose(U, np.roll(pr.U0, -1, axis=3), rtol=1e-13, atol=1e-15)
    o2 = O.Oracle(pr)
    U = o2.shift_grid(pr.U0, -dx)
    assert np.allclose(U, np.roll(pr.U0, 1, axis=3), rtol=1e-13, atol=1e-15)


def test_second_order_for_a_smooth_profile():
    errs = []
    for n in (32, 64, 128):
        f = np.linspace(0.0, 1.0, n + 1)
        # exact cell averages of 2 + sin(2 pi x) (density) on the old and the shifted grid
        def avg(a, b):
            return 2.0 + (np.cos(2 * np.pi * a) - np.cos(2 * np.pi * b)) / (2 * np.pi * (b - a))
        U = np.zeros((5, 1, 1, n))
        U[0, 0, 0] = avg(f[:-1], f[1:])
        U[4, 0, 0] = 10.0
        pr = _cart1d(f, U, bc=("periodic", "periodic"))
        d = 0.3 / n
        Un = O.Oracle(pr).shift_grid(pr.U0, d)
        errs.append(np.abs(Un[0, 0, 0] - avg(f[:-1] + d, f[1:] + d)).mean())
    rates = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(rates) > 1.8, (errs, rates)


@pytest.mark.parametrize("d", [0.04, -0.07])
def test_transmissive_slabs_leave_and_enter(d):
    """Transmissive boundaries copy the edge cells, whose profiles are therefore flat: shifting a
    linear state by d changes each total by d (U_last - U_first) (the slab entering at one end
    minus the slab leaving at the other), and a uniform state stays uniform."""
    n = 20
    f = np.linspace(0.0, 2.0, n + 1)
    xc = 0.5 * (f[:-1] + f[1:])
    U = _linear_state(xc, COEF)
    pr = _cart1d(f, U)
    o = O.Oracle(pr)
    t0 = o.totals(U)
    Un = o.shift_grid(U, d)
    t1 = o.totals(Un)  # on the shifted faces (the oracle's faces moved with it)
    assert np.allclose(t1 - t0, d * (U[:, 0, 0, -1] - U[:, 0, 0, 0]), rtol=1e-11, atol=1e-14)
    V = np.broadcast_to(np.array([1.5, 0.3, 0.0, 0.0, 4.0])[:, None, None, None], U.shape).copy()
    Vn = O.Oracle(pr).shift_grid(V, d)
    assert np.allclose(Vn, V, rtol=1e-14, atol=0)


def test_uniform_state_stays_uniform_spherical():
    n = 24
    f = 1.0 * 5.0 ** (np.arange(n + 1) / n)
    U = np.zeros((5, 1, 1, n))
    U[0] = 0.7
    U[4] = 3.0
    pr = _sph1d(f, U)
    Un = O.Oracle(pr).shift_grid(U, 0.9 * np.diff(f).min())
    assert np.allclose(Un, U, rtol=1e-13, atol=1e-15)


def test_positive_across_a_blast():
    pr = P.sedov3d(n=16)
    o = O.Oracle(pr)
    U = pr.U0
    for d in (0.1, -0.12):
        Un = O.Oracle(pr).shift_grid(U, d)
        e = Un[4] - 0.5 * (Un[1] ** 2 + Un[2] ** 2 + Un[3] ** 2) / Un[0]
        assert np.all(Un[0] > 0) and np.all(e > 0)
        assert np.allclose(o.totals(Un)[0], o.totals(U)[0], rtol=1e-12)  # uniform density near the edges


def test_shift_limits():
    pr = P.random_periodic(n=(10, 4, 4), ndim=3, nscalar=1, seed=84)
    with pytest.raises(ValueError):
        O.Oracle(pr).shift_grid(pr.U0, 0.11)
    w = P.static_wedge()
    with pytest.raises(ValueError):
        O.Oracle(w).shift_grid(w.U0, -1.5)
