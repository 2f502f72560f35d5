"""Pins of the FP64 oracle against what the paper and the mathematics fix: closed forms,
invariants, exact solutions, special cases and brute force on tiny inputs."""
import math

import numpy as np
import pytest

from oracle import exact
from oracle import oracle as O
from paper_2503_04428_amd import problems as P


# ---------------------------------------------------------------------------- limiters

@pytest.mark.parametrize("a,b,vl,mm,va", [
    (1.0, 3.0, 1.5, 1.0, 1.2),
    (3.0, 1.0, 1.5, 1.0, 1.2),
    (-2.0, -2.0, -2.0, -2.0, -2.0),
    (-1.0, -4.0, -1.6, -1.0, -5.0 * 4.0 / 17.0),
    (1.0, -1.0, 0.0, 0.0, 0.0),
    (0.0, 5.0, 0.0, 0.0, 0.0),
])
def test_limiter_closed_forms(a, b, vl, mm, va):
    assert O.limiter("vanleer", a, b) == pytest.approx(vl, rel=1e-15)
    assert O.limiter("minmod", a, b) == pytest.approx(mm, rel=1e-15)
    assert O.limiter("vanalbada", a, b) == pytest.approx(va, rel=1e-15)
    assert O.limiter("none", a, b) == 0.0


def test_limiters_lie_in_tvd_region():
    rng = np.random.default_rng(0)
    for _ in range(2000):
        a, b = rng.normal(size=2)
        for name in ("vanleer", "minmod", "vanalbada"):
            s = O.limiter(name, a, b)
            if a * b <= 0:
                assert s == 0.0
            else:
                # Sweby: 0 <= s/a <= min(2, 2 b/a)
                phi = s / a
                assert -1e-15 <= phi <= min(2.0, 2.0 * b / a) + 1e-12


# ---------------------------------------------------------------------------- Riemann solvers

def _cons(rho, u, p, f=(), g=1.4):
    u = np.asarray(u, dtype=float)
    return np.array([rho, rho * u[0], rho * u[1], rho * u[2],
                     p / (g - 1) + 0.5 * rho * float(u @ u)] + [rho * x for x in f])


def _phys(q, d, g=1.4):
    rho = q[0]
    u = q[1:4] / rho
    p = (g - 1) * (q[4] - 0.5 * rho * float(u @ u))
    F = np.array([q[1 + d], q[1 + d] * u[0], q[1 + d] * u[1], q[1 + d] * u[2], u[d] * (q[4] + p)]
                 + [q[1 + d] * q[v] / rho for v in range(5, len(q))])
    F[1 + d] += p
    return F


@pytest.mark.parametrize("solver", ["hll", "hllc"])
@pytest.mark.parametrize("d", [0, 1, 2])
def test_riemann_consistency(solver, d):
    rng = np.random.default_rng(d)
    for _ in range(50):
        q = _cons(rng.uniform(0.1, 3), rng.uniform(-2, 2, 3), rng.uniform(0.1, 3), [rng.uniform()])
        F = O.riemann_flux(solver, d, 1.4, q, q)
        assert np.allclose(F, _phys(q, d), rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("d", [0, 1, 2])
def test_hllc_resolves_isolated_contact_exactly(d):
    """A contact (equal p and normal u, jumps in rho, tangential u, scalar) is an exact HLLC
    solution: the flux is the upwind physical flux.  HLL smears it."""
    u = np.zeros(3)
    u[d] = 0.3
    uL = u.copy(); uR = u.copy()
    uL[(d + 1) % 3] = 0.7
    uR[(d + 1) % 3] = -0.4
    qL = _cons(2.0, uL, 1.0, [1.0])
    qR = _cons(0.5, uR, 1.0, [0.0])
    F = O.riemann_flux("hllc", d, 1.4, qL, qR)
    assert np.allclose(F, _phys(qL, d), rtol=1e-13, atol=1e-14)
    Fh = O.riemann_flux("hll", d, 1.4, qL, qR)
    assert not np.allclose(Fh, _phys(qL, d), rtol=1e-3)


@pytest.mark.parametrize("solver", ["hll", "hllc"])
def test_riemann_mirror_symmetry_and_wall(solver):
    """Mirror images give mirrored fluxes; a state against its own mirror (a reflective wall)
    gives zero mass, energy and scalar flux (S* = 0 exactly; the F + S (U* - U) form leaves
    round-off)."""
    rng = np.random.default_rng(5)
    for _ in range(50):
        qL = _cons(rng.uniform(0.1, 3), rng.uniform(-2, 2, 3), rng.uniform(0.1, 3), [rng.uniform()])
        qR = _cons(rng.uniform(0.1, 3), rng.uniform(-2, 2, 3), rng.uniform(0.1, 3), [rng.uniform()])
        M = np.ones(6); M[1] = -1
        F = O.riemann_flux(solver, 0, 1.4, qL, qR)
        Fm = O.riemann_flux(solver, 0, 1.4, qR * M, qL * M)
        assert np.allclose(Fm, -F * M, rtol=1e-12, atol=1e-12)
        Fw = O.riemann_flux(solver, 0, 1.4, qL * M, qL)
        scale = np.abs(_phys(qL, 0)).max() + abs(qL[0]) * 10
        assert abs(Fw[0]) < 1e-15 * scale and abs(Fw[4]) < 1e-15 * scale and abs(Fw[5]) < 1e-15 * scale


def test_hllc_supersonic_upwinding():
    qL = _cons(1.0, [5.0, 0, 0], 1.0)
    qR = _cons(0.5, [4.0, 0, 0], 0.3)
    assert np.array_equal(O.riemann_flux("hllc", 0, 1.4, qL, qR), _phys(qL, 0))
    assert np.array_equal(O.riemann_flux("hll", 0, 1.4, qR * [1, -1, 1, 1, 1], qL * [1, -1, 1, 1, 1])[:1],
                          _phys(qL * [1, -1, 1, 1, 1], 0)[:1])


def test_hllc_flux_close_to_godunov_for_weak_waves():
    """For a weak Riemann problem the HLLC flux agrees with the exact Godunov flux to second
    order in the jump."""
    g = 1.4
    for eps in (1e-2, 5e-3):
        rL, uL, pL = 1.0, 0.1, 1.0
        rR, uR, pR = 1.0 + eps, 0.1 - eps, 1.0 + 2 * eps
        r, u, p = exact.sample(rL, uL, pL, rR, uR, pR, np.array([0.0]), g)
        qs = _cons(r[0], [u[0], 0, 0], p[0])
        Fex = _phys(qs, 0)
        F = O.riemann_flux("hllc", 0, g, _cons(rL, [uL, 0, 0], pL), _cons(rR, [uR, 0, 0], pR))
        assert np.max(np.abs(F - Fex)) < 3 * eps * eps


# ---------------------------------------------------------------------------- 1D Sod

def _sod_l1(n, limiter="vanleer"):
    pr = P.sod(n, limiter=limiter)
    o = O.Oracle(pr)
    U, t, steps, _ = o.run(pr.U0.copy(), t_end=0.2)
    f = pr.faces[0][pr.ng:pr.ng + n + 1]
    r, u, p = exact.cell_average(1.0, 0.0, 1.0, 0.125, 0.0, 0.1, f, 0.5, 0.2, sub=16)
    return np.abs(U[0, 0, 0] - r).mean(), U, steps


def test_sod_converges_to_exact_solution():
    errs = [(_sod_l1(n)[0]) for n in (128, 256, 512)]
    assert errs[0] < 4e-3
    assert errs[1] < errs[0] / 1.5 and errs[2] < errs[1] / 1.5


def test_sod_1024_accuracy_and_wave_widths():
    err, U, steps = _sod_l1(1024)
    assert err < 6e-4
    assert 500 < steps < 620
    rho = U[0, 0, 0]
    x = (np.arange(1024) + 0.5) / 1024
    # shock at 0.85044: transition 0.26557 -> 0.125 within a few cells (paper: ~2 cells)
    mid = (rho > 0.14) & (rho < 0.25) & (x > 0.8)
    assert mid.sum() <= 3
    # contact at 0.68549: 0.42632 -> 0.26557 (paper: ~4 cells; second-order vL smears a bit more)
    mid = (rho > 0.28) & (rho < 0.41) & (x > 0.6) & (x < 0.8)
    assert mid.sum() <= 16


def test_first_order_matches_plain_godunov_loop():
    """With zero slopes the MUSCL-Hancock step is Godunov's first-order scheme:
    U_i <- U_i + dt/dx (F(U_{i-1}, U_i) - F(U_i, U_{i+1})), with the oracle's flux function."""
    pr = P.sod(16, limiter="none")
    o = O.Oracle(pr)
    U = pr.U0.copy()
    dx = 1.0 / 16
    for _ in range(5):
        dt, _ = o.compute_dt(U)
        Un, st = o.step(U, dt)
        q = U[:, 0, 0, :].T
        qg = np.vstack([q[:1], q, q[-1:]])
        ref = np.empty_like(q)
        for i in range(16):
            Fm = O.riemann_flux("hllc", 0, 1.4, qg[i], qg[i + 1])
            Fp = O.riemann_flux("hllc", 0, 1.4, qg[i + 1], qg[i + 2])
            ref[i] = q[i] + dt / dx * (Fm - Fp)
        # the scheme feeds the solver cons(prim(U)), equal to U up to round-off
        assert np.allclose(Un[:, 0, 0, :].T, ref, rtol=1e-14, atol=1e-15)
        U = Un


# ---------------------------------------------------------------------------- invariants

@pytest.mark.parametrize("ndim", [1, 2, 3])
@pytest.mark.parametrize("riemann", ["hll", "hllc"])
def test_conservation_periodic(ndim, riemann):
    n = {1: (64,), 2: (20, 14), 3: (10, 9, 8)}[ndim]
    pr = P.random_periodic(n=n, ndim=ndim, nscalar=2, seed=ndim, riemann=riemann)
    o = O.Oracle(pr)
    U = pr.U0.copy()
    t0 = o.totals(U)
    U, _, _, _ = o.run(U, nsteps=40)
    t1 = o.totals(U)
    scale = np.abs(pr.U0).reshape(pr.nvar, -1).max(axis=1)
    assert np.all(np.abs(t1 - t0) <= 1e-13 * scale)


def test_free_stream_stays_uniform():
    pr = P.random_periodic(n=(8, 7, 6), ndim=3, nscalar=1)
    U = pr.U0.copy()
    vals = np.array([1.3, 0.4, -0.2, 0.7, 3.1, 0.6])
    U[:] = vals[:, None, None, None]
    o = O.Oracle(pr)
    U1, _, _, _ = o.run(U, nsteps=20)
    assert np.all(U1 == U1[:, :1, :1, :1])
    assert np.allclose(U1[:, 0, 0, 0], vals, rtol=1e-14, atol=1e-15)


def test_mirror_and_permutation_symmetry_sedov():
    pr = P.sedov3d(n=12, nsteps=10)
    o = O.Oracle(pr)
    U, _, _, _ = o.run(pr.U0.copy(), nsteps=15)
    scale = np.maximum(np.abs(U).reshape(pr.nvar, -1).max(axis=1), 1e-300)[:, None, None, None]
    # x -> -x mirror: density even, x-momentum odd
    Ux = U[:, :, :, ::-1].copy()
    Ux[1] *= -1
    assert np.max(np.abs(U - Ux) / scale) < 1e-13
    # x <-> y permutation: swap the axes and the momenta
    Up = U.transpose(0, 1, 3, 2).copy()
    Up[[1, 2]] = Up[[2, 1]]
    assert np.max(np.abs(U - Up) / scale) < 1e-13


def test_3d_with_1d_data_equals_1d_run_bitwise():
    n = 32
    p1 = P.sod(n)
    U1 = p1.U0.copy()
    p3 = P.random_periodic(n=(n, 5, 4), ndim=3, nscalar=0, bc=[["transmissive"] * 2, ["periodic"] * 2,
                                                                   ["reflective"] * 2])
    U3 = np.broadcast_to(U1, (5, 4, 5, n)).copy()
    o1, o3 = O.Oracle(p1), O.Oracle(p3)
    for _ in range(8):
        dt, _ = o1.compute_dt(U1)
        U1, _ = o1.step(U1, dt)
        U3, _ = o3.step(U3, dt)
    assert np.array_equal(U3, np.broadcast_to(U1, U3.shape))


def test_free_fall_under_uniform_gravity_is_exact():
    """Uniform periodic state under uniform g: no flux differences, so momentum grows as
    rho g t and the energy as E0 + rho g^2 t^2 / 2 (the half-step source makes the momentum
    update midpoint-exact).  Pins the sign and the time-centring of the gravity source."""
    pr = P.free_fall()
    o = O.Oracle(pr)
    U = pr.U0.copy()
    dt = 0.01
    U1, _, steps, _ = o.run(U, nsteps=25, dt_fixed=dt)
    t = steps * dt
    g = np.array(pr.g0)
    rho = pr.U0[0, 0, 0, 0]
    for d in range(3):
        assert np.allclose(U1[1 + d], rho * g[d] * t, rtol=1e-12, atol=1e-15)
    assert np.allclose(U1[4], pr.U0[4] + 0.5 * rho * float(g @ g) * t * t, rtol=1e-13)
    assert np.allclose(U1[0], rho, rtol=1e-15)


def test_dt_closed_form():
    pr = P.random_periodic(n=(6, 5, 4), ndim=3, nscalar=0)
    U = pr.U0.copy()
    rho, u, p = 2.0, np.array([0.3, -0.5, 0.1]), 1.5
    U[0] = rho; U[1:4] = (rho * u)[:, None, None, None]; U[4] = p / 0.4 + 0.5 * rho * u @ u
    o = O.Oracle(pr)
    dt, st = o.compute_dt(U)
    c = math.sqrt(1.4 * p / rho)
    s = (abs(u[0]) + c) * 6 + (abs(u[1]) + c) * 5 + (abs(u[2]) + c) * 4
    assert st == 0 and dt == pytest.approx(0.5 / s, rel=1e-14)


@pytest.mark.parametrize("what", ["rho", "p", "nan"])
def test_nonphysical_state_is_reported(what):
    pr = P.random_periodic(n=(6, 5, 4), ndim=3, nscalar=0)
    U = pr.U0.copy()
    if what == "rho":
        U[0, 1, 2, 3] = -1.0
    elif what == "p":
        U[4, 1, 2, 3] = 0.0
    else:
        U[2, 1, 2, 3] = np.nan
    o = O.Oracle(pr)
    _, st = o.compute_dt(U)
    assert st == O.ENONPHYS
    _, st = o.step(U, 1e-3)
    assert st == O.ENONPHYS


def test_step_box_matches_full_step():
    pr = P.random_wedge(nr=9, nth=7, nph=6, gravity="point_monopole", bc=[["reflective", "transmissive"],
                                                                         ["reflective"] * 2, ["periodic"] * 2])
    o = O.Oracle(pr)
    U = pr.U0
    dt, _ = o.compute_dt(U)
    full, _ = o.step(U, dt)
    for lo, hi in [((0, 0, 0), (1, 1, 1)), ((3, 2, 1), (9, 5, 6)), ((8, 6, 5), (9, 7, 6))]:
        box, _ = o.step_box(U, dt, lo, hi)
        assert np.array_equal(box, full[:, lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]])


# ---------------------------------------------------------------------------- spherical

def test_static_wedge_stays_static():
    """Uniform rho and P at rest with reflective walls: the pressure terms of the geometric
    sources must cancel the flux divergence of P on every face."""
    pr = P.static_wedge()
    o = O.Oracle(pr)
    U, _, _, _ = o.run(pr.U0.copy(), nsteps=50)
    cs = math.sqrt(5.0 / 3.0)
    assert np.max(np.abs(U[1:4] / U[0])) < 1e-13 * cs
    assert np.max(np.abs(U[0] - 1.0)) < 1e-13


@pytest.mark.parametrize("ndim", [2, 3])
def test_wedge_mass_and_angular_momentum(ndim):
    """Reflective r/theta walls and periodic phi: mass, energy and the discrete angular momentum
    L_z = sum R_i S_j (rho u_phi) dV (R = mean face radius, S = mean face sin(theta)) are
    conserved; the eq. source_terms_1 discretisation makes the latter telescope."""
    pr = P.random_wedge(nr=10, nth=8, nph=6, ndim=ndim, bc=[["reflective"] * 2, ["reflective"] * 2,
                                                            ["periodic"] * 2])
    o = O.Oracle(pr)
    fr = pr.faces[0][pr.ng:pr.ng + pr.n[0] + 1]
    ft = pr.faces[1][pr.ng:pr.ng + pr.n[1] + 1] if ndim >= 2 else pr.faces[1]
    fp = pr.faces[2][pr.ng:pr.ng + pr.n[2] + 1] if ndim >= 3 else pr.faces[2]
    R = 0.5 * (fr[1:] + fr[:-1])
    S = 0.5 * (np.sin(ft[1:]) + np.sin(ft[:-1]))
    dV = ((fr[1:] ** 3 - fr[:-1] ** 3) / 3)[None, None, :] * (np.cos(ft[:-1]) - np.cos(ft[1:]))[None, :, None] \
        * np.diff(fp)[:, None, None]
    lever = R[None, None, :] * S[None, :, None]

    def inv(U):
        return np.array([(U[0] * dV).sum(), (U[4] * dV).sum(), (U[3] * lever * dV).sum()])

    U = pr.U0.copy()
    i0 = inv(U)
    U, _, _, _ = o.run(U, nsteps=30)
    i1 = inv(U)
    assert abs(i1[0] - i0[0]) < 1e-13 * abs(i0[0])
    assert abs(i1[1] - i0[1]) < 1e-13 * abs(i0[1])
    scale = (np.abs(U[3]) * lever * dV).sum()
    assert abs(i1[2] - i0[2]) < 1e-13 * scale


def test_point_gravity_first_step():
    """From rest with uniform rho and P, one step changes the radial momentum by dt rho g(r_c)
    with g = -G Mc / r_c^2 (eq. point_gravity, pointing inward), up to the second-order effect of
    the half-step velocity on the pressure terms.  Cells next to the reflective r walls are
    excluded: there the wall pushes back on the falling gas."""
    pr = P.static_wedge().with_(gravity="point", G=1.0, Mc=2.0)
    o = O.Oracle(pr)
    dt = 1e-4
    U1, _ = o.step(pr.U0, dt)
    fr = pr.faces[0][pr.ng:pr.ng + pr.n[0] + 1]
    rc = 0.5 * (fr[1:] + fr[:-1])
    expect = -dt * 1.0 * 2.0 / rc ** 2
    assert np.allclose(U1[1][:, :, 1:-1], expect[None, None, 1:-1], rtol=1e-6)


def test_enclosed_mass_closed_form():
    """Uniform density: M(r_i) = (4 pi/3) rho [(r_{i-1/2}^3 - r_0^3) + (r_{i+1/2}^3 - r_{i-1/2}^3)/2]."""
    pr = P.static_wedge(nr=12).with_(gravity="point_monopole", G=1.0, Mc=1.0)
    U = pr.U0.copy()
    U[0] = 0.7
    m = O.Oracle(pr).enclosed_mass(U)
    fr = pr.faces[0][pr.ng:pr.ng + pr.n[0] + 1]
    expect = 4 * math.pi / 3 * 0.7 * ((fr[:-1] ** 3 - fr[0] ** 3) + 0.5 * (fr[1:] ** 3 - fr[:-1] ** 3))
    assert np.allclose(m, expect, rtol=1e-13)


def test_spherical_sedov_1d_shock_radius():
    """Paper App. C.4: 1D spherical Sedov with E1 = 1, gamma = 1.4; the shock follows
    d_sh = xi0 (E t^2/rho0)^(1/5)."""
    pr = P.sedov_sph1d(n=200)
    o = O.Oracle(pr)
    t_end = 0.3
    U, t, steps, _ = o.run(pr.U0.copy(), t_end=t_end)
    fr = pr.faces[0][pr.ng:pr.ng + pr.n[0] + 1]
    rc = 0.5 * (fr[1:] + fr[:-1])
    r_peak = rc[np.argmax(U[0, 0, 0])]
    r_ex = exact.sedov_radius(1.0, 1.0, t_end, 1.4)
    assert abs(r_peak - r_ex) < 3 * (fr[1] - fr[0])
    # total energy conserved (the outer boundary is not reached)
    dV = 4 * math.pi * (fr[1:] ** 3 - fr[:-1] ** 3) / 3
    e0 = (pr.U0[4, 0, 0] * dV).sum()
    assert abs((U[4, 0, 0] * dV).sum() - e0) < 1e-12 * e0


@pytest.mark.slow
def test_cartesian_sedov_3d_shock_radius():
    pr = P.sedov3d(n=32)
    o = O.Oracle(pr)
    t_end = 0.06
    U, t, steps, _ = o.run(pr.U0.copy(), t_end=t_end)
    f = pr.faces[0][pr.ng:pr.ng + 33]
    xc = 0.5 * (f[1:] + f[:-1])
    Z, Y, X = np.meshgrid(xc, xc, xc, indexing="ij")
    r = np.sqrt(X * X + Y * Y + Z * Z)
    bins = np.linspace(0, 1, 33)
    idx = np.digitize(r.ravel(), bins)
    prof = np.array([U[0].ravel()[idx == k].mean() if np.any(idx == k) else 0 for k in range(1, 33)])
    r_peak = 0.5 * (bins[:-1] + bins[1:])[np.argmax(prof)]
    r_ex = exact.sedov_radius(1.0, 1.0, t_end, 1.4)
    assert abs(r_peak - r_ex) < 0.1 * r_ex


# ---------------------------------------------------------------------------- MLP limiter

def _mlp_const(b3):
    w = np.zeros(O.MLP_NPARAM)
    w[1248] = b3
    return w


def test_mlp_torch_reference_forward_and_grad():
    """The oracle's network equals torch's Linear/GELU(tanh)/sigmoid composition in FP64, and
    its hand-written backward equals autograd."""
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(1)
    w = rng.normal(scale=0.5, size=O.MLP_NPARAM)
    B = 16
    x = rng.uniform(-1, 1, size=(B, 4))
    a = rng.uniform(-1, 1, size=B)
    t = rng.uniform(-1, 1, size=B)
    wt = rng.uniform(0.5, 1.5, size=B)
    tw = torch.tensor(w, requires_grad=True)
    W1 = tw[:128].view(32, 4); b1 = tw[128:160]; W2 = tw[160:1184].view(32, 32); b2 = tw[1184:1216]
    w3 = tw[1216:1248]; b3 = tw[1248]
    tx = torch.tensor(x)
    gelu = lambda z: torch.nn.functional.gelu(z, approximate="tanh")
    phi = 2 * torch.sigmoid(gelu(gelu(tx @ W1.T + b1) @ W2.T + b2) @ w3 + b3)
    for b in range(4):
        assert O.mlp_phi(w, x[b]) == pytest.approx(float(phi[b]), rel=1e-13)
    ta, tt, twt = torch.tensor(a), torch.tensor(t), torch.tensor(wt)
    L = (twt * (phi * ta - tt) ** 2).sum() / twt.sum()
    L.backward()
    loss, g = O.mlp_loss_grad(w, x, a, t, wt)
    assert loss == pytest.approx(float(L), rel=1e-13)
    assert np.allclose(g, tw.grad.numpy(), rtol=1e-11, atol=1e-14)


def test_mlp_gradient_finite_differences():
    rng = np.random.default_rng(2)
    w = rng.normal(scale=0.4, size=O.MLP_NPARAM)
    B = 8
    x = rng.uniform(-1, 1, size=(B, 4)); a = rng.uniform(-1, 1, size=B); t = rng.uniform(-1, 1, size=B)
    wt = np.ones(B)
    _, g = O.mlp_loss_grad(w, x, a, t, wt)
    for k in rng.choice(O.MLP_NPARAM, size=40, replace=False):
        h = 1e-6
        wp = w.copy(); wp[k] += h
        wm = w.copy(); wm[k] -= h
        fd = (O.mlp_loss_grad(wp, x, a, t, wt)[0] - O.mlp_loss_grad(wm, x, a, t, wt)[0]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(g[k])) + 1e-9


def test_mlp_slope_special_cases():
    """phi = 0 gives zero slopes; phi = 2 gives 2a where 2 <= 2r and van Leer elsewhere; the network
    is skipped (zero slope) wherever the TVD region forces it."""
    w0, w2 = _mlp_const(-1000.0), _mlp_const(1000.0)
    rng = np.random.default_rng(3)
    for _ in range(500):
        d = rng.normal(size=4)
        cm, cp = rng.uniform(0.3, 0.7, size=2)
        a, b = cm * d[1], cp * d[2]
        assert O.mlp_slope(w0, d, cm, cp) == 0.0
        s2 = O.mlp_slope(w2, d, cm, cp)
        if d[1] * d[2] <= 0:
            assert s2 == 0.0
        elif b / a >= 1.0:
            assert s2 == 2.0 * a
        else:
            assert s2 == pytest.approx(O.limiter("vanleer", a, b), rel=1e-15)


def test_mlp_phi0_equals_first_order_scheme():
    pr = P.random_periodic(n=(9, 8, 7), ndim=3, nscalar=1, ng=3)
    o_none = O.Oracle(pr.with_(limiter="none"))
    o_mlp = O.Oracle(pr.with_(limiter="mlp"), mlp_weights=_mlp_const(-1000.0))
    U = pr.U0
    dt, _ = o_none.compute_dt(U)
    a, _ = o_none.step(U, dt)
    b, _ = o_mlp.step(U, dt)
    assert np.array_equal(a, b)


# ---------------------------------------------------------------------------- learned-limiter samples

def _fine_batch(prims, nf):
    """[5][nrows][nf] conserved state from per-row primitive profiles (rho, u, p) callables."""
    xf = (np.arange(nf) + 0.5) / nf
    U = np.zeros((5, len(prims), nf))
    for r, (rho, u, p) in enumerate(prims):
        R, V, Pp = rho(xf), u(xf), p(xf)
        U[0, r] = R
        U[1, r] = R * V
        U[4, r] = Pp / 0.4 + 0.5 * R * V * V
    return U


def test_mlp_samples_linear_profiles():
    """A linear fine profile of a conserved density restricts to a linear coarse profile: all four
    differences equal (x = +-1), and the least-squares label slope equals the coarse difference
    (t = a), so phi = 1 is the exact answer there."""
    nf, R = 64, 4
    U = _fine_batch([(lambda x: 1 + 0.5 * x, lambda x: 0 * x, lambda x: 1 + 0 * x),
                     (lambda x: 2 - x, lambda x: 0 * x, lambda x: 0.5 + 0 * x)], nf)
    x, a, t, wt = O.mlp_features(U, R, 1.4)
    x = x.reshape(2, nf // R, 5, 4)
    a, t, wt = (v.reshape(2, nf // R, 5) for v in (a, t, wt))
    inner = slice(2, nf // R - 2)
    assert np.all(wt[:, inner, 0] == 1) and np.all(wt[:, :2] == 0) and np.all(wt[:, -2:] == 0)
    sign = np.array([1.0, -1.0])[:, None]
    assert np.allclose(x[:, inner, 0], sign[:, :, None], rtol=1e-13)
    assert np.allclose(a[:, inner, 0], sign, rtol=1e-13)
    assert np.allclose(t[:, inner, 0], sign, rtol=1e-12)
    # flat velocity and pressure: no sample
    assert np.all(wt[:, :, 1:] == 0)


def test_mlp_samples_piecewise_constant_fine_data_has_zero_label():
    """Fine data constant inside every coarse cell (a staircase) has zero least-squares slope."""
    nf, R = 64, 4
    stairs = lambda x: 1.0 + np.floor(x * nf / R) * 0.1
    U = _fine_batch([(stairs, lambda x: 0 * x, lambda x: 1 + 0 * x)], nf)
    x, a, t, wt = O.mlp_features(U, R, 1.4)
    live = wt > 0
    assert live.sum() > 0
    assert np.all(np.abs(t[live]) < 1e-12)
    assert np.allclose(a[live], 1.0)


def test_mlp_samples_skip_extrema():
    """At a density maximum the two central differences change sign: no sample (TVD forces 0)."""
    nf, R = 64, 4
    U = _fine_batch([(lambda x: 1.0 + np.exp(-((x - 0.5) / 0.1) ** 2), lambda x: 0 * x, lambda x: 1 + 0 * x)], nf)
    x, a, t, wt = O.mlp_features(U, R, 1.4)
    wt = wt.reshape(nf // R, 5)[:, 0]
    xx = x.reshape(nf // R, 5, 4)[:, 0]
    peak = np.argmax(U[0, 0].reshape(-1, R).mean(axis=1))
    assert wt[peak] == 0
    assert np.all(np.abs(xx[wt > 0]) <= 1.0 + 1e-15)
