"""Seeded synthetic problem setups (initial conditions and grids).

This module only builds inputs: face coordinates (including ghost faces) and
the initial conserved state U0 with layout [nvar][n3][n2][n1] (x fastest,
interior cells only), plus the run parameters.  It contains none of the
solver's arithmetic; the FP64 oracle and the HIP library both consume what
it returns and each derive their own geometry, primitives and fluxes.

Conserved variables (paper Sect. 2.1, eqs. continuity/momentum/energy/passive
scalar): U = (rho, rho*u1, rho*u2, rho*u3, E, rho*f_1 .. rho*f_ns), all three
momentum components carried in every dimension.

Configuration values are plain strings so that neither consumer depends on
the other's enum numbering:
  geom     'cart' | 'sph'            (sph: x1 = r, x2 = theta, x3 = phi)
  riemann  'hll' | 'hllc'
  limiter  'none' | 'minmod' | 'vanleer' | 'vanalbada' | 'mlp'
  bc       'periodic' | 'transmissive' | 'reflective'   per axis (lo, hi)
  gravity  'none' | 'uniform' | 'point' | 'point_monopole'
  precision 'fp64' | 'fp32'
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

GHOSTS_DEFAULT = 2
GHOSTS_MLP = 3


@dataclass
class Problem:
    name: str
    ndim: int
    geom: str
    n: tuple                      # (n1, n2, n3); inactive axes have n = 1
    ng: int
    faces: list                   # per axis float64 arrays (ghost faces incl.)
    nscalar: int
    gamma: float
    cfl: float
    riemann: str
    limiter: str
    bc: list                      # [[lo, hi]] * 3
    U0: np.ndarray                # float64 [nvar][n3][n2][n1]
    precision: str = "fp64"
    gravity: str = "none"
    g0: tuple = (0.0, 0.0, 0.0)
    G: float = 0.0
    Mc: float = 0.0
    t_end: float = 0.0
    nsteps: int = 0
    meta: dict = field(default_factory=dict)
    dual_energy: bool = False     # last field = monitored internal energy e (Sect. 2.5)
    de_eps: float = 1e-6          # criterion of the blend factor alpha
    eos: str = "gas"              # "gas" (eq. eos_gas) or "gas_rad" (gas + radiation, Sect. 2.3)
    eos_R: float = 0.0            # gas + radiation: specific gas constant k_b / (mu m_u)
    eos_arad: float = 0.0         # gas + radiation: radiation constant
    ni_heating: bool = False      # 56Ni decay heating (Sect. 2.4, eq. heating_ni)
    ni_scalar: int = 0            # the passive scalar carrying rho f_Ni
    ni_Q: tuple = (0.0, 0.0)      # energy per decay of 56Ni and 56Co
    ni_tau: tuple = (1.0, 2.0)    # lifetimes of 56Ni and 56Co
    ni_m: float = 1.0             # mass of a 56Ni nucleus (56 m_u)
    centroid: bool = False        # reconstruction about the volume centroids of spherical cells

    @property
    def nvar(self) -> int:
        return 5 + self.nscalar + (1 if self.dual_energy else 0)

    @property
    def ncells(self) -> int:
        return int(self.n[0]) * int(self.n[1]) * int(self.n[2])

    def with_(self, **kw) -> "Problem":
        d = dict(self.__dict__)
        d.update(kw)
        return Problem(**d)


# ----------------------------------------------------------------------------
# grids
# ----------------------------------------------------------------------------

def ghost_faces(f: np.ndarray, ng: int, bclo: str, bchi: str) -> np.ndarray:
    """Extend interior faces f[0..n] by ng ghost faces on each side.

    Periodic: the ghost cells take the geometry of the cells they wrap to.
    Reflective and transmissive: ghost cells are the mirror images of the
    boundary cells, so their widths mirror the interior widths.
    """
    f = np.asarray(f, dtype=np.float64)
    n = len(f) - 1
    lo = np.empty(ng)
    hi = np.empty(ng)
    for k in range(1, ng + 1):
        if bclo == "periodic":
            lo[ng - k] = f[0] - (f[n] - f[n - k])
        else:
            lo[ng - k] = f[0] - (f[k] - f[0])
        if bchi == "periodic":
            hi[k - 1] = f[n] + (f[k] - f[0])
        else:
            hi[k - 1] = f[n] + (f[n] - f[n - k])
    return np.concatenate([lo, f, hi])


def uniform_faces(a: float, b: float, n: int) -> np.ndarray:
    return a + (b - a) * np.arange(n + 1, dtype=np.float64) / n


def build_faces(interior: list, ndim: int, ng: int, bc: list, geom: str) -> list:
    out = []
    for d in range(3):
        if d < ndim:
            out.append(ghost_faces(interior[d], ng, bc[d][0], bc[d][1]))
        else:
            out.append(np.asarray(interior[d], dtype=np.float64))
    return out


def centers(f: np.ndarray, ng: int, n: int) -> np.ndarray:
    """Interior cell centres (face midpoints) from a ghosted face array."""
    fi = f[ng:ng + n + 1] if len(f) != n + 1 else f
    return 0.5 * (fi[:-1] + fi[1:])


def _inactive(geom: str, d: int) -> np.ndarray:
    if geom == "sph":
        return np.array([0.0, math.pi] if d == 1 else [0.0, 2.0 * math.pi])
    return np.array([0.0, 1.0])


def _pack(rho, u1, u2, u3, p, scal, gamma) -> np.ndarray:
    rho = np.asarray(rho, dtype=np.float64)
    shape = rho.shape
    nvar = 5 + len(scal)
    U = np.empty((nvar,) + shape, dtype=np.float64)
    U[0] = rho
    U[1] = rho * u1
    U[2] = rho * u2
    U[3] = rho * u3
    U[4] = p / (gamma - 1.0) + 0.5 * rho * (np.asarray(u1) ** 2 + np.asarray(u2) ** 2 + np.asarray(u3) ** 2)
    for s, f in enumerate(scal):
        U[5 + s] = rho * f
    return U


def _mk(name, ndim, geom, n, interior, ng, bc, U0, **kw) -> Problem:
    n = tuple(int(x) for x in n)
    faces = build_faces(interior, ndim, ng, bc, geom)
    return Problem(name=name, ndim=ndim, geom=geom, n=n, ng=ng, faces=faces, bc=bc,
                   U0=np.ascontiguousarray(U0), **kw)


# ----------------------------------------------------------------------------
# the five workloads
# ----------------------------------------------------------------------------

def sod(n: int = 1024, limiter: str = "vanleer", riemann: str = "hllc", ng: int = GHOSTS_DEFAULT) -> Problem:
    """1D Sod shock tube (paper App. C.1): gamma 1.4, [0,1], interface on face n/2."""
    f = uniform_faces(0.0, 1.0, n)
    xc = 0.5 * (f[:-1] + f[1:])
    left = np.arange(n) < n // 2
    rho = np.where(left, 1.0, 0.125)
    p = np.where(left, 1.0, 0.1)
    z = np.zeros(n)
    U = _pack(rho, z, z, z, p, [], 1.4).reshape(5, 1, 1, n)
    bc = [["transmissive"] * 2, ["periodic"] * 2, ["periodic"] * 2]
    return _mk("sod", 1, "cart", (n, 1, 1), [f, _inactive("cart", 1), _inactive("cart", 2)], ng, bc, U,
               nscalar=0, gamma=1.4, cfl=0.8, riemann=riemann, limiter=limiter, t_end=0.2,
               meta={"xc": xc})


def sedov3d(n: int = 256, precision: str = "fp64", nsteps: int = 200, limiter: str = "vanleer",
            ng: int = GHOSTS_DEFAULT, bc: str = "transmissive") -> Problem:
    """3D Cartesian Sedov blast on [-1,1]^3: rho 1, p 1e-5, E=1 in the central 2^3 cells,
    2 passive scalars (f1 = [r < 0.1], f2 = 1 - f1)."""
    assert n % 2 == 0
    f = uniform_faces(-1.0, 1.0, n)
    xc = 0.5 * (f[:-1] + f[1:])
    Z, Y, X = np.meshgrid(xc, xc, xc, indexing="ij")
    r = np.sqrt(X * X + Y * Y + Z * Z)
    gamma = 1.4
    rho = np.ones((n, n, n))
    p = np.full((n, n, n), 1e-5)
    z = np.zeros((n, n, n))
    f1 = (r < 0.1).astype(np.float64)
    U = _pack(rho, z, z, z, p, [f1, 1.0 - f1], gamma)
    dV = (2.0 / n) ** 3
    c = n // 2
    U[4, c - 1:c + 1, c - 1:c + 1, c - 1:c + 1] += 0.125 / dV
    bcs = [[bc, bc]] * 3
    return _mk("sedov", 3, "cart", (n, n, n), [f, f, f], ng, [list(b) for b in bcs], U,
               nscalar=2, gamma=gamma, cfl=0.5, riemann="hllc", limiter=limiter,
               precision=precision, nsteps=nsteps, meta={"E1": 1.0, "rho0": 1.0})


def rt3d(nx: int = 128, ny: int = 128, nz: int = 512, seed: int = 3, precision: str = "fp32",
         nsteps: int = 500, ng: int = GHOSTS_DEFAULT) -> Problem:
    """3D Rayleigh-Taylor stand-in: cubic cells dx = 1/512 scaled to nz; heavy (2) over light (1)
    at z = 0.5, g = -0.1 e_z, piecewise-linear hydrostatic p (p = 2.5 at the interface),
    v_z = 0.01 U(-1,1) within 0.05 of the interface, one scalar marking the heavy fluid."""
    dx = 1.0 / nz
    fx = uniform_faces(0.0, nx * dx, nx)
    fy = uniform_faces(0.0, ny * dx, ny)
    fz = uniform_faces(0.0, 1.0, nz)
    xc = 0.5 * (fx[:-1] + fx[1:])
    yc = 0.5 * (fy[:-1] + fy[1:])
    zc = 0.5 * (fz[:-1] + fz[1:])
    g = 0.1
    rho1 = np.where(zc > 0.5, 2.0, 1.0)
    p1 = 2.5 - g * rho1 * (zc - 0.5)
    rho = np.broadcast_to(rho1[:, None, None], (nz, ny, nx)).copy()
    p = np.broadcast_to(p1[:, None, None], (nz, ny, nx)).copy()
    rng = np.random.Generator(np.random.PCG64(seed))
    vz = 0.01 * rng.uniform(-1.0, 1.0, size=(nz, ny, nx))
    band = (np.abs(zc - 0.5) < 0.05)[:, None, None]
    vz = np.where(band, vz, 0.0)
    z = np.zeros_like(rho)
    fs = np.broadcast_to((zc > 0.5).astype(np.float64)[:, None, None], (nz, ny, nx)).copy()
    U = _pack(rho, z, z, vz, p, [fs], 1.4)
    bc = [["periodic"] * 2, ["periodic"] * 2, ["reflective"] * 2]
    return _mk("rt", 3, "cart", (nx, ny, nz), [fx, fy, fz], ng, bc, U,
               nscalar=1, gamma=1.4, cfl=0.5, riemann="hllc", limiter="vanleer",
               precision=precision, gravity="uniform", g0=(0.0, 0.0, -g), nsteps=nsteps)


def wedge3d(nr: int = 1024, nth: int = 128, nph: int = 128, seed: int = 4, precision: str = "fp32",
            nsteps: int = 300, ng: int = GHOSTS_DEFAULT) -> Problem:
    """Spherical wedge stand-in for the paper's red-supergiant run: log-spaced r in [1, 100],
    theta in [pi/3, 2pi/3], phi in [0, pi/3], gamma 5/3, rho = 0.01 r^-2.5 with a seeded 1%
    lognormal perturbation, hydrostatic p for point mass + enclosed mass (G = Mc = 1),
    thermal bomb (p x10) in the inner 20 shells, 4 composition shells split at r = 3, 10, 30."""
    gamma = 5.0 / 3.0
    fr = 100.0 ** (np.arange(nr + 1, dtype=np.float64) / nr)
    fth = math.pi / 3.0 + (math.pi / 3.0) * np.arange(nth + 1, dtype=np.float64) / nth
    fph = (math.pi / 3.0) * np.arange(nph + 1, dtype=np.float64) / nph
    rc = 0.5 * (fr[:-1] + fr[1:])
    rho0 = 0.01
    G, Mc = 1.0, 1.0
    rhobar = rho0 * rc ** -2.5
    # enclosed mass of the unperturbed profile, 4 pi int_1^r rho0 r^-0.5 dr
    menc = Mc + 8.0 * math.pi * rho0 * (np.sqrt(rc) - 1.0)
    p = np.empty(nr)
    p[-1] = rhobar[-1] * G * menc[-1] / (3.5 * rc[-1])
    for i in range(nr - 2, -1, -1):   # trapezoid integration of dp/dr = -rho G M / r^2, inward
        a = rhobar[i] * G * menc[i] / rc[i] ** 2
        b = rhobar[i + 1] * G * menc[i + 1] / rc[i + 1] ** 2
        p[i] = p[i + 1] + 0.5 * (a + b) * (rc[i + 1] - rc[i])
    p[:20] *= 10.0
    rng = np.random.Generator(np.random.PCG64(seed))
    zeta = rng.standard_normal(size=(nph, nth, nr))
    rho = rhobar[None, None, :] * np.exp(0.01 * zeta - 0.00005)
    P = np.broadcast_to(p[None, None, :], (nph, nth, nr)).copy()
    z = np.zeros_like(rho)
    R = np.broadcast_to(rc[None, None, :], (nph, nth, nr))
    f1 = (R < 3.0).astype(np.float64)
    f2 = ((R >= 3.0) & (R < 10.0)).astype(np.float64)
    f3 = ((R >= 10.0) & (R < 30.0)).astype(np.float64)
    f4 = (R >= 30.0).astype(np.float64)
    U = _pack(rho, z, z, z, P, [f1, f2, f3, f4], gamma)
    bc = [["reflective", "transmissive"], ["reflective"] * 2, ["reflective"] * 2]
    return _mk("wedge", 3, "sph", (nr, nth, nph), [fr, fth, fph], ng, bc, U,
               nscalar=4, gamma=gamma, cfl=0.5, riemann="hllc", limiter="vanleer",
               precision=precision, gravity="point_monopole", G=G, Mc=Mc, nsteps=nsteps)


def riemann_states(rng: np.random.Generator, count: int, ncomp: int = 3):
    """Random states drawn from the learned-limiter training distribution:
    rho log-uniform in [0.1, 10], p log-uniform in [0.01, 10], velocity U(-2, 2)."""
    rho = np.exp(rng.uniform(math.log(0.1), math.log(10.0), size=count))
    p = np.exp(rng.uniform(math.log(0.01), math.log(10.0), size=count))
    u = rng.uniform(-2.0, 2.0, size=(count, ncomp))
    return rho, u, p


def riemann_batch(nrows: int = 64, n: int = 1024, seed: int = 1000, cfl: float = 0.8,
                  precision: str = "fp64", limiter: str = "vanleer", ng: int = GHOSTS_DEFAULT,
                  mirror: bool = False) -> Problem:
    """A batch of independent 1D Riemann problems on [0, 1] (interface at 0.5), one per row of a
    Cartesian ndim-1 grid with n[1] = nrows: left/right states drawn from the learned-limiter
    training distribution (rho log-U[0.1,10], p log-U[0.01,10], u U(-2,2)), gamma 1.4,
    transmissive ends.  With mirror=True the second half of the rows are the mirror images
    (x -> -x) of the first half."""
    f = uniform_faces(0.0, 1.0, n)
    rng = np.random.Generator(np.random.PCG64(seed))
    if mirror:
        assert nrows % 2 == 0
        h = nrows // 2
        r0, u0, p0 = riemann_states(rng, 2 * h, ncomp=1)
        # rows [0, h): (left, right) = (first, second) draw; rows [h, 2h): swapped, velocity negated
        rho_s = np.concatenate([r0[:h], r0[h:], r0[h:], r0[:h]])
        p_s = np.concatenate([p0[:h], p0[h:], p0[h:], p0[:h]])
        u_s = np.concatenate([u0[:h], u0[h:], -u0[h:], -u0[:h]])
        order = np.concatenate([np.arange(h), np.arange(2 * h, 3 * h), np.arange(h, 2 * h), np.arange(3 * h, 4 * h)])
        rho_s, u_s, p_s = rho_s[order], u_s[order], p_s[order]
    else:
        rho_s, u_s, p_s = riemann_states(rng, 2 * nrows, ncomp=1)
    left = (np.arange(n) < n // 2)[None, :]
    rho = np.where(left, rho_s[:nrows, None], rho_s[nrows:, None])
    u = np.where(left, u_s[:nrows, 0][:, None], u_s[nrows:, 0][:, None])
    p = np.where(left, p_s[:nrows, None], p_s[nrows:, None])
    z = np.zeros_like(rho)
    U = _pack(rho, u, z, z, p, [], 1.4).reshape(5, 1, nrows, n)
    bc = [["transmissive"] * 2, ["periodic"] * 2, ["periodic"] * 2]
    smax = float(np.max(np.abs(u_s[:, 0]) + np.sqrt(1.4 * p_s / rho_s)))
    return _mk("riemann_batch", 1, "cart", (n, nrows, 1), [f, _inactive("cart", 1), _inactive("cart", 2)], ng, bc,
               U, nscalar=0, gamma=1.4, cfl=cfl, riemann="hllc", limiter=limiter, precision=precision,
               meta={"smax": smax, "left": (rho_s[:nrows], u_s[:nrows, 0], p_s[:nrows]),
                     "right": (rho_s[nrows:], u_s[nrows:, 0], p_s[nrows:])})


def riemann_row(batch: Problem, row: int) -> Problem:
    """One row of a batch as a stand-alone 1D problem (same grid and parameters)."""
    return batch.with_(n=(batch.n[0], 1, 1), U0=np.ascontiguousarray(batch.U0[:, :, row:row + 1, :]),
                       name=f"riemann_row{row}")


def quadrant3d(n: int = 256, seed: int = 2000, octant: bool = False, precision: str = "fp32",
               limiter: str = "vanleer", ng: int = GHOSTS_MLP, nsteps: int = 0) -> Problem:
    """Learned-limiter evaluation problem: [0,1]^3, split at x, y (and z for octants) = 0.5,
    each region a random state of the training distribution, transmissive, 5 fields."""
    f = uniform_faces(0.0, 1.0, n)
    rng = np.random.Generator(np.random.PCG64(seed))
    nreg = 8 if octant else 4
    rho_s, u_s, p_s = riemann_states(rng, nreg)
    idx = (np.arange(n) >= n // 2).astype(np.int64)
    I = idx[None, None, :]
    J = idx[None, :, None]
    K = idx[:, None, None] if octant else np.zeros((n, 1, 1), dtype=np.int64)
    reg = np.broadcast_to(I + 2 * J + 4 * K, (n, n, n))
    rho = rho_s[reg]
    p = p_s[reg]
    U = _pack(rho, u_s[reg, 0], u_s[reg, 1], u_s[reg, 2], p, [], 1.4)
    smax = float(np.max(np.abs(u_s).max(axis=1) + np.sqrt(1.4 * p_s / rho_s)))
    bc = [["transmissive"] * 2] * 3
    return _mk("learned", 3, "cart", (n, n, n), [f, f, f], ng, [list(b) for b in bc], U,
               nscalar=0, gamma=1.4, cfl=0.5, riemann="hllc", limiter=limiter,
               precision=precision, t_end=0.4 / smax, nsteps=nsteps)


# ----------------------------------------------------------------------------
# validation problems (paper Sect. 4 and App. C) and test fixtures
# ----------------------------------------------------------------------------

def random_periodic(n=(12, 10, 8), ndim=3, nscalar=2, seed=7, geom="cart", amp=0.2, ng=GHOSTS_DEFAULT,
                    limiter="vanleer", riemann="hllc", bc=None, gravity="none", g0=(0.0, 0.0, 0.0),
                    G=0.0, Mc=0.0, faces=None, precision="fp64") -> Problem:
    """Smooth-plus-noise random state on a small grid; the default is periodic Cartesian.
    Used for conservation, parity and edge-case tests."""
    n = tuple(list(n[:ndim]) + [1] * (3 - ndim))
    rng = np.random.Generator(np.random.PCG64(seed))
    shape = (n[2], n[1], n[0])
    rho = 1.0 + amp * rng.uniform(-1, 1, size=shape)
    p = 1.0 + amp * rng.uniform(-1, 1, size=shape)
    u = [amp * rng.uniform(-1, 1, size=shape) for _ in range(3)]
    for d in range(ndim, 3):
        u[d] = np.zeros(shape)
    scal = [rng.uniform(0, 1, size=shape) for _ in range(nscalar)]
    U = _pack(rho, u[0], u[1], u[2], p, scal, 1.4)
    if bc is None:
        bc = [["periodic"] * 2 for _ in range(3)]
    if faces is None:
        faces = []
        for d in range(3):
            if d < ndim:
                faces.append(uniform_faces(0.0, 1.0, n[d]))
            else:
                faces.append(_inactive(geom, d))
    return _mk("random", ndim, geom, n, faces, ng, bc, U, nscalar=nscalar, gamma=1.4, cfl=0.5,
               riemann=riemann, limiter=limiter, gravity=gravity, g0=g0, G=G, Mc=Mc,
               precision=precision)


def expansion(n=(32, 1, 1), ndim=1, V=2.0, p0=1e-3, width=3.0, nscalar=0, rho_amp=0.0, seed=9,
              axis=0, limiter="vanleer", riemann="hllc", ng=GHOSTS_DEFAULT, precision="fp64",
              bc="transmissive", gamma=1.4) -> Problem:
    """A cold gas flying apart from the centre of [0,1]^ndim: rho 1 (times 1 + rho_amp U(-1,1),
    seeded), P p0, outward velocity V tanh(r / (width cells)) along the radius r from the centre
    (in 1D along x, or along `axis` of a grid whose other axes are inactive-like copies), passive
    scalars f_s = 1 / (1 + (s + 1) r^2).  Where the expansion is steep and cold, the Hancock half
    step of a limited reconstruction drives face-state pressures (or densities) negative, so the
    positivity fallback of the step takes over in those cells."""
    n = tuple(list(n[:3]) + [1] * (3 - len(n)))
    rng = np.random.Generator(np.random.PCG64(seed))
    shape = (n[2], n[1], n[0])
    fs = [uniform_faces(0.0, 1.0, n[d]) if d < ndim else _inactive("cart", d) for d in range(3)]
    cs = [0.5 * (f[:-1] + f[1:]) - 0.5 if d < ndim else np.zeros(1) for d, f in enumerate(fs)]
    Z, Y, X = np.meshgrid(cs[2], cs[1], cs[0], indexing="ij")
    comp = [X, Y, Z]
    if ndim == 1 and axis != 0:
        raise ValueError("a 1D expansion runs along axis 0")
    r = np.sqrt(X * X + Y * Y + Z * Z)
    hcell = 1.0 / max(n[d] for d in range(ndim))
    speed = V * np.tanh(r / (width * hcell))
    with np.errstate(invalid="ignore", divide="ignore"):
        u = [np.where(r > 0, speed * comp[d] / r, 0.0) if d < ndim else np.zeros(shape) for d in range(3)]
    rho = np.ones(shape)
    if rho_amp:
        rho = rho * (1.0 + rho_amp * rng.uniform(-1, 1, size=shape))
    p = np.full(shape, p0)
    scal = [1.0 / (1.0 + (s + 1) * r * r) for s in range(nscalar)]
    U = _pack(rho, u[0], u[1], u[2], p, scal, gamma)
    bcs = [[bc, bc] for _ in range(3)]
    return _mk("expansion", ndim, "cart", n, fs, ng, bcs, U, nscalar=nscalar, gamma=gamma, cfl=0.5,
               riemann=riemann, limiter=limiter, precision=precision)


def sedov_sph1d(n: int = 400, ng: int = GHOSTS_DEFAULT) -> Problem:
    """1D spherical Sedov (paper App. C.4): r in [0,1], rho 1, E 1e-12 except E1 = 1 in the
    first shell, gamma 1.4, reflective centre, transmissive outer boundary."""
    fr = uniform_faces(0.0, 1.0, n)
    gamma = 1.4
    rho = np.ones(n)
    z = np.zeros(n)
    vol0 = (4.0 * math.pi / 3.0) * fr[1] ** 3
    E = np.full(n, 1e-12)
    E[0] = 1.0 / vol0
    U = np.zeros((5, 1, 1, n))
    U[0, 0, 0] = rho
    U[4, 0, 0] = E
    bc = [["reflective", "transmissive"], ["reflective"] * 2, ["periodic"] * 2]
    return _mk("sedov_sph1d", 1, "sph", (n, 1, 1), [fr, _inactive("sph", 1), _inactive("sph", 2)], ng, bc, U,
               nscalar=0, gamma=gamma, cfl=0.5, riemann="hllc", limiter="vanleer", t_end=0.7,
               meta={"E1": 1.0, "rho0": 1.0})


def static_wedge(nr=10, nth=8, nph=6, ng=GHOSTS_DEFAULT, bc_phi="reflective", rin=1.0, rout=3.0,
                 th=(math.pi / 4, 3 * math.pi / 4), ph=(0.0, math.pi / 2), log_r=True) -> Problem:
    """Uniform rho, p at rest in a spherical wedge with reflective walls."""
    if log_r:
        fr = rin * (rout / rin) ** (np.arange(nr + 1, dtype=np.float64) / nr)
    else:
        fr = uniform_faces(rin, rout, nr)
    fth = uniform_faces(th[0], th[1], nth)
    fph = uniform_faces(ph[0], ph[1], nph)
    shape = (nph, nth, nr)
    z = np.zeros(shape)
    U = _pack(np.ones(shape), z, z, z, np.ones(shape), [np.full(shape, 0.5)], 5.0 / 3.0)
    bc = [["reflective"] * 2, ["reflective"] * 2, [bc_phi] * 2]
    return _mk("static_wedge", 3, "sph", (nr, nth, nph), [fr, fth, fph], ng, bc, U,
               nscalar=1, gamma=5.0 / 3.0, cfl=0.5, riemann="hllc", limiter="vanleer")


def random_wedge(nr=10, nth=8, nph=6, seed=11, ng=GHOSTS_DEFAULT, bc=None, gravity="none", G=1.0, Mc=1.0,
                 amp=0.2, th=(math.pi / 4, 3 * math.pi / 4), ph=(0.0, math.pi / 2), nscalar=1,
                 limiter="vanleer", riemann="hllc", ndim=3, precision="fp64") -> Problem:
    """Random smooth state on a small log-r spherical wedge (with rotation in u_phi)."""
    fr = 1.0 * 3.0 ** (np.arange(nr + 1, dtype=np.float64) / nr)
    n = [nr, nth if ndim >= 2 else 1, nph if ndim >= 3 else 1]
    fth = uniform_faces(th[0], th[1], nth) if ndim >= 2 else _inactive("sph", 1)
    fph = uniform_faces(ph[0], ph[1], nph) if ndim >= 3 else _inactive("sph", 2)
    rng = np.random.Generator(np.random.PCG64(seed))
    shape = (n[2], n[1], n[0])
    rho = 1.0 + amp * rng.uniform(-1, 1, size=shape)
    p = 1.0 + amp * rng.uniform(-1, 1, size=shape)
    u = [amp * rng.uniform(-1, 1, size=shape) for _ in range(3)]
    scal = [rng.uniform(0, 1, size=shape) for _ in range(nscalar)]
    U = _pack(rho, u[0], u[1], u[2], p, scal, 5.0 / 3.0)
    if bc is None:
        bc = [["reflective"] * 2, ["reflective"] * 2, ["periodic"] * 2]
    return _mk("random_wedge", ndim, "sph", tuple(n), [fr, fth, fph], ng, bc, U,
               nscalar=nscalar, gamma=5.0 / 3.0, cfl=0.5, riemann=riemann, limiter=limiter,
               gravity=gravity, G=G, Mc=Mc, precision=precision)


def liska(n: int = 64, ng: int = GHOSTS_DEFAULT) -> Problem:
    """Liska-Wendroff implosion (paper App. C.3), [0,0.3]^2, reflective walls."""
    f = uniform_faces(0.0, 0.3, n)
    xc = 0.5 * (f[:-1] + f[1:])
    Y, X = np.meshgrid(xc, xc, indexing="ij")
    # the printed threshold x + z >= 0.015 is read as 0.15 (the usual Liska-Wendroff setup);
    # the inner (rho, P) = (0.14, 0.125) are the paper's printed values
    inner = (X + Y) < 0.15
    rho = np.where(inner, 0.14, 1.0)
    p = np.where(inner, 0.125, 1.0)
    z = np.zeros_like(rho)
    U = _pack(rho, z, z, z, p, [], 1.4).reshape(5, 1, n, n)
    bc = [["reflective"] * 2, ["reflective"] * 2, ["periodic"] * 2]
    return _mk("liska", 2, "cart", (n, n, 1), [f, f, _inactive("cart", 2)], ng, bc, U,
               nscalar=0, gamma=1.4, cfl=0.5, riemann="hllc", limiter="vanleer", t_end=2.5)


def free_fall(n=(6, 5, 4), ndim=3, g0=(0.3, -0.2, -0.5), ng=GHOSTS_DEFAULT) -> Problem:
    """Uniform state in a periodic box under uniform gravity (free fall)."""
    n = tuple(list(n[:ndim]) + [1] * (3 - ndim))
    shape = (n[2], n[1], n[0])
    z = np.zeros(shape)
    U = _pack(np.full(shape, 1.3), z, z, z, np.full(shape, 0.9), [np.full(shape, 0.25)], 1.4)
    faces = [uniform_faces(0.0, 1.0, n[d]) if d < ndim else _inactive("cart", d) for d in range(3)]
    bc = [["periodic"] * 2 for _ in range(3)]
    g = tuple(g0[d] if d < ndim else 0.0 for d in range(3))
    return _mk("free_fall", ndim, "cart", n, faces, ng, bc, U, nscalar=1, gamma=1.4, cfl=0.5,
               riemann="hllc", limiter="vanleer", gravity="uniform", g0=g)


def rt2d(nx: int = 32, nz: int = 64, ng: int = GHOSTS_DEFAULT, h0: float = 0.01, width: float = 0.005) -> Problem:
    """2D single-mode Rayleigh-Taylor (paper App. C.2): x in [-0.5,0.5], z in [-1,1],
    g = -0.5 e_z, rho 2 over 1, P0 = 10/7 + 1/4, interface h0 cos(4 pi x) smoothed by tanh."""
    fx = uniform_faces(-0.5, 0.5, nx)
    fz = uniform_faces(-1.0, 1.0, nz)
    xc = 0.5 * (fx[:-1] + fx[1:])
    zc = 0.5 * (fz[:-1] + fz[1:])
    Zc, Xc = np.meshgrid(zc, xc, indexing="ij")
    g = 0.5
    h = h0 * np.cos(4.0 * math.pi * Xc)
    s = 0.5 * (1.0 + np.tanh((Zc - h) / width))
    rho = 1.0 + s
    P0 = 10.0 / 7.0 + 0.25
    # hydrostatic pressure of the unperturbed step profile, integrated from z = -1
    zz = zc
    pz = np.where(zz < 0.0, P0 - g * 1.0 * (zz + 1.0), P0 - g * 1.0 - g * 2.0 * zz)
    p = np.broadcast_to(pz[:, None], rho.shape).copy()
    z = np.zeros_like(rho)
    U = _pack(rho, z, z, z, p, [s], 1.4).reshape(6, 1, nz, nx)
    # 2D in the (x, y) index plane; the paper's z axis is mapped to axis 2 here
    bc = [["periodic"] * 2, ["reflective"] * 2, ["periodic"] * 2]
    return _mk("rt2d", 2, "cart", (nx, nz, 1), [fx, fz, _inactive("cart", 2)], ng, bc, U,
               nscalar=1, gamma=1.4, cfl=0.5, riemann="hllc", limiter="vanleer",
               gravity="uniform", g0=(0.0, -g, 0.0), t_end=1.5, meta={"h0": h0, "A": 1.0 / 3.0, "g": g,
                                                                       "kappa": 4.0 * math.pi})


WORKLOADS = {
    "sod": sod,
    "sedov": sedov3d,
    "rt": rt3d,
    "wedge": wedge3d,
    "learned": quadrant3d,
}


def with_internal_energy(prob: Problem, eps: float = 1e-6) -> Problem:
    """The same problem with the internal-energy monitor of Sect. 2.5: one more field, initialised
    to e = E - |m|^2 / (2 rho)."""
    U = prob.U0
    e = U[4] - 0.5 * (U[1] * U[1] + U[2] * U[2] + U[3] * U[3]) / U[0]
    return prob.with_(name=prob.name + "+e", U0=np.concatenate([U, e[None]], axis=0), dual_energy=True,
                      de_eps=float(eps), riemann="hllc")


def boosted_sedov3d(n: int = 64, boost=(1.0, 0.5, 0.25), eps: float = 1e-6, **kw) -> Problem:
    """Sedov blast in a medium moving at a uniform velocity (periodic box): the ambient gas is at
    Mach ~300, so its internal energy is 1e-5 of its kinetic energy and the monitor's alpha
    switches between its branches across the domain."""
    p = sedov3d(n=n, **kw)
    U = p.U0.copy()
    rho = U[0]
    for d in range(3):
        U[1 + d] = U[1 + d] + rho * boost[d]
    U[4] = U[4] + 0.5 * rho * float(np.dot(boost, boost))
    q = p.with_(name="boosted_sedov", U0=U, bc=[["periodic"] * 2 for _ in range(3)],
                faces=[ghost_faces(np.linspace(-1.0, 1.0, n + 1), p.ng, "periodic", "periodic") for _ in range(3)])
    return with_internal_energy(q, eps)


def acoustic_wave1d(n: int = 128, amp: float = 1e-3, ng: int = 2, limiter: str = "vanleer") -> Problem:
    """Smooth isentropic right-going acoustic wave on a periodic unit interval (rho = 1, P = 1/gamma,
    c = 1): a smooth flow where the internal-energy equation and the total-energy equation must
    agree to the scheme's order."""
    gamma = 1.4
    f = np.linspace(0.0, 1.0, n + 1)
    x = 0.5 * (f[:-1] + f[1:])
    s = amp * np.sin(2.0 * np.pi * x)
    rho = 1.0 + s
    u = s  # c0 = 1, right-going: u = c0 drho / rho0
    p = (1.0 / gamma) * rho ** gamma
    U = np.zeros((5, 1, 1, n))
    U[0, 0, 0] = rho
    U[1, 0, 0] = rho * u
    U[4, 0, 0] = p / (gamma - 1.0) + 0.5 * rho * u * u
    return Problem(name="acoustic1d", ndim=1, geom="cart", n=(n, 1, 1), ng=ng,
                   faces=[ghost_faces(f, ng, "periodic", "periodic"), np.array([0.0, 1.0]), np.array([0.0, 1.0])],
                   nscalar=0, gamma=gamma, cfl=0.5, riemann="hllc", limiter=limiter,
                   bc=[["periodic"] * 2, ["periodic"] * 2, ["periodic"] * 2], U0=U)



def with_gas_rad(prob: Problem, R: float = 1.0, arad: float = 30.0) -> Problem:
    """The same problem with the gas + radiation EoS (Sect. 2.3), re-initialised so that its
    pressures (hence its dynamics) are those of the ideal-gas state: each cell's temperature solves
    P = rho R T + arad T^4 / 3 and E = e(T) + |m|^2 / (2 rho).  With R = 1, arad = 30, rho = 1 and
    T = 1, P_r / P_g = 10: radiation-dominated."""
    U = prob.U0.copy()
    g = prob.gamma
    ke = 0.5 * (U[1] ** 2 + U[2] ** 2 + U[3] ** 2) / U[0]
    p = (g - 1.0) * (U[4] - ke)
    rho = U[0]
    # temperature from P by bisection on the monotone residual (host-side set-up only): the gas-only
    # and radiation-only temperatures bound the root from above, and half the smaller one (each
    # term of P is below P) from below, so 60 halvings reach full precision
    T = np.empty_like(p)
    pf, cgf, Tf = p.reshape(-1), (rho * R).reshape(-1), T.reshape(-1)
    for a in range(0, pf.size, 1 << 16):  # cache-sized chunks
        pc, cg = pf[a:a + (1 << 16)], cgf[a:a + (1 << 16)]
        with np.errstate(divide="ignore"):
            hi = np.minimum(pc / cg, (3.0 * pc / arad) ** 0.25) * (1 + 1e-12)
        lo = 0.5 * hi
        mid = np.empty_like(pc)
        f = np.empty_like(pc)
        for _ in range(60):
            np.add(lo, hi, out=mid)
            mid *= 0.5
            np.multiply(mid, mid, out=f)
            f *= f
            f *= arad / 3.0
            f += cg * mid
            f -= pc
            up = f > 0
            np.copyto(hi, mid, where=up)
            np.copyto(lo, mid, where=~up)
        Tf[a:a + (1 << 16)] = 0.5 * (lo + hi)
    U[4] = rho * R * T / (g - 1.0) + arad * T ** 4 + ke
    return prob.with_(name=prob.name + "+rad", U0=U, eos="gas_rad", eos_R=float(R), eos_arad=float(arad))


def rad_wall1d(n: int = 400, u0: float = -3.0, R: float = 1.0, arad: float = 30.0) -> Problem:
    """Uniform radiation-dominated gas (rho 1, T 1, P_r / P_g = 10) streaming at u0 into a
    reflective wall at x = 0: a strong shock whose compression tends to 7 (adiabatic index 4/3)."""
    g = 5.0 / 3.0
    f = np.linspace(0.0, 1.0, n + 1)
    U = np.zeros((5, 1, 1, n))
    rho, T = 1.0, 1.0
    U[0] = rho
    U[1] = rho * u0
    U[4] = rho * R * T / (g - 1.0) + arad * T ** 4 + 0.5 * rho * u0 * u0
    return Problem(name="rad_wall", ndim=1, geom="cart", n=(n, 1, 1), ng=2,
                   faces=[ghost_faces(f, 2, "reflective", "transmissive"), np.array([0.0, 1.0]), np.array([0.0, 1.0])],
                   nscalar=0, gamma=g, cfl=0.5, riemann="hllc", limiter="vanleer",
                   bc=[["reflective", "transmissive"], ["periodic"] * 2, ["periodic"] * 2], U0=U,
                   eos="gas_rad", eos_R=R, eos_arad=arad)


# 56Ni -> 56Co -> 56Fe in CGS: energies per decay (1.75 and 3.73 MeV, gamma rays and positrons) and
# lifetimes (8.8 and 111.3 days) as Sect. 2.4 gives them; the mass of a 56Ni nucleus is 56 m_u
MEV_ERG = 1.602176634e-6
M_U_G = 1.66053906660e-24
DAY_S = 86400.0
NI_CGS = dict(ni_Q=(1.75 * MEV_ERG, 3.73 * MEV_ERG), ni_tau=(8.8 * DAY_S, 111.3 * DAY_S), ni_m=56.0 * M_U_G)


def with_ni_heating(prob: Problem, scalar: int = 0, Q=(1.0, 2.0), tau=(0.05, 0.6), m: float = 1.0) -> Problem:
    """The same problem with 56Ni decay heating (Sect. 2.4, eq. heating_ni): passive scalar `scalar`
    carries rho f_Ni.  The defaults are code units in which the decay is fast enough to matter in a
    short run; NI_CGS holds the physical constants."""
    return prob.with_(name=prob.name + "+ni", ni_heating=True, ni_scalar=int(scalar), ni_Q=tuple(Q),
                      ni_tau=tuple(tau), ni_m=float(m))


def ni_blob3d(n=(24, 20, 16), seed: int = 61, eos: str = "gas") -> Problem:
    """Random periodic 3D flow with a 56Ni-rich blob (scalar 0 = rho f_Ni, f_Ni up to 0.8 in a
    Gaussian blob, 0.05 outside; scalar 1 an ordinary tracer), with decay heating in code units."""
    base = random_periodic(n=n, ndim=3, nscalar=2, seed=seed)
    U = base.U0.copy()
    x = [centers(base.faces[d], base.ng, n[d]) for d in range(3)]
    Z, Y, X = np.meshgrid(x[2], x[1], x[0], indexing="ij")
    c = [0.5 * (x[d][0] + x[d][-1]) for d in range(3)]
    r2 = (X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2
    f = 0.05 + 0.75 * np.exp(-r2 / 0.02)
    U[5] = U[0] * f
    pr = with_ni_heating(base.with_(U0=U, name="ni_blob"))
    return with_gas_rad(pr) if eos == "gas_rad" else pr


def hybrid_linlog_faces(r0: float, rb: float, r1: float, n_lin: int, n_log: int) -> np.ndarray:
    """Hybrid linear-log radial faces (the grid of the paper's 3D SN runs, Sect. 5): n_lin uniform
    cells on [r0, rb], then n_log cells on [rb, r1] whose widths grow by a constant factor q
    chosen so that the first of them is as wide as a uniform cell (the spacing is continuous)."""
    dr = (rb - r0) / n_lin
    lin = r0 + dr * np.arange(n_lin + 1, dtype=np.float64)
    span = r1 - rb
    if not span > n_log * dr:
        raise ValueError("the log part must widen: need r1 - rb > n_log * (rb - r0) / n_lin")
    lo, hi = 1.0, 2.0
    while dr * (hi ** n_log - 1.0) / (hi - 1.0) < span:
        hi *= 2.0
    for _ in range(200):  # bisection for q: dr (q^n - 1) / (q - 1) = span
        q = 0.5 * (lo + hi)
        if dr * (q ** n_log - 1.0) / (q - 1.0) < span:
            lo = q
        else:
            hi = q
    q = 0.5 * (lo + hi)
    k = np.arange(1, n_log + 1, dtype=np.float64)
    log = rb + dr * (q ** k - 1.0) / (q - 1.0)
    log[-1] = r1
    return np.concatenate([lin, log])


def sn_wedge3d(n_lin: int = 64, n_log: int = 64, nth: int = 32, nph: int = 32, seed: int = 5,
               ndim: int = 3, ng: int = GHOSTS_DEFAULT) -> Problem:
    """Stand-in for the paper's 3D SN ejecta runs (Sect. 5 setup: gas + radiation EoS, 56Ni decay
    heating, point-mass gravity, internal-energy monitor, minmod, HLLC, reflective inner and
    transmissive outer radius, hybrid linear-log radial grid), in code units.

    r in [0.1, 10], linear to r = 1 then logarithmic; theta in [pi/4, 3pi/4], phi in [0, pi/2]
    (periodic). A homologously expanding shocked core (r < 0.5: u_r = 2 r, rho 3 r^-1.5, P 2)
    inside a static envelope (rho = r^-2.5 with a seeded 5 % lognormal perturbation, P = 1e-3
    rho^(5/3)); scalar 0 carries 56Ni (f = 0.2 for r < 0.25), scalar 1 the envelope (r > 0.5).
    Gas + radiation EoS with R = 1, a = 10 (temperatures from the pressures above), G Mc = 0.5,
    56Ni lifetimes 0.5 and 6.3 time units (the physical ratio), Q = (0.175, 0.373)."""
    gamma = 5.0 / 3.0
    fr = hybrid_linlog_faces(0.1, 1.0, 10.0, n_lin, n_log)
    nr = n_lin + n_log
    th = (math.pi / 4.0, 3.0 * math.pi / 4.0)
    fth = uniform_faces(th[0], th[1], nth) if ndim >= 2 else _inactive("sph", 1)
    fph = uniform_faces(0.0, math.pi / 2.0, nph) if ndim >= 3 else _inactive("sph", 2)
    n = (nr, nth if ndim >= 2 else 1, nph if ndim >= 3 else 1)
    rc = 0.5 * (fr[:-1] + fr[1:])
    rng = np.random.Generator(np.random.PCG64(seed))
    shape = (n[2], n[1], n[0])
    R = np.broadcast_to(rc[None, None, :], shape)
    core = R < 0.5
    rho = np.where(core, 3.0 * R ** -1.5, R ** -2.5) * np.exp(0.05 * rng.standard_normal(size=shape))
    P = np.where(core, 2.0, 1e-3 * rho ** gamma)
    ur = np.where(core, 2.0 * R, 0.0)
    z = np.zeros(shape)
    fni = np.where(R < 0.25, 0.2, 0.0)
    fenv = (R > 0.5).astype(np.float64)
    U = _pack(rho, ur, z, z, P, [fni, fenv], gamma)
    bc = [["reflective", "transmissive"], ["reflective"] * 2, ["periodic"] * 2]
    pr = _mk("sn_wedge", ndim, "sph", n, [fr, fth, fph], ng, bc, U, nscalar=2, gamma=gamma, cfl=0.5,
             riemann="hllc", limiter="minmod", gravity="point", G=1.0, Mc=0.5)
    pr = with_gas_rad(pr, R=1.0, arad=10.0)
    pr = with_ni_heating(pr, scalar=0, Q=(0.175, 0.373), tau=(0.5, 6.3), m=1.0)
    return with_internal_energy(pr, eps=1e-6).with_(name="sn_wedge")
