"""ctypes binding of the FP64 C oracle (liboracle.so).

TEST INFRASTRUCTURE ONLY.  The caller passes a problem description (any
object with the attributes of paper_2503_04428_amd.problems.Problem, or a
dict); this module never imports the product package.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
OMP_LIB_PATH = os.path.join(HERE, "liboracle_omp.so")  # same source, OpenMP over z planes
OPCOUNT_LIB_PATH = os.path.join(HERE, "liboracle_opcount.so")

GEOM = {"cart": 0, "sph": 1}
RIEMANN = {"hll": 0, "hllc": 1}
LIMITER = {"none": 0, "minmod": 1, "vanleer": 2, "vanalbada": 3, "mlp": 4}
BC = {"periodic": 0, "transmissive": 1, "reflective": 2}
GRAVITY = {"none": 0, "uniform": 1, "point": 2, "point_monopole": 3}
EOS = {"gas": 0, "gas_rad": 1}
OK, EINVAL, ENONPHYS, ENOMEM = 0, -1, -3, -5
MLP_NPARAM = 1249

_DP = C.POINTER(C.c_double)


class OrConfig(C.Structure):
    _fields_ = [
        ("ndim", C.c_int), ("geom", C.c_int), ("n", C.c_int * 3), ("ng", C.c_int),
        ("faces", _DP * 3), ("nscalar", C.c_int), ("gamma", C.c_double), ("cfl", C.c_double),
        ("riemann", C.c_int), ("limiter", C.c_int), ("bc", (C.c_int * 2) * 3),
        ("gravity", C.c_int), ("g0", C.c_double * 3), ("G", C.c_double), ("Mc", C.c_double),
        ("mlp", _DP), ("dual_energy", C.c_int), ("de_eps", C.c_double),
        ("eos", C.c_int), ("eos_R", C.c_double), ("eos_arad", C.c_double),
        ("ni_heating", C.c_int), ("ni_scalar", C.c_int), ("ni_Q", C.c_double * 2), ("ni_tau", C.c_double * 2),
        ("ni_m", C.c_double), ("time", C.c_double), ("centroid", C.c_int),
    ]


_libs = {}


def lib(path: str = LIB_PATH):
    """The oracle's C library (or a library with the same entry points, e.g. the op-counting
    build), loaded once per path."""
    if path not in _libs:
        if not os.path.exists(path):
            from . import build_oracle
            if path == LIB_PATH:
                build_oracle.build()
            elif path == OMP_LIB_PATH:
                build_oracle.build(openmp=True)
            elif path == OPCOUNT_LIB_PATH:
                build_oracle.build_opcount()
        L = C.CDLL(path)
        cp = C.POINTER(OrConfig)
        L.or_step.argtypes = [cp, _DP, C.c_double, _DP]
        L.or_step_box.argtypes = [cp, _DP, C.c_double, C.POINTER(C.c_int), C.POINTER(C.c_int), _DP]
        L.or_step_box_fb.argtypes = [cp, _DP, C.c_double, C.POINTER(C.c_int), C.POINTER(C.c_int), _DP,
                                     C.POINTER(C.c_ubyte)]
        L.or_compute_dt.argtypes = [cp, _DP, _DP]
        L.or_compute_dt_box.argtypes = [cp, _DP, C.POINTER(C.c_int), C.POINTER(C.c_int), _DP]
        L.or_face_states.argtypes = [cp, _DP, C.c_int, C.c_int, C.c_int, C.c_int, _DP, _DP]
        L.or_num_threads.argtypes = []
        L.or_num_threads.restype = C.c_int
        L.or_totals.argtypes = [cp, _DP, _DP]
        L.or_totals.restype = None
        L.or_enclosed_mass.argtypes = [cp, _DP, _DP]
        L.or_riemann_flux.argtypes = [C.c_int, C.c_int, C.c_int, C.c_double, _DP, _DP, _DP]
        L.or_riemann_flux.restype = None
        L.or_eos_state.argtypes = [C.POINTER(OrConfig), C.c_double, C.c_double, _DP, _DP]
        L.or_eos_state.restype = C.c_double
        L.or_eos_energy.argtypes = [C.POINTER(OrConfig), C.c_double, C.c_double]
        L.or_eos_energy.restype = C.c_double
        L.or_shift_grid.argtypes = [C.POINTER(OrConfig), _DP, C.c_double, _DP]
        L.or_shift_grid.restype = C.c_int
        L.or_ni_rate.argtypes = [C.POINTER(OrConfig), C.c_double]
        L.or_ni_rate.restype = C.c_double
        L.or_de_alpha.argtypes = [C.c_double, C.c_double, C.c_double]
        L.or_de_alpha.restype = C.c_double
        L.or_limiter.argtypes = [C.c_int, C.c_double, C.c_double]
        L.or_limiter.restype = C.c_double
        L.or_mlp_phi.argtypes = [_DP, _DP]
        L.or_mlp_phi.restype = C.c_double
        L.or_mlp_slope.argtypes = [_DP, _DP, C.c_double, C.c_double]
        L.or_mlp_slope.restype = C.c_double
        L.or_mlp_loss_grad.argtypes = [_DP, C.c_int, _DP, _DP, _DP, _DP, _DP]
        L.or_mlp_loss_grad.restype = C.c_double
        L.or_mlp_features.argtypes = [_DP, C.c_int, C.c_int, C.c_int, C.c_double, _DP, _DP, _DP, _DP]
        L.or_mlp_features.restype = None
        if hasattr(L, "or_opcount"):
            L.or_opcount.argtypes = [C.POINTER(C.c_ulonglong)]
            L.or_opcount.restype = None
            L.or_opcount_reset.argtypes = []
            L.or_opcount_reset.restype = None
        _libs[path] = L
    return _libs[path]


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_DP)


def _get(p, k):
    return p[k] if isinstance(p, dict) else getattr(p, k)


def _opt(p, k, default):
    return p.get(k, default) if isinstance(p, dict) else getattr(p, k, default)


class Oracle:
    """FP64 oracle bound to one problem description."""

    def __init__(self, prob, mlp_weights: np.ndarray | None = None, library: str = LIB_PATH):
        self.prob = prob
        self._L = lib(library)
        self.ndim = int(_get(prob, "ndim"))
        self.n = tuple(int(v) for v in _get(prob, "n"))
        self.nscalar = int(_get(prob, "nscalar"))
        dual = bool(getattr(prob, "dual_energy", False)) if not isinstance(prob, dict) else bool(prob.get("dual_energy", False))
        self.nvar = 5 + self.nscalar + (1 if dual else 0)
        self._faces = [np.ascontiguousarray(f, dtype=np.float64) for f in _get(prob, "faces")]
        c = OrConfig()
        c.ndim = self.ndim
        c.geom = GEOM[_get(prob, "geom")]
        for d in range(3):
            c.n[d] = self.n[d]
            c.faces[d] = _ptr(self._faces[d])
            c.bc[d][0] = BC[_get(prob, "bc")[d][0]]
            c.bc[d][1] = BC[_get(prob, "bc")[d][1]]
            c.g0[d] = float(_get(prob, "g0")[d])
        c.ng = int(_get(prob, "ng"))
        c.nscalar = self.nscalar
        c.gamma = float(_get(prob, "gamma"))
        c.cfl = float(_get(prob, "cfl"))
        c.riemann = RIEMANN[_get(prob, "riemann")]
        c.limiter = LIMITER[_get(prob, "limiter")]
        c.gravity = GRAVITY[_get(prob, "gravity")]
        c.G = float(_get(prob, "G"))
        c.Mc = float(_get(prob, "Mc"))
        c.dual_energy = 1 if dual else 0
        c.eos = EOS[_opt(prob, "eos", "gas")]
        c.eos_R = float(_opt(prob, "eos_R", 0.0))
        c.eos_arad = float(_opt(prob, "eos_arad", 0.0))
        c.ni_heating = 1 if _opt(prob, "ni_heating", False) else 0
        c.ni_scalar = int(_opt(prob, "ni_scalar", 0))
        for i in range(2):
            c.ni_Q[i] = float(_opt(prob, "ni_Q", (0.0, 0.0))[i])
            c.ni_tau[i] = float(_opt(prob, "ni_tau", (1.0, 2.0))[i])
        c.ni_m = float(_opt(prob, "ni_m", 1.0))
        c.centroid = 1 if _opt(prob, "centroid", False) else 0
        c.de_eps = float(getattr(prob, "de_eps", 1e-6)) if not isinstance(prob, dict) else float(prob.get("de_eps", 1e-6))
        self._mlp = None
        if mlp_weights is not None:
            self.set_mlp(mlp_weights)
        self.cfg = c

    def set_mlp(self, w: np.ndarray):
        self._mlp = np.ascontiguousarray(w, dtype=np.float64)
        assert self._mlp.size == MLP_NPARAM
        if hasattr(self, "cfg"):
            self.cfg.mlp = _ptr(self._mlp)
        else:
            pass

    def _cfgp(self):
        if self._mlp is not None:
            self.cfg.mlp = _ptr(self._mlp)
        return C.byref(self.cfg)

    def shape(self):
        return (self.nvar, self.n[2], self.n[1], self.n[0])

    def step(self, U: np.ndarray, dt: float, t: float = 0.0) -> tuple[np.ndarray, int]:
        """One step from time t (the decay clock of the 56Ni heating; unused otherwise)."""
        U = np.ascontiguousarray(U, dtype=np.float64).reshape(self.shape())
        self.cfg.time = float(t)
        out = np.empty_like(U)
        st = self._L.or_step(self._cfgp(), _ptr(U), float(dt), _ptr(out))
        if st == EINVAL:
            raise ValueError("oracle: invalid configuration")
        if st == ENOMEM:
            raise MemoryError("oracle: out of memory")
        return out, st

    def step_box(self, U: np.ndarray, dt: float, lo, hi, t: float = 0.0) -> tuple[np.ndarray, int]:
        U = np.ascontiguousarray(U, dtype=np.float64).reshape(self.shape())
        self.cfg.time = float(t)
        lo3 = (C.c_int * 3)(*[int(v) for v in lo])
        hi3 = (C.c_int * 3)(*[int(v) for v in hi])
        ext = [int(hi[d]) - int(lo[d]) for d in range(3)]
        out = np.empty((self.nvar, ext[2], ext[1], ext[0]))
        st = self._L.or_step_box(self._cfgp(), _ptr(U), float(dt), lo3, hi3, _ptr(out))
        if st == EINVAL:
            raise ValueError("oracle: invalid box or configuration")
        return out, st

    def step_fallback(self, U: np.ndarray, dt: float, lo=None, hi=None, t: float = 0.0):
        """The step over the box [lo, hi) (default: the whole grid) and the positivity-fallback mask
        of its cells (1 where the cell's own half step was replaced by first order); returns
        (Unew, mask [k][j][i] as bool, status)."""
        U = np.ascontiguousarray(U, dtype=np.float64).reshape(self.shape())
        lo = (0, 0, 0) if lo is None else lo
        hi = self.n if hi is None else hi
        self.cfg.time = float(t)
        lo3 = (C.c_int * 3)(*[int(v) for v in lo])
        hi3 = (C.c_int * 3)(*[int(v) for v in hi])
        ext = [int(hi[d]) - int(lo[d]) for d in range(3)]
        out = np.empty((self.nvar, ext[2], ext[1], ext[0]))
        fb = np.zeros((ext[2], ext[1], ext[0]), dtype=np.uint8)
        st = self._L.or_step_box_fb(self._cfgp(), _ptr(U), float(dt), lo3, hi3, _ptr(out),
                                    fb.ctypes.data_as(C.POINTER(C.c_ubyte)))
        if st == EINVAL:
            raise ValueError("oracle: invalid box or configuration")
        return out, fb.astype(bool), st

    def compute_dt(self, U: np.ndarray) -> tuple[float, int]:
        U = np.ascontiguousarray(U, dtype=np.float64).reshape(self.shape())
        dt = C.c_double(0.0)
        st = self._L.or_compute_dt(self._cfgp(), _ptr(U), C.byref(dt))
        if st == EINVAL:
            raise ValueError("oracle: invalid configuration")
        return dt.value, st

    def face_states(self, U: np.ndarray, i: int, j: int, k: int, d: int):
        """Limited face primitives (lower, upper) of cell (i, j, k) along axis d, before the half step."""
        U = np.ascontiguousarray(U, dtype=np.float64).reshape(self.shape())
        wm = np.zeros(self.nvar)
        wp = np.zeros(self.nvar)
        st = self._L.or_face_states(self._cfgp(), _ptr(U), int(i), int(j), int(k), int(d), _ptr(wm), _ptr(wp))
        if st == EINVAL:
            raise ValueError("oracle: invalid cell, axis or configuration")
        return wm, wp

    def num_threads(self) -> int:
        """Threads of the library's step (OpenMP team size; 1 for the serial build)."""
        return int(self._L.or_num_threads())

    def compute_dt_box(self, U: np.ndarray, lo, hi) -> tuple[float, int]:
        """The CFL step over the cells of the box [lo, hi) (x, y, z order) only."""
        U = np.ascontiguousarray(U, dtype=np.float64).reshape(self.shape())
        dt = C.c_double(0.0)
        lo3 = (C.c_int * 3)(*[int(v) for v in lo])
        hi3 = (C.c_int * 3)(*[int(v) for v in hi])
        st = self._L.or_compute_dt_box(self._cfgp(), _ptr(U), lo3, hi3, C.byref(dt))
        if st == EINVAL:
            raise ValueError("oracle: invalid box or configuration")
        return dt.value, st

    def totals(self, U: np.ndarray) -> np.ndarray:
        U = np.ascontiguousarray(U, dtype=np.float64).reshape(self.shape())
        out = np.zeros(self.nvar)
        self._L.or_totals(self._cfgp(), _ptr(U), _ptr(out))
        return out

    def enclosed_mass(self, U: np.ndarray) -> np.ndarray:
        U = np.ascontiguousarray(U, dtype=np.float64).reshape(self.shape())
        out = np.zeros(self.n[0])
        st = self._L.or_enclosed_mass(self._cfgp(), _ptr(U), _ptr(out))
        if st:
            raise ValueError("oracle: enclosed mass needs a spherical grid")
        return out

    def run(self, U: np.ndarray, nsteps: int | None = None, t_end: float | None = None,
            dt_fixed: float | None = None, t0: float = 0.0):
        """Advance from time t0 with the CFL time step (or a fixed one), the last step clipped to
        t_end; returns (U, t, steps, dts)."""
        t = t0
        steps = 0
        dts = []
        while True:
            if nsteps is not None and steps >= nsteps:
                break
            if t_end is not None and t >= t_end * (1 - 1e-14):
                break
            if dt_fixed is not None:
                dt = dt_fixed
            else:
                dt, st = self.compute_dt(U)
                if st:
                    raise FloatingPointError("oracle: nonphysical state at dt")
            if t_end is not None:
                dt = min(dt, t_end - t)
            U, st = self.step(U, dt, t)
            if st:
                raise FloatingPointError(f"oracle: nonphysical state after step {steps}")
            t += dt
            steps += 1
            dts.append(dt)
        return U, t, steps, dts

    def eos_state(self, rho: float, e: float):
        """(T, P, c_s) of internal energy e per unit volume at density rho (Sect. 2.3)."""
        P, cs = C.c_double(), C.c_double()
        T = self._L.or_eos_state(self._cfgp(), float(rho), float(e), C.byref(P), C.byref(cs))
        return T, P.value, cs.value

    def shift_grid(self, U: np.ndarray, delta: float) -> np.ndarray:
        """Move every face of axis 0 by delta and carry U over conservatively (Sect. 3.1.1, moving
        grid); the oracle's own faces move with it."""
        U = np.ascontiguousarray(U, dtype=np.float64).reshape(self.shape())
        out = np.empty_like(U)
        st = self._L.or_shift_grid(self._cfgp(), _ptr(U), float(delta), _ptr(out))
        if st == EINVAL:
            raise ValueError("oracle: invalid grid shift")
        self._faces[0] = self._faces[0] + float(delta)
        self.cfg.faces[0] = _ptr(self._faces[0])
        return out

    def ni_rate(self, t: float) -> float:
        """56Ni decay heating per unit mass of 56Ni at time t (eq. heating_ni)."""
        return self._L.or_ni_rate(self._cfgp(), float(t))

    def eos_energy(self, rho: float, P: float) -> float:
        return self._L.or_eos_energy(self._cfgp(), float(rho), float(P))


def riemann_flux(solver: str, d: int, gamma: float, qL, qR) -> np.ndarray:
    qL = np.ascontiguousarray(qL, dtype=np.float64)
    qR = np.ascontiguousarray(qR, dtype=np.float64)
    out = np.zeros_like(qL)
    lib().or_riemann_flux(RIEMANN[solver], d, qL.size, float(gamma), _ptr(qL), _ptr(qR), _ptr(out))
    return out


def limiter(name: str, a: float, b: float) -> float:
    return lib().or_limiter(LIMITER[name], float(a), float(b))


def mlp_phi(w: np.ndarray, x) -> float:
    w = np.ascontiguousarray(w, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    return lib().or_mlp_phi(_ptr(w), _ptr(x))


def mlp_slope(w: np.ndarray, d4, cm: float = 0.5, cp: float = 0.5) -> float:
    w = np.ascontiguousarray(w, dtype=np.float64)
    d4 = np.ascontiguousarray(d4, dtype=np.float64)
    return lib().or_mlp_slope(_ptr(w), _ptr(d4), float(cm), float(cp))


def mlp_loss_grad(w, x, a, t, wt):
    w = np.ascontiguousarray(w, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    a = np.ascontiguousarray(a, dtype=np.float64)
    t = np.ascontiguousarray(t, dtype=np.float64)
    wt = np.ascontiguousarray(wt, dtype=np.float64)
    g = np.zeros(MLP_NPARAM)
    loss = lib().or_mlp_loss_grad(_ptr(w), int(a.size), _ptr(x), _ptr(a), _ptr(t), _ptr(wt), _ptr(g))
    return loss, g


def mlp_features(U, ratio: int, gamma: float):
    """Training samples of a batch of 1D fine solutions U [5][nrows][nf] (see hydro_oracle.h)."""
    U = np.ascontiguousarray(U, dtype=np.float64)
    _, nrows, nf = U.shape
    n = nrows * (nf // ratio) * 5
    x = np.zeros(4 * n)
    a = np.zeros(n)
    t = np.zeros(n)
    wt = np.zeros(n)
    lib().or_mlp_features(_ptr(U), nrows, nf, ratio, float(gamma), _ptr(x), _ptr(a), _ptr(t), _ptr(wt))
    return x.reshape(n, 4), a, t, wt


def bf16_round(w) -> np.ndarray:
    """Round FP32 values to the nearest BF16 (ties to even), returned as float64."""
    f = np.ascontiguousarray(w, dtype=np.float32).view(np.uint32).astype(np.uint64)
    f = (f + 0x7FFF + ((f >> 16) & 1)) & 0xFFFF0000
    return f.astype(np.uint32).view(np.float32).astype(np.float64)


OPCOUNT_FIELDS = ("add", "mul", "div", "sqrt", "cmp", "minmax_abs", "transc")


def opcount_step(prob, U: np.ndarray, dt: float) -> dict:
    """Operations of the oracle's step on state U (op-counting build of the same C source): a dict
    of counts per category of the algorithm's work, plus 'flops' = add + mul + div + sqrt, and
    'repeated' with the same counts for the work the oracle repeats (the second evaluation of
    every face flux), which is not part of the algorithm's work."""
    o = Oracle(prob, library=OPCOUNT_LIB_PATH)
    L = o._L
    L.or_opcount_reset()
    out, st = o.step(U, dt)
    c = (C.c_ulonglong * 14)()
    L.or_opcount(c)
    res = {k: int(v) for k, v in zip(OPCOUNT_FIELDS, c[:7])}
    res["flops"] = res["add"] + res["mul"] + res["div"] + res["sqrt"]
    rep = {k: int(v) for k, v in zip(OPCOUNT_FIELDS, c[7:])}
    rep["flops"] = rep["add"] + rep["mul"] + rep["div"] + rep["sqrt"]
    res["repeated"] = rep
    res["state"] = out
    res["status"] = st
    return res


def de_alpha(e: float, ek: float, eps: float) -> float:
    """Blend factor of the internal-energy monitor (Sect. 2.5)."""
    return lib().or_de_alpha(float(e), float(ek), float(eps))

