"""Python binding of libhydro.so (the gfx950 MUSCL-Hancock step behind the C ABI of
include/hydro.h).  Argument marshalling only: every step of the method runs in the library's
HIP kernels.  PyTorch provides device memory and the HIP stream.

The binding refuses to work without the built library and a HIP device: there is no CPU path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# HX_LIB_PATH selects another build of the same library (tuning experiments)
LIB_PATH = os.environ.get("HX_LIB_PATH") or os.path.join(HERE, "libhydro.so")

OK, EINVAL, EHIP, ENONPHYS, ESTATE, ENOSPACE = 0, -1, -2, -3, -4, -5
MLP_NPARAM = 1249

GEOM = {"cart": 0, "sph": 1}
RIEMANN = {"hll": 0, "hllc": 1}
LIMITER = {"none": 0, "minmod": 1, "vanleer": 2, "vanalbada": 3, "mlp": 4}
PRECISION = {"fp64": 0, "fp32": 1}
BC = {"periodic": 0, "transmissive": 1, "reflective": 2}
GRAVITY = {"none": 0, "uniform": 1, "point": 2, "point_monopole": 3}
EOS = {"gas": 0, "gas_rad": 1}

_DP = C.POINTER(C.c_double)


class HxConfig(C.Structure):
    _fields_ = [
        ("ndim", C.c_int), ("geom", C.c_int), ("n", C.c_int * 3), ("nghost", C.c_int),
        ("faces", _DP * 3), ("nscalar", C.c_int), ("gamma", C.c_double), ("cfl", C.c_double),
        ("riemann", C.c_int), ("limiter", C.c_int), ("precision", C.c_int),
        ("bc", (C.c_int * 2) * 3), ("gravity", C.c_int), ("g0", C.c_double * 3),
        ("G", C.c_double), ("Mc", C.c_double), ("dual_energy", C.c_int), ("de_eps", C.c_double),
        ("eos", C.c_int), ("eos_R", C.c_double), ("eos_arad", C.c_double),
        ("ni_heating", C.c_int), ("ni_scalar", C.c_int), ("ni_Q", C.c_double * 2), ("ni_tau", C.c_double * 2),
        ("ni_m", C.c_double), ("centroid", C.c_int),
    ]


class HydroError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"hydro status {status}: {msg}")
        self.status = status


class NonPhysicalState(HydroError):
    pass


_lib = None

# names of the exported entry points, as declared in include/hydro.h
EXPORTS = ["hx_workspace_bytes", "hx_create", "hx_set_state", "hx_get_state", "hx_compute_dt",
           "hx_compute_dt_device", "hx_step", "hx_step_device", "hx_run_1d", "hx_totals", "hx_check", "hx_set_mlp",
           "hx_set_zchunk", "hx_get_zchunk", "hx_set_time", "hx_get_time", "hx_shift_grid", "hx_enclosed_mass", "hx_arith_check", "hx_mlp_eval", "hx_mlp_features",
           "hx_mlp_grad_workspace_bytes", "hx_mlp_grad", "hx_mlp_grad_noalloc", "hx_mlp_adam", "hx_last_error",
           "hx_destroy"]


def load_library():
    """Load libhydro.so; raises if it has not been built (no fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with python -m paper_2503_04428_amd.build")
    L = C.CDLL(LIB_PATH)
    cfgp = C.POINTER(HxConfig)
    vp = C.c_void_p
    L.hx_workspace_bytes.argtypes = [cfgp]
    L.hx_workspace_bytes.restype = C.c_size_t
    L.hx_create.argtypes = [cfgp, vp, C.c_size_t, vp, C.POINTER(vp)]
    L.hx_set_state.argtypes = [vp, vp]
    L.hx_get_state.argtypes = [vp, vp]
    L.hx_compute_dt.argtypes = [vp, _DP]
    L.hx_compute_dt_device.argtypes = [vp, vp]
    L.hx_step.argtypes = [vp, C.c_double]
    L.hx_step_device.argtypes = [vp, vp]
    L.hx_run_1d.argtypes = [vp, C.c_double, C.c_double, C.c_int, _DP, C.POINTER(C.c_int)]
    L.hx_totals.argtypes = [vp, _DP]
    L.hx_check.argtypes = [vp]
    L.hx_set_mlp.argtypes = [vp, C.POINTER(C.c_float), C.c_size_t]
    L.hx_set_zchunk.argtypes = [vp, C.c_int]
    L.hx_get_zchunk.argtypes = [vp, C.POINTER(C.c_int)]
    L.hx_set_time.argtypes = [vp, C.c_double]
    L.hx_shift_grid.argtypes = [vp, C.c_double]
    L.hx_get_time.argtypes = [vp, C.POINTER(C.c_double)]
    L.hx_enclosed_mass.argtypes = [vp, _DP]
    L.hx_arith_check.argtypes = [vp, vp, C.c_longlong, vp, vp, vp]
    L.hx_mlp_eval.argtypes = [vp, vp, C.c_longlong, vp, vp]
    L.hx_mlp_features.argtypes = [vp, C.c_int, C.c_int, C.c_int, C.c_double, vp, vp, vp, vp, vp]
    L.hx_mlp_grad_workspace_bytes.argtypes = [C.c_longlong]
    L.hx_mlp_grad_workspace_bytes.restype = C.c_size_t
    L.hx_mlp_grad.argtypes = [vp, vp, vp, vp, vp, C.c_longlong, vp, vp, vp, C.c_size_t, vp]
    L.hx_mlp_grad_noalloc.argtypes = [vp, vp, vp, vp, vp, C.c_longlong, vp, vp, vp]
    L.hx_mlp_adam.argtypes = [vp, vp, vp, vp, C.c_int, C.c_float, C.c_float, C.c_float, C.c_float, vp]
    L.hx_last_error.argtypes = []
    L.hx_last_error.restype = C.c_char_p
    L.hx_destroy.argtypes = [vp]
    L.hx_destroy.restype = None
    for name in EXPORTS:
        if name not in ("hx_workspace_bytes", "hx_last_error", "hx_destroy", "hx_mlp_grad_workspace_bytes"):
            getattr(L, name).restype = C.c_int
    _lib = L
    return L


def _get(p, k):
    return p[k] if isinstance(p, dict) else getattr(p, k)


def _opt(p, k, default):
    return p.get(k, default) if isinstance(p, dict) else getattr(p, k, default)


def make_config(prob, precision: str | None = None):
    """hx_config for a problem description (see problems.Problem); returns (config, keepalive)."""
    c = HxConfig()
    ndim = int(_get(prob, "ndim"))
    c.ndim = ndim
    c.geom = GEOM[_get(prob, "geom")]
    faces = [np.ascontiguousarray(f, dtype=np.float64) for f in _get(prob, "faces")]
    for d in range(3):
        c.n[d] = int(_get(prob, "n")[d])
        c.faces[d] = faces[d].ctypes.data_as(_DP)
        c.bc[d][0] = BC[_get(prob, "bc")[d][0]]
        c.bc[d][1] = BC[_get(prob, "bc")[d][1]]
        c.g0[d] = float(_get(prob, "g0")[d])
    c.nghost = int(_get(prob, "ng"))
    c.nscalar = int(_get(prob, "nscalar"))
    c.gamma = float(_get(prob, "gamma"))
    c.cfl = float(_get(prob, "cfl"))
    c.riemann = RIEMANN[_get(prob, "riemann")]
    c.limiter = LIMITER[_get(prob, "limiter")]
    c.precision = PRECISION[precision or _get(prob, "precision")]
    c.gravity = GRAVITY[_get(prob, "gravity")]
    c.G = float(_get(prob, "G"))
    c.Mc = float(_get(prob, "Mc"))
    c.dual_energy = 1 if _opt(prob, "dual_energy", False) else 0
    c.de_eps = float(_opt(prob, "de_eps", 1e-6))
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
    return c, faces


def workspace_bytes(prob, precision: str | None = None) -> int:
    L = load_library()
    c, keep = make_config(prob, precision)
    n = L.hx_workspace_bytes(C.byref(c))
    if n == 0:
        raise HydroError(EINVAL, L.hx_last_error().decode())
    return int(n)


class Solver:
    """One solver context on a torch CUDA (HIP) device and stream."""

    def __init__(self, prob, precision: str | None = None, device="cuda", stream=None, zchunk: int | None = None):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("hydro.Solver needs a HIP device; there is no CPU path")
        self.torch = torch
        self.L = load_library()
        self.prob = prob
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.cfg, self._faces = make_config(prob, precision)
        self.nvar = 5 + int(_get(prob, "nscalar")) + (1 if _opt(prob, "dual_energy", False) else 0)
        n = [int(v) for v in _get(prob, "n")]
        self.shape = (self.nvar, n[2], n[1], n[0])
        nbytes = self.L.hx_workspace_bytes(C.byref(self.cfg))
        if nbytes == 0:
            raise HydroError(EINVAL, self.L.hx_last_error().decode())
        # over-allocate so the workspace can be aligned to 256 bytes
        self._ws_raw = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self._ws_raw.data_ptr()
        self._ws_ptr = (base + 255) // 256 * 256
        self.workspace_bytes = nbytes
        ctx = C.c_void_p()
        self._call(self.L.hx_create(C.byref(self.cfg), C.c_void_p(self._ws_ptr), C.c_size_t(nbytes),
                                    C.c_void_p(self.stream.cuda_stream), C.byref(ctx)))
        self.ctx = ctx
        self._dt_dev = torch.zeros(1, dtype=torch.float64, device=self.device)
        if zchunk is not None:
            self.set_zchunk(zchunk)

    def _call(self, st: int):
        if st != OK:
            msg = self.L.hx_last_error().decode()
            if st == ENONPHYS:
                raise NonPhysicalState(st, msg)
            raise HydroError(st, msg)

    def close(self):
        if getattr(self, "ctx", None):
            self.L.hx_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ----------------------------------------------------------------- state
    def set_state(self, U):
        torch = self.torch
        if isinstance(U, np.ndarray):
            t = torch.from_numpy(np.ascontiguousarray(U, dtype=np.float64).reshape(self.shape)).to(self.device)
        else:
            t = U.to(device=self.device, dtype=torch.float64).contiguous().reshape(self.shape)
        self._state_in = t  # keep alive until the async copy has run
        with torch.cuda.stream(self.stream):
            self._call(self.L.hx_set_state(self.ctx, C.c_void_p(t.data_ptr())))

    def get_state(self, out=None):
        torch = self.torch
        if out is None:
            out = torch.empty(self.shape, dtype=torch.float64, device=self.device)
        self._call(self.L.hx_get_state(self.ctx, C.c_void_p(out.data_ptr())))
        return out

    def state_numpy(self) -> np.ndarray:
        t = self.get_state()
        self.stream.synchronize()
        return t.cpu().numpy()

    def state(self) -> np.ndarray:
        """The current conserved state as a host FP64 array [nvar][n3][n2][n1]."""
        return self.state_numpy()

    # ----------------------------------------------------------------- stepping
    def compute_dt(self) -> float:
        dt = C.c_double(0.0)
        self._call(self.L.hx_compute_dt(self.ctx, C.byref(dt)))
        return dt.value

    def compute_dt_device(self, d_dt=None):
        d_dt = self._dt_dev if d_dt is None else d_dt
        self._call(self.L.hx_compute_dt_device(self.ctx, C.c_void_p(d_dt.data_ptr())))
        return d_dt

    def step(self, dt: float):
        self._call(self.L.hx_step(self.ctx, C.c_double(float(dt))))

    def step_device(self, d_dt=None):
        d_dt = self._dt_dev if d_dt is None else d_dt
        self._call(self.L.hx_step_device(self.ctx, C.c_void_p(d_dt.data_ptr())))

    def advance(self, nsteps: int):
        """nsteps CFL steps without host synchronisation (dt computed on the device)."""
        for _ in range(nsteps):
            self.compute_dt_device()
            self.step_device()

    def run(self, t_end: float | None = None, nsteps: int | None = None, t0: float = 0.0):
        """Advance from time t0 with the CFL time step, the last step clipped to t_end (host time
        step: one synchronisation per step); returns (t, steps).  The decay clock of the 56Ni
        heating is set to t0 first."""
        if t_end is None and nsteps is None:
            raise ValueError("run needs t_end or nsteps")
        self.set_time(t0)
        t, steps = t0, 0
        while (nsteps is None or steps < nsteps) and (t_end is None or t < t_end * (1 - 1e-14)):
            dt = self.compute_dt()
            if t_end is not None:
                dt = min(dt, t_end - t)
            self.step(dt)
            t += dt
            steps += 1
        return t, steps

    def run_1d(self, t_end: float, max_steps: int = 1 << 30, t0: float = 0.0):
        """The same time loop as run(t_end) for a 1D row, inside one workgroup on the device (no
        launch or synchronisation per step); returns (t, steps)."""
        t = C.c_double(0.0)
        n = C.c_int(0)
        self._call(self.L.hx_run_1d(self.ctx, C.c_double(float(t0)), C.c_double(float(t_end)), int(max_steps),
                                    C.byref(t), C.byref(n)))
        return t.value, n.value

    def totals(self) -> np.ndarray:
        out = np.zeros(self.nvar)
        self._call(self.L.hx_totals(self.ctx, out.ctypes.data_as(_DP)))
        return out

    def check(self):
        self._call(self.L.hx_check(self.ctx))

    def set_mlp(self, w):
        w = np.ascontiguousarray(w, dtype=np.float32)
        self._call(self.L.hx_set_mlp(self.ctx, w.ctypes.data_as(C.POINTER(C.c_float)), C.c_size_t(w.size)))

    def set_zchunk(self, kz: int):
        """z planes per workgroup of the 3D sweep (0: automatic)."""
        self._call(self.L.hx_set_zchunk(self.ctx, int(kz)))

    def zchunk(self) -> int:
        """z planes per workgroup in use (0 before the first automatic 3D step)."""
        v = C.c_int(0)
        self._call(self.L.hx_get_zchunk(self.ctx, C.byref(v)))
        return v.value

    def shift_grid(self, delta: float):
        """Move the faces of axis 0 by delta and carry the state over (moving grid)."""
        self._call(self.L.hx_shift_grid(self.ctx, float(delta)))

    def set_time(self, t: float):
        """Set the decay clock of the 56Ni heating (every step advances it by its dt)."""
        self._call(self.L.hx_set_time(self.ctx, float(t)))

    def time(self) -> float:
        v = C.c_double(0.0)
        self._call(self.L.hx_get_time(self.ctx, C.byref(v)))
        return v.value

    def enclosed_mass(self) -> np.ndarray:
        out = np.zeros(int(_get(self.prob, "n")[0]))
        self._call(self.L.hx_enclosed_mass(self.ctx, out.ctypes.data_as(_DP)))
        return out


# ----------------------------------------------------------------------------- learned limiter

def _check(L, st):
    if st != OK:
        raise HydroError(st, L.hx_last_error().decode())


def _stream_ptr(torch, stream):
    return C.c_void_p((stream or torch.cuda.current_stream()).cuda_stream)


def arith_check(a, b, stream=None):
    """The sweeps' FP64 division and square root on device FP64 tensors: (a / b, sqrt(|a|))."""
    import torch

    L = load_library()
    a = a.contiguous().double()
    b = b.contiguous().double()
    n = a.numel()
    q = torch.empty_like(a)
    r = torch.empty_like(a)
    _check(L, L.hx_arith_check(C.c_void_p(a.data_ptr()), C.c_void_p(b.data_ptr()), C.c_longlong(n),
                               C.c_void_p(q.data_ptr()), C.c_void_p(r.data_ptr()), _stream_ptr(torch, stream)))
    return q, r


def mlp_eval(w, x, stream=None):
    """phi of the normalised stencils x [n, 4] (device FP32 tensors) with parameters w [1249]."""
    import torch

    L = load_library()
    w = w.contiguous().float()
    x = x.contiguous().float()
    n = x.shape[0]
    phi = torch.empty(n, dtype=torch.float32, device=x.device)
    _check(L, L.hx_mlp_eval(C.c_void_p(w.data_ptr()), C.c_void_p(x.data_ptr()), C.c_longlong(n),
                            C.c_void_p(phi.data_ptr()), _stream_ptr(torch, stream)))
    return phi


def mlp_features(fine, ratio: int, gamma: float, stream=None):
    """Training samples (x [n,4], a, t, wt) from a device FP64 batch of 1D fine states [5, rows, nf]."""
    import torch

    L = load_library()
    fine = fine.contiguous().double()
    _, rows, nf = fine.shape
    n = rows * (nf // ratio) * 5
    dev = fine.device
    x = torch.empty((n, 4), dtype=torch.float32, device=dev)
    a, t, wt = (torch.empty(n, dtype=torch.float32, device=dev) for _ in range(3))
    _check(L, L.hx_mlp_features(C.c_void_p(fine.data_ptr()), rows, nf, ratio, float(gamma),
                                C.c_void_p(x.data_ptr()), C.c_void_p(a.data_ptr()), C.c_void_p(t.data_ptr()),
                                C.c_void_p(wt.data_ptr()), _stream_ptr(torch, stream)))
    return x, a, t, wt


class MlpTrainer:
    """FP32 master weights, Adam moments and gradient scratch on the device."""

    def __init__(self, w0, n_max: int, device="cuda", stream=None):
        import torch

        self.torch = torch
        self.L = load_library()
        self.w = torch.as_tensor(np.asarray(w0, dtype=np.float32)).to(device).contiguous()
        self.m = torch.zeros_like(self.w)
        self.v = torch.zeros_like(self.w)
        self.grad = torch.zeros_like(self.w)
        self.loss = torch.zeros(1, dtype=torch.float32, device=device)
        nb = int(self.L.hx_mlp_grad_workspace_bytes(C.c_longlong(n_max)))
        self.work = torch.empty(max(nb, 4), dtype=torch.uint8, device=device)
        self.stream = stream
        self.step_count = 0

    def gradient(self, x, a, t, wt):
        n = x.shape[0]
        _check(self.L, self.L.hx_mlp_grad(
            C.c_void_p(self.w.data_ptr()), C.c_void_p(x.data_ptr()), C.c_void_p(a.data_ptr()),
            C.c_void_p(t.data_ptr()), C.c_void_p(wt.data_ptr()), C.c_longlong(n),
            C.c_void_p(self.grad.data_ptr()), C.c_void_p(self.loss.data_ptr()),
            C.c_void_p(self.work.data_ptr()), C.c_size_t(self.work.numel()), _stream_ptr(self.torch, self.stream)))
        return self.grad, self.loss

    def gradient_noalloc(self, x, a, t, wt):
        """gradient() through the allocation-free entry point (the library's static scratch)."""
        n = x.shape[0]
        _check(self.L, self.L.hx_mlp_grad_noalloc(
            C.c_void_p(self.w.data_ptr()), C.c_void_p(x.data_ptr()), C.c_void_p(a.data_ptr()),
            C.c_void_p(t.data_ptr()), C.c_void_p(wt.data_ptr()), C.c_longlong(n),
            C.c_void_p(self.grad.data_ptr()), C.c_void_p(self.loss.data_ptr()), _stream_ptr(self.torch, self.stream)))
        return self.grad, self.loss

    def adam(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.step_count += 1
        _check(self.L, self.L.hx_mlp_adam(
            C.c_void_p(self.w.data_ptr()), C.c_void_p(self.grad.data_ptr()), C.c_void_p(self.m.data_ptr()),
            C.c_void_p(self.v.data_ptr()), self.step_count, float(lr), float(beta1), float(beta2), float(eps),
            _stream_ptr(self.torch, self.stream)))
