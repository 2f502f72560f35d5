"""Helpers shared by the GPU parity tests (test infrastructure)."""
import sys

import numpy as np


def announce(msg: str):
    """Name the case before a GPU step, so that a failing run says which case it was."""
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def parity_tolerance(Uo: np.ndarray, rel: float = 1e-12, absf: float = 1e-14, flow_scale: bool = False) -> np.ndarray:
    """Per cell |dU| <= rel |U_oracle| + absf * scale of that field, scale = max_cells |U_oracle|.
    With flow_scale, the three momenta share one scale, at least sqrt(max rho * max E) (the momentum
    of the flow's energy), so that a momentum that is ~0 everywhere is not judged on its own size."""
    nv = Uo.shape[0]
    scale = np.abs(Uo).reshape(nv, -1).max(axis=1)
    if flow_scale:
        ms = max(scale[1:4].max(), np.sqrt(scale[0] * scale[4]))
        scale[1:4] = ms
    return rel * np.abs(Uo) + absf * scale.reshape((nv,) + (1,) * (Uo.ndim - 1))


def assert_parity(Ug: np.ndarray, Uo: np.ndarray, rel: float = 1e-12, absf: float = 1e-14, what: str = "",
                  flow_scale: bool = False):
    assert Ug.shape == Uo.shape, (Ug.shape, Uo.shape)
    assert np.all(np.isfinite(Ug)), f"{what}: non-finite GPU values"
    tol = parity_tolerance(Uo, rel, absf, flow_scale)
    err = np.abs(Ug - Uo)
    bad = err > tol
    if bad.any():
        idx = np.argwhere(bad)
        v, *cell = idx[0]
        worst = np.unravel_index(np.argmax(err / np.maximum(tol, 1e-300)), err.shape)
        raise AssertionError(
            f"{what}: {bad.sum()} of {bad.size} values outside tolerance; first at var {v} cell {cell}: "
            f"gpu {Ug[tuple(idx[0])]!r} oracle {Uo[tuple(idx[0])]!r}; worst ratio "
            f"{(err / np.maximum(tol, 1e-300))[worst]:.3g} at {worst}")


def max_rel(Ug, Uo):
    nv = Uo.shape[0]
    scale = np.abs(Uo).reshape(nv, -1).max(axis=1).reshape((nv,) + (1,) * (Uo.ndim - 1))
    return float(np.max(np.abs(Ug - Uo) / np.maximum(np.abs(Uo), 1e-300 + 1e-14 * scale)))
