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
    of the flow's energy), so that a momentum that is ~0 everywhere is not measured against its own size."""
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


def tol_ratio(Ug, Uo, rel: float = 1e-12, absf: float = 1e-14, flow_scale: bool = False) -> float:
    """Largest |dU| over its tolerance (1 at the bar)."""
    tol = parity_tolerance(Uo, rel, absf, flow_scale)
    return float(np.max(np.abs(Ug - Uo) / np.maximum(tol, 1e-300)))


def max_rel(Ug, Uo):
    nv = Uo.shape[0]
    scale = np.abs(Uo).reshape(nv, -1).max(axis=1).reshape((nv,) + (1,) * (Uo.ndim - 1))
    return float(np.max(np.abs(Ug - Uo) / np.maximum(np.abs(Uo), 1e-300 + 1e-14 * scale)))


def active_box(U: np.ndarray, margin: int = 3):
    """The smallest box [lo, hi) (x, y, z order) holding every cell whose state differs from the
    state of cell (0, 0, 0), widened by `margin` cells and clipped to the grid; None if there is no
    such cell."""
    amb = U[(slice(None),) + (0,) * (U.ndim - 1)]
    diff = np.any(U != amb.reshape((-1,) + (1,) * (U.ndim - 1)), axis=0)
    if not diff.any():
        return None
    idx = np.argwhere(diff)  # [k, j, i]
    n = diff.shape[::-1]
    lo = [max(int(idx[:, 2 - d].min()) - margin, 0) for d in range(3)]
    hi = [min(int(idx[:, 2 - d].max()) + margin + 1, n[d]) for d in range(3)]
    return tuple(lo), tuple(hi)


def boxed_step(o, U: np.ndarray, dt: float, margin: int = 3):
    """One oracle step of a state that is uniform and at rest outside a compact region (a blast in a
    quiet ambient, no gravity): the oracle advances only the box of cells within `margin` of the
    region, and every other cell keeps its state.  That is the whole-grid step exactly: a cell
    depends on cells at most two away along each axis (the flux stencil and the transverse slopes
    of its neighbours' half steps), so a cell outside the box sees a uniform state, whose slopes
    are zero and whose two face fluxes along each axis are the same numbers; the update adds their
    difference, exactly 0.  (Pinned against the whole-grid step in the CPU tests.)"""
    box = active_box(U, margin)
    Un = U.copy()
    if box is None:
        return Un, 0
    lo, hi = box
    out, st = o.step_box(U, dt, lo, hi)
    Un[:, lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]] = out
    return Un, st


def boxed_dt(o, U: np.ndarray, margin: int = 3):
    """The oracle's CFL step over the active box: the grid's step when the box holds an ambient
    cell, since every cell outside the box has the ambient state (a maximum of the same rates)."""
    box = active_box(U, margin)
    if box is None:
        return o.compute_dt(U)
    lo, hi = box
    amb = U[(slice(None),) + (0,) * (U.ndim - 1)]
    sub = U[:, lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]]
    assert np.all(sub[:, 0, 0, 0] == amb), "the box must hold an ambient cell"
    return o.compute_dt_box(U, lo, hi)


class BoxedRun:
    """Oracle steps of a blast in a quiet ambient at full size, in place: `box` bounds every cell
    that differs from the ambient state (cell (0, 0, 0) at the start), so a step advances only the
    box widened by `margin` (boxed_step's argument) and scans only that for the new box (a step
    changes cells at most two away from the changed region)."""

    def __init__(self, o, U: np.ndarray, margin: int = 3):
        self.o, self.U, self.margin = o, U, margin
        self.amb = U[(slice(None),) + (0,) * (U.ndim - 1)].copy()
        self.n = U.shape[1:][::-1]
        self.box = active_box(U, 0)

    def _ext(self):
        lo, hi = self.box
        return (tuple(max(lo[d] - self.margin, 0) for d in range(3)),
                tuple(min(hi[d] + self.margin, self.n[d]) for d in range(3)))

    def compute_dt(self):
        lo, hi = self._ext()
        sub = self.U[:, lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]]
        assert np.all(sub[:, 0, 0, 0] == self.amb), "the widened box must hold an ambient cell"
        return self.o.compute_dt_box(self.U, lo, hi)

    def step(self, dt: float):
        lo, hi = self._ext()
        out, st = self.o.step_box(self.U, dt, lo, hi)
        self.U[:, lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]] = out
        diff = np.any(out != self.amb.reshape((-1, 1, 1, 1)), axis=0)
        idx = np.argwhere(diff)
        self.box = (tuple(lo[d] + int(idx[:, 2 - d].min()) for d in range(3)),
                    tuple(lo[d] + int(idx[:, 2 - d].max()) + 1 for d in range(3)))
        # the changed region must stay off the widened box's faces, or cells outside could change
        for d in range(3):
            assert self.box[0][d] - lo[d] >= 2 or lo[d] == 0
            assert hi[d] - self.box[1][d] >= 2 or hi[d] == self.n[d]
        return st
