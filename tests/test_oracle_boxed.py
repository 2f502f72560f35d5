"""The boxed oracle step used by the full-size GPU parity runs equals the whole-grid oracle step bit
for bit (CPU): a blast in a quiet ambient, advanced over the box of cells within three of the
non-ambient region, leaves every other cell exactly as it was, because a cell depends on cells at
most two away along each axis and a uniform state's update adds a flux difference of exactly 0.
Also the boxed CFL step equals the whole grid's, and the OpenMP build of the oracle gives the same
bits as the serial one on these runs."""
import numpy as np

from oracle import oracle as O
from paper_2503_04428_amd import problems as P

from parity import BoxedRun, active_box, boxed_dt, boxed_step


def test_boxed_step_equals_whole_grid_sedov():
    prob = P.sedov3d(n=48)
    o = O.Oracle(prob)
    U = prob.U0.copy()
    Ub = prob.U0.copy()
    for n in range(30):
        dt, st = o.compute_dt(U)
        dtb, stb = boxed_dt(o, Ub)
        assert st == 0 and stb == 0 and dtb == dt
        U, st = o.step(U, dt)
        Ub, stb = boxed_step(o, Ub, dtb)
        assert st == 0 and stb == 0
        assert np.array_equal(U, Ub), f"step {n}"
    lo, hi = active_box(U)
    # the blast has spread but is still compact: the shortcut has something to skip
    assert all(hi[d] - lo[d] < 48 for d in range(3))


def test_boxed_run_equals_whole_grid_sedov():
    prob = P.sedov3d(n=40)
    o = O.Oracle(prob)
    U = prob.U0.copy()
    run = BoxedRun(o, prob.U0.copy())
    for n in range(25):
        dt, st = o.compute_dt(U)
        dtb, stb = run.compute_dt()
        assert st == 0 and stb == 0 and dtb == dt
        U, st = o.step(U, dt)
        assert run.step(dtb) == 0
        assert np.array_equal(U, run.U), f"step {n}"


def test_boxed_step_needs_a_margin():
    """Without a margin the box misses cells that the step changes (the blast front moves into
    the ambient), so the comparison above is not vacuous."""
    prob = P.sedov3d(n=40)
    o = O.Oracle(prob)
    U = prob.U0.copy()
    dt, _ = o.compute_dt(U)
    U, _ = o.step(U, dt)
    dt, _ = o.compute_dt(U)
    full, _ = o.step(U, dt)
    thin, _ = boxed_step(o, U, dt, margin=0)
    assert not np.array_equal(full, thin)
    assert np.array_equal(full, boxed_step(o, U, dt, margin=3)[0])


def test_openmp_oracle_matches_serial_on_sedov():
    prob = P.sedov3d(n=32)
    a = O.Oracle(prob)
    b = O.Oracle(prob, library=O.OMP_LIB_PATH)
    Ua = prob.U0.copy()
    Ub = prob.U0.copy()
    for _ in range(10):
        dta, _ = a.compute_dt(Ua)
        dtb, _ = b.compute_dt(Ub)
        assert dta == dtb
        Ua, _ = a.step(Ua, dta)
        Ub, _ = b.step(Ub, dtb)
    assert np.array_equal(Ua, Ub)
