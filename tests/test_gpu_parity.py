"""GPU parity: the HIP library (through the C ABI) against the FP64 CPU oracle on the same seeded
inputs.  FP64 bar: per cell |dU| <= 1e-12 |U_oracle| + 1e-14 max|U_oracle,field|, after up to 100
steps, on small grids spanning several workgroup tiles with ragged tails, every boundary type,
limiter, Riemann solver, gravity mode, geometry and scalar count; and at full size on sampled
cells of the first step."""
import math
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2503_04428_amd import problems as P

from parity import announce, assert_parity, max_rel, tol_ratio

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2503_04428_amd import hydro
    hydro.load_library()
    return hydro


def run_pair(H, prob, nsteps, zchunk=None, check_dt=True):
    o = O.Oracle(prob)
    s = H.Solver(prob, zchunk=zchunk)
    U = prob.U0.copy()
    s.set_state(U)
    for n in range(nsteps):
        dt, st = o.compute_dt(U)
        assert st == 0
        if check_dt and n in (0, nsteps - 1):
            dtg = s.compute_dt()
            assert dtg == pytest.approx(dt, rel=1e-14, abs=0), (dtg, dt)
        U, st = o.step(U, dt)
        assert st == 0
        s.step(dt)
    Ug = s.state_numpy()
    s.close()
    return Ug, U


CASES = {
    # 1D
    "sod1024_vl_hllc_100": (lambda: P.sod(1024), 100, None),
    "sod300_minmod_hll": (lambda: P.sod(300, limiter="minmod", riemann="hll"), 40, None),
    "sod300_vanalbada_hllc": (lambda: P.sod(300, limiter="vanalbada"), 40, None),
    "sod300_none_hllc": (lambda: P.sod(300, limiter="none"), 40, None),
    "rand1d_periodic_s2": (lambda: P.random_periodic(n=(131,), ndim=1, nscalar=2, seed=21), 40, None),
    # 2D
    "rand2d_periodic_s1": (lambda: P.random_periodic(n=(37, 29), ndim=2, nscalar=1, seed=22), 40, None),
    "rand2d_mixed_hll_s3": (lambda: P.random_periodic(
        n=(30, 17), ndim=2, nscalar=3, seed=23, riemann="hll", limiter="minmod",
        bc=[["transmissive", "reflective"], ["reflective", "transmissive"], ["periodic"] * 2]), 40, None),
    "liska40": (lambda: P.liska(40), 40, None),
    "rt2d_24x48_gravity": (lambda: P.rt2d(24, 48), 40, None),
    # 3D
    "rand3d_periodic_s2_kz8": (lambda: P.random_periodic(n=(31, 23, 19), ndim=3, nscalar=2, seed=24), 30, 8),
    "rand3d_mixed_s3_kz5": (lambda: P.random_periodic(
        n=(17, 20, 13), ndim=3, nscalar=3, seed=25, limiter="vanalbada",
        bc=[["transmissive"] * 2, ["reflective"] * 2, ["periodic"] * 2]), 30, 5),
    "rand3d_hll_s0_kz32": (lambda: P.random_periodic(n=(15, 16, 33), ndim=3, nscalar=0, seed=26,
                                                       riemann="hll"), 30, 32),
    "sedov32_100": (lambda: P.sedov3d(n=32), 100, 8),
    "rt3d_16x16x48": (lambda: P.rt3d(16, 16, 48, precision="fp64"), 50, 12),
    "free_fall3d": (lambda: P.free_fall(), 20, 2),
    # spherical
    "wedge3d_monopole_s4": (lambda: P.random_wedge(
        nr=17, nth=15, nph=13, nscalar=4, gravity="point_monopole",
        bc=[["reflective", "transmissive"], ["reflective"] * 2, ["periodic"] * 2]), 30, 4),
    "wedge3d_point_refl": (lambda: P.random_wedge(
        nr=16, nth=9, nph=20, nscalar=1, gravity="point",
        bc=[["reflective"] * 2, ["reflective"] * 2, ["reflective"] * 2]), 30, 7),
    "wedge2d_point": (lambda: P.random_wedge(nr=20, nth=18, ndim=2, nscalar=1, gravity="point",
                                             bc=[["reflective", "transmissive"], ["reflective"] * 2,
                                                 ["periodic"] * 2]), 30, None),
    "sedov_sph1d_100": (lambda: P.sedov_sph1d(100), 100, None),
    "static_wedge": (lambda: P.static_wedge(), 30, 3),
}


# FP32-form tolerance, from its arithmetic: FP32 rounding (6e-8) through one step of ~10^3 operations
# per cell, relative to the value, plus a floor for fields that cancel; momenta are floored on the
# flow's momentum scale (a component that is ~0 everywhere has no scale of its own)
FP32_REL, FP32_ABS = 2e-5, 2e-6


@pytest.mark.parametrize("name", list(CASES))
def test_fp64_parity_small(H, name):
    make, nsteps, kz = CASES[name]
    prob = make()
    announce(f"fp64 parity {name} n={prob.n} nvar={prob.nvar} steps={nsteps} kz={kz}")
    Ug, Uo = run_pair(H, prob, nsteps, zchunk=kz)
    assert_parity(Ug, Uo, what=name)
    print(f"{name}: max relative difference {max_rel(Ug, Uo):.3e}")


@pytest.mark.parametrize("name", list(CASES))
def test_fp32_form_parity_small(H, name):
    """The FP32 form on every small case (each dimension, geometry, boundary type, limiter,
    Riemann solver, gravity mode and field count, so every FP32 instantiation the cases reach),
    20 steps at most with the oracle's time steps, at the FP32-form bar against the FP64 oracle; its
    own time step agrees with the oracle's to FP32 rounding."""
    make, nsteps, kz = CASES[name]
    prob = make()
    nsteps = min(nsteps, 20)
    announce(f"fp32 form parity {name} n={prob.n} nvar={prob.nvar} steps={nsteps} kz={kz}")
    o = O.Oracle(prob)
    s = H.Solver(prob, precision="fp32", zchunk=kz)
    U = prob.U0.copy()
    s.set_state(U)
    for n in range(nsteps):
        dt, st = o.compute_dt(U)
        assert st == 0
        if n in (0, nsteps - 1):
            assert s.compute_dt() == pytest.approx(dt, rel=1e-5), n
        U, st = o.step(U, dt)
        assert st == 0
        s.step(dt)
    G = s.state_numpy()
    s.check()
    s.close()
    assert_parity(G, U, rel=FP32_REL, absf=FP32_ABS, what=f"fp32 {name}", flow_scale=True)
    print(f"{name} fp32: largest difference {tol_ratio(G, U, FP32_REL, FP32_ABS, True):.3f} of the bar")


def test_fp64_parity_full_size_sedov_sampled(H):
    """Sedov 256^3 in the benchmark's launch configuration: the first step on sampled boxes (the
    blast centre, random interior boxes, tile and chunk seams, the domain corners)."""
    prob = P.sedov3d(n=256)
    announce("fp64 full-size sedov 256^3 first step")
    o = O.Oracle(prob)
    U0 = prob.U0
    dt, st = o.compute_dt(U0)
    s = H.Solver(prob)
    s.set_state(U0)
    dtg = s.compute_dt()
    assert dtg == pytest.approx(dt, rel=1e-14, abs=0)
    s.step(dt)
    Ug = s.state_numpy()
    s.close()
    rng = np.random.default_rng(0)
    boxes = [((124, 124, 124), (132, 132, 132)), ((0, 0, 0), (3, 3, 3)), ((253, 253, 253), (256, 256, 256)),
             ((12, 12, 30), (17, 17, 34)), ((138, 26, 62), (142, 30, 66))]
    for _ in range(6):
        lo = rng.integers(0, 252, size=3)
        boxes.append((tuple(int(v) for v in lo), tuple(int(v) + 4 for v in lo)))
    for lo, hi in boxes:
        ob, st = o.step_box(U0, dt, lo, hi)
        gb = Ug[:, lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]]
        assert_parity(gb, ob, what=f"sedov256 box {lo}-{hi}")


def test_fp64_parity_full_size_sedov_200_steps(H):
    """Sedov 256^3 in the benchmark's launch configuration, 200 steps (the workload's length) on
    both sides, every cell compared at the FP64 bar after 100 and after 200 steps, and every time
    step equal to the oracle's.  The oracle advances only the box around the blast (every other
    cell keeps the ambient state exactly; pinned against whole-grid steps in the CPU tests)."""
    from parity import BoxedRun
    prob = P.sedov3d(n=256)
    announce("fp64 full-size sedov 256^3, 200 steps, every cell")
    lib = O.OMP_LIB_PATH if os.path.exists(O.OMP_LIB_PATH) else O.LIB_PATH
    run = BoxedRun(O.Oracle(prob, library=lib), prob.U0.copy())
    s = H.Solver(prob)
    s.set_state(prob.U0)
    for n in range(1, 201):
        dt, st = run.compute_dt()
        assert st == 0
        assert s.compute_dt() == dt, f"step {n}"
        assert run.step(dt) == 0
        s.step(dt)
        if n in (100, 200):
            Ug = s.state_numpy()
            assert_parity(Ug, run.U, what=f"sedov256 after {n} steps")
            lo, hi = run.box
            print(f"sedov 256^3 step {n}: blast box {lo}-{hi}, max relative difference "
                  f"{max_rel(Ug, run.U):.3e}")
            del Ug
    s.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_dt_and_totals_match_oracle(H, precision):
    """Time step, conserved totals and enclosed masses against the oracle; the FP32 form's totals
    and enclosed masses are FP64 sums of its (exactly widened) FP32 state, so they match the
    oracle's on the FP32-rounded state to FP64 summation order, and its time step matches to FP32
    rounding."""
    prob = P.random_wedge(nr=21, nth=11, nph=9, nscalar=2, gravity="point_monopole",
                          bc=[["reflective", "transmissive"], ["reflective"] * 2, ["periodic"] * 2])
    announce(f"dt/totals/enclosed-mass parity {precision}")
    U0 = prob.U0 if precision == "fp64" else prob.U0.astype(np.float32).astype(np.float64)
    o = O.Oracle(prob)
    s = H.Solver(prob, precision=precision)
    s.set_state(prob.U0)
    dt, _ = o.compute_dt(U0)
    if precision == "fp64":
        assert s.compute_dt() == dt
    else:
        assert s.compute_dt() == pytest.approx(dt, rel=1e-5)
    tg = s.totals()
    to = o.totals(U0)
    assert np.allclose(tg, to, rtol=1e-13, atol=0)
    s.step(dt)
    s.check()
    me = s.enclosed_mass()
    mo = o.enclosed_mass(U0)
    assert np.allclose(me, mo, rtol=1e-13)
    s.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_nonphysical_state_reported(H, precision):
    """A negative density is reported by the time step and a NaN by the check after a step, in
    either form; a fresh valid state clears the report."""
    prob = P.random_periodic(n=(20, 18, 9), ndim=3, nscalar=1)
    announce(f"non-physical state report {precision}")
    U = prob.U0.copy()
    U[0, 3, 4, 5] = -1.0
    s = H.Solver(prob, precision=precision)
    s.set_state(U)
    with pytest.raises(H.NonPhysicalState):
        s.compute_dt()
    # a fresh valid state clears the report
    s.set_state(prob.U0)
    assert s.compute_dt() > 0
    U = prob.U0.copy()
    U[4, 1, 2, 3] = np.nan
    s.set_state(U)
    s.step(1e-4)
    with pytest.raises(H.NonPhysicalState):
        s.check()
    s.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32", "learned"])
def test_checkpoint_resume_bitwise(H, precision):
    """A state fetched mid-run and loaded into a fresh context continues with the same bits."""
    learned_form = precision == "learned"
    prob = P.random_periodic(n=(23, 19, 17), ndim=3, nscalar=2, seed=3,
                             **(dict(limiter="mlp", ng=3, precision="fp32") if learned_form else {}))
    w = None
    if learned_form:
        from paper_2503_04428_amd import learned
        try:
            w = learned.load_weights()
        except OSError:
            w = np.random.default_rng(6).normal(scale=0.4, size=O.MLP_NPARAM).astype(np.float32)
        precision = "fp32"
    announce(f"checkpoint/resume {precision}{' learned' if learned_form else ''}")

    def solver():
        x = H.Solver(prob, precision=precision)
        if w is not None:
            x.set_mlp(w)
        return x

    a = solver()
    a.set_state(prob.U0)
    a.advance(10)
    ref = a.state_numpy()
    b = solver()
    b.set_state(prob.U0)
    b.advance(5)
    mid = b.get_state()
    c = solver()
    c.set_state(mid)
    c.advance(5)
    assert np.array_equal(c.state_numpy(), ref)
    for x in (a, b, c):
        x.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_device_dt_loop_equals_host_dt_loop(H, precision):
    """The time step kept on the device (hx_compute_dt_device + hx_step_device) gives the same bits
    as the host loop of hx_compute_dt + hx_step."""
    prob = P.sedov3d(n=32)
    announce(f"device-dt loop {precision}")
    a = H.Solver(prob, precision=precision)
    a.set_state(prob.U0)
    for _ in range(12):
        a.step(a.compute_dt())
    b = H.Solver(prob, precision=precision)
    b.set_state(prob.U0)
    b.advance(12)
    assert np.array_equal(a.state_numpy(), b.state_numpy())


@pytest.mark.parametrize("form", ["fp64", "fp32", "learned"])
def test_zchunk_does_not_change_results(H, form):
    """Every form gives the same bits whatever the z planes per workgroup (each cell's arithmetic
    does not depend on the launch layout)."""
    kw = dict(limiter="mlp", ng=3) if form == "learned" else {}
    prob = P.random_periodic(n=(18, 17, 29), ndim=3, nscalar=1, seed=9,
                             precision="fp64" if form == "fp64" else "fp32",
                             bc=[["reflective"] * 2, ["transmissive"] * 2, ["reflective"] * 2], **kw)
    w = None
    if form == "learned":
        from paper_2503_04428_amd import learned
        try:
            w = learned.load_weights()
        except OSError:
            w = np.random.default_rng(5).normal(scale=0.4, size=O.MLP_NPARAM).astype(np.float32)
    announce(f"z-chunk invariance, {form}")
    outs = []
    for kz in (1, 3, 29, 64):
        s = H.Solver(prob, zchunk=kz)
        if w is not None:
            s.set_mlp(w)
        s.set_state(prob.U0)
        for _ in range(5):
            s.step(2e-3)
        outs.append(s.state_numpy())
        s.close()
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])


# ---------------------------------------------------------------------------- full-size workloads

def _sampled_first_step(H, prob, precision, boxes, rel, absf, weights=None, oracle_weights=None, flow_scale=False):
    o = O.Oracle(prob, mlp_weights=oracle_weights)
    U0 = prob.U0
    dt, st = o.compute_dt(U0)
    assert st == 0
    s = H.Solver(prob, precision=precision)
    if weights is not None:
        s.set_mlp(weights)
    s.set_state(U0)
    s.step(dt)
    Ug = s.state_numpy()
    s.close()
    worst = 0.0
    for lo, hi in boxes:
        ob, st = o.step_box(U0, dt, lo, hi)
        gb = Ug[:, lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]]
        assert_parity(gb, ob, rel=rel, absf=absf, what=f"{prob.name} {precision} box {lo}-{hi}",
                      flow_scale=flow_scale)
        worst = max(worst, max_rel(gb, ob))
    return worst


def _boxes(n, centre, rng, k=5, size=4):
    out = [(tuple(max(0, c - 3) for c in centre), tuple(min(n[d], centre[d] + 3) for d in range(3))),
           ((0, 0, 0), (min(3, n[0]), min(3, n[1]), min(3, n[2]))),
           (tuple(n[d] - min(3, n[d]) for d in range(3)), tuple(n))]
    for _ in range(k):
        lo = [int(rng.integers(0, n[d] - size + 1)) for d in range(3)]
        out.append((tuple(lo), tuple(lo[d] + size for d in range(3))))
    return out


def test_full_size_sedov_fp32_form_200_steps(H):
    """The FP32 form on the headline workload (Sedov 256^3 in the benchmark's launch configuration):
    200 steps with the oracle's time steps against the oracle's boxed run, every cell at the
    FP32-form bar and each field's L1 within 1e-5 of the oracle's, and the form's own time step
    within 1e-5 of the oracle's at the first and the last step."""
    from parity import BoxedRun
    prob = P.sedov3d(n=256)
    announce("fp32 form, full-size sedov 256^3, 200 steps, every cell")
    lib = O.OMP_LIB_PATH if os.path.exists(O.OMP_LIB_PATH) else O.LIB_PATH
    run = BoxedRun(O.Oracle(prob, library=lib), prob.U0.copy())
    s = H.Solver(prob, precision="fp32")
    s.set_state(prob.U0)
    for n in range(1, 201):
        dt, st = run.compute_dt()
        assert st == 0
        if n in (1, 200):
            assert s.compute_dt() == pytest.approx(dt, rel=1e-5), n
        assert run.step(dt) == 0
        s.step(dt)
    G = s.state_numpy()
    s.check()
    s.close()
    U = run.U
    assert_parity(G, U, rel=FP32_REL, absf=FP32_ABS, what="sedov256 fp32 after 200 steps", flow_scale=True)
    nv = U.shape[0]
    l1 = np.abs(G - U).reshape(nv, -1).sum(axis=1) / np.abs(U).reshape(nv, -1).sum(axis=1)
    print(f"sedov 256^3 fp32, 200 steps: L1 relative per field {l1}, largest difference "
          f"{tol_ratio(G, U, FP32_REL, FP32_ABS, True):.3f} of the bar")
    assert np.all(l1 < 1e-5)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_full_size_rt_sampled(H, precision):
    prob = P.rt3d()
    announce(f"full-size RT 128x128x512 {precision} first step")
    rng = np.random.default_rng(1)
    rel, absf = (1e-12, 1e-14) if precision == "fp64" else (FP32_REL, FP32_ABS)
    w = _sampled_first_step(H, prob, precision, _boxes(prob.n, (64, 64, 256), rng) +
                            [((60, 60, 0), (68, 68, 3)), ((0, 60, 508), (4, 68, 512))], rel, absf,
                            flow_scale=precision == "fp32")
    print(f"RT {precision}: max relative difference on samples {w:.3e}")


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_full_size_wedge_sampled(H, precision):
    prob = P.wedge3d()
    announce(f"full-size wedge 1024x128x128 {precision} first step")
    rng = np.random.default_rng(2)
    rel, absf = (1e-12, 1e-14) if precision == "fp64" else (FP32_REL, FP32_ABS)
    w = _sampled_first_step(H, prob, precision, _boxes(prob.n, (18, 64, 64), rng) +
                            [((0, 0, 60), (4, 4, 64)), ((1020, 124, 124), (1024, 128, 128))], rel, absf,
                            flow_scale=precision == "fp32")
    print(f"wedge {precision}: max relative difference on samples {w:.3e}")


def test_full_size_learned_sampled(H):
    """Learned form at 256^3 with the trained network: BF16 inference vs the FP64 oracle network
    (BF16-rounded parameters) on sampled boxes around the quadrant interfaces."""
    from paper_2503_04428_amd import learned
    try:
        w = learned.load_weights()
    except OSError:
        pytest.skip("no trained weights")
    prob = P.quadrant3d(n=256, limiter="mlp", precision="fp32")
    announce("full-size learned 256^3 first step")
    rng = np.random.default_rng(3)
    boxes = [((124, 124, 0), (132, 132, 4)), ((125, 30, 100), (131, 36, 104)), ((30, 125, 7), (36, 131, 11))]
    boxes += _boxes(prob.n, (128, 128, 128), rng, k=3)
    # BF16 inference perturbs phi by ~1e-3, which moves the slopes of monotone stencils by that
    # relative amount; one step carries ~dt/dx of it into the state
    _sampled_first_step(H, prob, "fp32", boxes, 2e-3, 2e-4, weights=w, oracle_weights=O.bf16_round(w),
                        flow_scale=True)


# ---------------------------------------------------------------------------- FP32 form accuracy

def test_fp32_form_accuracy_sod_and_sedov(H):
    """FP32 form: L1 error against the FP64 oracle and against the exact Sod solution (reported;
    the FP32 error must be far below the discretisation error)."""
    from oracle import exact
    announce("fp32 form accuracy")
    pr = P.sod(1024)
    o = O.Oracle(pr)
    Uo, t, steps, dts = o.run(pr.U0.copy(), t_end=0.2)
    s = H.Solver(pr, precision="fp32")
    s.set_state(pr.U0)
    for dt in dts:
        s.step(dt)
    Ug = s.state_numpy()
    f = pr.faces[0][pr.ng:pr.ng + 1025]
    r, u, p = exact.cell_average(1.0, 0.0, 1.0, 0.125, 0.0, 0.1, f, 0.5, 0.2, sub=16)
    e_fp32_oracle = np.abs(Ug[0, 0, 0] - Uo[0, 0, 0]).mean()
    e_oracle_exact = np.abs(Uo[0, 0, 0] - r).mean()
    e_fp32_exact = np.abs(Ug[0, 0, 0] - r).mean()
    print(f"Sod 1024 rho L1: fp32-vs-oracle {e_fp32_oracle:.3e}, oracle-vs-exact {e_oracle_exact:.3e}, "
          f"fp32-vs-exact {e_fp32_exact:.3e}")
    assert e_fp32_oracle < 1e-2 * e_oracle_exact
    assert abs(e_fp32_exact - e_oracle_exact) < 1e-2 * e_oracle_exact
    # Sedov: FP32 vs FP64 oracle after 100 steps at 32^3
    pr = P.sedov3d(n=32)
    o = O.Oracle(pr)
    Uo, t, steps, dts = o.run(pr.U0.copy(), nsteps=100)
    s = H.Solver(pr, precision="fp32")
    s.set_state(pr.U0)
    for dt in dts:
        s.step(dt)
    Ug = s.state_numpy()
    rel = np.abs(Ug - Uo).reshape(7, -1).mean(axis=1) / np.maximum(np.abs(Uo).reshape(7, -1).mean(axis=1), 1e-300)
    print("Sedov 32^3 100 steps, fp32 form L1 relative error per field:", rel)
    assert np.all(rel[[0, 4, 5, 6]] < 1e-4)


def test_fp64_parity_beyond_32bit_offsets(H):
    """A 704^3 random state with 7 fields (2.44e9 values per state, beyond 32-bit element offsets;
    19.5 GB per FP64 state): the first step on sampled boxes, including the far corner whose last
    field sits above 2^31 elements, against the oracle.  The time step is fixed (the signal speed
    is below 5 cells per unit time here), so the oracle only evaluates the boxes."""
    import torch
    n = 704
    prob = P.random_periodic(n=(n, n, n), ndim=3, nscalar=2, seed=71)
    assert prob.nvar * prob.ncells > 2 ** 31
    announce("fp64 704^3 random periodic first step (64-bit offsets)")
    o = O.Oracle(prob)
    U0 = prob.U0
    dt = 0.05 / n
    s = H.Solver(prob)
    s.set_state(U0)
    s.step(dt)
    G = s.get_state()
    s.stream.synchronize()
    rng = np.random.default_rng(3)
    boxes = [((n - 4, n - 4, n - 4), (n, n, n)), ((0, 0, 0), (4, 4, 4)), ((0, n - 3, n - 5), (5, n, n)),
             ((348, 350, 352), (353, 355, 357))]
    for _ in range(4):
        lo = rng.integers(0, n - 4, size=3)
        boxes.append((tuple(int(v) for v in lo), tuple(int(v) + 4 for v in lo)))
    for lo, hi in boxes:
        ob, st = o.step_box(U0, dt, lo, hi)
        assert st == 0
        gb = G[:, lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]].cpu().numpy()
        assert_parity(gb, ob, what=f"704^3 box {lo}-{hi}")
    del G
    s.close()
    torch.cuda.empty_cache()


def test_run_to_t_end(H):
    """Sod to t = 0.2 with the last step clipped: the same step sequence and final time as the
    oracle's run, the state to the FP64 bar."""
    prob = P.sod(n=400)
    announce("run to t_end (Sod 400)")
    Uo, to, no, _ = O.Oracle(prob).run(prob.U0.copy(), t_end=0.2)
    s = H.Solver(prob)
    s.set_state(prob.U0)
    t, n = s.run(t_end=0.2)
    G = s.state_numpy()
    s.close()
    assert n == no and t == to and abs(t - 0.2) < 1e-15
    assert_parity(G, Uo, what="sod run to t_end")


def test_fp32_form_high_mach_advected_flow(H):
    """FP32 form on a smooth flow advected at Mach ~250 (internal energy 6e-5 of the total): the
    FP64 energy recovery (taken wherever the kinetic energy dominates) keeps every pressure
    positive and the positivity test (exact sign for the FP32 face states) takes no cell to first
    order, as in the FP64 oracle; conserved fields at the FP32-form bar, pressure within the
    resolution of an FP32 total energy (|dE| / e ~ 6e-8 E / e)."""
    prob = P.random_periodic(n=(20, 18, 16), ndim=3, nscalar=2, seed=41, precision="fp32")
    U0 = prob.U0.copy()
    boost = (240.0, 80.0, 40.0)
    for d in range(3):
        U0[4] = U0[4] + U0[1 + d] * boost[d] + 0.5 * U0[0] * boost[d] ** 2
        U0[1 + d] = U0[1 + d] + U0[0] * boost[d]
    U0 = U0.astype(np.float32).astype(np.float64)
    prob = prob.with_(U0=U0)
    announce("fp32 form, high-Mach advected flow")
    o = O.Oracle(prob)
    s = H.Solver(prob, precision="fp32", zchunk=4)
    s.set_state(U0)
    U = U0.copy()
    for _ in range(10):
        dt, st = o.compute_dt(U)
        assert st == 0
        U, fb, st = o.step_fallback(U, dt)
        assert st == 0 and not fb.any()
        s.step(dt)
    G = s.state_numpy()
    s.check()
    s.close()
    assert_parity(G, U, rel=FP32_REL, absf=FP32_ABS, what="fp32 high mach", flow_scale=True)
    pg = 0.4 * (G[4] - 0.5 * (G[1] ** 2 + G[2] ** 2 + G[3] ** 2) / G[0])
    po = 0.4 * (U[4] - 0.5 * (U[1] ** 2 + U[2] ** 2 + U[3] ** 2) / U[0])
    ratio = float(np.max(U[4] / (po / 0.4)))
    assert ratio > 1e4
    assert np.all(pg > 0)
    assert np.max(np.abs(pg - po) / po) < 50 * 6e-8 * ratio, np.max(np.abs(pg - po) / po)
    print(f"fp32 high Mach: E/e up to {ratio:.3g}, max relative pressure difference "
          f"{np.max(np.abs(pg - po) / po):.3e}")


def test_fp32_form_mixed_mach_shear_flow(H):
    """FP32 form on a shear flow whose Mach number runs from 0 to about 12 across the grid, so
    that in the same waves some cells recover the internal energy in FP32 and others (kinetic
    energy above 3/4 of E) take the FP64 island: conserved fields at the FP32-form bar against the
    FP64 oracle after 10 steps, every pressure positive and within the resolution of an FP32 total
    energy of the oracle's."""
    prob = P.random_periodic(n=(24, 20, 12), ndim=3, nscalar=1, seed=43, precision="fp32")
    U0 = prob.U0.copy()
    nz, ny, nx = U0.shape[1:]
    y = (np.arange(ny) + 0.5) / ny
    ux = 12.0 * np.sin(2 * np.pi * y)[None, :, None] * np.ones((nz, ny, nx))
    U0[4] = U0[4] + U0[1] * ux + 0.5 * U0[0] * ux ** 2
    U0[1] = U0[1] + U0[0] * ux
    U0 = U0.astype(np.float32).astype(np.float64)
    prob = prob.with_(U0=U0)
    ke = 0.5 * (U0[1] ** 2 + U0[2] ** 2 + U0[3] ** 2) / U0[0]
    island = ke > 0.75 * U0[4]
    assert island.any() and (~island).any()
    announce("fp32 form, mixed-Mach shear flow")
    o = O.Oracle(prob)
    s = H.Solver(prob, precision="fp32", zchunk=3)
    s.set_state(U0)
    U = U0.copy()
    for _ in range(10):
        dt, st = o.compute_dt(U)
        assert st == 0
        U, st = o.step(U, dt)
        assert st == 0
        s.step(dt)
    G = s.state_numpy()
    s.check()
    s.close()
    assert_parity(G, U, rel=FP32_REL, absf=FP32_ABS, what="fp32 mixed mach", flow_scale=True)
    pg = 0.4 * (G[4] - 0.5 * (G[1] ** 2 + G[2] ** 2 + G[3] ** 2) / G[0])
    po = 0.4 * (U[4] - 0.5 * (U[1] ** 2 + U[2] ** 2 + U[3] ** 2) / U[0])
    ratio = U[4] / (po / 0.4)
    assert np.all(pg > 0)
    rel = np.abs(pg - po) / po
    assert np.all(rel < 50 * 6e-8 * ratio + 1e-4), float(np.max(rel / (50 * 6e-8 * ratio + 1e-4)))
    print(f"fp32 mixed Mach: {island.mean():.0%} of the cells start in the FP64 island, E/e up to "
          f"{ratio.max():.3g}, max relative pressure difference {rel.max():.3e}")
