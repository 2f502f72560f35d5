"""Benchmark: zone-cycles/s of the MUSCL-Hancock step on one MI355X.

Workload: 3D Cartesian Sedov blast, 256^3 cells, 7 fields (5 conserved + 2 passive scalars),
HLLC, van Leer, CFL 0.5 -- the plain FP64 path (the headline value) and the FP32 form, each a
sequence of steps; one step = the CFL dt reduction + the fused sweep, with the time step kept on
the device (no host synchronisation inside the timed loop).  Inputs are synthetic and resident in
HBM before the timed region starts.  Every form is timed `repeats` times (default 5) over exactly
`steps` steps after `warmup` steps; the median run is reported.  Beside the headline:
  forms.rt, forms.wedge   RT 128x128x512 and the spherical wedge 1024x128x128, FP64 and FP32, with
                          the FP32 form's L1 against the FP64 path;
  forms.learned           the learned limiter on seeded 2D quadrant and 3D octant Riemann problems
                          in a 256^3 box beside FP32 and FP64 van Leer: timing, and every form's L1
                          at t_end against the FP64 van Leer solution on 512^3 restricted to 256^3;
  accuracy_vs_exact       Sod 1024 at t = 0.2 against the exact Riemann solution and the Sedov
                          shock radius and density profile on 128^3 against the self-similar
                          solution, FP64 and FP32 (exact values from tests/golden).

Prints one JSON line (see the contract in the repository's documentation).  The roofline block
refers to the dominant kernel, the fused sweep: algorithmic bytes per launch = 2 * nvar * b * cells
(U^n read once, U^{n+1} written once), divided by the sweep's average duration measured with HIP
events on the stream it runs on; roofline.traffic is the measured HBM bytes per launch (rocprofv3
FETCH_SIZE + WRITE_SIZE, calibrated on a plain copy, recorded in profiles/) over the same duration,
reported only while the kernel sources match the recorded ones.  The cpu_baseline block times the
FP64 oracle as it stands: its OpenMP build on the whole first step with every host thread, and the
serial build on a central slab (one_core).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# vector peaks: 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA) x 2.4 GHz (FP64), twice that with
# packed FP32
FP64_VECTOR_PEAK_TFLOPS = 78.6
FP32_VECTOR_PEAK_TFLOPS = 157.3


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def run_form(hydro, torch, prob, form, steps, warmup, zchunk, weights=None, repeats=1):
    """`repeats` runs of the same timed loop on one solver: each restarts from the initial state,
    takes `warmup` untimed steps, then exactly `steps` timed steps (compute_dt_device + step_device,
    HIP events around each sweep on the solver's stream, wall clock around the loop bracketed by
    device synchronisations).  Returns the run with the median wall time, every run's wall time,
    and the state after the last run."""
    s = hydro.Solver(prob, precision=form, zchunk=zchunk)
    if weights is not None:
        s.set_mlp(weights)
    stream = s.stream
    runs = []
    for _ in range(max(1, repeats)):
        s.set_state(prob.U0)
        s.advance(warmup)
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        t_start = torch.cuda.Event(enable_timing=True)
        t_end = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        wall0 = time.perf_counter()
        with torch.cuda.stream(stream):
            t_start.record(stream)
            for a, b in evs:
                s.compute_dt_device()
                a.record(stream)
                s.step_device()
                b.record(stream)
            t_end.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - wall0
        sweep_ms = [a.elapsed_time(b) for a, b in evs]
        runs.append({"wall_s": wall, "gpu_ms": t_start.elapsed_time(t_end),
                     "sweep_ms_avg": sum(sweep_ms) / len(sweep_ms), "sweep_ms_min": min(sweep_ms)})
    s.check()
    state = s.get_state()
    torch.cuda.synchronize()
    order = sorted(range(len(runs)), key=lambda i: runs[i]["wall_s"])
    med = runs[order[len(runs) // 2]]
    out = dict(med)
    out.update({"form": form, "ms_per_step": med["wall_s"] * 1e3 / steps, "zchunk": s.zchunk(), "state": state,
                "repeats": len(runs), "wall_s_all": [r["wall_s"] for r in runs],
                "sweep_ms_all": [r["sweep_ms_avg"] for r in runs]})
    s.close()
    return out


def run_shift(hydro, torch, prob, nshift):
    """Grid shifts (moving grid) of the workload's state, alternating +/- half the narrowest radial
    cell; HIP events around each call (the remap kernel and the geometry upload)."""
    import numpy as np

    s = hydro.Solver(prob)
    s.set_state(prob.U0)
    d = 0.5 * float(np.diff(prob.faces[0]).min())
    stream = s.stream
    s.shift_grid(d)
    s.shift_grid(-d)
    ms = []
    for k in range(nshift):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        with torch.cuda.stream(stream):
            a.record(stream)
            s.shift_grid(d if k % 2 == 0 else -d)
            b.record(stream)
        torch.cuda.synchronize()
        ms.append(a.elapsed_time(b))
    s.check()
    s.close()
    avg = sum(ms) / len(ms)
    alg = 2 * prob.nvar * 8 * prob.ncells
    return {"calls": nshift, "ms_avg": avg, "ms_min": min(ms), "algorithmic_bytes": alg,
            "GB/s": alg / (avg * 1e-3) / 1e9, "frac_of_hbm": alg / (avg * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "delta": d}


def monotone_fraction(torch, U, gamma):
    """Share of (cell, axis, primitive) stencils with differences of one sign on both sides, i.e.
    where the learned limiter evaluates its network (interior cells only)."""
    rho = U[0]
    inv = 1.0 / rho
    u = U[1:4] * inv
    p = (gamma - 1.0) * (U[4] - 0.5 * (U[1:4] * u).sum(dim=0))
    W = torch.stack([rho, u[0], u[1], u[2], p])
    tot, hit = 0, 0
    for ax in (1, 2, 3):
        d = torch.diff(W, dim=ax)
        sl = [slice(None)] * 4
        sl[ax] = slice(0, -1)
        dm = d[tuple(sl)]
        sl[ax] = slice(1, None)
        dp = d[tuple(sl)]
        hit += int((dm * dp > 0).sum().item())
        tot += dm.numel()
    return hit / tot


def l1_rel(a, b):
    """Per-field relative L1 distance of device states a and b [nvar, ...]: mean |a - b| / mean |b|."""
    nv = b.shape[0]
    return ((a - b).abs().reshape(nv, -1).mean(dim=1) / b.abs().reshape(nv, -1).mean(dim=1).clamp(min=1e-300)
            ).cpu().numpy().tolist()


def state_at(hydro, prob, t_end, precision=None, weights=None):
    """The library's state at t_end (CFL steps, the last one clipped) on the device, and the step count."""
    s = hydro.Solver(prob, precision=precision)
    if weights is not None:
        s.set_mlp(weights)
    s.set_state(prob.U0)
    _, nsteps = s.run(t_end=t_end)
    U = s.get_state()
    s.stream.synchronize()
    s.check()
    s.close()
    return U, nsteps


LEARNED_FORMS = [("learned_fp32", "mlp", "fp32"), ("vanleer_fp32", "vanleer", "fp32"), ("vanleer_fp64", "vanleer", "fp64")]
LEARNED_SEEDS = [(2000, False), (2001, False), (2002, True), (2003, True)]


def run_learned(hydro, torch, problems, steps, warmup, n, n_ref, zchunk, repeats, accuracy=True):
    """Learned-limiter form on seeded random Riemann problems in a n^3 box (2D quadrant states, split
    at x, y = 1/2, and 3D octant states, split at x, y, z = 1/2; 5 fields, transmissive, HLLC, CFL
    0.5), beside the FP32 and FP64 van Leer paths.  Timing: `steps` timed steps (median of
    `repeats`) on the first quadrant and the first octant seed.  Accuracy: every seed run to its
    t_end = 0.4 / (largest initial signal speed) by the three forms, each compared per field with the
    FP64 van Leer solution on the n_ref^3 grid restricted to n^3 (conserved variables averaged over
    the (n_ref/n)^3 fine cells of each coarse cell)."""
    from paper_2503_04428_amd import learned

    try:
        w = learned.load_weights()
    except (OSError, AssertionError) as e:
        log(f"learned form skipped: no trained weights ({e})")
        return None
    r = n_ref // n
    out = {"workload": (f"random 2D Riemann quadrants and 3D octants in a {n}^3 box (5 fields, transmissive, HLLC, "
                        f"CFL 0.5), seeds {[sd for sd, _ in LEARNED_SEEDS]}"),
           "reference": f"FP64 van Leer on {n_ref}^3, restricted to {n}^3 by averaging {r}^3 cells",
           "timing": {}, "accuracy": []}
    cells = n ** 3
    for seed, octant in LEARNED_SEEDS:
        kind = "octant" if octant else "quadrant"
        base = problems.quadrant3d(n=n, seed=seed, octant=octant, precision="fp32", limiter="mlp", ng=3)
        if steps > 0 and kind not in out["timing"]:
            timing = {}
            for name, lim, prec in LEARNED_FORMS:
                pr = base.with_(limiter=lim, precision=prec)
                rr = run_form(hydro, torch, pr, prec, steps, warmup, zchunk, weights=w if lim == "mlp" else None,
                              repeats=repeats)
                b = 8 if prec == "fp64" else 4
                timing[name] = {"zone_cycles_per_s": cells * steps / rr["wall_s"], "ms_per_step": rr["ms_per_step"],
                                "sweep_ms": rr["sweep_ms_avg"],
                                "sweep_hbm_gbs_algorithmic": 2 * 5 * b * cells / (rr["sweep_ms_avg"] * 1e-3) / 1e9,
                                "zchunk": rr["zchunk"], "repeats": rr["repeats"]}
                if name == "learned_fp32":
                    timing["monotone_stencil_fraction"] = monotone_fraction(torch, rr["state"], 1.4)
                log(f"{kind} seed {seed} {name}: {rr['ms_per_step']:.3f} ms/step, sweep {rr['sweep_ms_avg']:.3f} ms, "
                    f"{cells * steps / rr['wall_s']:.3e} zone-cycles/s, kz {rr['zchunk']}")
                del rr["state"]
            for name, _, _ in LEARNED_FORMS:
                timing[name]["speedup_vs_vanleer_fp64"] = (timing[name]["zone_cycles_per_s"] /
                                                            timing["vanleer_fp64"]["zone_cycles_per_s"])
            timing["steps"] = steps
            timing["seed"] = seed
            out["timing"][kind] = timing
        if not accuracy:
            continue
        t_end = base.t_end
        fine = problems.quadrant3d(n=n_ref, seed=seed, octant=octant, precision="fp64", limiter="vanleer", ng=2)
        Uf, nf = state_at(hydro, fine, t_end)
        del fine
        ref = Uf.reshape(5, n, r, n, r, n, r).mean(dim=(2, 4, 6))
        del Uf
        acc = {"seed": seed, "kind": kind, "t_end": t_end, "reference_steps": nf, "steps": {}, "l1_rel_vs_reference": {}}
        for name, lim, prec in LEARNED_FORMS:
            pr = base.with_(limiter=lim, precision=prec)
            U, ns = state_at(hydro, pr, t_end, precision=prec, weights=w if lim == "mlp" else None)
            acc["steps"][name] = ns
            acc["l1_rel_vs_reference"][name] = l1_rel(U, ref)
            del U
        e = acc["l1_rel_vs_reference"]
        acc["ratio_learned_over_vanleer_fp32"] = [a / b if b > 0 else None for a, b in
                                                  zip(e["learned_fp32"], e["vanleer_fp32"])]
        log(f"{kind} seed {seed}: L1 vs restricted {n_ref}^3 (rho, m, E) learned "
            f"{e['learned_fp32'][0]:.3e} {e['learned_fp32'][1]:.3e} {e['learned_fp32'][4]:.3e}, van Leer FP32 "
            f"{e['vanleer_fp32'][0]:.3e} {e['vanleer_fp32'][1]:.3e} {e['vanleer_fp32'][4]:.3e}")
        out["accuracy"].append(acc)
        del ref
        torch.cuda.empty_cache()
    # geometric mean over the seeds of the learned / van Leer FP32 error ratio, per field
    import math
    gm = []
    for v in range(5 if out["accuracy"] else 0):
        vals = [a["ratio_learned_over_vanleer_fp32"][v] for a in out["accuracy"]
                if a["ratio_learned_over_vanleer_fp32"][v]]
        gm.append(math.exp(sum(math.log(x) for x in vals) / len(vals)) if vals else None)
    out["ratio_learned_over_vanleer_fp32_geomean"] = gm
    return out


def sod_exact(hydro, problems):
    """Sod 1024 (paper App. C.1) to t = 0.2 in FP64 and in the FP32 form, run inside one workgroup
    (hx_run_1d): L1 of (rho, u, P) against the exact solution's cell averages
    (tests/golden/sod1024_exact_t0.2.txt, written from the exact Riemann solver), the FP32 form's
    L1 against the FP64 path, and the zone-cycle rate of that device-side loop beside the host loop
    (hx_compute_dt + hx_step per step), which is bound by launch latency at this size."""
    import numpy as np
    import torch

    ex = np.loadtxt(os.path.join(ROOT, "tests", "golden", "sod1024_exact_t0.2.txt"))
    prob = problems.sod(1024)
    out, prims = {}, {}
    for form in ("fp64", "fp32"):
        s = hydro.Solver(prob, precision=form)
        rates = {}
        for loop in ("host", "host", "device", "device"):  # the second run of each loop is the timed one
            s.set_state(prob.U0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, ns = s.run(t_end=0.2) if loop == "host" else s.run_1d(0.2)
            torch.cuda.synchronize()
            rates[loop] = prob.ncells * ns / (time.perf_counter() - t0)
        U = s.state_numpy().reshape(5, -1)
        s.check()
        s.close()
        rho = U[0]
        u = U[1] / rho
        p = (prob.gamma - 1.0) * (U[4] - 0.5 * U[1] * u)
        prims[form] = np.stack([rho, u, p], axis=1)
        out[form] = {"steps": ns, "l1_vs_exact": np.abs(prims[form] - ex).mean(axis=0).tolist(),
                     "zone_cycles_per_s_one_workgroup_loop": rates["device"],
                     "zone_cycles_per_s_host_loop": rates["host"]}
    out["fp32"]["l1_vs_fp64"] = np.abs(prims["fp32"] - prims["fp64"]).mean(axis=0).tolist()
    out["fields"] = ["rho", "u", "P"]
    out["note"] = "L1 = mean over the 1024 cells of |q - q_exact| (the integral over [0, 1])"
    return out


def sedov_exact(hydro, problems, n=128, t_end=0.16):
    """Sedov blast on n^3 cells of [-1, 1]^3 to t_end (shock radius near 0.5), FP64 and the FP32
    form: the shock radius (peak of the angle-averaged density) against xi0 (E t^2 / rho0)^(1/5)
    (Sect. 4.3, xi0(1.4) from tests/golden/sedov_xi0_gamma1.4.txt), and the density's relative L1
    against the self-similar profile (tests/golden/sedov_profile_gamma1.4.txt)."""
    import numpy as np

    xi0 = float(np.loadtxt(os.path.join(ROOT, "tests", "golden", "sedov_xi0_gamma1.4.txt")))
    prof = np.loadtxt(os.path.join(ROOT, "tests", "golden", "sedov_profile_gamma1.4.txt"))
    prob = problems.sedov3d(n=n)
    E, rho0 = prob.meta["E1"], prob.meta["rho0"]
    R = xi0 * (E * t_end ** 2 / rho0) ** 0.2
    f = prob.faces[0][prob.ng:prob.ng + n + 1]
    xc = 0.5 * (f[1:] + f[:-1])
    Z, Y, X = np.meshgrid(xc, xc, xc, indexing="ij")
    r = np.sqrt(X * X + Y * Y + Z * Z)
    rho_ex = np.where(r < R, rho0 * np.interp(r / R, prof[:, 0], prof[:, 1]), rho0)
    bins = np.linspace(0.0, 1.0, n // 2 + 1)
    idx = np.digitize(r.ravel(), bins)
    out = {"workload": f"sedov3d-{n}^3 to t = {t_end}", "radius_exact": R, "xi0": xi0}
    dens = {}
    for form in ("fp64", "fp32"):
        U, ns = state_at(hydro, prob, t_end, precision=form)
        rho = U[0].cpu().numpy()
        dens[form] = rho
        sums = np.bincount(idx, weights=rho.ravel(), minlength=len(bins) + 1)
        cnt = np.bincount(idx, minlength=len(bins) + 1)
        prof_num = sums[1:len(bins)] / np.maximum(cnt[1:len(bins)], 1)
        r_peak = 0.5 * (bins[:-1] + bins[1:])[int(np.argmax(prof_num))]
        out[form] = {"steps": ns, "shock_radius": r_peak, "radius_rel_error": (r_peak - R) / R,
                     "rho_l1_rel_vs_self_similar": float(np.abs(rho - rho_ex).mean() / np.abs(rho_ex).mean())}
    out["fp32"]["rho_l1_rel_vs_fp64"] = float(np.abs(dens["fp32"] - dens["fp64"]).mean() / np.abs(dens["fp64"]).mean())
    out["note"] = f"radius bins of width {bins[1]:.4f}; cell width {f[1] - f[0]:.4f}"
    return out


def recorded_traffic(form):
    """HBM bytes per sweep launch from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE record, valid
    only while the kernel sources are the ones the counters were taken on (else None)."""
    from paper_2503_04428_amd.srchash import kernel_source_hash

    path = os.path.join(ROOT, "profiles", "sweep_sedov256_hbm_traffic.md")
    try:
        for line in open(path):
            if "TRAFFIC_JSON" in line:
                rec = json.loads(line.split("TRAFFIC_JSON", 1)[1])
                if rec.get("source_hash") != kernel_source_hash():
                    return None
                return rec.get(f"{form}_bytes")
    except OSError:
        return None
    return None


def recorded_flops(name="sweep_sedov256_flops.md"):
    """Algorithmic FP64 flops of one zone-cycle of a workload from its committed op-count record
    (the oracle's own operations, each face flux counted once), or None."""
    path = os.path.join(ROOT, "profiles", name)
    try:
        for line in open(path):
            if line.startswith("FLOPS_JSON"):
                return json.loads(line.split("FLOPS_JSON", 1)[1])["per_zone_cycle"]["flops"]
    except (OSError, KeyError, ValueError):
        return None
    return None


def cpu_baseline(prob, nz_slab):
    """The FP64 oracle as it stands (plain C, no tuning) on the host: the OpenMP build (the same
    source, cell loops shared over z planes, bitwise the serial results) on the whole first step,
    with every thread it starts, and the serial build on a central slab of nz_slab planes."""
    import numpy as np

    from oracle import oracle as O

    n = prob.n
    out = None
    if os.path.exists(O.OMP_LIB_PATH):
        o = O.Oracle(prob, library=O.OMP_LIB_PATH)
        threads = o.num_threads()
        dt, _ = o.compute_dt(prob.U0)
        t0 = time.perf_counter()
        _, st = o.step(prob.U0, dt)
        el = time.perf_counter() - t0
        cells = n[0] * n[1] * n[2]
        out = {"value": cells / el, "unit": "zone-cycles/s", "cores": threads, "kind": "oracle",
               "sample": (f"the whole first step of the {n[0]}x{n[1]}x{n[2]} Sedov state ({cells} cells, {el:.2f} s "
                          f"on {threads} threads, OpenMP build of the oracle)")}
    o1 = O.Oracle(prob)
    dt, _ = o1.compute_dt(prob.U0)
    nz_slab = min(nz_slab, n[2])
    z0 = n[2] // 2 - nz_slab // 2
    lo, hi = (0, 0, z0), (n[0], n[1], z0 + nz_slab)
    t0 = time.perf_counter()
    _, st = o1.step_box(prob.U0, dt, lo, hi)
    el = time.perf_counter() - t0
    cells = n[0] * n[1] * nz_slab
    one = {"value": cells / el, "unit": "zone-cycles/s", "cores": 1, "kind": "oracle",
           "sample": f"one step of the {n[0]}x{n[1]}x{nz_slab} central slab of the Sedov state ({cells} cells, {el:.2f} s)"}
    if out is None:
        return one
    out["one_core"] = one
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--repeats", type=int, default=5, help="timed runs per form; the median is reported")
    ap.add_argument("--n", type=int, default=256, help="cells per axis of the Sedov cube")
    ap.add_argument("--workload", default="sedov", choices=["sedov", "rt", "wedge", "sod", "boosted", "rad", "sn"],
                    help="sedov (default, the headline line with every form and accuracy block); rt, wedge, "
                         "sod, boosted (Sedov in a moving medium with the internal-energy monitor, FP64), rad "
                         "(Sedov with the gas + radiation EoS, FP64), sn (spherical wedge in the paper's SN "
                         "configuration: gas + radiation EoS, monitor, 56Ni heating, point mass, hybrid grid; "
                         "FP64) time that workload alone")
    ap.add_argument("--forms", default="fp64,fp32")
    ap.add_argument("--zchunk", type=int, default=None)
    ap.add_argument("--cpu-slab", type=int, default=32,
                    help="z planes of the serial oracle's timed slab (0: skip the CPU baseline)")
    ap.add_argument("--learned-steps", type=int, default=100,
                    help="timed steps of the learned-limiter comparison (0: skip the learned block)")
    ap.add_argument("--learned-n", type=int, default=256)
    ap.add_argument("--learned-ref", type=int, default=512, help="cells per axis of the learned block's reference")
    ap.add_argument("--learned-timing-only", action="store_true", help="skip the learned block's accuracy runs")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the RT and wedge forms and the accuracy blocks (Sod, Sedov radius)")
    ap.add_argument("--copy-ref-mib", type=int, default=0,
                    help="also run a plain device copy of this many MiB (reference for HBM counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU domain decomposition exists as a design, not as code)", file=sys.stderr)
        sys.exit(2)
    if os.environ.get("WORLD_SIZE", "1") not in ("", "1"):
        print("bench.py runs as a single process on one GPU", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2503_04428_amd import hydro, problems

    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        sys.exit(1)
    hydro.load_library()
    if args.workload == "sedov":
        prob = problems.sedov3d(n=args.n)
        wl = f"sedov3d-{args.n}^3 (5 conserved + 2 passive scalars, HLLC, van Leer, CFL 0.5)"
    elif args.workload == "boosted":
        prob = problems.boosted_sedov3d(n=args.n, eps=1e-3)
        wl = (f"boosted-sedov3d-{args.n}^3 with the internal-energy monitor (periodic, 8 fields, HLLC, "
              f"van Leer, eps 1e-3)")
        args.forms = "fp64"
    elif args.workload == "rad":
        prob = problems.with_gas_rad(problems.sedov3d(n=args.n))
        wl = (f"sedov3d-{args.n}^3 with the gas + radiation EoS (R 1, a 30; 7 fields, HLLC, van Leer, "
              f"CFL 0.5)")
        args.forms = "fp64"
    elif args.workload == "sn":
        prob = problems.sn_wedge3d(n_lin=256, n_log=256, nth=128, nph=128)
        wl = ("sn-wedge 512x128x128 spherical (hybrid linear-log r, gas + radiation EoS, internal-energy "
              "monitor, 56Ni heating, point mass, minmod, HLLC; 8 fields)")
        args.forms = "fp64"
    elif args.workload == "rt":
        prob = problems.rt3d()
        wl = "rt3d-128x128x512 (uniform gravity, 1 scalar, periodic x/y, reflective z, HLLC, van Leer)"
    elif args.workload == "wedge":
        prob = problems.wedge3d()
        wl = "wedge-1024x128x128 spherical (point + enclosed-mass gravity, 4 scalars, HLLC, van Leer)"
    else:
        prob = problems.sod(1024)
        wl = "sod-1024 (1D, HLLC, van Leer, CFL 0.8)"
    headline = args.workload == "sedov"
    if not headline:
        args.cpu_slab = 0
        args.learned_steps = 0
        args.no_extra = True
    cells = prob.ncells
    nvar = prob.nvar
    log(f"workload: {wl}, nvar {nvar}, steps {args.steps}, warmup {args.warmup}, repeats {args.repeats}")

    def summary(r, c, nv, ref_wall=None):
        b = 8 if r["form"] == "fp64" else 4
        return {"zone_cycles_per_s": c * args.steps / r["wall_s"], "ms_per_step": r["ms_per_step"],
                "sweep_ms": r["sweep_ms_avg"], "sweep_ms_min": r["sweep_ms_min"],
                "sweep_hbm_gbs_algorithmic": 2 * nv * b * c / (r["sweep_ms_avg"] * 1e-3) / 1e9,
                "sweep_hbm_frac": 2 * nv * b * c / (r["sweep_ms_avg"] * 1e-3) / 1e9 / HBM_PEAK_GBS,
                "zchunk": r["zchunk"], "repeats": r["repeats"],
                "zone_cycles_per_s_all": [c * args.steps / w for w in r["wall_s_all"]],
                "speedup_vs_fp64": (ref_wall / r["wall_s"]) if ref_wall else None}

    results = {}
    for form in [f.strip() for f in args.forms.split(",") if f.strip()]:
        r = run_form(hydro, torch, prob, form, args.steps, args.warmup, args.zchunk, repeats=args.repeats)
        log(f"{form}: {r['ms_per_step']:.3f} ms/step (median of {r['repeats']}), sweep {r['sweep_ms_avg']:.3f} ms "
            f"(min {r['sweep_ms_min']:.3f}), {cells * args.steps / r['wall_s']:.3e} zone-cycles/s, kz {r['zchunk']}")
        results[form] = r

    shift_out = None
    if args.workload == "sn":
        shift_out = run_shift(hydro, torch, prob, 20)
        log(f"grid shift: {shift_out['ms_avg']:.3f} ms per call, {shift_out['GB/s']:.0f} GB/s algorithmic")

    # accuracy of the FP32 form against the FP64 path (same initial state, same number of steps)
    l1 = None
    if "fp64" in results and "fp32" in results:
        l1 = l1_rel(results["fp32"]["state"], results["fp64"]["state"])
    for r in results.values():
        del r["state"]

    head = results.get("fp64") or next(iter(results.values()))
    rb = 8 if head["form"] == "fp64" else 4
    value = cells * args.steps / head["wall_s"]
    alg_bytes = 2 * nvar * rb * cells
    achieved = alg_bytes / (head["sweep_ms_avg"] * 1e-3) / 1e9
    ref_wall = results["fp64"]["wall_s"] if "fp64" in results else None
    forms = {f: summary(r, cells, nvar, ref_wall) for f, r in results.items()}
    if l1 is not None:
        forms["fp32"]["l1_rel_vs_fp64_per_field"] = l1

    # the other configurations: RT 128x128x512 and the spherical wedge 1024x128x128, FP64 and FP32
    workloads = {}
    if not args.no_extra:
        for key, pr, desc in [
                ("rt", problems.rt3d(), "rt3d-128x128x512 (uniform gravity, 1 scalar, periodic x/y, reflective z)"),
                ("wedge", problems.wedge3d(), "wedge-1024x128x128 spherical (point + enclosed-mass gravity, 4 scalars)")]:
            rs = {}
            for form in ("fp64", "fp32"):
                rs[form] = run_form(hydro, torch, pr, form, args.steps, args.warmup, args.zchunk, repeats=args.repeats)
                log(f"{key} {form}: {rs[form]['ms_per_step']:.3f} ms/step, sweep {rs[form]['sweep_ms_avg']:.3f} ms, "
                    f"{pr.ncells * args.steps / rs[form]['wall_s']:.3e} zone-cycles/s")
            wl_out = {"workload": desc, "cells": pr.ncells, "nvar": pr.nvar, "steps": args.steps}
            for form in ("fp64", "fp32"):
                wl_out[form] = summary(rs[form], pr.ncells, pr.nvar, rs["fp64"]["wall_s"])
            wl_out["fp32"]["l1_rel_vs_fp64_per_field"] = l1_rel(rs["fp32"]["state"], rs["fp64"]["state"])
            workloads[key] = wl_out
            del rs
            torch.cuda.empty_cache()
    if workloads:
        forms["rt"] = workloads["rt"]
        forms["wedge"] = workloads["wedge"]

    learned_out = None
    if args.learned_steps > 0:
        learned_out = run_learned(hydro, torch, problems, args.learned_steps, args.warmup, args.learned_n,
                                  args.learned_ref, args.zchunk, args.repeats,
                                  accuracy=not args.learned_timing_only)
    if learned_out is not None:
        forms["learned"] = learned_out

    accuracy = None
    if not args.no_extra:
        log("accuracy against exact solutions ...")
        accuracy = {"sod": sod_exact(hydro, problems), "sedov": sedov_exact(hydro, problems)}
        log(f"sod L1 rho: fp64 {accuracy['sod']['fp64']['l1_vs_exact'][0]:.3e}, fp32 "
            f"{accuracy['sod']['fp32']['l1_vs_exact'][0]:.3e}; sod fp64 zone-cycles/s one-workgroup loop "
            f"{accuracy['sod']['fp64']['zone_cycles_per_s_one_workgroup_loop']:.3e}, host loop "
            f"{accuracy['sod']['fp64']['zone_cycles_per_s_host_loop']:.3e}; sedov radius error fp64 "
            f"{accuracy['sedov']['fp64']['radius_rel_error']:.3e}")

    if args.copy_ref_mib > 0:
        nb = args.copy_ref_mib * 1024 * 1024
        src = torch.ones(nb // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy reference: {args.copy_ref_mib} MiB read + {args.copy_ref_mib} MiB written")
        del src, dst

    sedov256 = args.n == 256 and args.workload == "sedov"
    traffic_bytes = recorded_traffic(head["form"]) if sedov256 else None
    flops_zc = recorded_flops() if sedov256 else None
    # the EoS sweeps are bound by ALU issue (Newton steps); their headline view is the ALU one
    alu_bound = args.workload in ("rad", "sn")
    if alu_bound:
        flops_zc = recorded_flops({"rad": "sweep_sedov_gas_rad_flops.md", "sn": "sweep_sn_wedge_flops.md"}[args.workload])
    alu = None
    if flops_zc is not None:
        peak = FP64_VECTOR_PEAK_TFLOPS if head["form"] == "fp64" else FP32_VECTOR_PEAK_TFLOPS
        tf = flops_zc * cells / (head["sweep_ms_avg"] * 1e-3) / 1e12
        alu = {"achieved": tf, "peak": peak, "unit": "TFLOP/s", "frac": tf / peak,
               "flops_per_zone_cycle": flops_zc, "algorithmic_flops_per_launch": flops_zc * cells}
    traffic = traffic_bytes / (head["sweep_ms_avg"] * 1e-3) / 1e9 if traffic_bytes else None

    cpu = None
    if args.cpu_slab > 0:
        log("timing the CPU oracle ...")
        cpu = cpu_baseline(prob, args.cpu_slab)
        log(f"oracle: {cpu['value']:.3e} zone-cycles/s on {cpu['cores']} threads")

    line = {
        "metric": "zone-cycles/s on 1 GPU (FP64 vs FP32 vs learned limiter) at stated L1 error",
        "value": value,
        "unit": "zone-cycles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if head["form"] == "fp64" else "f32",
        "data": "synthetic",
        "config": {"workload": wl,
                   "cells": cells, "nvar": nvar, "form": head["form"], "dt": "CFL, on device every step",
                   "repeats": args.repeats, "value_is": "median of the repeats"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "traffic_bytes_per_launch": traffic_bytes,
                     "kernel": "hx::sweep_kernel (fused MUSCL-Hancock sweep)",
                     "algorithmic_bytes_per_launch": alg_bytes,
                     "alu": alu},
        "cpu_baseline": cpu,
        "forms": forms,
        "accuracy_vs_exact": accuracy,
    }
    if alu_bound and alu is not None:
        hbm = dict(line["roofline"])
        hbm.pop("alu")
        line["roofline"] = {"bound": "alu", "achieved": alu["achieved"], "peak": alu["peak"], "unit": "TFLOP/s",
                            "frac": alu["frac"], "traffic": None, "kernel": hbm["kernel"],
                            "flops_per_zone_cycle": alu["flops_per_zone_cycle"],
                            "algorithmic_flops_per_launch": alu["algorithmic_flops_per_launch"], "hbm": hbm}
    if shift_out is not None:
        line["grid_shift"] = shift_out
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
