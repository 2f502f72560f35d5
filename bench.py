"""Benchmark: zone-cycles/s of the MUSCL-Hancock step on one MI355X.

Workload: 3D Cartesian Sedov blast, 256^3 cells, 7 fields (5 conserved + 2 passive scalars),
HLLC, van Leer, CFL 0.5 -- the plain FP64 path (the headline value) and the FP32 form, each a
sequence of steps; one step = the CFL dt reduction + the fused sweep, with the time step kept on
the device (no host synchronisation inside the timed loop).  Inputs are synthetic and resident in
HBM before the timed region starts.  The learned-limiter form runs on its own workload (2D Riemann
quadrants in a 256^3 box, 5 fields) beside FP32 and FP64 van Leer on the same problem, reported under
forms.learned with its L1 difference from the FP64 van Leer run and the share of stencils where the
network is evaluated.

Prints one JSON line (see the contract in the repository's documentation).  The roofline block
refers to the dominant kernel, the fused sweep: algorithmic bytes per launch = 2 * nvar * b * cells
(U^n read once, U^{n+1} written once), divided by the sweep's average duration measured with HIP
events on the stream it runs on; roofline.traffic is the measured HBM bytes per launch (rocprofv3
FETCH_SIZE + WRITE_SIZE, calibrated on a plain copy, recorded in profiles/) over the same duration,
reported only while the kernel sources match the recorded ones.  The cpu_baseline block times the
FP64 oracle (single-threaded, as it stands) on a bounded slab of the same first step.
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


def run_form(hydro, torch, prob, form, steps, warmup, zchunk, weights=None):
    s = hydro.Solver(prob, precision=form, zchunk=zchunk)
    if weights is not None:
        s.set_mlp(weights)
    s.set_state(prob.U0)
    stream = s.stream
    s.advance(warmup)
    torch.cuda.synchronize()
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
    gpu_ms = t_start.elapsed_time(t_end)
    sweep_ms = [a.elapsed_time(b) for a, b in evs]
    s.check()
    state = s.get_state()
    torch.cuda.synchronize()
    out = {
        "form": form,
        "wall_s": wall,
        "gpu_ms": gpu_ms,
        "ms_per_step": wall * 1e3 / steps,
        "sweep_ms_avg": sum(sweep_ms) / len(sweep_ms),
        "sweep_ms_min": min(sweep_ms),
        "zchunk": s.zchunk(),
        "state": state,
    }
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


def run_learned(hydro, torch, problems, steps, warmup, n, zchunk):
    """Learned-limiter form on the quadrant Riemann workload, beside FP32 and FP64 van Leer."""
    from paper_2503_04428_amd import learned

    try:
        w = learned.load_weights()
    except (OSError, AssertionError) as e:
        log(f"learned form skipped: no trained weights ({e})")
        return None
    base = problems.quadrant3d(n=n, seed=2000, octant=False, precision="fp32", limiter="mlp", ng=3)
    cells = base.ncells
    runs = {}
    for name, lim, prec in [("learned_fp32", "mlp", "fp32"), ("vanleer_fp32", "vanleer", "fp32"),
                            ("vanleer_fp64", "vanleer", "fp64")]:
        pr = base.with_(limiter=lim, precision=prec)
        r = run_form(hydro, torch, pr, prec, steps, warmup, zchunk, weights=w if lim == "mlp" else None)
        log(f"{name}: {r['ms_per_step']:.3f} ms/step, sweep {r['sweep_ms_avg']:.3f} ms, "
            f"{cells * steps / r['wall_s']:.3e} zone-cycles/s, kz {r['zchunk']}")
        runs[name] = r
    ref = runs["vanleer_fp64"]["state"]
    out = {"workload": f"2D Riemann quadrants in a {n}^3 box (5 fields, transmissive, HLLC, CFL 0.5), seed 2000",
           "steps": steps}
    for name, r in runs.items():
        b = 8 if name.endswith("fp64") else 4
        diff = (r["state"] - ref).abs().reshape(5, -1).mean(dim=1) / ref.abs().reshape(5, -1).mean(dim=1)
        out[name] = {"zone_cycles_per_s": cells * steps / r["wall_s"], "ms_per_step": r["ms_per_step"],
                     "sweep_ms": r["sweep_ms_avg"],
                     "sweep_hbm_gbs_algorithmic": 2 * 5 * b * cells / (r["sweep_ms_avg"] * 1e-3) / 1e9,
                     "zchunk": r["zchunk"],
                     "l1_rel_vs_vanleer_fp64_per_field": diff.cpu().numpy().tolist(),
                     "speedup_vs_vanleer_fp64": runs["vanleer_fp64"]["wall_s"] / r["wall_s"]}
    out["monotone_stencil_fraction"] = monotone_fraction(torch, runs["learned_fp32"]["state"][:, :, :, :], 1.4)
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
    """FP64 oracle (single-threaded C, as it stands) on an nx*ny*nz_slab slab of the first step."""
    import numpy as np

    from oracle import oracle as O

    o = O.Oracle(prob)
    dt, _ = o.compute_dt(prob.U0)
    n = prob.n
    nz_slab = min(nz_slab, n[2])
    z0 = n[2] // 2 - nz_slab // 2
    lo, hi = (0, 0, z0), (n[0], n[1], z0 + nz_slab)
    t0 = time.perf_counter()
    _, st = o.step_box(prob.U0, dt, lo, hi)
    el = time.perf_counter() - t0
    cells = n[0] * n[1] * nz_slab
    what = (f"the whole first step of the {n[0]}x{n[1]}x{n[2]} Sedov state" if nz_slab == n[2] else
            f"one step of the {n[0]}x{n[1]}x{nz_slab} central slab of the {n[0]}x{n[1]}x{n[2]} Sedov state")
    return {"value": cells / el, "unit": "zone-cycles/s", "cores": 1, "kind": "oracle",
            "sample": f"{what} ({cells} cells, {el:.1f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=256, help="cells per axis of the Sedov cube")
    ap.add_argument("--workload", default="sedov", choices=["sedov", "rt", "wedge", "sod", "boosted", "rad", "sn"],
                    help="sedov (default, the headline line); rt, wedge, sod, boosted (Sedov in a moving "
                         "medium with the internal-energy monitor, FP64), rad (Sedov with the gas + "
                         "radiation EoS, FP64), sn (spherical wedge in the paper's SN configuration: "
                         "gas + radiation EoS, monitor, 56Ni heating, point mass, hybrid grid; FP64) "
                         "measure the other workloads")
    ap.add_argument("--forms", default="fp64,fp32")
    ap.add_argument("--zchunk", type=int, default=None)
    ap.add_argument("--cpu-slab", type=int, default=256,
                    help="z planes of the oracle's timed slab (0: skip; the default times the whole first step)")
    ap.add_argument("--learned-steps", type=int, default=100,
                    help="timed steps of the learned-limiter comparison (0: skip)")
    ap.add_argument("--learned-n", type=int, default=256)
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

    import numpy as np
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
    if args.workload != "sedov":
        args.cpu_slab = 0
        args.learned_steps = 0
    cells = prob.ncells
    nvar = prob.nvar
    log(f"workload: {wl}, nvar {nvar}, steps {args.steps}, warmup {args.warmup}")

    results = {}
    for form in [f.strip() for f in args.forms.split(",") if f.strip()]:
        r = run_form(hydro, torch, prob, form, args.steps, args.warmup, args.zchunk)
        log(f"{form}: {r['ms_per_step']:.3f} ms/step, sweep {r['sweep_ms_avg']:.3f} ms "
            f"(min {r['sweep_ms_min']:.3f}), {cells * args.steps / r['wall_s']:.3e} zone-cycles/s, kz {r['zchunk']}")
        results[form] = r

    shift_out = None
    if args.workload == "sn":
        shift_out = run_shift(hydro, torch, prob, 20)
        log(f"grid shift: {shift_out['ms_avg']:.3f} ms per call, {shift_out['GB/s']:.0f} GB/s algorithmic")

    learned_out = None
    if args.learned_steps > 0:
        learned_out = run_learned(hydro, torch, problems, args.learned_steps, args.warmup, args.learned_n,
                                  args.zchunk)

    # accuracy of the FP32 form against the FP64 path (same initial state, same number of steps)
    l1 = None
    if "fp64" in results and "fp32" in results:
        a = results["fp64"]["state"]
        b = results["fp32"]["state"]
        diff = (b - a).abs().reshape(nvar, -1).mean(dim=1)
        ref = a.abs().reshape(nvar, -1).mean(dim=1)
        l1 = (diff / ref).cpu().numpy().tolist()
    for r in results.values():
        del r["state"]

    head = results.get("fp64") or next(iter(results.values()))
    rb = 8 if head["form"] == "fp64" else 4
    value = cells * args.steps / head["wall_s"]
    alg_bytes = 2 * nvar * rb * cells
    achieved = alg_bytes / (head["sweep_ms_avg"] * 1e-3) / 1e9
    forms = {}
    for f, r in results.items():
        b = 8 if f == "fp64" else 4
        forms[f] = {
            "zone_cycles_per_s": cells * args.steps / r["wall_s"],
            "ms_per_step": r["ms_per_step"],
            "sweep_ms": r["sweep_ms_avg"],
            "sweep_hbm_gbs_algorithmic": 2 * nvar * b * cells / (r["sweep_ms_avg"] * 1e-3) / 1e9,
            "zchunk": r["zchunk"],
            "speedup_vs_fp64": (results["fp64"]["wall_s"] / r["wall_s"]) if "fp64" in results else None,
        }
    if l1 is not None:
        forms["fp32"]["l1_rel_vs_fp64_per_field"] = l1
    if learned_out is not None:
        forms["learned"] = learned_out

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
        log(f"oracle: {cpu['value']:.3e} zone-cycles/s on 1 core")

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
                   "cells": cells, "nvar": nvar, "form": head["form"], "dt": "CFL, on device every step"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "traffic_bytes_per_launch": traffic_bytes,
                     "kernel": "hx::sweep_kernel (fused MUSCL-Hancock sweep)",
                     "algorithmic_bytes_per_launch": alg_bytes,
                     "alu": alu},
        "cpu_baseline": cpu,
        "forms": forms,
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
