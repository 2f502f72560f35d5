"""Algorithmic floating-point work of one zone-cycle, counted on the oracle (TEST INFRASTRUCTURE).

Runs the op-counting build of the oracle (opcount.cpp: the same C source with a counting FP64
type) for the first step of a workload and writes the per-cell counts to a record under
profiles/, which the benchmark reads as the algorithmic flops of one zone-cycle (add, mul, div
and sqrt count one flop each).

    python -m oracle.count_flops [--n 256] [--out profiles/sweep_sedov256_flops.md]
    python -m oracle.count_flops --workload rad --n 64 --out profiles/sweep_sedov_gas_rad_flops.md
    python -m oracle.count_flops --workload sn --n 64 --out profiles/sweep_sn_wedge_flops.md
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2503_04428_amd import problems as P  # noqa: E402


def count(prob) -> dict:
    o = O.Oracle(prob)
    dt, _ = o.compute_dt(prob.U0)
    t0 = time.perf_counter()
    r = O.opcount_step(prob, prob.U0, dt)
    el = time.perf_counter() - t0
    cells = prob.ncells
    per = {k: r[k] / cells for k in (*O.OPCOUNT_FIELDS, "flops")}
    return {"workload": prob.name, "n": list(prob.n), "nvar": prob.nvar, "limiter": prob.limiter,
            "riemann": prob.riemann, "cells": cells, "seconds": el,
            "per_zone_cycle": {k: round(v, 4) for k, v in per.items()}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--out", default=os.path.join(ROOT, "profiles", "sweep_sedov256_flops.md"))
    ap.add_argument("--workload", default="sedov", choices=["sedov", "rad", "sn"])
    a = ap.parse_args()
    if a.workload == "sedov":
        prob = P.sedov3d(n=a.n)
        title = f"Sedov {a.n}^3 (7 fields, HLLC, van Leer)"
    elif a.workload == "rad":
        prob = P.with_gas_rad(P.sedov3d(n=a.n))
        title = f"Sedov {a.n}^3 with the gas + radiation EoS (7 fields, HLLC, van Leer; R 1, a 30)"
    else:
        prob = P.sn_wedge3d(n_lin=a.n, n_log=a.n, nth=a.n // 4, nph=a.n // 4)
        title = (f"SN wedge {2 * a.n}x{a.n // 4}x{a.n // 4} (gas + radiation EoS, internal-energy monitor, "
                 f"56Ni heating, point mass, minmod, HLLC; 8 fields)")
    rec = count(prob)
    pz = rec["per_zone_cycle"]
    lines = [
        f"# Algorithmic FP64 work per zone-cycle: {title}",
        "",
        "Counted by the op-counting build of the oracle (oracle/opcount.cpp, the oracle's C source",
        "with a counting FP64 type) over the first step of the workload; one flop each for add/sub,",
        "mul, div and sqrt.  Command (repository root):",
        "",
        f"    python -m oracle.count_flops --workload {a.workload} --n {a.n}"
        + ("" if a.workload == "sedov" else f" --out {os.path.relpath(a.out, ROOT)}"),
        "",
        "| add/sub | mul | div | sqrt | flops | comparisons | min/max/abs |",
        "|---|---|---|---|---|---|---|",
        f"| {pz['add']:.2f} | {pz['mul']:.2f} | {pz['div']:.2f} | {pz['sqrt']:.2f} | {pz['flops']:.2f} | "
        f"{pz['cmp']:.2f} | {pz['minmax_abs']:.2f} |",
        "",
        "FLOPS_JSON " + json.dumps(rec),
        "",
    ]
    with open(a.out, "w") as f:
        f.write("\n".join(lines))
    print("\n".join(lines))


if __name__ == "__main__":
    main()
