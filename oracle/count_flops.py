"""Algorithmic floating-point work of one zone-cycle, counted on the oracle (TEST INFRASTRUCTURE).

Runs the op-counting build of the oracle (opcount.cpp: the same C source with a counting FP64
type) for the first step of a workload and writes the per-cell counts to a record under
profiles/, which the benchmark reads as the algorithmic flops of one zone-cycle (add, mul, div
and sqrt count one flop each).

    python -m oracle.count_flops [--n 256] [--out profiles/sweep_sedov256_flops.md]
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
    a = ap.parse_args()
    rec = count(P.sedov3d(n=a.n))
    pz = rec["per_zone_cycle"]
    lines = [
        f"# Algorithmic FP64 work per zone-cycle: Sedov {a.n}^3 (7 fields, HLLC, van Leer)",
        "",
        "Counted by the op-counting build of the oracle (oracle/opcount.cpp, the oracle's C source",
        "with a counting FP64 type) over the first step of the workload; one flop each for add/sub,",
        "mul, div and sqrt.  Command (repository root):",
        "",
        f"    python -m oracle.count_flops --n {a.n}",
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
