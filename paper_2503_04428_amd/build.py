"""Build libhydro.so (gfx950) in-tree with hipcc.

Each HIP translation unit is compiled separately (no relocatable device code):
  hx_sweep_fp64*.hip FP64 sweep, -ffp-contract=off so its rounding matches the FP64 oracle
  hx_sweep_fp32*.hip FP32-form sweep (contraction allowed)
  (the *_hllc_vl units fix HLLC + van Leer at compile time; the others take them at run time;
   hx_sweep_fp32_mlp.hip is the learned-limiter form, hx_sweep_fp64_de.hip the FP64 sweep with the
   internal-energy monitor, hx_sweep_fp64_rad.hip the FP64 sweep with the gas + radiation EoS,
   hx_sweep_fp64_de_rad.hip both; hx_sweep_fp64_3d_ilp.hip the 3D one-wave-per-SIMD FP64 sweeps
   built with the ILP machine scheduler)
  hx_reduce.hip      dt / totals / enclosed-mass reductions, -ffp-contract=off
  hx_shift.hip       grid shift along axis 0 (conservative remap), -ffp-contract=off
  hx_mlp.hip         learned limiter: BF16-MFMA evaluation, training samples, FP32 training
  hx_run1d_fp64.hip  persistent one-workgroup run of a 1D problem to t_end, -ffp-contract=off
  hx_run1d_fp32.hip  the same for the FP32 form (the FP32 sweep's flags)
  hx_arith.hip       the sweeps' FP64 division and square root over arrays (checked against IEEE)
  hx_abi.hip         C ABI host code
Packed FP32 instructions are disabled for all device code.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libhydro.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-I", os.path.join(ROOT, "include"),
          "-I", CSRC, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wno-unused-command-line-argument"]
SCHED_ILP = ["-mllvm", "-amdgpu-sched-strategy=iterative-ilp"]
UNITS = {
    "hx_sweep_fp64.hip": ["-ffp-contract=off"],
    "hx_sweep_fp64_hllc_vl.hip": ["-ffp-contract=off"],
    "hx_sweep_fp64_de.hip": ["-ffp-contract=off"],
    "hx_sweep_fp64_rad.hip": ["-ffp-contract=off"],
    "hx_sweep_fp64_de_rad.hip": ["-ffp-contract=off"],
    "hx_sweep_fp64_3d_ilp.hip": ["-ffp-contract=off", "-mllvm", "-amdgpu-sched-strategy=iterative-ilp"],
    "hx_sweep_fp32.hip": [],
    "hx_sweep_fp32_hllc_vl.hip": [],
    "hx_sweep_fp32_mlp.hip": [],
    "hx_reduce.hip": ["-ffp-contract=off"],
    "hx_shift.hip": ["-ffp-contract=off"],
    "hx_mlp.hip": ["-ffp-contract=off"],
    "hx_run1d_fp64.hip": ["-ffp-contract=off"],
    "hx_run1d_fp32.hip": [],
    "hx_arith.hip": ["-ffp-contract=off"],
    "hx_abi.hip": ["-ffp-contract=off"],
}


def _compile(src: str, extra: list) -> str:
    obj = os.path.join(BUILD, src.replace(".hip", ".o"))
    # optional extra flags for tuning experiments (e.g. -DHX_MINW_FP64=2)
    tune = os.environ.get("HX_EXTRA_FLAGS", "").split()
    cmd = [HIPCC, *COMMON, *extra, *tune, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and SCHED_ILP[1] in cmd:
        # the ILP scheduler is an optional code-generation choice: without it the unit computes the
        # same results, so a compiler that cannot build it with that scheduler builds it without
        k = cmd.index(SCHED_ILP[1])
        cmd = cmd[:k - 1] + cmd[k + 1:]
        print(f"note: {src} built without {SCHED_ILP[1]} (the compiler failed with it)", file=sys.stderr)
        r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr[-6000:]}")
    return obj


def build(verbose: bool = False, out: str | None = None) -> str:
    global BUILD
    if out is not None:
        BUILD = os.path.join(os.path.dirname(os.path.abspath(out)), "_build_" + os.path.basename(out))
    os.makedirs(BUILD, exist_ok=True)
    jobs = min(len(UNITS), int(os.environ.get("MAX_JOBS", "8")))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda kv: _compile(*kv), UNITS.items()))
    lib = out or LIB
    tmp = lib + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr[-4000:]}")
    os.replace(tmp, lib)
    if verbose:
        print(lib)
    return lib


if __name__ == "__main__":
    build(verbose=True, out=sys.argv[1] if len(sys.argv) > 1 else None)
    sys.exit(0)
