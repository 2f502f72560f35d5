"""Host-side checks of the benchmark script (no GPU): it refuses more than one GPU before touching a
device, and the committed records it reads (algorithmic flops per zone-cycle, measured HBM bytes
per launch) parse to the values the profiles state."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


@pytest.mark.parametrize("n", [2, 8])
def test_more_than_one_gpu_is_refused(n):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", str(n)],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""  # no JSON line


def test_flop_records():
    sedov = bench.recorded_flops("sweep_sedov256_flops.md")
    rad = bench.recorded_flops("sweep_sedov_gas_rad_flops.md")
    sn = bench.recorded_flops("sweep_sn_wedge_flops.md")
    # the ideal-gas count is the oracle's own work on the first Sedov step; the EoS workloads add
    # temperature solves, and the SN configuration the monitor, heating and spherical sources
    assert 800 < sedov < 1200
    assert sedov < rad < sn
    assert bench.recorded_flops("no_such_record.md") is None


def test_traffic_record():
    """The record's bytes exceed the algorithmic bytes of a launch (U read and written once): the
    counters see every byte the kernel moves, halo re-reads included."""
    path = os.path.join(ROOT, "profiles", "sweep_sedov256_hbm_traffic.md")
    rec = None
    for line in open(path):
        if "TRAFFIC_JSON" in line:
            rec = json.loads(line.split("TRAFFIC_JSON", 1)[1])
    assert rec is not None and len(rec["source_hash"]) == 16
    cells, nvar = 256 ** 3, 7
    assert rec["fp64_bytes"] > 2 * nvar * 8 * cells
    assert rec["fp32_bytes"] > 2 * nvar * 4 * cells
    # bench.py reports them only while the kernel sources are the ones the counters were taken on
    from paper_2503_04428_amd.srchash import kernel_source_hash
    expect = rec["fp64_bytes"] if rec["source_hash"] == kernel_source_hash() else None
    assert bench.recorded_traffic("fp64") == expect


def test_source_hash_does_not_depend_on_the_tree_location(tmp_path):
    """The hash that ties the traffic record to the kernel sources must be the same wherever the
    repository sits (the bench runs from another path than the one the record was written in)."""
    import shutil
    import subprocess
    import sys

    from paper_2503_04428_amd.srchash import kernel_source_hash

    pkg = os.path.join(ROOT, "paper_2503_04428_amd")
    dst = tmp_path / "elsewhere"
    dst.mkdir()
    shutil.copytree(pkg, dst / "paper_2503_04428_amd",
                    ignore=shutil.ignore_patterns("_build*", "*.so", "__pycache__"))
    out = subprocess.run([sys.executable, "-c",
                          "from paper_2503_04428_amd.srchash import kernel_source_hash as k; print(k())"],
                         cwd=dst, capture_output=True, text=True, check=True).stdout.strip()
    assert out == kernel_source_hash()
