"""Hash of the sources and build flags of the fused sweep, to tie recorded hardware-counter results
(HBM traffic per launch) to the kernel code they were taken on: the sweep's headers and units, the
launch-shape header and the flags its units are compiled with."""
import hashlib
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))
SWEEP_HEADERS = ("hx_device.h", "hx_launch.h", "hx_mlp.h", "hx_params.h", "hx_sweep.h", "hx_sweep_inst.h")


def kernel_source_hash() -> str:
    from . import build as B

    h = hashlib.sha256()
    csrc = os.path.join(HERE, "csrc")
    names = sorted(n for n in os.listdir(csrc)
                   if n in SWEEP_HEADERS or (n.startswith("hx_sweep_") and n.endswith(".hip")))
    for name in names:
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode())
            h.update(f.read())
    # the include paths are absolute: hash them relative to the repository root, so that the same
    # sources give the same hash wherever the tree sits
    common = [f.replace(B.ROOT, "<root>") for f in B.COMMON]
    flags = {"common": common, "units": {k: v for k, v in sorted(B.UNITS.items()) if k.startswith("hx_sweep")}}
    h.update(json.dumps(flags, sort_keys=True).encode())
    return h.hexdigest()[:16]


if __name__ == "__main__":
    import sys
    sys.path.insert(0, os.path.dirname(HERE))
    from paper_2503_04428_amd.srchash import kernel_source_hash as k
    print(k())
