"""Build the plain-C oracle into oracle/liboracle.so (gcc, FP64, no FMA contraction).

TEST INFRASTRUCTURE ONLY.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
LIB_OMP = os.path.join(HERE, "liboracle_omp.so")
CFLAGS = ["-O2", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-Wall"]


def build(openmp: bool = False) -> str:
    """liboracle.so (serial), or with openmp=True liboracle_omp.so: the same source with its cell
    loops shared over z planes by OpenMP threads (bitwise the same results)."""
    src = os.path.join(HERE, "hydro_oracle.c")
    lib = LIB_OMP if openmp else LIB
    cmd = ["gcc", *CFLAGS, *(["-fopenmp"] if openmp else []), "-o", lib + ".tmp", src, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(lib + ".tmp", lib)
    return lib


def build_opcount() -> str:
    """The oracle compiled as C++ with a counting FP64 type (opcount.cpp): same entry points plus
    or_opcount / or_opcount_reset, same arithmetic."""
    lib = os.path.join(HERE, "liboracle_opcount.so")
    src = os.path.join(HERE, "opcount.cpp")
    flags = [f for f in CFLAGS if not f.startswith("-std=")]
    cmd = ["g++", *flags, "-std=gnu++17", "-I", HERE, "-o", lib + ".tmp", src, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(lib + ".tmp", lib)
    return lib


if __name__ == "__main__":
    print(build())
    sys.exit(0)
