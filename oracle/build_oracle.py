"""Build the plain-C oracle into oracle/liboracle.so (gcc, FP64, no FMA contraction).

TEST INFRASTRUCTURE ONLY.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
CFLAGS = ["-O2", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-Wall"]


def build(openmp: bool = False) -> str:
    src = os.path.join(HERE, "hydro_oracle.c")
    cmd = ["gcc", *CFLAGS, "-o", LIB + ".tmp", src, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


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
