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


if __name__ == "__main__":
    print(build())
    sys.exit(0)
