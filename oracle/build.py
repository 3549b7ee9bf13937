"""Build the CPU oracle (test infrastructure) into oracle/liboracle.so.

Plain gcc, -O2 -ffp-contract=off (no fusing beyond the explicit fma()
calls of the branch), no -ffast-math, OpenMP for the column-chunked form.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
SOURCES = ["gpp_oracle.c", "gpp_oracle_ld.c"]
CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11",
          "-fPIC", "-shared", "-fopenmp", "-Wall", "-Wextra"]


def build(verbose: bool = False) -> str:
    srcs = [os.path.join(HERE, s) for s in SOURCES]
    tmp = LIB + ".tmp"
    cmd = ["gcc", *CFLAGS, "-o", tmp, *srcs, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


def is_stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(os.path.join(HERE, s)) > t for s in SOURCES)


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
