"""Build the FP64 CPU oracle library (test infrastructure only).

Compiles ``lbm_oracle.c`` with gcc at -O2 and without floating-point contraction, so that every
multiply and add rounds separately, in the order the source states. Test infrastructure only.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbm_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")


def build(force=True):
    """Compile the oracle; returns the path of the shared library.

    Sites are independent within each sweep, so the OpenMP loops over z give bit-identical
    results at any thread count (OMP_NUM_THREADS); global sums stay serial."""
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-std=c11", "-fopenmp", "-Wall", "-Wextra", "-shared",
           "-fPIC",
           "-o", LIB + ".tmp", SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build())
