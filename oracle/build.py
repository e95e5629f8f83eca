"""Build the CPU oracle library (oracle/liboracle.so) with gcc.

TEST INFRASTRUCTURE ONLY: the oracle is the reference the GPU path is checked
against. -ffp-contract=off keeps every single-precision multiply and add of the
decision geometry separately rounded (fused operations appear only where fmaf()
is written), which the bit-exact binning comparison relies on.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["ora_geom32.c", "ora_sh.c", "ora_raster.c", "ora_loss.c"]
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", "-Wall", "-Wno-unused-function", "-o", LIB + ".tmp"]
    cmd += [os.path.join(HERE, s) for s in SOURCES] + ["-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
