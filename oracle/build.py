"""Build step of the CPU oracle (test infrastructure): gcc, FP64, no contraction.

Two libraries from the same sources: liboracle.so, the oracle the GPU path is
compared with, and liboracle_mut.so (-DORC_MUTANTS), which adds the planted-
mistake switches that only the pins' self-check (tests/test_oracle_mutants.py)
uses.
"""
from __future__ import annotations

import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["hydro_oracle.c", "mlp_oracle.c", "surface_oracle.c", "spectra_oracle.c"]
LIBS = {"liboracle.so": [], "liboracle_mut.so": ["-DORC_MUTANTS"]}


def build(verbose: bool = False) -> str:
    srcs = [os.path.join(_HERE, s) for s in SOURCES if os.path.exists(os.path.join(_HERE, s))]
    for name, extra in LIBS.items():
        out = os.path.join(_HERE, name)
        tmp = out + ".tmp"
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
               "-std=c11", "-D_DEFAULT_SOURCE", "-Wall"] + extra + ["-o", tmp] + srcs + ["-lm"]
        if verbose:
            print(" ".join(cmd))
        subprocess.run(cmd, check=True)
        os.replace(tmp, out)
    return os.path.join(_HERE, "liboracle.so")


if __name__ == "__main__":
    print(build(verbose=True))
