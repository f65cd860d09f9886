"""Build step of the CPU oracle (test infrastructure): gcc, FP64, no contraction."""
from __future__ import annotations

import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["hydro_oracle.c", "mlp_oracle.c", "surface_oracle.c", "spectra_oracle.c"]


def build(verbose: bool = False) -> str:
    out = os.path.join(_HERE, "liboracle.so")
    srcs = [os.path.join(_HERE, s) for s in SOURCES if os.path.exists(os.path.join(_HERE, s))]
    tmp = out + ".tmp"
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
           "-std=c11", "-D_DEFAULT_SOURCE", "-Wall", "-o", tmp] + srcs + ["-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
