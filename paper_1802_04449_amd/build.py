"""Build step: compile the HIP library libktmi.so for gfx950 (in-tree).

The stencil passes are compiled per (pass, arithmetic type) from
csrc/ktmi_stencil.hip, in parallel with the host file, the network kernels and
the freeze-out surface finder, and the spectra kernels, then linked into one shared library.  Objects go to
_build/ next to this file.
"""
from __future__ import annotations

import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

_HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(_HERE)
CSRC = os.path.join(_HERE, "csrc")
OBJDIR = os.path.join(_HERE, "_build")
LIB = os.path.join(_HERE, "libktmi.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"),
]
NUM_PASSES = 11  # first estimate, stage1 (viscous, ideal), stage2 pi, stage2 T (viscous, ideal),
#                 stage1 viscous and stage2 pi with the lambda_1 term, stage1 / stage2 pi /
#                 stage2 T with bulk pressure and baryon density


def _jobs():
    jobs = [("ktmi", os.path.join(CSRC, "ktmi.hip"), []),
            ("ktmi_mlp", os.path.join(CSRC, "ktmi_mlp.hip"), []),
            ("ktmi_surface", os.path.join(CSRC, "ktmi_surface.hip"), []),
            ("ktmi_spectra", os.path.join(CSRC, "ktmi_spectra.hip"), [])]
    for p in range(NUM_PASSES):
        for rt, tag in (("double", "f64"), ("float", "f32")):
            jobs.append((f"stencil_p{p}_{tag}", os.path.join(CSRC, "ktmi_stencil.hip"),
                         [f"-DKTMI_PASS={p}", f"-DKTMI_RT={rt}",
                          f"-DKTMI_LAUNCH_FN=launch_pass{p}_{tag}"]))
    return jobs


def build(verbose: bool = False, extra=(), workers: int | None = None) -> str:
    os.makedirs(OBJDIR, exist_ok=True)
    workers = workers or max(1, min(16, os.cpu_count() or 1))

    def compile_one(job):
        name, src, defs = job
        obj = os.path.join(OBJDIR, name + ".o")
        cmd = [HIPCC] + FLAGS + list(extra) + defs + ["-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"compiling {name} failed:\n{r.stderr}")
        return obj

    with ThreadPoolExecutor(max_workers=workers) as ex:
        objs = list(ex.map(compile_one, _jobs()))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
