"""Build step for libabacus_nf.so (gfx950), in-tree next to this file.

``python -m paper_2110_11392_amd.build`` or ``build()`` compiles every HIP
source under ``csrc/`` with hipcc for gfx950 and links the shared library that
the Python binding loads, then builds the plain-C example program
``examples/nbody_step`` against the C ABI alone.  Compilation runs even when a
library already exists.
"""
from __future__ import annotations

import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libabacus_nf.so")
ARCH = "gfx950"
EXAMPLE_SRC = os.path.join(HERE, "examples", "nbody_step.c")
EXAMPLE = os.path.join(HERE, "examples", "nbody_step")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")

SOURCES = ["common.hip", "bin.hip", "plan.hip", "pairs.hip", "pairs64.hip", "vjp.hip", "vjp64.hip",
           "reduce.hip",
           "tune.hip",
           "multipoles.hip", "kdk.hip", "api.hip"]

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # One IEEE rounding per written operation: cell assignment must match the
    # FP64 definition bit for bit, and the pair kernels use explicit fmaf.
    "-ffp-contract=off",
    # No packed FP32 instructions anywhere in this library.
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-command-line-argument",
    f"-I{INCLUDE}", f"-I{CSRC}",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    return "hipcc"


def build(verbose: bool = False) -> str:
    cc = hipcc()
    with tempfile.TemporaryDirectory(prefix="anf_build_") as tmp:
        procs = []
        objs = []
        for src in SOURCES:
            obj = os.path.join(tmp, src.replace(".hip", ".o"))
            cmd = [cc, *HIPCC_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE,
                                                stderr=subprocess.STDOUT, text=True)))
            objs.append(obj)
        failed = []
        for src, p in procs:
            out, _ = p.communicate()
            noise = [ln for ln in out.splitlines() if "packed-fp32-ops" not in ln and ln.strip()]
            if p.returncode != 0:
                failed.append((src, out))
            elif noise and verbose:
                print("\n".join(noise))
        if failed:
            msg = "\n".join(f"--- {s}\n{o}" for s, o in failed)
            raise RuntimeError(f"hipcc failed:\n{msg}")
        tmp_lib = os.path.join(tmp, "libabacus_nf.so")
        cmd = [cc, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp_lib]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
        os.replace(tmp_lib, LIB)
    build_example(verbose)
    return LIB


def build_example(verbose: bool = False) -> str:
    """The C example: plain C99 host code (no HIP kernels of its own), built
    with the system C compiler against include/abacus_nf.h, the library and
    the HIP runtime, with the library found next to it at run time."""
    cmd = [os.environ.get("CC", "gcc"), "-std=c99", "-O2", "-Wall", "-Wextra",
           "-D__HIP_PLATFORM_AMD__", f"-I{INCLUDE}", f"-I{ROCM}/include", EXAMPLE_SRC,
           f"-L{HERE}", "-labacus_nf", f"-L{ROCM}/lib", "-lamdhip64", "-lm",
           "-Wl,-rpath,$ORIGIN/..", f"-Wl,-rpath,{ROCM}/lib", "-o", EXAMPLE + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"example build failed:\n{r.stdout}\n{r.stderr}")
    os.replace(EXAMPLE + ".tmp", EXAMPLE)
    return EXAMPLE


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
