"""The plain-C example program (paper_2110_11392_amd/examples/nbody_step.c): a
few leapfrog steps through the C ABI alone -- binning, forces with the FP64
momentum sums, the adjoint, kick-drift with the Eq. 1 statistics and the time
step -- built here with the system C compiler against include/abacus_nf.h and
run as its own process.  Its exit status checks every call and that the
momentum residual of every step stays below 1e-5 (pair antisymmetry, Eq. 3)."""
import os
import subprocess
import sys

import pytest

from paper_2110_11392_amd import build as B

pytestmark = pytest.mark.gpu


def test_c_example_runs_through_the_c_abi(tmp_path):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    assert os.path.exists(B.LIB), "libabacus_nf.so is not built"
    exe = str(tmp_path / "nbody_step")
    cmd = [os.environ.get("CC", "gcc"), "-std=c99", "-O2", "-Wall", "-Wextra",
           "-D__HIP_PLATFORM_AMD__", f"-I{B.INCLUDE}", f"-I{B.ROCM}/include", B.EXAMPLE_SRC,
           f"-L{B.HERE}", "-labacus_nf", f"-L{B.ROCM}/lib", "-lamdhip64", "-lm",
           f"-Wl,-rpath,{B.HERE}", f"-Wl,-rpath,{B.ROCM}/lib", "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    print("[example] n=32768 K=8, 3 steps", flush=True)
    sys.stdout.flush()
    r = subprocess.run([exe, "32768", "8", "3"], capture_output=True, text=True, timeout=120)
    print(r.stdout, r.stderr, flush=True)
    assert r.returncode == 0, r.stdout + r.stderr
    lines = r.stdout.strip().splitlines()
    assert lines[-1] == "ok"
    assert sum(ln.startswith("step ") for ln in lines) == 3
