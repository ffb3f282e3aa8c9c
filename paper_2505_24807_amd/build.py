"""Build libseqx.so (HIP for gfx950) in-tree.

    python -m paper_2505_24807_amd.build        # or: python paper_2505_24807_amd/build.py

Every source is compiled with hipcc for gfx950 only, with packed FP32
instructions disabled (-packed-fp32-ops), then linked against rocSOLVER and
rocBLAS.  Objects go to paper_2505_24807_amd/_build/, the library next to this file.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libseqx.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")

SOURCES = ["model.cpp", "integrals.hip", "gemm.hip", "fock.hip", "linalg.hip", "scf.hip", "sigma.hip",
           "davidson.hip", "skinny.hip", "batch.hip", "mlp.hip", "small_dense.hip", "spectrum.hip", "gradient.hip", "abi.cpp"]

CFLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-x", "hip",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-mllvm", "-amdgpu-mfma-vgpr-form",
          "-Wall", "-Wno-unused-function", "-Wno-unused-variable", "-Wno-unused-result",
          f"-I{ROCM}/include", f"-I{os.path.join(HERE, '..', 'include')}"]


def _hipcc() -> str:
    cand = os.path.join(ROCM, "bin", "hipcc")
    return cand if os.path.exists(cand) else "hipcc"


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [_hipcc(), *CFLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    warn = "\n".join(line for line in r.stderr.splitlines() if "packed-fp32-ops" not in line and line.strip())
    if warn.strip():
        sys.stderr.write(warn + "\n")
    return obj


def build(verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = min(len(SOURCES), int(os.environ.get("MAX_JOBS", "8")))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [_hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs,
           f"-L{ROCM}/lib", "-lrocsolver", "-lrocblas", f"-Wl,-rpath,{ROCM}/lib"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build()
