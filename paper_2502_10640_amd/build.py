"""Build the gfx950 shared library ``libpp_hip.so`` from ``csrc/`` with hipcc.

Every HIP source is compiled with packed FP32 instructions disabled
(``-Xclang -target-feature -Xclang -packed-fp32-ops``).  On gfx950 plain FP32
FMA still issues 108 lane operations per clock per CU, 85% of the 128 that the
packed FP32 peak assumes (``bench.py --mode ubench``,
``profiles/valu_issue_rates.md``).
"""
from __future__ import annotations

import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB_PATH = os.path.join(HERE, "libpp_hip.so")
BUILD_DIR = os.path.join(ROOT, "_build")

SOURCES = ["pp_kernels.hip", "pp_sym.hip", "pp_sym64.hip", "pp_sort.hip", "pp_runtime.hip", "pp_noalloc.hip", "pp_fused.hip"]
ARCH = "gfx950"
HIPCC_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wextra",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", INCLUDE, "-I", CSRC,
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the HIP library cannot be built")


def _compile(src: str) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    obj = os.path.join(BUILD_DIR, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc(), *HIPCC_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    """Compile every source and link the shared library; returns its path."""
    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB_PATH + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB_PATH)
    if verbose:
        print("built", LIB_PATH)
    return LIB_PATH


UBENCH_SRC = "pp_ubench.hip"
UBENCH_PATH = os.path.join(HERE, "libpp_ubench.so")


def build_ubench(verbose: bool = False) -> str:
    """The vector-ALU micro-benchmarks (``bench.py --mode ubench``): a library
    of their own, outside the C ABI of include/pp.h."""
    obj = _compile(UBENCH_SRC)
    tmp = UBENCH_PATH + ".tmp"
    r = subprocess.run([hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, obj],
                       capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, UBENCH_PATH)
    if verbose:
        print("built", UBENCH_PATH)
    return UBENCH_PATH


def device_asm(src: str = "pp_kernels.hip") -> str:
    """gfx950 assembly of one source (for inspecting instruction selection)."""
    out = os.path.join(BUILD_DIR, os.path.splitext(src)[0] + ".s")
    os.makedirs(BUILD_DIR, exist_ok=True)
    cmd = [hipcc(), *HIPCC_FLAGS, "--cuda-device-only", "-S", os.path.join(CSRC, src), "-o", out]
    subprocess.run(cmd, check=True, capture_output=True)
    return out


if __name__ == "__main__":
    build(verbose=True)
    build_ubench(verbose=True)
