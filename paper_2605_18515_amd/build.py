"""Build libcbspmv.so in-tree for gfx950.

    python -m paper_2605_18515_amd.build

Host converter (C++17, g++), HIP kernels and the C ABI (hipcc for gfx950,
packed-FP32 instructions disabled, hardware FP atomics), linked into
paper_2605_18515_amd/libcbspmv.so next to this file.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
SRC = os.path.join(PKG, "csrc")
INC = os.path.join(ROOT, "include")
OUT = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libcbspmv.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

HIP_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-munsafe-fp-atomics",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result", "-I", INC, "-I", SRC,
]
CXX_FLAGS = ["-O3", "-std=c++17", "-fPIC", "-pthread", "-Wall", "-Wextra", "-Wno-unused-parameter", "-I", INC,
             "-I", SRC]


def _run(cmd: list[str]) -> None:
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("build step failed:\n" + " ".join(cmd) + "\n" + r.stdout + r.stderr)


def build(verbose: bool = False) -> str:
    os.makedirs(OUT, exist_ok=True)
    jobs = [
        ["g++", *CXX_FLAGS, "-c", os.path.join(SRC, "convert.cpp"), "-o", os.path.join(OUT, "convert.o")],
        [HIPCC, *HIP_FLAGS, "-c", os.path.join(SRC, "capi.cpp"), "-o", os.path.join(OUT, "capi.o")],
        [HIPCC, *HIP_FLAGS, "-c", os.path.join(SRC, "kernels.hip"), "-o", os.path.join(OUT, "kernels.o")],
        [HIPCC, *HIP_FLAGS, "-c", os.path.join(SRC, "solver.hip"), "-o", os.path.join(OUT, "solver.o")],
        [HIPCC, *HIP_FLAGS, "-c", os.path.join(SRC, "serve.hip"), "-o", os.path.join(OUT, "serve.o")],
        [HIPCC, *HIP_FLAGS, "-c", os.path.join(SRC, "tune.hip"), "-o", os.path.join(OUT, "tune.o")],
    ]
    with ThreadPoolExecutor(max_workers=len(jobs)) as ex:
        for f in [ex.submit(_run, j) for j in jobs]:
            f.result()
    tmp = LIB + ".tmp"
    _run([HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-pthread", "-o", tmp,
          os.path.join(OUT, "convert.o"), os.path.join(OUT, "capi.o"), os.path.join(OUT, "kernels.o"),
          os.path.join(OUT, "solver.o"), os.path.join(OUT, "serve.o"), os.path.join(OUT, "tune.o")])
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
